// Stencil tables: derivatives of 1/r at the stencil offsets, and the
// interaction tensors T_d[k][n] = (-1)^|k| D_{k+n}(-d) at unit spacing.
//
// The derivatives are computed on the host, exactly up to one final rounding:
// D_m = P_m(x, y, z) / r^(2|m|+1) with P_m a homogeneous integer polynomial of
// degree |m| (the quotient rule gives P_0 = 1 and
//   P_{m+e} = r^2 dP_m/dx_e - (2|m| + 1) x_e P_m),
// so at an integer point the numerator P_m(X) is an exact integer and
// D_m = P_m(X) / (r2^|m| sqrt(r2)) is evaluated in 64-bit-mantissa extended
// precision (three roundings of 2^-64 each) and rounded once to float64:
// at most one unit in the last place from the correctly rounded value, for
// every entry, including those that alternating sums would cancel. Spacing h
// enters later as exact powers of two: D_m(h R) = h^(-1-|m|) D_m(R).
#include <cmath>
#include <vector>

#include "kernels.h"

namespace fmm {

namespace {

// Integer numerator polynomials P_m, |m| <= order, each a dense array over the
// exponents (a, b, c) of its degree |m| (position mindex(a, b, c) - ncomp(|m| - 1)).
struct NumeratorTable {
  int order;
  std::vector<std::vector<__int128>> P;   // by mindex(m)
};

NumeratorTable make_numerators(int order) {
  NumeratorTable t{order, std::vector<std::vector<__int128>>(ncomp(order))};
  auto deg_off = [](int n) { return n == 0 ? 0 : ncomp(n - 1); };
  t.P[0] = {1};
  for (int n = 0; n < order; ++n) {
    for (int idx = deg_off(n); idx < ncomp(n); ++idx) {
      const MI m = mi_of(idx);
      const std::vector<__int128>& Pm = t.P[idx];
      for (int e = 0; e < 3; ++e) {
        const int mx[3] = {m.x + (e == 0), m.y + (e == 1), m.z + (e == 2)};
        const int dst = mindex(mx[0], mx[1], mx[2]);
        if (!t.P[dst].empty()) continue;   // built from an earlier axis
        std::vector<__int128> Q((size_t)(ncomp(n + 1) - deg_off(n + 1)), 0);
        for (int j = deg_off(n); j < ncomp(n); ++j) {
          const __int128 c = Pm[(size_t)(j - deg_off(n))];
          if (c == 0) continue;
          const MI a = mi_of(j);
          const int ex[3] = {a.x, a.y, a.z};
          // r^2 dP/dx_e: the term's exponent of x_e drops by one, then + 2 on each axis
          if (ex[e] > 0) {
            for (int q = 0; q < 3; ++q) {
              int ey[3] = {ex[0], ex[1], ex[2]};
              ey[e] -= 1;
              ey[q] += 2;
              Q[(size_t)(mindex(ey[0], ey[1], ey[2]) - deg_off(n + 1))] += c * ex[e];
            }
          }
          // - (2n + 1) x_e P
          int ez[3] = {ex[0], ex[1], ex[2]};
          ez[e] += 1;
          Q[(size_t)(mindex(ez[0], ez[1], ez[2]) - deg_off(n + 1))] -= c * (2 * n + 1);
        }
        t.P[dst] = std::move(Q);
      }
    }
  }
  return t;
}

}  // namespace

std::vector<double> host_derivative_tables(const int* stencil, int ns, int order) {
  static const NumeratorTable num = make_numerators(kMaxOrderD);
  const int nd = ncomp(order);
  std::vector<double> D((size_t)ns * nd);
  auto deg_off = [](int n) { return n == 0 ? 0 : ncomp(n - 1); };
  for (int s = 0; s < ns; ++s) {
    const long long X[3] = {-stencil[3 * s], -stencil[3 * s + 1], -stencil[3 * s + 2]};
    const long long r2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
    // powers of the coordinates up to the order
    __int128 pw[3][kMaxOrderD + 1];
    for (int q = 0; q < 3; ++q) {
      pw[q][0] = 1;
      for (int i = 1; i <= order; ++i) pw[q][i] = pw[q][i - 1] * X[q];
    }
    const long double sq = std::sqrt((long double)r2);
    long double r2n = 1.0L;
    for (int n = 0; n <= order; ++n, r2n *= (long double)r2) {
      for (int idx = deg_off(n); idx < ncomp(n); ++idx) {
        const std::vector<__int128>& Pm = num.P[idx];
        __int128 v = 0;
        for (int j = deg_off(n); j < ncomp(n); ++j) {
          const __int128 c = Pm[(size_t)(j - deg_off(n))];
          if (c == 0) continue;
          const MI a = mi_of(j);
          v += c * pw[0][a.x] * pw[1][a.y] * pw[2][a.z];
        }
        // |v| < 2^63 for |m| <= 8 and |d| <= 6: exact in the 64-bit mantissa
        D[(size_t)s * nd + idx] = (double)((long double)(long long)v / (r2n * sq));
      }
    }
  }
  return D;
}

// T[s][k][n] = (-1)^|k| D_{k+n}(-d_s) for |k|, |n| <= p; D has ncomp(order_d) per offset
__global__ void build_tensors_kernel(const double* __restrict__ D, int ns, int order_d, int p,
                                     double* __restrict__ T) {
  const int C = ncomp(p);
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns * C * C) return;
  int n = i % C;
  int k = (i / C) % C;
  int s = i / (C * C);
  MI mk = mi_of(k), mn = mi_of(n);
  double val = D[(size_t)s * ncomp(order_d) + mindex(mk.x + mn.x, mk.y + mn.y, mk.z + mn.z)];
  T[i] = ((mk.x + mk.y + mk.z) & 1) ? -val : val;
}

hipError_t launch_build_tensors(const double* d_D, int order_d, int p, double* d_T, hipStream_t s) {
  const int C = ncomp(p);
  const int total = kNStencil * C * C;
  hipLaunchKernelGGL(build_tensors_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d_D,
                     kNStencil, order_d, p, d_T);
  return hipGetLastError();
}

}  // namespace fmm
