// P2M (leaf moments about cell centres) and its adjoint with respect to the
// particle masses. Both are HBM-bound: one thread per frame cell.
//
//   M_k(j)   = sum_i m_i a_i^k / k!,      a_i = y_i - c_j, c_j = (j + 1/2) h
//   dm_i     = sum_k dM_k(j) a_i^k / k!
//
// The paper approximates each leaf cell by a monopole at its centre (Sec. IV-C,
// "Octo-Tiger"); that is the a = 0 case of these moments.
#include "kernels.h"

namespace fmm {

constexpr int kP2MThreads = 256;
constexpr int kCellBlocks = kNCell / kP2MThreads;   // 54
static_assert(kNCell % kP2MThreads == 0, "cells per block");

template <int P>
__device__ __forceinline__ void monomials(double ax, double ay, double az, double* out) {
  double px[P + 1], py[P + 1], pz[P + 1];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= P; ++i) {
    px[i] = px[i - 1] * ax;
    py[i] = py[i - 1] * ay;
    pz[i] = pz[i - 1] * az;
  }
#pragma unroll
  for (int c = 0; c < ncomp(P); ++c) {
    const MI k = mi_of(c);
    out[c] = px[k.x] * py[k.y] * pz[k.z] * (inv_fact(k.x) * inv_fact(k.y) * inv_fact(k.z));
  }
}

template <int P>
__device__ void p2m_cell(const DevDesc& d, const double* __restrict__ pos,
                         const double* __restrict__ mass, int ppc, double* __restrict__ M,
                         int cell) {
  constexpr int C = ncomp(P);
  const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
  double* out = M + d.m_off + cell;
  if (!block_present(d.mask, jx, jy, jz)) {
#pragma unroll
    for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = 0.0;
    return;
  }
  const double h = ldexp(1.0, -d.log2_inv_h);
  const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  const int64_t p0 = d.part_off + (int64_t)cell * ppc;
  for (int i = 0; i < ppc; ++i) {
    const double m = mass[p0 + i];
    const double* y = pos + 3 * (p0 + i);
    double mono[C];
    monomials<P>(y[0] - cx, y[1] - cy, y[2] - cz, mono);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = __builtin_fma(m, mono[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = acc[c];
}

__global__ void __launch_bounds__(kP2MThreads) p2m_kernel(const DevDesc* __restrict__ desc,
                                                          const double* __restrict__ pos,
                                                          const double* __restrict__ mass, int ppc,
                                                          double* __restrict__ M) {
  const int b = blockIdx.x / kCellBlocks;
  const int cell = (blockIdx.x % kCellBlocks) * kP2MThreads + threadIdx.x;
  const DevDesc d = desc[b];
  switch (d.p) {
    case 2: p2m_cell<2>(d, pos, mass, ppc, M, cell); break;
    case 3: p2m_cell<3>(d, pos, mass, ppc, M, cell); break;
    case 4: p2m_cell<4>(d, pos, mass, ppc, M, cell); break;
    default: break;
  }
}

template <int P>
__device__ void p2m_bwd_cell(const DevDesc& d, const double* __restrict__ pos, int ppc,
                             const double* __restrict__ dM, double* __restrict__ dmass, int cell) {
  constexpr int C = ncomp(P);
  const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
  const int64_t p0 = d.part_off + (int64_t)cell * ppc;
  if (!block_present(d.mask, jx, jy, jz)) {
    for (int i = 0; i < ppc; ++i) dmass[p0 + i] = 0.0;
    return;
  }
  double g[C];
  const double* src = dM + d.m_off + cell;
#pragma unroll
  for (int c = 0; c < C; ++c) g[c] = src[(size_t)c * kNCell];
  const double h = ldexp(1.0, -d.log2_inv_h);
  const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
  for (int i = 0; i < ppc; ++i) {
    const double* y = pos + 3 * (p0 + i);
    double mono[C];
    monomials<P>(y[0] - cx, y[1] - cy, y[2] - cz, mono);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) s = __builtin_fma(g[c], mono[c], s);
    dmass[p0 + i] = s;
  }
}

__global__ void __launch_bounds__(kP2MThreads) p2m_bwd_kernel(const DevDesc* __restrict__ desc,
                                                              const double* __restrict__ pos, int ppc,
                                                              const double* __restrict__ dM,
                                                              double* __restrict__ dmass) {
  const int b = blockIdx.x / kCellBlocks;
  const int cell = (blockIdx.x % kCellBlocks) * kP2MThreads + threadIdx.x;
  const DevDesc d = desc[b];
  switch (d.p) {
    case 2: p2m_bwd_cell<2>(d, pos, ppc, dM, dmass, cell); break;
    case 3: p2m_bwd_cell<3>(d, pos, ppc, dM, dmass, cell); break;
    case 4: p2m_bwd_cell<4>(d, pos, ppc, dM, dmass, cell); break;
    default: break;
  }
}

hipError_t launch_p2m(const DevDesc* d_desc, int64_t nsub, const double* pos, const double* mass,
                      int ppc, double* M, hipStream_t s) {
  const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks);
  for (int64_t b0 = 0; b0 < nsub; b0 += per_launch) {
    const int64_t n = nsub - b0 < per_launch ? nsub - b0 : per_launch;
    hipLaunchKernelGGL(p2m_kernel, dim3((unsigned)(n * kCellBlocks)), dim3(kP2MThreads), 0, s,
                       d_desc + b0, pos, mass, ppc, M);
  }
  return hipGetLastError();
}

hipError_t launch_p2m_backward(const DevDesc* d_desc, int64_t nsub, const double* pos, int ppc,
                               const double* dM, double* dmass, hipStream_t s) {
  const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks);
  for (int64_t b0 = 0; b0 < nsub; b0 += per_launch) {
    const int64_t n = nsub - b0 < per_launch ? nsub - b0 : per_launch;
    hipLaunchKernelGGL(p2m_bwd_kernel, dim3((unsigned)(n * kCellBlocks)), dim3(kP2MThreads), 0, s,
                       d_desc + b0, pos, ppc, dM, dmass);
  }
  return hipGetLastError();
}

}  // namespace fmm
