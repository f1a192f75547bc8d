// Reference M2L kernels on the vector ALU: one thread per output cell, a
// plain loop over the stencil. Slow but simple; kept as the second, independent
// GPU implementation that the matrix-core kernels are checked against, and as
// the fallback selectable with FMM_OPT_M2L_KERNEL = 1.
//
// Forward:  L_n(t) = h^(-1-|n|) sum_{d in S} sum_k [h^-|k| M_k(t + d)] T_d[k][n]
// Adjoint:  dM_k(s) = h^-|k| sum_{e in S} sum_n [h^(-1-|n|) dL_n(s + e)] T_e[n][k]
// The adjoint uses T_{-d} = T_d^T (D_m(-R) = (-1)^|m| D_m(R)), so it is the
// forward operator on dL placed in the target block, evaluated on the frame.
#include "kernels.h"

namespace fmm {

template <int P>
__global__ void __launch_bounds__(256) m2l_ref_fwd_kernel(const DevDesc* __restrict__ desc,
                                                          const int* __restrict__ ids,
                                                          const int* __restrict__ stencil,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ M,
                                                          double* __restrict__ L) {
  constexpr int C = ncomp(P);
  const int b = ids[blockIdx.x / 2];
  const int t = (blockIdx.x % 2) * 256 + threadIdx.x;
  const DevDesc d = desc[b];
  const int jx = t % kBlock + kBlock, jy = (t / kBlock) % kBlock + kBlock, jz = t / 64 + kBlock;
  const int l2 = d.log2_inv_h;
  double acc[C];
#pragma unroll
  for (int n = 0; n < C; ++n) acc[n] = 0.0;
  const double* src = M + d.m_off;
  for (int s = 0; s < kNStencil; ++s) {
    const int sx = jx + stencil[3 * s], sy = jy + stencil[3 * s + 1], sz = jz + stencil[3 * s + 2];
    if (!block_present(d.mask, sx, sy, sz)) continue;
    const int cell = sx + kFrame * sy + kFrame * kFrame * sz;
    double v[C];
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = ldexp(src[(size_t)k * kNCell + cell], l2 * order_of(k));
    const double* Ts = T + (size_t)s * C * C;
#pragma unroll
    for (int k = 0; k < C; ++k)
#pragma unroll
      for (int n = 0; n < C; ++n) acc[n] = __builtin_fma(v[k], Ts[k * C + n], acc[n]);
  }
  double* out = L + d.l_off + t;
#pragma unroll
  for (int n = 0; n < C; ++n) out[(size_t)n * kNTarget] = ldexp(acc[n], l2 * (1 + order_of(n)));
}

template <int P>
__global__ void __launch_bounds__(256) m2l_ref_bwd_kernel(const DevDesc* __restrict__ desc,
                                                          const int* __restrict__ ids,
                                                          const int* __restrict__ stencil,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ dL,
                                                          double* __restrict__ dM) {
  constexpr int C = ncomp(P);
  constexpr int kBlocksPerSub = kNCell / 256;
  const int b = ids[blockIdx.x / kBlocksPerSub];
  const int cell = (blockIdx.x % kBlocksPerSub) * 256 + threadIdx.x;
  const DevDesc d = desc[b];
  const int sx = cell % kFrame, sy = (cell / kFrame) % kFrame, sz = cell / (kFrame * kFrame);
  double* out = dM + d.m_off + cell;
  const bool in_window = sx >= kWin0 && sx < kWin0 + kWin && sy >= kWin0 && sy < kWin0 + kWin &&
                         sz >= kWin0 && sz < kWin0 + kWin;
  if (!in_window || !block_present(d.mask, sx, sy, sz)) {
#pragma unroll
    for (int k = 0; k < C; ++k) out[(size_t)k * kNCell] = 0.0;
    return;
  }
  const int l2 = d.log2_inv_h;
  double acc[C];
#pragma unroll
  for (int k = 0; k < C; ++k) acc[k] = 0.0;
  const double* src = dL + d.l_off;
  for (int e = 0; e < kNStencil; ++e) {
    const int tx = sx + stencil[3 * e] - kBlock, ty = sy + stencil[3 * e + 1] - kBlock,
              tz = sz + stencil[3 * e + 2] - kBlock;
    if ((unsigned)tx >= (unsigned)kBlock || (unsigned)ty >= (unsigned)kBlock ||
        (unsigned)tz >= (unsigned)kBlock)
      continue;
    const int t = tx + kBlock * ty + kBlock * kBlock * tz;
    double w[C];
#pragma unroll
    for (int n = 0; n < C; ++n) w[n] = ldexp(src[(size_t)n * kNTarget + t], l2 * (1 + order_of(n)));
    const double* Te = T + (size_t)e * C * C;
#pragma unroll
    for (int n = 0; n < C; ++n)
#pragma unroll
      for (int k = 0; k < C; ++k) acc[k] = __builtin_fma(w[n], Te[n * C + k], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < C; ++k) out[(size_t)k * kNCell] = ldexp(acc[k], l2 * order_of(k));
}

hipError_t launch_m2l_ref(int p, bool backward, const DevDesc* d_desc, const int* d_ids, int count,
                          const int* d_stencil, const double* d_T, const double* src, double* out,
                          hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!backward) {
    dim3 grid((unsigned)count * 2);
    switch (p) {
      case 2: hipLaunchKernelGGL(m2l_ref_fwd_kernel<2>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      case 3: hipLaunchKernelGGL(m2l_ref_fwd_kernel<3>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      case 4: hipLaunchKernelGGL(m2l_ref_fwd_kernel<4>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    dim3 grid((unsigned)count * (kNCell / 256));
    switch (p) {
      case 2: hipLaunchKernelGGL(m2l_ref_bwd_kernel<2>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      case 3: hipLaunchKernelGGL(m2l_ref_bwd_kernel<3>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      case 4: hipLaunchKernelGGL(m2l_ref_bwd_kernel<4>, grid, dim3(256), 0, s, d_desc, d_ids, d_stencil, d_T, src, out); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace fmm
