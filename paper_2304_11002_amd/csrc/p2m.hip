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

// ---------------------------------------------------------------------------
// 8 particles per cell: one kernel per order (so p = 3 is not held to p = 4's
// registers), 128-cell workgroups. The workgroup's particles are read with
// coalesced 16-byte loads into LDS (cell stride padded to 25 doubles against
// bank conflicts), then each thread works on its own cell from LDS.
// Particles of absent blocks are not read.
// ---------------------------------------------------------------------------

constexpr int kPpc8 = 8;
constexpr int kT8 = 128;                     // cells (threads) per workgroup
constexpr int kCellBlocks8 = kNCell / kT8;   // 108
constexpr int kPosStride = 3 * kPpc8 + 1;    // doubles per cell in LDS
static_assert(kNCell % kT8 == 0, "cells per block");

__device__ __forceinline__ bool cell_present(uint32_t mask, int cell) {
  return block_present(mask, cell % kFrame, (cell / kFrame) % kFrame, cell / (kFrame * kFrame));
}

__device__ __forceinline__ void stage_pos8(const DevDesc& d, const double* __restrict__ pos, int cell0,
                                           double* s_pos) {
  // 128 cells x 24 doubles = 1536 double2, 12 per thread
  const double2* src = reinterpret_cast<const double2*>(pos + 3 * (d.part_off + (int64_t)cell0 * kPpc8));
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int v = threadIdx.x + i * kT8;
    const int c = v / 12, w = v % 12;
    if (cell_present(d.mask, cell0 + c)) {
      const double2 x = src[v];
      s_pos[c * kPosStride + 2 * w] = x.x;
      s_pos[c * kPosStride + 2 * w + 1] = x.y;
    }
  }
}

template <int P>
__global__ void __launch_bounds__(kT8) p2m8_kernel(const DevDesc* __restrict__ desc,
                                                   const int* __restrict__ ids,
                                                   const double* __restrict__ pos,
                                                   const double* __restrict__ mass,
                                                   double* __restrict__ M) {
  constexpr int C = ncomp(P);
  __shared__ double s_pos[kT8 * kPosStride];
  __shared__ double s_mass[kT8 * kPpc8];
  const DevDesc d = desc[ids[blockIdx.x / kCellBlocks8]];
  const int cell0 = (blockIdx.x % kCellBlocks8) * kT8;
  stage_pos8(d, pos, cell0, s_pos);
  const double2* msrc = reinterpret_cast<const double2*>(mass + d.part_off + (int64_t)cell0 * kPpc8);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = threadIdx.x + i * kT8;
    if (cell_present(d.mask, cell0 + v / 4)) {
      const double2 x = msrc[v];
      s_mass[2 * v] = x.x;
      s_mass[2 * v + 1] = x.y;
    }
  }
  __syncthreads();
  const int cell = cell0 + threadIdx.x;
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
  const double* y = s_pos + threadIdx.x * kPosStride;
#pragma unroll 2
  for (int i = 0; i < kPpc8; ++i) {
    const double m = s_mass[threadIdx.x * kPpc8 + i];
    double mono[C];
    monomials<P>(y[3 * i] - cx, y[3 * i + 1] - cy, y[3 * i + 2] - cz, mono);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = __builtin_fma(m, mono[c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = acc[c];
}

template <int P>
__global__ void __launch_bounds__(kT8) p2m8_bwd_kernel(const DevDesc* __restrict__ desc,
                                                       const int* __restrict__ ids,
                                                       const double* __restrict__ pos,
                                                       const double* __restrict__ dM,
                                                       double* __restrict__ dmass) {
  constexpr int C = ncomp(P);
  __shared__ double s_pos[kT8 * kPosStride];
  __shared__ double s_out[kT8 * (kPpc8 + 1)];
  const DevDesc d = desc[ids[blockIdx.x / kCellBlocks8]];
  const int cell0 = (blockIdx.x % kCellBlocks8) * kT8;
  stage_pos8(d, pos, cell0, s_pos);
  __syncthreads();
  const int cell = cell0 + threadIdx.x;
  const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
  if (!block_present(d.mask, jx, jy, jz)) {
#pragma unroll
    for (int i = 0; i < kPpc8; ++i) s_out[threadIdx.x * (kPpc8 + 1) + i] = 0.0;
  } else {
    double g[C];
    const double* src = dM + d.m_off + cell;
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = src[(size_t)c * kNCell];
    const double h = ldexp(1.0, -d.log2_inv_h);
    const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
    const double* y = s_pos + threadIdx.x * kPosStride;
#pragma unroll 2
    for (int i = 0; i < kPpc8; ++i) {
      double mono[C];
      monomials<P>(y[3 * i] - cx, y[3 * i + 1] - cy, y[3 * i + 2] - cz, mono);
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) sum = __builtin_fma(g[c], mono[c], sum);
      s_out[threadIdx.x * (kPpc8 + 1) + i] = sum;
    }
  }
  __syncthreads();
  // coalesced write of the workgroup's 128 x 8 gradients
  double2* dst = reinterpret_cast<double2*>(dmass + d.part_off + (int64_t)cell0 * kPpc8);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = threadIdx.x + i * kT8;
    const int c = v / 4, w = v % 4;
    dst[v] = make_double2(s_out[c * (kPpc8 + 1) + 2 * w], s_out[c * (kPpc8 + 1) + 2 * w + 1]);
  }
}

// The 8-particle kernels use 16-byte loads: they need 16-byte aligned particle
// arrays (always true for part_off of a whole sub-grid and hipMalloc'd buffers).
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

hipError_t launch_p2m(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids, const int* counts,
                      const double* pos, const double* mass, int ppc, double* M, bool all_aligned,
                      hipStream_t s) {
  const bool fast = ppc == kPpc8 && all_aligned && aligned16(pos) && aligned16(mass);
  if (fast) {
    // one launch per order present, over that order's sub-grids
    const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks8);
    for (int p = 2; p <= kMaxP; ++p) {
      for (int64_t b0 = 0; b0 < counts[p]; b0 += per_launch) {
        const int64_t n = counts[p] - b0 < per_launch ? counts[p] - b0 : per_launch;
        const dim3 grid((unsigned)(n * kCellBlocks8));
        if (p == 2) hipLaunchKernelGGL(p2m8_kernel<2>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, mass, M);
        if (p == 3) hipLaunchKernelGGL(p2m8_kernel<3>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, mass, M);
        if (p == 4) hipLaunchKernelGGL(p2m8_kernel<4>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, mass, M);
      }
    }
    return hipGetLastError();
  }
  const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks);
  for (int64_t b0 = 0; b0 < nsub; b0 += per_launch) {
    const int64_t n = nsub - b0 < per_launch ? nsub - b0 : per_launch;
    hipLaunchKernelGGL(p2m_kernel, dim3((unsigned)(n * kCellBlocks)), dim3(kP2MThreads), 0, s,
                       d_desc + b0, pos, mass, ppc, M);
  }
  return hipGetLastError();
}

hipError_t launch_p2m_backward(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids,
                               const int* counts, const double* pos, int ppc, const double* dM,
                               double* dmass, bool all_aligned, hipStream_t s) {
  const bool fast = ppc == kPpc8 && all_aligned && aligned16(pos) && aligned16(dmass);
  if (fast) {
    const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks8);
    for (int p = 2; p <= kMaxP; ++p) {
      for (int64_t b0 = 0; b0 < counts[p]; b0 += per_launch) {
        const int64_t n = counts[p] - b0 < per_launch ? counts[p] - b0 : per_launch;
        const dim3 grid((unsigned)(n * kCellBlocks8));
        if (p == 2) hipLaunchKernelGGL(p2m8_bwd_kernel<2>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, dM, dmass);
        if (p == 3) hipLaunchKernelGGL(p2m8_bwd_kernel<3>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, dM, dmass);
        if (p == 4) hipLaunchKernelGGL(p2m8_bwd_kernel<4>, grid, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, pos, dM, dmass);
      }
    }
    return hipGetLastError();
  }
  const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks);
  for (int64_t b0 = 0; b0 < nsub; b0 += per_launch) {
    const int64_t n = nsub - b0 < per_launch ? nsub - b0 : per_launch;
    hipLaunchKernelGGL(p2m_bwd_kernel, dim3((unsigned)(n * kCellBlocks)), dim3(kP2MThreads), 0, s,
                       d_desc + b0, pos, ppc, dM, dmass);
  }
  return hipGetLastError();
}

}  // namespace fmm
