// P2M (leaf moments about cell centres) and its adjoint with respect to the
// particle masses. Both are HBM-bound: one thread per frame cell.
//
//   M_k(j)   = sum_i m_i a_i^k / k!,      a_i = y_i - c_j, c_j = (j + 1/2) h
//   dm_i     = sum_k dM_k(j) a_i^k / k!
//
// The paper approximates each leaf cell by a monopole at its centre (Sec. IV-C,
// "Octo-Tiger"); that is the a = 0 case of these moments.
#include "kernels.h"
#include "p2m_common.h"

namespace fmm {

constexpr int kP2MThreads = 256;
constexpr int kCellBlocks = kNCell / kP2MThreads;   // 54
static_assert(kNCell % kP2MThreads == 0, "cells per block");

// The frame rows (y, z) in [2, 22)^2, all 24 cells of each: they hold the
// reachable window [2, 22)^3, the only cells M2L reads, and whole rows keep
// the stores to M in whole cache lines (a partial line costs more than it
// saves).
__device__ __forceinline__ bool in_window(int cell) {
  const unsigned y = (cell / kFrame) % kFrame - kWin0, z = cell / (kFrame * kFrame) - kWin0;
  return y < (unsigned)kWin && z < (unsigned)kWin;
}

template <int P>
__device__ void p2m_cell(const DevDesc& d, const double* __restrict__ pos,
                         const double* __restrict__ mass, int ppc, double* __restrict__ M,
                         int cell, bool window) {
  constexpr int C = ncomp(P);
  const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
  if (window && !in_window(cell)) return;
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
    const double* y = pos + 3 * (p0 + i);
    p2m_accumulate<P>(mass[p0 + i], y[0] - cx, y[1] - cy, y[2] - cz, acc);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = acc[c];
}

__global__ void __launch_bounds__(kP2MThreads) p2m_kernel(const DevDesc* __restrict__ desc,
                                                          const double* __restrict__ pos,
                                                          const double* __restrict__ mass, int ppc,
                                                          double* __restrict__ M, bool window) {
  const int b = blockIdx.x / kCellBlocks;
  const int cell = (blockIdx.x % kCellBlocks) * kP2MThreads + threadIdx.x;
  const DevDesc d = desc[b];
  switch (d.p) {
    case 2: p2m_cell<2>(d, pos, mass, ppc, M, cell, window); break;
    case 3: p2m_cell<3>(d, pos, mass, ppc, M, cell, window); break;
    case 4: p2m_cell<4>(d, pos, mass, ppc, M, cell, window); break;
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
    dmass[p0 + i] = monomial_dot<P>(g, y[0] - cx, y[1] - cy, y[2] - cz);
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
// registers), blocks of 128 cells. A block's particles are read with coalesced
// 16-byte loads and staged through LDS (cell stride padded to 25 doubles
// against bank conflicts), then each thread works on its own cell from LDS.
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
// WIN: only the window rows' cells are read and written; their z range
// [2, 22) is blocks 9 .. 98 of the 108 blocks of 128 cells
constexpr int kWinBlock0 = (kWin0 * kFrame * kFrame) / 128;                            // 9
constexpr int kWinBlocks = ((kWin0 + kWin) * kFrame * kFrame + 127) / 128 - kWinBlock0;   // 90

// Each workgroup takes K cell blocks (strided by the grid; K = 4 measured best of 4, 8, 16). The coalesced loads
// of the next block are issued into registers before this block's moments are
// computed, so every workgroup keeps loads in flight through its compute and
// store phases (4 workgroups fit a CU by LDS). p = 4 needs those registers for
// its moments and takes one block per workgroup.
template <int P, int K, bool WIN>
__global__ void __launch_bounds__(kT8) p2m8_kernel(const DevDesc* __restrict__ desc,
                                                   const int* __restrict__ ids, int nblocks,
                                                   const double* __restrict__ pos,
                                                   const double* __restrict__ mass,
                                                   double* __restrict__ M) {
  constexpr int C = ncomp(P);
  __shared__ double s_pos[kT8 * kPosStride];
  __shared__ double s_mass[kT8 * kPpc8];
  constexpr int NB = WIN ? kWinBlocks : kCellBlocks8;   // blocks per sub-grid
  constexpr int B0 = WIN ? kWinBlock0 : 0;
  const int tid = threadIdx.x;
  double2 rp[12], rm[4];
  // coalesced loads of block B's positions (12 double2 per thread) and masses (4)
#define P2M8_USE(MASK, C) (cell_present((MASK), (C)) && (!WIN || in_window(C)))
#define P2M8_ISSUE(B)                                                                          \
  {                                                                                            \
    const DevDesc dn = desc[ids[(B) / NB]];                                                    \
    const int c0 = ((B) % NB + B0) * kT8;                                                      \
    const double2* ps = reinterpret_cast<const double2*>(pos + 3 * (dn.part_off + (int64_t)c0 * kPpc8)); \
    const double2* ms = reinterpret_cast<const double2*>(mass + dn.part_off + (int64_t)c0 * kPpc8); \
    _Pragma("unroll") for (int i = 0; i < 12; ++i) {                                           \
      const int v = tid + i * kT8;                                                             \
      rp[i] = P2M8_USE(dn.mask, c0 + v / 12) ? ps[v] : make_double2(0.0, 0.0);                 \
    }                                                                                          \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                            \
      const int v = tid + i * kT8;                                                             \
      rm[i] = P2M8_USE(dn.mask, c0 + v / 4) ? ms[v] : make_double2(0.0, 0.0);                  \
    }                                                                                          \
  }
  int blk = blockIdx.x;
  P2M8_ISSUE(blk);
  for (int k = 0; k < K && blk < nblocks; ++k, blk += gridDim.x) {
    if (k > 0) __syncthreads();   // the previous block's LDS reads are done
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const int v = tid + i * kT8;
      const int c = v / 12, w = v % 12;
      s_pos[c * kPosStride + 2 * w] = rp[i].x;
      s_pos[c * kPosStride + 2 * w + 1] = rp[i].y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = tid + i * kT8;
      s_mass[2 * v] = rm[i].x;
      s_mass[2 * v + 1] = rm[i].y;
    }
    __syncthreads();
    const int nb = blk + (int)gridDim.x;
    if (k + 1 < K && nb < nblocks) P2M8_ISSUE(nb);
    const DevDesc d = desc[ids[blk / NB]];
    const int cell = (blk % NB + B0) * kT8 + tid;
    const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
    double* out = M + d.m_off + cell;
    if (WIN && !in_window(cell)) {
      // outside the window: neither read nor written
    } else if (!block_present(d.mask, jx, jy, jz)) {
#pragma unroll
      for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = 0.0;
    } else {
      const double h = ldexp(1.0, -d.log2_inv_h);
      const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
      double acc[C];
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = 0.0;
      const double* y = s_pos + tid * kPosStride;
#pragma unroll 2
      for (int i = 0; i < kPpc8; ++i)
        p2m_accumulate<P>(s_mass[tid * kPpc8 + i], y[3 * i] - cx, y[3 * i + 1] - cy, y[3 * i + 2] - cz, acc);
#pragma unroll
      for (int c = 0; c < C; ++c) out[(size_t)c * kNCell] = acc[c];
    }
  }
#undef P2M8_ISSUE
#undef P2M8_USE
}

// Adjoint: K cell blocks per workgroup as in the forward; the next block's
// positions and moment gradients are loaded while this block's are used.
template <int P, int K>
__global__ void __launch_bounds__(kT8) p2m8_bwd_kernel(const DevDesc* __restrict__ desc,
                                                       const int* __restrict__ ids, int nblocks,
                                                       const double* __restrict__ pos,
                                                       const double* __restrict__ dM,
                                                       double* __restrict__ dmass) {
  constexpr int C = ncomp(P);
  __shared__ double s_pos[kT8 * kPosStride];
  __shared__ double s_out[kT8 * (kPpc8 + 1)];
  const int tid = threadIdx.x;
  double2 rp[12];
  double rg[C];
  // coalesced loads of block B's positions, and this thread's cell's C gradients
#define P2M8B_ISSUE(B)                                                                         \
  {                                                                                            \
    const DevDesc dn = desc[ids[(B) / kCellBlocks8]];                                          \
    const int c0 = ((B) % kCellBlocks8) * kT8;                                                 \
    const double2* ps = reinterpret_cast<const double2*>(pos + 3 * (dn.part_off + (int64_t)c0 * kPpc8)); \
    _Pragma("unroll") for (int i = 0; i < 12; ++i) {                                           \
      const int v = tid + i * kT8;                                                             \
      rp[i] = cell_present(dn.mask, c0 + v / 12) ? ps[v] : make_double2(0.0, 0.0);             \
    }                                                                                          \
    const bool on_ = cell_present(dn.mask, c0 + tid);                                          \
    const double* gs = dM + dn.m_off + c0 + tid;                                               \
    _Pragma("unroll") for (int c = 0; c < C; ++c) rg[c] = on_ ? gs[(size_t)c * kNCell] : 0.0;  \
  }
  int blk = blockIdx.x;
  P2M8B_ISSUE(blk);
  for (int k = 0; k < K && blk < nblocks; ++k, blk += gridDim.x) {
    if (k > 0) __syncthreads();   // the previous block's LDS reads are done
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const int v = tid + i * kT8;
      const int c = v / 12, w = v % 12;
      s_pos[c * kPosStride + 2 * w] = rp[i].x;
      s_pos[c * kPosStride + 2 * w + 1] = rp[i].y;
    }
    double g[C];
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = rg[c];
    __syncthreads();
    const int nb = blk + (int)gridDim.x;
    if (k + 1 < K && nb < nblocks) P2M8B_ISSUE(nb);
    const DevDesc d = desc[ids[blk / kCellBlocks8]];
    const int cell0 = (blk % kCellBlocks8) * kT8;
    const int cell = cell0 + tid;
    const int jx = cell % kFrame, jy = (cell / kFrame) % kFrame, jz = cell / (kFrame * kFrame);
    if (!block_present(d.mask, jx, jy, jz)) {
#pragma unroll
      for (int i = 0; i < kPpc8; ++i) s_out[tid * (kPpc8 + 1) + i] = 0.0;
    } else {
      const double h = ldexp(1.0, -d.log2_inv_h);
      const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
      const double* y = s_pos + tid * kPosStride;
#pragma unroll 2
      for (int i = 0; i < kPpc8; ++i)
        s_out[tid * (kPpc8 + 1) + i] = monomial_dot<P>(g, y[3 * i] - cx, y[3 * i + 1] - cy, y[3 * i + 2] - cz);
    }
    __syncthreads();
    // coalesced write of the block's 128 x 8 gradients
    double2* dst = reinterpret_cast<double2*>(dmass + d.part_off + (int64_t)cell0 * kPpc8);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = tid + i * kT8;
      const int c = v / 4, w = v % 4;
      dst[v] = make_double2(s_out[c * (kPpc8 + 1) + 2 * w], s_out[c * (kPpc8 + 1) + 2 * w + 1]);
    }
  }
#undef P2M8B_ISSUE
}

// The 8-particle kernels use 16-byte loads: they need 16-byte aligned particle
// arrays (always true for part_off of a whole sub-grid and hipMalloc'd buffers).
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

hipError_t launch_p2m(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids, const int* counts,
                      const double* pos, const double* mass, int ppc, double* M, bool all_aligned,
                      bool window, hipStream_t s) {
  const bool fast = ppc == kPpc8 && all_aligned && aligned16(pos) && aligned16(mass);
  if (fast) {
    // one launch per order present, over that order's sub-grids
    const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks8);
    for (int p = 2; p <= kMaxP; ++p) {
      for (int64_t b0 = 0; b0 < counts[p]; b0 += per_launch) {
        const int64_t n = counts[p] - b0 < per_launch ? counts[p] - b0 : per_launch;
        const int nblocks = (int)(n * (window ? kWinBlocks : kCellBlocks8));
        const dim3 grid4((unsigned)((nblocks + 3) / 4)), grid1((unsigned)nblocks);
        const int* ids = d_ids[p] + b0;
        if (window) {
          if (p == 2) hipLaunchKernelGGL((p2m8_kernel<2, 4, true>), grid4, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
          if (p == 3) hipLaunchKernelGGL((p2m8_kernel<3, 4, true>), grid4, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
          if (p == 4) hipLaunchKernelGGL((p2m8_kernel<4, 1, true>), grid1, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
        } else {
          if (p == 2) hipLaunchKernelGGL((p2m8_kernel<2, 4, false>), grid4, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
          if (p == 3) hipLaunchKernelGGL((p2m8_kernel<3, 4, false>), grid4, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
          if (p == 4) hipLaunchKernelGGL((p2m8_kernel<4, 1, false>), grid1, dim3(kT8), 0, s, d_desc, ids, nblocks, pos, mass, M);
        }
      }
    }
    return hipGetLastError();
  }
  const int64_t per_launch = (int64_t)(0x7fffffff / kCellBlocks);
  for (int64_t b0 = 0; b0 < nsub; b0 += per_launch) {
    const int64_t n = nsub - b0 < per_launch ? nsub - b0 : per_launch;
    hipLaunchKernelGGL(p2m_kernel, dim3((unsigned)(n * kCellBlocks)), dim3(kP2MThreads), 0, s,
                       d_desc + b0, pos, mass, ppc, M, window);
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
        const int nblocks = (int)(n * kCellBlocks8);
        const dim3 grid8((unsigned)((nblocks + 7) / 8)), grid1((unsigned)nblocks);
        if (p == 2) hipLaunchKernelGGL((p2m8_bwd_kernel<2, 8>), grid8, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, nblocks, pos, dM, dmass);
        if (p == 3) hipLaunchKernelGGL((p2m8_bwd_kernel<3, 8>), grid8, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, nblocks, pos, dM, dmass);
        if (p == 4) hipLaunchKernelGGL((p2m8_bwd_kernel<4, 1>), grid1, dim3(kT8), 0, s, d_desc, d_ids[p] + b0, nblocks, pos, dM, dmass);
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
