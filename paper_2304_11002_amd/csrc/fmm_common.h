// Shared definitions of the HIP library (host and device). gfx950 only.
//
// Geometry of one sub-grid (the N = 8 sub-grid of the paper's Octo-Tiger
// subsection, Sec. IV-C): a 24^3 frame of cells, x fastest, linear index
// x + 24 y + 576 z; the 8^3 target block is [8,16)^3; neighbour block of a
// cell is j / 8 per axis with mask bit bx + 3 by + 9 bz. The interaction
// stencil is the shell 5 <= |d|^2 <= 36 (892 offsets), so only the 20^3
// window [2,22)^3 of the frame is ever read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmm.h"

namespace fmm {

constexpr int kFrame = 24;
constexpr int kBlock = 8;
constexpr int kNCell = kFrame * kFrame * kFrame;     // 13824
constexpr int kNTarget = kBlock * kBlock * kBlock;   // 512
constexpr int kWin0 = 2;                             // reachable window [2, 22)
constexpr int kWin = 20;
constexpr int kRad = 6;
constexpr int kNStencil = 892;
constexpr int kMaxP = 4;
constexpr int kMaxOrderD = 2 * kMaxP;                // derivatives up to order 8
constexpr uint32_t kFullMask = (1u << 27) - 1u;
constexpr int kCentreBit = 13;

__host__ __device__ constexpr int ncomp(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Graded multi-index enumeration: order n ascending, then kx descending,
// then ky descending (kz is the remainder). Returns the position of
// (a, b, c) in that list.
__host__ __device__ constexpr int mindex(int a, int b, int c) {
  int n = a + b + c;
  int base = n * (n + 1) * (n + 2) / 6;              // entries of order < n
  // entries of order n with kx > a: sum_{kx=a+1..n} (n - kx + 1)
  int before_x = 0;
  for (int kx = n; kx > a; --kx) before_x += n - kx + 1;
  return base + before_x + (n - a - b);              // ky runs from n-a down to b
}

struct MI { int x, y, z; };

// Inverse of mindex for compile-time loops.
__host__ __device__ constexpr MI mi_of(int idx) {
  int n = 0;
  while ((n + 1) * (n + 2) * (n + 3) / 6 <= idx) ++n;
  int r = idx - n * (n + 1) * (n + 2) / 6;
  for (int kx = n; kx >= 0; --kx) {
    int cnt = n - kx + 1;
    if (r < cnt) return MI{kx, n - kx - r, r};
    r -= cnt;
  }
  return MI{0, 0, 0};
}

// Order |k| of the multi-index at position idx: the number of orders whose
// whole block ends at or before idx (blocks end at ncomp(n) = 1, 4, 10, ...).
// Branch-free for the orders used here (idx < ncomp(9) = 220).
__host__ __device__ constexpr int order_of(int idx) {
  return (idx >= 1) + (idx >= 4) + (idx >= 10) + (idx >= 20) + (idx >= 35) + (idx >= 56) +
         (idx >= 84) + (idx >= 120) + (idx >= 165);
}
static_assert(order_of(0) == 0 && order_of(3) == 1 && order_of(4) == 2 && order_of(19) == 3 &&
                  order_of(20) == 4 && order_of(34) == 4 && order_of(164) == 8 && order_of(165) == 9,
              "order_of");

__host__ __device__ constexpr double inv_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}

// Device copy of one descriptor (same bytes as fmm_subgrid).
struct DevDesc {
  int32_t p;
  int32_t log2_inv_h;
  uint32_t mask;
  int32_t reserved;
  int64_t m_off;
  int64_t l_off;
  int64_t part_off;
};
static_assert(sizeof(DevDesc) == sizeof(fmm_subgrid), "descriptor layout");

__host__ __device__ inline bool block_present(uint32_t mask, int jx, int jy, int jz) {
  int bit = (jx / kBlock) + 3 * (jy / kBlock) + 9 * (jz / kBlock);
  return (mask >> bit) & 1u;
}

}  // namespace fmm
