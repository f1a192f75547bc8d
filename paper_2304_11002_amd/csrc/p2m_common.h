// Leaf moments of one cell (Sec. IV-C, the leaves of the bottom-up pass of
// Sec. VII-C), shared by the P2M kernels and by the matrix-core kernel that
// computes each sub-grid's moments itself before its M2L.
//
//   M_k(j) = sum_i m_i a_i^k / k!,   a_i = y_i - c_j
#pragma once

#include "fmm_common.h"

namespace fmm {

// sum_c g[c] a^k / k!, in component order, each monomial a^k / k! formed as
// (x^kx y^ky z^kz) / (kx! ky! kz!) and consumed at once
template <int P>
__device__ __forceinline__ double monomial_dot(const double* g, double ax, double ay, double az) {
  double px[P + 1], py[P + 1], pz[P + 1];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= P; ++i) {
    px[i] = px[i - 1] * ax;
    py[i] = py[i - 1] * ay;
    pz[i] = pz[i - 1] * az;
  }
  double sum = 0.0;
#pragma unroll
  for (int c = 0; c < ncomp(P); ++c) {
    const MI k = mi_of(c);
    sum = __builtin_fma(g[c], px[k.x] * py[k.y] * pz[k.z] * (inv_fact(k.x) * inv_fact(k.y) * inv_fact(k.z)), sum);
  }
  return sum;
}

// acc[c - C0] += m a^k / k! for the components c in [C0, C1). The mass and the
// factorials ride on the powers (xm_i = m ax^i / i!, yf_i = ay^i / i!,
// zf_i = az^i / i!), so a component costs one product of an x and a y power
// (shared by every kz) and one fma: 41 operations per particle for all 20
// components at p = 3, against 89 with monomial_dot's monomials. Each
// component's value does not depend on the range it is computed in.
template <int P, int C0 = 0, int C1 = ncomp(P)>
__device__ __forceinline__ void p2m_accumulate(double m, double ax, double ay, double az,
                                               double* acc) {
  constexpr int PO = C1 <= 1 ? 0 : order_of(C1 - 1);   // highest order needed
  double xm[P + 1], yf[P + 1], zf[P + 1];
  xm[0] = m;
  yf[0] = zf[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= PO; ++i) {
    const double inv = 1.0 / i;   // exact for i = 1; folded at compile time
    xm[i] = i == 1 ? xm[0] * ax : xm[i - 1] * (ax * inv);
    yf[i] = i == 1 ? ay : yf[i - 1] * (ay * inv);
    zf[i] = i == 1 ? az : zf[i - 1] * (az * inv);
  }
#pragma unroll
  for (int c = C0; c < C1; ++c) {
    const MI k = mi_of(c);
    const double xy = k.y == 0 ? xm[k.x] : xm[k.x] * yf[k.y];
    acc[c - C0] = k.z == 0 ? acc[c - C0] + xy : __builtin_fma(xy, zf[k.z], acc[c - C0]);
  }
}

// ---------------------------------------------------------------------------
// One 512-thread workgroup computes the moments of a whole sub-grid's frame
// rows (y, z) in [2, 22)^2 (all 24 cells of each row: they hold the reachable
// window, the only cells M2L reads), 8 particles per cell, in steps of half a
// z plane's rows (240 cells, contiguous in memory). A step's particles are
// read with coalesced 16-byte loads and staged through LDS transposed, one row
// of 241 doubles per particle coordinate or mass (so a wave's reads are
// consecutive doubles); two register sets take turns, so the loads of step k + 2 are
// in flight while step k's moments are computed and step k + 1's loads land.
// Each cell is shared by two waves: even waves sum the components of orders
// below p, odd waves those of order p, so a thread holds at most 20 sums and
// two sets of 8 loads (this runs inside a kernel with registers of its own).
// Cells of absent blocks get zero moments and their particles are not read:
// their loads read the always present centre cell instead, and what lands is
// never used. Every vector memory operation of the loop is unconditional, so
// each wait covers exactly the loads it needs and not the set still in flight.
// Needs 16-byte aligned particle blocks (even part_off) and kP2MRowsLds
// doubles of LDS.
// ---------------------------------------------------------------------------
constexpr int kRowsPlane = kWin * kFrame;                          // 480 cells per z plane
constexpr int kRowsStep = kRowsPlane / 2;                          // 240 cells per step
constexpr int kRowsSteps = 2 * kWin;                               // 40
constexpr int kRowsLd = kRowsStep + 1;                             // LDS row: one value per cell
constexpr int kP2MRowsLds = 32 * kRowsLd;                          // 24 coordinate + 8 mass rows
constexpr int kP2MRowsThreads = 512;

template <int P, int C0, int C1>
__device__ __forceinline__ void p2m_rows_cell(const DevDesc& d, double h, const double* s_pos,
                                              const double* s_mass, int lc, int jx, int jy, int jz,
                                              double* M) {
  constexpr int CP = C1 - C0;
  double acc[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) acc[c] = 0.0;
  if (block_present(d.mask, jx, jy, jz)) {
    const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
    const double* y = s_pos + lc;
#pragma unroll 1
    for (int i = 0; i < 8; ++i)
      p2m_accumulate<P, C0, C1>(s_mass[i * kRowsLd + lc], y[(3 * i) * kRowsLd] - cx,
                                y[(3 * i + 1) * kRowsLd] - cy, y[(3 * i + 2) * kRowsLd] - cz, acc);
  }
  double* out = M + d.m_off + jx + kFrame * jy + kFrame * kFrame * jz;
#pragma unroll
  for (int c = 0; c < CP; ++c) out[(size_t)(C0 + c) * kNCell] = acc[c];
}

template <int P>
__device__ __forceinline__ void p2m_window_rows(const DevDesc& d, const double* __restrict__ pos,
                                                const double* __restrict__ mass, double* M,
                                                double* lds) {
  constexpr int NT = kP2MRowsThreads;
  constexpr int NPC = kRowsStep * 12, NMC = kRowsStep * 4;   // 16-byte chunks per step
  constexpr int NP = (NPC + NT - 1) / NT;                    // position loads per thread (6)
  constexpr int NM = (NMC + NT - 1) / NT;                    // mass loads per thread (2)
  static_assert(2 * kRowsStep <= NT && kRowsSteps % 2 == 0, "two threads per cell, steps in pairs");
  double* s_pos = lds;                  // [3 * particle + coordinate][cell]
  double* s_mass = lds + 24 * kRowsLd;  // [particle][cell]
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lc = (wave >> 1) * 64 + (tid & 63);   // this thread's cell in the step
  const bool high = wave & 1;                     // order p (odd waves) or the lower orders
  const double h = ldexp(1.0, -d.log2_inv_h);
  const bool full = d.mask == kFullMask;
  const int centre = kBlock * (1 + kFrame + kFrame * kFrame);   // cell (8, 8, 8)
  const double2* pcentre = reinterpret_cast<const double2*>(pos + 3 * (d.part_off + (int64_t)centre * 8));
  const double2* mcentre = reinterpret_cast<const double2*>(mass + d.part_off + (int64_t)centre * 8);
  // step s: z plane kWin0 + s / 2, its rows' cells [r0, r0 + 240) with r0 = (s % 2) * 240
  auto issue = [&](int step, double2* rp, double2* rm) {
    step = min(step, kRowsSteps - 1);   // past the end: a harmless reload of the last step
    const int z = kWin0 + (step >> 1), r0 = (step & 1) * kRowsStep;
    const int base = z * kFrame * kFrame + kWin0 * kFrame + r0;    // the step's first cell
    const uint32_t pm = (d.mask >> (9 * (z / kBlock))) & 511u;     // the plane's 3 x 3 blocks
    const double2* ps = reinterpret_cast<const double2*>(pos + 3 * (d.part_off + (int64_t)base * 8));
    const double2* ms = reinterpret_cast<const double2*>(mass + d.part_off + (int64_t)base * 8);
    int t = tid;
    asm volatile("" : "+v"(t));   // recomputed per step, not kept live
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int v = t + i * NT, r = r0 + v / 12;
      const bool on = v < NPC && (full || ((pm >> ((r % kFrame) / kBlock + 3 * ((kWin0 + r / kFrame) / kBlock))) & 1u));
      rp[i] = *(on ? ps + v : pcentre);
    }
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      const int v = t + i * NT, r = r0 + v / 4;
      const bool on = v < NMC && (full || ((pm >> ((r % kFrame) / kBlock + 3 * ((kWin0 + r / kFrame) / kBlock))) & 1u));
      rm[i] = *(on ? ms + v : mcentre);
    }
  };
  // step's loads (landed in rp, rm) to LDS, the loads of step + 2 into the same
  // registers, then step's moments
  auto run = [&](int step, double2* rp, double2* rm) {
    __syncthreads();   // earlier readers of the LDS buffer are done
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int v = t + i * NT;
      if (v < NPC) {
        // chunk w of a cell holds its doubles 2w, 2w + 1 (x0 y0 z0 x1 ...): rows 2w, 2w + 1
        double* dst = s_pos + 2 * (v % 12) * kRowsLd + v / 12;
        dst[0] = rp[i].x;
        dst[kRowsLd] = rp[i].y;
      }
    }
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      const int v = t + i * NT;
      if (v < NMC) {
        double* dst = s_mass + 2 * (v % 4) * kRowsLd + v / 4;
        dst[0] = rm[i].x;
        dst[kRowsLd] = rm[i].y;
      }
    }
    __syncthreads();
    issue(step + 2, rp, rm);
    // lanes past the step's 240 cells repeat its last cell (same values, same address)
    const int lcc = min(lc, kRowsStep - 1);
    const int r = (step & 1) * kRowsStep + lcc;
    const int jx = r % kFrame, jy = kWin0 + r / kFrame, jz = kWin0 + (step >> 1);
    constexpr int CL = ncomp(P - 1);
    if (high) p2m_rows_cell<P, CL, ncomp(P)>(d, h, s_pos, s_mass, lcc, jx, jy, jz, M);
    else p2m_rows_cell<P, 0, CL>(d, h, s_pos, s_mass, lcc, jx, jy, jz, M);
  };
  double2 ap[NP], am[NM], bp[NP], bm[NM];
  issue(0, ap, am);
  issue(1, bp, bm);
  for (int step = 0; step < kRowsSteps; step += 2) {
    run(step, ap, am);
    run(step + 1, bp, bm);
  }
}

// ---------------------------------------------------------------------------
// The adjoint of P2M with respect to the masses for one sub-grid, by one
// 512-thread workgroup: dmass_i = sum_k dM_k(j) a_i^k / k!, for dM as the M2L
// adjoint writes it (zero outside the reachable window). Cells outside the
// frame rows (y, z) in [2, 22)^2 get zero gradients without any read; the
// rows go in the same half-plane steps as p2m_window_rows, positions and dM
// staged through LDS in rows of one value per cell, one register set of loads
// in flight during a step's arithmetic. Two threads share a cell, four of its
// particles each. Per particle the sum is monomial_dot<P>, as in the P2M
// adjoint kernels, so the results are the same bits. Particles of absent blocks get 0 and are not
// read. Needs 16-byte aligned particle blocks and kP2MAdjRowsLds doubles of LDS.
// ---------------------------------------------------------------------------
constexpr int kP2MAdjRowsLds = (24 + ncomp(kMaxP)) * kRowsLd;   // 14219 doubles

template <int P>
__device__ __forceinline__ void p2m_adjoint_rows(const DevDesc& d, const double* __restrict__ pos,
                                                 const double* dM, double* __restrict__ dmass,
                                                 double* lds) {
  constexpr int C = ncomp(P);
  constexpr int NT = kP2MRowsThreads;
  constexpr int NPC = kRowsStep * 12;                  // 16-byte position chunks per step
  constexpr int NGC = C * kRowsStep / 2;               // 16-byte dM chunks per step
  constexpr int NP = (NPC + NT - 1) / NT, NG = (NGC + NT - 1) / NT;
  static_assert(2 * kRowsStep <= NT && (24 + C) * kRowsLd <= kP2MAdjRowsLds, "layout");
  double* s_pos = lds;                  // [3 * particle + coordinate][cell]
  double* s_g = lds + 24 * kRowsLd;     // [component][cell]
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lc = (wave >> 1) * 64 + (tid & 63);   // this thread's cell in the step
  const int half = wave & 1;                      // its particles 4 half .. 4 half + 3
  const double h = ldexp(1.0, -d.log2_inv_h);
  const bool full = d.mask == kFullMask;
  double* dm = dmass + d.part_off;
  // zeros for every particle outside the rows: planes z < 2 and z >= 22 whole,
  // and in the others the two rows below and above [2, 22)
  {
    double2* dm2 = reinterpret_cast<double2*>(dm);
    constexpr int kPlane2 = kFrame * kFrame * 4;    // double2 per z plane (8 particles a cell)
    constexpr int kEdge2 = kWin0 * kFrame * 4;      // double2 of two rows
    const double2 z2 = make_double2(0.0, 0.0);
    for (int i = tid; i < kWin0 * kPlane2; i += NT) {
      dm2[i] = z2;
      dm2[(kWin0 + kWin) * kPlane2 + i] = z2;
    }
    for (int i = tid; i < kWin * 2 * kEdge2; i += NT) {
      const int z = kWin0 + i / (2 * kEdge2), k = i % (2 * kEdge2);
      dm2[z * kPlane2 + (k < kEdge2 ? k : kPlane2 - 2 * kEdge2 + k)] = z2;
    }
  }
  const int centre = kBlock * (1 + kFrame + kFrame * kFrame);
  const double2* pcentre = reinterpret_cast<const double2*>(pos + 3 * (d.part_off + (int64_t)centre * 8));
  const double* gsrc = dM + d.m_off;
  double2 rp[NP], rg[NG];
  auto issue = [&](int step) {
    step = min(step, kRowsSteps - 1);   // past the end: a harmless reload of the last step
    const int z = kWin0 + (step >> 1), r0 = (step & 1) * kRowsStep;
    const int base = z * kFrame * kFrame + kWin0 * kFrame + r0;
    const uint32_t pm = (d.mask >> (9 * (z / kBlock))) & 511u;
    const double2* ps = reinterpret_cast<const double2*>(pos + 3 * (d.part_off + (int64_t)base * 8));
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int v = t + i * NT, r = r0 + v / 12;
      const bool on = v < NPC && (full || ((pm >> ((r % kFrame) / kBlock + 3 * ((kWin0 + r / kFrame) / kBlock))) & 1u));
      rp[i] = *(on ? ps + v : pcentre);
    }
    // dM of the step's cells: component c is kRowsStep contiguous doubles at base
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int v = min(t + i * NT, NGC - 1);
      const int c = v / (kRowsStep / 2), w = v % (kRowsStep / 2);
      rg[i] = reinterpret_cast<const double2*>(gsrc + (size_t)c * kNCell + base)[w];
    }
  };
  issue(0);
  for (int step = 0; step < kRowsSteps; ++step) {
    __syncthreads();   // earlier readers of the LDS buffer are done
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int v = t + i * NT;
      if (v < NPC) {
        double* dst = s_pos + 2 * (v % 12) * kRowsLd + v / 12;
        dst[0] = rp[i].x;
        dst[kRowsLd] = rp[i].y;
      }
    }
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int v = t + i * NT;
      if (v < NGC) {
        const int c = v / (kRowsStep / 2), w = v % (kRowsStep / 2);
        s_g[c * kRowsLd + 2 * w] = rg[i].x;
        s_g[c * kRowsLd + 2 * w + 1] = rg[i].y;
      }
    }
    __syncthreads();
    issue(step + 1);
    // lanes past the step's 240 cells repeat its last cell (same values, same address)
    const int lcc = min(lc, kRowsStep - 1);
    const int r = (step & 1) * kRowsStep + lcc;
    const int jx = r % kFrame, jy = kWin0 + r / kFrame, jz = kWin0 + (step >> 1);
    const int cell = jx + kFrame * jy + kFrame * kFrame * jz;
    double res[4] = {0.0, 0.0, 0.0, 0.0};
    if (block_present(d.mask, jx, jy, jz)) {
      double g[C];
#pragma unroll
      for (int c = 0; c < C; ++c) g[c] = s_g[c * kRowsLd + lcc];
      const double cx = (jx + 0.5) * h, cy = (jy + 0.5) * h, cz = (jz + 0.5) * h;
      const double* y = s_pos + lcc;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pi = 4 * half + i;
        res[i] = monomial_dot<P>(g, y[(3 * pi) * kRowsLd] - cx, y[(3 * pi + 1) * kRowsLd] - cy,
                                 y[(3 * pi + 2) * kRowsLd] - cz);
      }
    }
    double2* out = reinterpret_cast<double2*>(dm + (int64_t)cell * 8 + 4 * half);
    out[0] = make_double2(res[0], res[1]);
    out[1] = make_double2(res[2], res[3]);
  }
}

}  // namespace fmm
