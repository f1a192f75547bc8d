// The multi-level gravity iteration on a uniform octree (the paper's
// three-step iteration, Sec. VII-C: bottom-up traversal, cell-to-cell
// interactions on every level, top-down traversal; Sec. IV-C: the octree's
// cells carry multipole moments).
//
// Domain: n^3 finest cells of spacing h; level l has n / 2^l cells per axis of
// spacing 2^l h, down to 4 per axis. Level arrays are [C][n_l][n_l][n_l]
// (x fastest), finest level first, back to back.
//
//   P2M  finest level: M_k(j) = sum_i m_i (y_i - c_j)^k / k!
//   M2M  M_k(J) = sum_{children j} sum_{q <= k} M_q(j) s^(k-q) / (k-q)!,  s = c_j - c_J
//   M2L  every level: L_n(t) = sum_{d in IL(t)} sum_k M_k(t + d) T_d[k][n] at the
//        level's spacing, IL(t) = {d : |d|^2 > 4, |floor((t mod 2 + d) / 2)|^2 <= 4}
//        (sources not near the target whose parents are near the target's
//        parent); on the 4-per-axis level every parent is near every other, so
//        the same lists give all non-near sources there. Sources outside the
//        domain are absent.
//   L2L  L_n(j) += sum_{m >= n} L_m(J) s^(m-n) / (m-n)!, coarsest level first.
//
// IL(t) depends only on the parity sigma of t: 231 offsets per parity, all
// inside the shell 5 <= |d|^2 <= 36 with |d_i| <= 5. The level M2L kernel
// gives each of its 8 waves one parity class of an 8^3 target block, so a
// wave's 64 targets (four 16-cell tiles, one per plane of that z parity) share
// one offset list and one table stream: v_mfma_f64_4x4x4_4b over
// [16 cells x 4 offsets] x [4 offsets x 4 columns] as in the single-level
// kernels, with the 18^3 source window of two moment components per round in
// LDS. The harmonic form (as FMM_FP64_HARMONIC: T_d is harmonic in both
// indices, so the moments fold onto the (p+1)^2 components with kz <= 1 and
// only those columns of L are computed, then expanded) uses the single-level
// form's fold plan per round and expansion of L.
#include <vector>

#include "kernels.h"
#include "m2l_mfma.h"
#include "p2m_common.h"

namespace fmm {

namespace {

constexpr int kTreeW = 18;                         // window (y, z): block cells -5 .. 12
constexpr int kTreeList = 231;                     // interaction-list length per parity
constexpr int kTreeQuads = (kTreeList + 3) / 4;    // 58 (the last quad has one empty slot)
constexpr int kTreeThreads = 512;
constexpr int kTreeMaxLevels = 8;
constexpr int kTreeWideMin = 64;                   // levels of at least this many cells per axis: NBLK = 2

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// b^i / i! per axis for i <= P
template <int P>
__device__ __forceinline__ void powers(double bx, double by, double bz, double (&px)[P + 1],
                                       double (&py)[P + 1], double (&pz)[P + 1]) {
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= P; ++i) {
    px[i] = px[i - 1] * bx * (1.0 / i);
    py[i] = py[i - 1] * by * (1.0 / i);
    pz[i] = pz[i - 1] * bz * (1.0 / i);
  }
}

// The (k, q) pairs with q <= k componentwise and their difference r = k - q,
// built at compile time so the shift loops unroll into straight-line code.
template <int P>
struct ShiftTerms {
  int n;
  signed char k[ncomp(P) * ncomp(P)], q[ncomp(P) * ncomp(P)];
  signed char rx[ncomp(P) * ncomp(P)], ry[ncomp(P) * ncomp(P)], rz[ncomp(P) * ncomp(P)];
};
template <int P>
constexpr ShiftTerms<P> make_shift_terms() {
  ShiftTerms<P> t{};
  for (int ck = 0; ck < ncomp(P); ++ck) {
    const MI k = mi_of(ck);
    for (int cq = 0; cq < ncomp(P); ++cq) {
      const MI q = mi_of(cq);
      if (q.x <= k.x && q.y <= k.y && q.z <= k.z) {
        t.k[t.n] = (signed char)ck;
        t.q[t.n] = (signed char)cq;
        t.rx[t.n] = (signed char)(k.x - q.x);
        t.ry[t.n] = (signed char)(k.y - q.y);
        t.rz[t.n] = (signed char)(k.z - q.z);
        ++t.n;
      }
    }
  }
  return t;
}

template <int P>
__global__ void __launch_bounds__(256) p2m_grid_kernel(const double* __restrict__ pos,
                                                       const double* __restrict__ mass, int ppc,
                                                       int n, double h, double* __restrict__ M) {
  constexpr int C = ncomp(P);
  const int64_t n3 = (int64_t)n * n * n;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n3) return;
  const int x = (int)(j % n), y = (int)((j / n) % n), z = (int)(j / ((int64_t)n * n));
  const double cx = (x + 0.5) * h, cy = (y + 0.5) * h, cz = (z + 0.5) * h;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  for (int i = 0; i < ppc; ++i) {
    const int64_t pi = j * ppc + i;
    p2m_accumulate<P>(mass[pi], pos[3 * pi] - cx, pos[3 * pi + 1] - cy, pos[3 * pi + 2] - cz, acc);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) M[c * n3 + j] = acc[c];
}

// One parent cell per thread; its 8 children's moments shifted to its centre.
template <int P>
__global__ void __launch_bounds__(256) m2m_kernel(const double* __restrict__ Mc,
                                                  double* __restrict__ Mp, int nc, double hc) {
  constexpr int C = ncomp(P);
  const int np = nc / 2;
  const int64_t np3 = (int64_t)np * np * np, nc3 = (int64_t)nc * nc * nc;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np3) return;
  const int X = (int)(i % np), Y = (int)((i / np) % np), Z = (int)(i / ((int64_t)np * np));
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
#pragma unroll 1
  for (int o = 0; o < 8; ++o) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
    const int64_t g = (2 * X + ox) + (int64_t)nc * (2 * Y + oy) + (int64_t)nc * nc * (2 * Z + oz);
    double mc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) mc[c] = Mc[c * nc3 + g];
    double px[P + 1], py[P + 1], pz[P + 1];
    powers<P>((ox - 0.5) * hc, (oy - 0.5) * hc, (oz - 0.5) * hc, px, py, pz);
    constexpr ShiftTerms<P> T = make_shift_terms<P>();
#pragma unroll
    for (int e = 0; e < T.n; ++e)
      acc[T.k[e]] = __builtin_fma(mc[T.q[e]], px[T.rx[e]] * py[T.ry[e]] * pz[T.rz[e]], acc[T.k[e]]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) Mp[c * np3 + i] = acc[c];
}

// One child cell per thread: adds its parent's local polynomial re-expanded
// about the child centre.
template <int P>
__global__ void __launch_bounds__(256) l2l_kernel(const double* __restrict__ Lp,
                                                  double* __restrict__ Lc, int nc, double hc) {
  constexpr int C = ncomp(P);
  const int np = nc / 2;
  const int64_t np3 = (int64_t)np * np * np, nc3 = (int64_t)nc * nc * nc;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= nc3) return;
  const int x = (int)(j % nc), y = (int)((j / nc) % nc), z = (int)(j / ((int64_t)nc * nc));
  const int64_t G = (x >> 1) + (int64_t)np * (y >> 1) + (int64_t)np * np * (z >> 1);
  double lp[C];
#pragma unroll
  for (int c = 0; c < C; ++c) lp[c] = Lp[c * np3 + G];
  double px[P + 1], py[P + 1], pz[P + 1];
  powers<P>(((x & 1) - 0.5) * hc, ((y & 1) - 0.5) * hc, ((z & 1) - 0.5) * hc, px, py, pz);
  // child n from parent m >= n: the terms (k, q) = (m, n) of the shift table
  constexpr ShiftTerms<P> T = make_shift_terms<P>();
  double s[C];
#pragma unroll
  for (int c = 0; c < C; ++c) s[c] = 0.0;
#pragma unroll
  for (int e = 0; e < T.n; ++e)
    s[T.q[e]] = __builtin_fma(lp[T.k[e]], px[T.rx[e]] * py[T.ry[e]] * pz[T.rz[e]], s[T.q[e]]);
#pragma unroll
  for (int c = 0; c < C; ++c) Lc[c * nc3 + j] += s[c];
}

// Tables of the level kernel, per order p:
//   B[sigma][round][quad][c2][group][kk * 4 + j] = T_d[2 round + c2][4 group + j]
// at unit spacing, d = the kk-th offset of the quad in sigma's list (zero for
// the empty slot, k >= C or n >= C). Built from the canonical [892][C][C]
// tables with the map sidx[sigma][quad][kk] (stencil index or -1).
__global__ void pack_tree_kernel(const double* __restrict__ T, int C, const int* __restrict__ sidx,
                                 double* __restrict__ B) {
  const int NG = (C + 3) / 4, R = (C + 1) / 2;
  const int64_t total = (int64_t)8 * R * kTreeQuads * 2 * NG * 16;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r_ = e;
    const int v = (int)(r_ % 16); r_ /= 16;
    const int g = (int)(r_ % NG); r_ /= NG;
    const int c2 = (int)(r_ % 2); r_ /= 2;
    const int q = (int)(r_ % kTreeQuads); r_ /= kTreeQuads;
    const int r = (int)(r_ % R);
    const int sigma = (int)(r_ / R);
    const int kk = v >> 2, j = v & 3;
    const int k = 2 * r + c2, nn = 4 * g + j;
    const int s = sidx[(sigma * kTreeQuads + q) * 4 + kk];
    B[e] = (s >= 0 && k < C && nn < C) ? T[((int64_t)s * C + k) * C + nn] : 0.0;
  }
}

// Harmonic tables: Bh[sigma][round][quad][c2][group][kk * 4 + j] =
// T_d[rowk[2 round + c2]][colk[4 group + j]] (zero where a map is -1).
struct TreeHMaps {
  int rowk[32];
  int colk[32];
};
__global__ void pack_tree_h_kernel(const double* __restrict__ T, int C, int R, int NG,
                                   const int* __restrict__ sidx, TreeHMaps mp, double* __restrict__ B) {
  const int64_t total = (int64_t)8 * R * kTreeQuads * 2 * NG * 16;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r_ = e;
    const int v = (int)(r_ % 16); r_ /= 16;
    const int g = (int)(r_ % NG); r_ /= NG;
    const int c2 = (int)(r_ % 2); r_ /= 2;
    const int q = (int)(r_ % kTreeQuads); r_ /= kTreeQuads;
    const int r = (int)(r_ % R);
    const int sigma = (int)(r_ / R);
    const int kk = v >> 2, j = v & 3;
    const int k = mp.rowk[2 * r + c2], nn = 4 * g + j < 32 ? mp.colk[4 * g + j] : -1;
    const int s = sidx[(sigma * kTreeQuads + q) * 4 + kk];
    B[e] = (s >= 0 && k >= 0 && nn >= 0) ? T[((int64_t)s * C + k) * C + nn] : 0.0;
  }
}

// Every level in one launch: the levels' blocks back to back, coarsest level
// first, so the few long-running blocks of the small levels start at once and
// overlap with the finest level's many blocks.
struct TreeLevels {
  int nlev;
  int first[kTreeMaxLevels + 1];   // first block of each level in launch order, then the total
  int n[kTreeMaxLevels];           // cells per axis
  int lg[kTreeMaxLevels];          // log2 of the spacing
  int64_t off[kTreeMaxLevels];     // element offset of the level in M and L
};

// NBLK: 8^3 target blocks per workgroup, side by side in x (the table operands
// of a quad then serve 4 NBLK tiles per wave)
template <int P, bool HARM, int NBLK>
__global__ void __launch_bounds__(kTreeThreads) m2l_level_kernel(
    const double* __restrict__ Mall, double* __restrict__ Lall, TreeLevels lv,
    const double* __restrict__ B, const int* __restrict__ doff, const HRound* __restrict__ hround,
    const HExp* __restrict__ hexp) {
  constexpr int C = ncomp(P);
  constexpr int CR = HARM ? (P + 1) * (P + 1) : C;   // contracted components (rows and columns)
  constexpr int NG = (CR + 3) / 4;
  constexpr int ROUNDS = (CR + 1) / 2;
  constexpr int WX = 8 * NBLK + 10;                   // window cells in x
  constexpr int WCELLS = WX * kTreeW * kTreeW;
  constexpr int STAGE = (WCELLS + kTreeThreads - 1) / kTreeThreads;
  constexpr int TPW = 4 * NBLK;                       // 16-cell tiles per wave
  // the window, and afterwards (harmonic form) the harmonic columns of the blocks
  constexpr int SMEM = HARM && NBLK * kNTarget * CR / 2 > WCELLS ? NBLK * kNTarget * CR / 2 : WCELLS;
  __shared__ double2 smem[SMEM];
  __shared__ int s_doff[8 * kTreeQuads * 4];
  int li = 0;
  while (li + 1 < lv.nlev && (int)blockIdx.x >= lv.first[li + 1]) ++li;
  const int n = lv.n[li], lg = lv.lg[li];
  const double* __restrict__ M = Mall + lv.off[li];
  double* __restrict__ L = Lall + lv.off[li];
  const int nb = n >= 8 ? n / 8 : 1;
  const int nbx = n >= 8 * NBLK ? n / (8 * NBLK) : 1;
  const int blk = (int)blockIdx.x - lv.first[li];
  const int B0x = 8 * NBLK * (blk % nbx), B0y = 8 * ((blk / nbx) % nb), B0z = 8 * (blk / (nbx * nb));
  const int64_t n3 = (int64_t)n * n * n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // parity class of this wave
  const int sx = wave & 1, sy = (wave >> 1) & 1, sz = wave >> 2;
  const int kk = lane >> 4, ci = lane & 15;
  // offsets of the lists, packed (dx + 8) | (dy + 8) << 5 | (dz + 8) << 10, as window deltas
  for (int i = tid; i < 8 * kTreeQuads * 4; i += kTreeThreads) {
    const int v = doff[i];
    s_doff[i] = ((v & 31) - 8) + WX * (((v >> 5) & 31) - 8) + WX * kTreeW * (((v >> 10) & 31) - 8);
  }

  // tile t: block t / 4, plane z = 2 (t % 4) + sz, cells (8 (t / 4) + 2 (ci & 3) + sx, 2 (ci >> 2) + sy)
  int abase[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int z = 2 * (t & 3) + sz, x = 8 * (t >> 2) + 2 * (ci & 3) + sx, y = 2 * (ci >> 2) + sy;
    abase[t] = (x + 5) + WX * (y + 5) + WX * kTreeW * (z + 5);
  }
  double acc[TPW][NG];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[t][g] = 0.0;

  const int* dq = s_doff + wave * kTreeQuads * 4 + kk;
  // this thread's window cells: global index, or -1 outside the domain
  // (n^3 <= 2^21 cells per level, so a cell index fits 32 bits)
  int wg[STAGE];
#pragma unroll
  for (int i = 0; i < STAGE; ++i) {
    const int c = tid + i * kTreeThreads;
    const int gx = B0x - 5 + c % WX, gy = B0y - 5 + (c / WX) % kTreeW,
              gz = B0z - 5 + c / (WX * kTreeW);
    wg[i] = (c < WCELLS && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n)
                ? gx + n * gy + n * n * gz
                : -1;
  }
  for (int r = 0; r < ROUNDS; ++r) {
    double s0, s1;
    double2 v[STAGE];
#pragma unroll
    for (int i = 0; i < STAGE; ++i) v[i] = make_double2(0.0, 0.0);
    if (HARM) {
      // the round's two folded components, each an integer combination of moment
      // components of one order
      const HRound& rd = hround[r];
      s0 = ldexp(1.0, -lg * rd.ord0);
      s1 = rd.ord1 >= 0 ? ldexp(1.0, -lg * rd.ord1) : 0.0;
      // two components at a time, so both sets of loads are in flight together
      // (an odd count's last pass reads its component twice, the second time
      // with zero coefficients)
      for (int u = 0; u < rd.nsup; u += 2) {
        const int u1 = u + 1 < rd.nsup ? u + 1 : u;
        const double* srcA = M + (int64_t)rd.comp[u] * n3;
        const double* srcB = M + (int64_t)rd.comp[u1] * n3;
        const double a0 = rd.c0[u], a1 = rd.c1[u];
        const double b0 = u1 != u ? rd.c0[u1] : 0.0, b1 = u1 != u ? rd.c1[u1] : 0.0;
        double ma[STAGE], mb[STAGE];
#pragma unroll
        for (int i = 0; i < STAGE; ++i) {
          ma[i] = wg[i] >= 0 ? srcA[wg[i]] : 0.0;
          mb[i] = wg[i] >= 0 ? srcB[wg[i]] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < STAGE; ++i) {
          v[i].x = __builtin_fma(b0, mb[i], __builtin_fma(a0, ma[i], v[i].x));
          v[i].y = __builtin_fma(b1, mb[i], __builtin_fma(a1, ma[i], v[i].y));
        }
      }
    } else {
      const int k0 = 2 * r, k1 = 2 * r + 1;
      s0 = ldexp(1.0, -lg * order_of(k0));
      s1 = k1 < C ? ldexp(1.0, -lg * order_of(k1)) : 0.0;
      const double* src0 = M + (int64_t)k0 * n3;
      const double* src1 = M + (int64_t)(k1 < C ? k1 : k0) * n3;
#pragma unroll
      for (int i = 0; i < STAGE; ++i) {
        if (wg[i] >= 0) {
          v[i].x = src0[wg[i]];
          v[i].y = src1[wg[i]];
        }
      }
    }
    __syncthreads();   // the previous round's window reads are done
#pragma unroll
    for (int i = 0; i < STAGE; ++i) {
      const int c = tid + i * kTreeThreads;
      if (c < WCELLS) smem[c] = make_double2(v[i].x * s0, v[i].y * s1);
    }
    __syncthreads();
    const double* Br = B + ((int64_t)(wave * ROUNDS + r) * kTreeQuads) * 2 * NG * 16 + kk * 4 + (lane & 3);
    // table operands are loaded two quads ahead of their products
    double nb0[NG], nb1[NG], mb0[NG], mb1[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      nb0[g] = Br[g * 16];
      nb1[g] = Br[(NG + g) * 16];
      mb0[g] = Br[2 * NG * 16 + g * 16];
      mb1[g] = Br[2 * NG * 16 + (NG + g) * 16];
    }
    for (int q = 0; q < kTreeQuads; ++q) {
      double b0[NG], b1[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        b0[g] = nb0[g];
        b1[g] = nb1[g];
        nb0[g] = mb0[g];
        nb1[g] = mb1[g];
      }
      if (q + 2 < kTreeQuads) {
        const double* Bn = Br + (int64_t)(q + 2) * 2 * NG * 16;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          mb0[g] = Bn[g * 16];
          mb1[g] = Bn[(NG + g) * 16];
        }
      }
      const int dl = dq[q * 4];
      double2 a[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) a[t] = smem[abase[t] + dl];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].x, b0[g], acc[t][g]);
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].y, b1[g], acc[t][g]);
      }
    }
  }

  // D layout: this lane holds cell (2 xi + sx, 2 yi + sy) of each tile, column j
  const int xi = lane >> 4, yi = (lane & 15) >> 2, j = lane & 3;
  if (!HARM) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int gx = B0x + 8 * (t >> 2) + 2 * xi + sx, gy = B0y + 2 * yi + sy, gz = B0z + 2 * (t & 3) + sz;
      if (gx >= n || gy >= n || gz >= n) continue;
      const int64_t g = gx + (int64_t)n * gy + (int64_t)n * n * gz;
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) {
        const int nn = 4 * gg + j;
        if (nn < C) L[nn * n3 + g] = ldexp(acc[t][gg], -lg * (1 + order_of(nn)));
      }
    }
    return;
  }
  // harmonic columns (column c has order floor(sqrt(c))) through LDS, then each
  // thread expands one target cell to all C components
  __syncthreads();                                  // the window is no longer read
  double* sh = reinterpret_cast<double*>(smem);     // [512 NBLK cells][CR], x fastest over 8 NBLK
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int cell = (8 * (t >> 2) + 2 * xi + sx) + 8 * NBLK * ((2 * yi + sy) + 8 * (2 * (t & 3) + sz));
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
      const int c = 4 * gg + j;
      if (c < CR) {
        int ord = 0;
        while ((ord + 1) * (ord + 1) <= c) ++ord;
        sh[cell * CR + c] = ldexp(acc[t][gg], -lg * (1 + ord));
      }
    }
  }
  __syncthreads();
  for (int cell = tid; cell < NBLK * kNTarget; cell += kTreeThreads) {
    const int gx = B0x + cell % (8 * NBLK), gy = B0y + (cell / (8 * NBLK)) % 8, gz = B0z + cell / (64 * NBLK);
    if (gx < n && gy < n && gz < n) {
      const int64_t g = gx + (int64_t)n * gy + (int64_t)n * n * gz;
      const double* lh = sh + cell * CR;
      for (int nn = 0; nn < C; ++nn) {
        const HExp& ex = hexp[nn];
        double v = 0.0;
        for (int u = 0; u < ex.nterm; ++u) v = __builtin_fma(ex.coef[u], lh[ex.col[u]], v);
        L[nn * n3 + g] = v;
      }
    }
  }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Interaction lists on the host: for each parity sigma (x + 2 y + 4 z bits),
// the offsets d (dz slowest, then dy, dx, ascending) with |d|^2 > 4 whose
// parents' offset floor((sigma + d) / 2) has squared length <= 4.
static std::vector<int> tree_lists() {
  std::vector<int> out;
  auto fl2 = [](int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); };   // floor(a / 2)
  for (int sigma = 0; sigma < 8; ++sigma) {
    const int sg[3] = {sigma & 1, (sigma >> 1) & 1, sigma >> 2};
    int count = 0;
    for (int dz = -6; dz <= 6; ++dz)
      for (int dy = -6; dy <= 6; ++dy)
        for (int dx = -6; dx <= 6; ++dx) {
          if (dx * dx + dy * dy + dz * dz <= 4) continue;
          const int Dx = fl2(sg[0] + dx), Dy = fl2(sg[1] + dy), Dz = fl2(sg[2] + dz);
          if (Dx * Dx + Dy * Dy + Dz * Dz > 4) continue;
          out.push_back(dx);
          out.push_back(dy);
          out.push_back(dz);
          ++count;
        }
    if (count != kTreeList) return {};
  }
  return out;
}

hipError_t tree_tables_create(TreeTables* tt, const double* const* d_T, const int* stencil_xyz,
                              int nstencil, hipStream_t s) {
  const std::vector<int> lists = tree_lists();
  if (lists.empty()) return hipErrorInvalidValue;
  std::vector<int> sidx(8 * kTreeQuads * 4, -1), doff(8 * kTreeQuads * 4, 8 | (8 << 5) | (8 << 10));
  for (int sigma = 0; sigma < 8; ++sigma)
    for (int e = 0; e < kTreeList; ++e) {
      const int* d = &lists[3 * (sigma * kTreeList + e)];
      int found = -1;
      for (int i = 0; i < nstencil; ++i)
        if (stencil_xyz[3 * i] == d[0] && stencil_xyz[3 * i + 1] == d[1] && stencil_xyz[3 * i + 2] == d[2]) {
          found = i;
          break;
        }
      if (found < 0) return hipErrorInvalidValue;
      sidx[sigma * kTreeQuads * 4 + e] = found;
      doff[sigma * kTreeQuads * 4 + e] = (d[0] + 8) | ((d[1] + 8) << 5) | ((d[2] + 8) << 10);
    }
  hipError_t e;
  int* d_sidx = nullptr;
  if ((e = hipMalloc(&tt->doff, sizeof(int) * doff.size())) != hipSuccess) return e;
  if ((e = hipMemcpy(tt->doff, doff.data(), sizeof(int) * doff.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_sidx, sizeof(int) * sidx.size())) != hipSuccess) return e;
  if ((e = hipMemcpy(d_sidx, sidx.data(), sizeof(int) * sidx.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(d_sidx);
    return e;
  }
  for (int p = 2; p <= kMaxP; ++p) {
    const int C = ncomp(p), NG = (C + 3) / 4, R = (C + 1) / 2;
    const size_t count = (size_t)8 * R * kTreeQuads * 2 * NG * 16;
    if ((e = hipMalloc(&tt->B[p], sizeof(double) * count)) != hipSuccess) break;
    hipLaunchKernelGGL(pack_tree_kernel, dim3(1024), dim3(256), 0, s, d_T[p], C, d_sidx, tt->B[p]);
    if ((e = hipGetLastError()) != hipSuccess) break;
    TreeHMaps mp;
    int rh = 0;
    if (!harmonic_plan_maps(p, mp.rowk, mp.colk, &rh) || rh != ((p + 1) * (p + 1) + 1) / 2) {
      e = hipErrorInvalidValue;
      break;
    }
    const int CRh = (p + 1) * (p + 1), NGh = (CRh + 3) / 4;
    const size_t counth = (size_t)8 * rh * kTreeQuads * 2 * NGh * 16;
    if ((e = hipMalloc(&tt->Bh[p], sizeof(double) * counth)) != hipSuccess) break;
    hipLaunchKernelGGL(pack_tree_h_kernel, dim3(1024), dim3(256), 0, s, d_T[p], C, rh, NGh, d_sidx, mp,
                       tt->Bh[p]);
    if ((e = hipGetLastError()) != hipSuccess) break;
  }
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(d_sidx);
  return e != hipSuccess ? e : e2;
}

void tree_tables_destroy(TreeTables* tt) {
  for (int p = 0; p <= kMaxP; ++p) {
    if (tt->B[p]) (void)hipFree(tt->B[p]);
    if (tt->Bh[p]) (void)hipFree(tt->Bh[p]);
  }
  if (tt->doff) (void)hipFree(tt->doff);
  *tt = TreeTables{};
}

hipError_t launch_tree_p2m(int p, const double* pos, const double* mass, int ppc, int n, double h,
                           double* M, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  const dim3 grid(blocks_for(n3, 256)), block(256);
  switch (p) {
    case 2: hipLaunchKernelGGL(p2m_grid_kernel<2>, grid, block, 0, s, pos, mass, ppc, n, h, M); break;
    case 3: hipLaunchKernelGGL(p2m_grid_kernel<3>, grid, block, 0, s, pos, mass, ppc, n, h, M); break;
    case 4: hipLaunchKernelGGL(p2m_grid_kernel<4>, grid, block, 0, s, pos, mass, ppc, n, h, M); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tree_m2m(int p, const double* Mc, double* Mp, int nc, double hc, hipStream_t s) {
  const int64_t np3 = (int64_t)(nc / 2) * (nc / 2) * (nc / 2);
  const dim3 grid(blocks_for(np3, 256)), block(256);
  switch (p) {
    case 2: hipLaunchKernelGGL(m2m_kernel<2>, grid, block, 0, s, Mc, Mp, nc, hc); break;
    case 3: hipLaunchKernelGGL(m2m_kernel<3>, grid, block, 0, s, Mc, Mp, nc, hc); break;
    case 4: hipLaunchKernelGGL(m2m_kernel<4>, grid, block, 0, s, Mc, Mp, nc, hc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tree_l2l(int p, const double* Lp, double* Lc, int nc, double hc, hipStream_t s) {
  const int64_t nc3 = (int64_t)nc * nc * nc;
  const dim3 grid(blocks_for(nc3, 256)), block(256);
  switch (p) {
    case 2: hipLaunchKernelGGL(l2l_kernel<2>, grid, block, 0, s, Lp, Lc, nc, hc); break;
    case 3: hipLaunchKernelGGL(l2l_kernel<3>, grid, block, 0, s, Lp, Lc, nc, hc); break;
    case 4: hipLaunchKernelGGL(l2l_kernel<4>, grid, block, 0, s, Lp, Lc, nc, hc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tree_m2l(int p, const TreeTables& tt, const MfmaTables& mt, bool harmonic,
                           const double* M, double* L, int nlev, const int* n, const int* lg,
                           const int64_t* off, hipStream_t s) {
  if (nlev < 1 || nlev > kTreeMaxLevels) return hipErrorInvalidValue;
  // Two 8^3 blocks per workgroup (NBLK = 2) where a level has many of them, one
  // (NBLK = 1) on the coarse levels and at p = 4 (registers). Each workgroup of a
  // launch has the same work, at one workgroup per CU, so a launch whose count is
  // just over a multiple of the CU count ends with a nearly idle wave: on 128^3,
  // 2304 wide workgroups for the 128 and 64 levels (9 full waves) then the 32..4
  // levels as 74 narrow ones (each ~0.6 of a wide one), instead of 2342 wide ones
  // in one launch (a tenth wave of 38).
  auto wide = [&](int l) { return p <= 3 && n[l] >= kTreeWideMin; };
  for (int pass = 0; pass < 2; ++pass) {
    const int nblk = pass == 0 ? 2 : 1;
    TreeLevels lv{};
    int total = 0, cnt = 0;
    for (int i = 0; i < nlev; ++i) {            // coarsest level first
      const int l = nlev - 1 - i;
      if (wide(l) != (pass == 0)) continue;
      const int nb = n[l] >= 8 ? n[l] / 8 : 1;
      const int nbx = n[l] >= 8 * nblk ? n[l] / (8 * nblk) : 1;
      lv.first[cnt] = total;
      lv.n[cnt] = n[l];
      lv.lg[cnt] = lg[l];
      lv.off[cnt] = off[l];
      total += nbx * nb * nb;
      ++cnt;
    }
    if (cnt == 0) continue;
    lv.nlev = cnt;
    lv.first[cnt] = total;
    const dim3 grid((unsigned)total), block(kTreeThreads);
#define TREE_LAUNCH(P, H, NB)                                                                   \
  hipLaunchKernelGGL((m2l_level_kernel<P, H, NB>), grid, block, 0, s, M, L, lv,                \
                     H ? tt.Bh[P] : tt.B[P], tt.doff, mt.hround[P], mt.hexp[P])
    switch ((p * 2 + (harmonic ? 1 : 0)) * 2 + pass) {
      case 8: TREE_LAUNCH(2, false, 2); break;
      case 9: TREE_LAUNCH(2, false, 1); break;
      case 10: TREE_LAUNCH(2, true, 2); break;
      case 11: TREE_LAUNCH(2, true, 1); break;
      case 12: TREE_LAUNCH(3, false, 2); break;
      case 13: TREE_LAUNCH(3, false, 1); break;
      case 14: TREE_LAUNCH(3, true, 2); break;
      case 15: TREE_LAUNCH(3, true, 1); break;
      case 17: TREE_LAUNCH(4, false, 1); break;
      case 19: TREE_LAUNCH(4, true, 1); break;
      default: return hipErrorInvalidValue;
    }
#undef TREE_LAUNCH
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fmm
