// Exact-slice M2L on gfx950 int8 matrix cores (FMM_EXACT_SLICE), harmonic form.
//
// The contraction L~[t][n'] = sum_{d, k'} Mh_k'(t + d) T_d[k'][n'] of the
// harmonic form is evaluated with the error-free splitting of Ozaki, Ogita,
// Oishi and Rump, using int8 slices and exact integer sums (the way Ootomo,
// Ozaki and Yokota run float64 products on integer units):
//   A = Mh 2^f 2^-e_A,  B = T 2^-f 2^-e_B(n'),  both in (-1, 1),
//   A = sum_{i<S} a_i 2^-7(i+1) + r,  B = sum_{j<S} b_j 2^-7(j+1) + r',
//   L~ = 2^(e_A + e_B(n')) sum_{i + j <= S} 2^-7(i+j+2) sum_{d, k'} a_i b_j.
// f is a fixed per-component prescale (the geometric bound of the folded
// moments), e_A one exponent per sub-grid (its largest prescaled folded
// moment over the reachable window), e_B one per table column. Every
// sum_{d, k'} a_i b_j is an exact integer below 2^31 (892 x 16 x 127^2 x 8).
//
// Kernels:
// * slice_window_kernel: one workgroup per sub-grid folds the moments of the
//   20^3 window (the round plan of the float64 harmonic kernels), finds e_A,
//   and writes S planes of [8000 cells][16 bytes] (slice i of the folded
//   components, round-plan order, zero past (p+1)^2 and on absent blocks).
// * m2l_fwd_slice_kernel: persistent, one workgroup of 4 waves per CU (one
//   wave per SIMD, up to 512 registers each). Wave w owns target planes
//   2w, 2w+1: eight 16-cell tiles. Per round i the workgroup stages slice
//   plane i in LDS (128,000 bytes); per offset quad each wave reads its 8 A
//   operands (16 bytes per lane: cell t + d of the lane's offset, 16 folded
//   components) and, for every j with i + j <= S, one B operand from the
//   L2-resident tables, and issues 8 v_mfma_i32_16x16x64_i8 into the int32
//   sums of (tile, j). At the end of the round the sums are added to float64
//   accumulators with weight 2^-7(i+j+2). The epilogue scales by
//   2^(e_A + e_B), expands L~ to all C components through LDS and applies
//   h^(-1-|n|).
//
// Operand lane layouts of v_mfma_i32_16x16x64_i8 (checked on gfx950):
//   A: lane l -> row l % 16, 16 bytes of the K range of lane group l / 16
//   B: lane l -> column l % 16, the same 16 bytes of K as A's lane group l / 16
//   D: lane l, v -> row 4 (l / 16) + v, column l % 16
// so the K index only has to agree between A and B: byte b of lane group g is
// folded component b of offset 4 q + g.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "kernels.h"
#include "m2l_mfma.h"

namespace fmm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWinCells = kWin * kWin * kWin;   // 8000
constexpr int kQuadsS = kNStencil / 4;          // 223
constexpr int kSliceThreads = 256;              // 4 waves: one per SIMD
constexpr int kPrepThreads = 512;

// per-order constants of the slicing (kernel argument)
struct SliceConst {
  int32_t f[2][16];    // [p - 2][byte]: prescale exponents of the folded rows
  int32_t eB[2][16];   // [p - 2][column]: table column exponents
};

__global__ void reset_slice_counter(unsigned* c) { *c = 0u; }

// The folded, h-scaled and prescaled moments of window cell c (zero on absent
// blocks), in round-plan order: byte 2 r + u is the round's u-th folded component.
template <int P>
__device__ __forceinline__ void fold_cell(const DevDesc& d, const double* __restrict__ src,
                                          const HRound* __restrict__ hr, const SliceConst& sc, int c,
                                          double (&v)[16]) {
  constexpr int R = ((P + 1) * (P + 1) + 1) / 2;
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  const int jx = c % kWin + kWin0, jy = (c / kWin) % kWin + kWin0, jz = c / (kWin * kWin) + kWin0;
  if (!block_present(d.mask, jx, jy, jz)) return;
  const int cell = jx + kFrame * jy + kFrame * kFrame * jz;
  const int l2 = d.log2_inv_h;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int nsup = hr[r].nsup;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int u = 0; u < kHMaxSup; ++u) {
      if (u < nsup) {
        const double x = src[(size_t)hr[r].comp[u] * kNCell + cell];
        a0 = __builtin_fma(hr[r].c0[u], x, a0);
        a1 = __builtin_fma(hr[r].c1[u], x, a1);
      }
    }
    v[2 * r] = ldexp(a0, l2 * hr[r].ord0 + sc.f[P - 2][2 * r]);
    if (2 * r + 1 < (P + 1) * (P + 1)) v[2 * r + 1] = ldexp(a1, l2 * hr[r].ord1 + sc.f[P - 2][2 * r + 1]);
  }
}

template <int P>
__device__ void slice_subgrid(const DevDesc& d, int b, const double* __restrict__ M,
                              const HRound* __restrict__ hr, const SliceConst& sc, int S,
                              int8_t* __restrict__ planes, int32_t* __restrict__ expo, int* s_e) {
  const int tid = threadIdx.x;
  const double* src = M + d.m_off;
  // pass 1: e_A = the frexp exponent of the largest |value| (max of the per-value exponents)
  int emax = INT_MIN;
  for (int c = tid; c < kWinCells; c += kPrepThreads) {
    double v[16];
    fold_cell<P>(d, src, hr, sc, c, v);
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (v[k] != 0.0) emax = max(emax, ilogb(v[k]) + 1);
  }
  atomicMax(s_e, emax);
  __syncthreads();
  const int eA = *s_e == INT_MIN ? 0 : *s_e;
  if (tid == 0) expo[b] = eA;
  // pass 2: the slices, 16 bytes per cell and slice
  int8_t* out = planes + (size_t)b * S * kSlicePlane;
  for (int c = tid; c < kWinCells; c += kPrepThreads) {
    double v[16];
    fold_cell<P>(d, src, hr, sc, c, v);
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = ldexp(v[k], -eA);   // |v| < 1
#pragma unroll
    for (int i = 0; i < kSliceMax; ++i) {
      if (i < S) {
        v4i w = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const double y = v[k] * 128.0;
          const double q = trunc(y);
          v[k] = y - q;
          w[k >> 2] |= ((int)q & 0xff) << (8 * (k & 3));
        }
        *reinterpret_cast<v4i*>(out + (size_t)i * kSlicePlane + (size_t)c * kSliceBytes) = w;
      }
    }
  }
}

__global__ void __launch_bounds__(kPrepThreads) slice_window_kernel(
    const DevDesc* __restrict__ desc, const double* __restrict__ M, const HRound* __restrict__ hr2,
    const HRound* __restrict__ hr3, SliceConst sc, int S, int8_t* __restrict__ planes,
    int32_t* __restrict__ expo) {
  __shared__ int s_e;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) s_e = INT_MIN;
  __syncthreads();
  const DevDesc d = desc[b];
  if (d.p == 2) slice_subgrid<2>(d, b, M, hr2, sc, S, planes, expo, &s_e);
  else if (d.p == 3) slice_subgrid<3>(d, b, M, hr3, sc, S, planes, expo, &s_e);
}

__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Part of one round (slice I of the moments) of one sub-grid: the products
// with the table slices j = J0 .. J0 + NJP - 1 over every live offset quad,
// then their sums into the float64 accumulators with weight 2^-7(I+j+2). A
// round runs its table slices (i + j <= S) in passes of at most 4, which keeps
// the int32 sums of the wave's 8 tiles in 128 registers; the window operands
// are read from LDS once per pass.
template <bool FULL, int I, int J0, int NJP>
__device__ __forceinline__ void slice_pass(const v4i* __restrict__ win, const v4i* __restrict__ Bt,
                                           const int* __restrict__ s_off, const uint64_t (&live)[4],
                                           const int (&abase)[8], int lane, double (&fa)[8][4]) {
  const int g = lane >> 4;
  v4i acc[NJP][8];
#pragma unroll
  for (int j = 0; j < NJP; ++j)
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[j][t] = v4i{0, 0, 0, 0};
  // Software pipeline (one wave per SIMD, so nothing else hides latency): the
  // table operands, from L2, are loaded four quads ahead into a ring of four
  // sets (each set reloaded right after its products are issued); the window
  // operands, from LDS, one quad ahead into two sets; the window offsets two
  // quads ahead. Loads are unconditional, with the
  // quad index clamped to the last quad, so every path into the products sees the
  // same outstanding loads; operands loaded past the last quad are never used.
  v4i a0[8], a1[8], b0[NJP], b1[NJP], b2[NJP], b3[NJP];
  int o0, o1;   // window offsets (this lane's offset of the quad) of the next two quads
  auto ldB = [&](v4i(&db)[NJP], int q) __attribute__((always_inline)) {
    q = min(q, kQuadsS - 1);
#pragma unroll
    for (int j = 0; j < NJP; ++j) db[j] = Bt[((size_t)(J0 + j) * kQuadsS + q) * 64 + lane];
  };
  auto ldA = [&](v4i(&da)[8], int off) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < 8; ++t) da[t] = win[abase[t] + off];
  };
  auto ldO = [&](int q) __attribute__((always_inline)) { return s_off[4 * min(q, kQuadsS - 1) + g]; };
  auto mma = [&](const v4i(&sa)[8], const v4i(&sb)[NJP]) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NJP; ++j)
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[j][t] = mfma_i8(sa[t], sb[j], acc[j][t]);
  };
  auto is_live = [&](int q) { return (live[q >> 6] >> (q & 63)) & 1ull; };
  // one step: the window operands of quad Q + 1 go to DA (its offset o0 was read
  // a step ago), the offset of quad Q + 3 is read, quad Q's products run from
  // (SA, SB), and SB, free again, takes the table operands of quad Q + 4
#define SL_STEP(SA, SB, DA, Q)                  \
  {                                             \
    ldA(DA, o0);                                \
    o0 = o1;                                    \
    o1 = ldO((Q) + 3);                          \
    if (FULL || is_live(Q)) mma(SA, SB);        \
    ldB(SB, (Q) + 4);                           \
  }
  static_assert(kQuadsS % 4 == 3, "groups of four quads, then three");
  // prologue: window operands of quad 0, offsets of quads 1 and 2, tables of quads 0-3
  ldA(a0, ldO(0));
  o0 = ldO(1);
  o1 = ldO(2);
  ldB(b0, 0);
  ldB(b1, 1);
  ldB(b2, 2);
  ldB(b3, 3);
#pragma unroll 1
  for (int q = 0; q + 4 < kQuadsS; q += 4) {
    SL_STEP(a0, b0, a1, q);
    SL_STEP(a1, b1, a0, q + 1);
    SL_STEP(a0, b2, a1, q + 2);
    SL_STEP(a1, b3, a0, q + 3);
  }
  SL_STEP(a0, b0, a1, kQuadsS - 3);
  SL_STEP(a1, b1, a0, kQuadsS - 2);
  SL_STEP(a0, b2, a1, kQuadsS - 1);
#undef SL_STEP
#pragma unroll
  for (int j = 0; j < NJP; ++j) {
    const double wgt = ldexp(1.0, -7 * (I + J0 + j + 2));
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) fa[t][v] = __builtin_fma((double)acc[j][t][v], wgt, fa[t][v]);
  }
}

// Round I: table slices j < NJ = min(S, S - I + 1), in passes of at most 4.
template <bool FULL, int I, int J0, int NJ>
__device__ __forceinline__ void slice_round(const v4i* __restrict__ win, const v4i* __restrict__ Bt,
                                            const int* __restrict__ s_off, const uint64_t (&live)[4],
                                            const int (&abase)[8], int lane, double (&fa)[8][4]) {
  if constexpr (J0 < NJ) {
    constexpr int NJP = NJ - J0 < 4 ? NJ - J0 : 4;
    slice_pass<FULL, I, J0, NJP>(win, Bt, s_off, live, abase, lane, fa);
    slice_round<FULL, I, J0 + NJP, NJ>(win, Bt, s_off, live, abase, lane, fa);
  }
}

template <bool FULL, int S, int I>
__device__ __forceinline__ void slice_rounds(const int8_t* __restrict__ pl, v4i* win,
                                             const v4i* __restrict__ Bt, const int* s_off,
                                             const uint64_t (&live)[4], const int (&abase)[8], int lane,
                                             double (&fa)[8][4]) {
  if constexpr (I < S) {
    __syncthreads();   // the previous round's reads of the window are done
    const v4i* gp = reinterpret_cast<const v4i*>(pl + (size_t)I * kSlicePlane);
    for (int c = threadIdx.x; c < kWinCells; c += kSliceThreads) win[c] = gp[c];
    __syncthreads();
    constexpr int NJ = (S - I + 1) < S ? (S - I + 1) : S;
    slice_round<FULL, I, 0, NJ>(win, Bt, s_off, live, abase, lane, fa);
    slice_rounds<FULL, S, I + 1>(pl, win, Bt, s_off, live, abase, lane, fa);
  }
}

template <int S>
__global__ void __launch_bounds__(kSliceThreads) m2l_fwd_slice_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, double* __restrict__ L, const int8_t* __restrict__ planes,
    const int32_t* __restrict__ expo, const v4i* __restrict__ Bt2, const v4i* __restrict__ Bt3,
    const int* __restrict__ lds_off, const uint32_t* __restrict__ touch, SliceConst sc,
    const HExp* __restrict__ he2, const HExp* __restrict__ he3) {
  __shared__ v4i win[kWinCells];            // 128,000 bytes: one slice plane of the window
  __shared__ int s_off[kNStencil];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ci = lane & 15;
  for (int i = tid; i < kNStencil; i += kSliceThreads) s_off[i] = lds_off[i];
  // tile t of this wave: target plane 2 wave + t / 4, 4x4 patch ((t & 1) * 4, ((t >> 1) & 1) * 4)
  int abase[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int x = (t & 1) * 4 + (ci & 3), y = ((t >> 1) & 1) * 4 + (ci >> 2), z = 2 * wave + (t >> 2);
    abase[t] = (x + 6) + kWin * (y + 6) + kWin * kWin * (z + 6);
  }
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= count) break;
    const int b = items[item].sub;
    const DevDesc d = desc[b];
    const int pi = d.p - 2;
    // live quads of this wave's two planes (some source block present)
    uint64_t live[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q = 64 * c + lane;
      bool on = false;
      if (q < kQuadsS) on = ((touch[(2 * wave) * kQuadsS + q] | touch[(2 * wave + 1) * kQuadsS + q]) & d.mask) != 0;
      live[c] = __ballot(on);
    }
    double fa[8][4];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) fa[t][v] = 0.0;
    const int8_t* pl = planes + (size_t)b * S * kSlicePlane;
    const v4i* Bt = pi == 0 ? Bt2 : Bt3;
    // sub-grids with every neighbour block present run the quad loop without skip tests
    if (d.mask == kFullMask) slice_rounds<true, S, 0>(pl, win, Bt, s_off, live, abase, lane, fa);
    else slice_rounds<false, S, 0>(pl, win, Bt, s_off, live, abase, lane, fa);
    // epilogue: L~ columns (scaled back) to LDS [n'][target], then each thread
    // expands two targets to all C components
    __syncthreads();   // every wave is done with the window
    double* lh = reinterpret_cast<double*>(win);
    const int n = lane & 15, g = lane >> 4;
    const double sc_n = ldexp(1.0, expo[b] + sc.eB[pi][n]);
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int x = (t & 1) * 4 + v, y = ((t >> 1) & 1) * 4 + g, z = 2 * wave + (t >> 2);
        lh[n * kNTarget + x + kBlock * y + kBlock * kBlock * z] = fa[t][v] * sc_n;
      }
    __syncthreads();
    const HExp* he = pi == 0 ? he2 : he3;
    const int C = ncomp(d.p);
    const int l2 = d.log2_inv_h;
    double* out = L + d.l_off;
    for (int k = 0; k < C; ++k) {
      const HExp e = he[k];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int tc = tid + r * kSliceThreads;
        double v = 0.0;
        for (int u = 0; u < e.nterm; ++u) v = __builtin_fma(e.coef[u], lh[e.col[u] * kNTarget + tc], v);
        out[(size_t)k * kNTarget + tc] = ldexp(v, l2 * (1 + order_of(k)));
      }
    }
    __syncthreads();   // s_item and the LDS are free for the next item
  }
}

// ---- host: the table operand

struct MIx {
  int x, y, z;
};

std::vector<MIx> graded(int p) {
  std::vector<MIx> v;
  for (int n = 0; n <= p; ++n)
    for (int kx = n; kx >= 0; --kx)
      for (int ky = n - kx; ky >= 0; --ky) v.push_back({kx, ky, n - kx - ky});
  return v;
}

double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

int frexp_exp(double x) {
  int e = 0;
  (void)std::frexp(x, &e);
  return x == 0.0 ? 0 : e;
}

}  // namespace

hipError_t slice_tables_create(SliceTables* st, double* const* d_T, hipStream_t s) {
  hipError_t e;
  for (int p = 2; p <= 3; ++p) {
    std::vector<HRound> rounds;
    int32_t rowk[32], colk[32];
    int nr = 0;
    if (!harmonic_rounds_host(p, &rounds) || !harmonic_plan_maps(p, rowk, colk, &nr))
      return hipErrorInvalidValue;
    const std::vector<MIx> ks = graded(p);
    const int C = ncomp(p), CR = (p + 1) * (p + 1);
    // prescale of each folded row: -floor(log2 b), b = sum over its moment components
    // of |coefficient| 2^-|k| / k! (|a| <= h/2 per axis)
    for (int r = 0; r < (int)rounds.size(); ++r)
      for (int u = 0; u < 2; ++u) {
        const int byte = 2 * r + u;
        if (byte >= CR) continue;
        double bnd = 0.0;
        for (int i = 0; i < rounds[r].nsup; ++i) {
          const double cf = u == 0 ? rounds[r].c0[i] : rounds[r].c1[i];
          const MIx k = ks[rounds[r].comp[i]];
          bnd += std::fabs(cf) * std::ldexp(1.0, -(k.x + k.y + k.z)) / (fact(k.x) * fact(k.y) * fact(k.z));
        }
        st->f[p][byte] = -(int)std::floor(std::log2(bnd));
      }
    std::vector<double> T((size_t)kNStencil * C * C);
    if ((e = hipMemcpyAsync(T.data(), d_T[p], sizeof(double) * T.size(), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    // scaled tables Tf[d][byte][n'] and their column exponents
    std::vector<double> Tf((size_t)kNStencil * 16 * 16, 0.0);
    for (int n = 0; n < CR; ++n) {
      double mx = 0.0;
      for (int d = 0; d < kNStencil; ++d)
        for (int b = 0; b < CR; ++b) {
          const double v = std::ldexp(T[((size_t)d * C + rowk[b]) * C + colk[n]], -st->f[p][b]);
          Tf[((size_t)d * 16 + b) * 16 + n] = v;
          mx = std::max(mx, std::fabs(v));
        }
      st->eB[p][n] = frexp_exp(mx);
    }
    // slices: [j][quad][lane][byte], lane = n' + 16 g for offset 4 quad + g
    std::vector<int8_t> host((size_t)kSliceMax * kQuadsS * 64 * 16, 0);
    for (int d = 0; d < kNStencil; ++d)
      for (int b = 0; b < 16; ++b)
        for (int n = 0; n < 16; ++n) {
          double y = std::ldexp(Tf[((size_t)d * 16 + b) * 16 + n], -st->eB[p][n]);
          const int q = d / 4, lane = n + 16 * (d % 4);
          for (int j = 0; j < kSliceMax; ++j) {
            y *= 128.0;
            const double t = std::trunc(y);
            y -= t;
            host[(((size_t)j * kQuadsS + q) * 64 + lane) * 16 + b] = (int8_t)t;
          }
        }
    if ((e = hipMalloc(&st->B[p], host.size())) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(st->B[p], host.data(), host.size(), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

void slice_tables_destroy(SliceTables* st) {
  for (int p = 0; p <= kMaxP; ++p)
    if (st->B[p]) {
      (void)hipFree(st->B[p]);
      st->B[p] = nullptr;
    }
}

hipError_t launch_m2l_slice(const MfmaTables& mt, const SliceTables& st, const WorkList& w,
                            const DevDesc* d_desc, int64_t nsub, const double* M, double* L, int S,
                            int8_t* planes, int32_t* expo, hipStream_t s) {
  if (nsub == 0 || w.count == 0) return hipSuccess;
  if (S < kSliceMin || S > kSliceMax || !st.B[2] || !st.B[3]) return hipErrorInvalidValue;
  SliceConst sc;
  for (int p = 2; p <= 3; ++p)
    for (int i = 0; i < 16; ++i) {
      sc.f[p - 2][i] = st.f[p][i];
      sc.eB[p - 2][i] = st.eB[p][i];
    }
  hipLaunchKernelGGL(slice_window_kernel, dim3((unsigned)nsub), dim3(kPrepThreads), 0, s, d_desc, M,
                     mt.hround[2], mt.hround[3], sc, S, planes, expo);
  hipLaunchKernelGGL(reset_slice_counter, dim3(1), dim3(1), 0, s, w.counter);
  const int grid = std::min(mt.num_cu, w.count);
  const v4i* b2 = reinterpret_cast<const v4i*>(st.B[2]);
  const v4i* b3 = reinterpret_cast<const v4i*>(st.B[3]);
#define SLICE_LAUNCH(SV)                                                                              \
  hipLaunchKernelGGL((m2l_fwd_slice_kernel<SV>), dim3(grid), dim3(kSliceThreads), 0, s, w.items,      \
                     w.count, w.counter, d_desc, L, planes, expo, b2, b3, mt.lds_off, mt.touch, sc,    \
                     mt.hexp[2], mt.hexp[3])
  switch (S) {
    case 6: SLICE_LAUNCH(6); break;
    case 7: SLICE_LAUNCH(7); break;
    case 8: SLICE_LAUNCH(8); break;
    default: return hipErrorInvalidValue;
  }
#undef SLICE_LAUNCH
  return hipGetLastError();
}

}  // namespace fmm
