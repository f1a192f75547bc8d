// Matrix-core M2L on gfx950: v_mfma_f64_4x4x4_4b (four independent 4x4x4
// products per instruction), persistent workgroups over a longest-first list
// of sub-grids.
//
// Forward (one workgroup owns one sub-grid's 512 targets for the whole sum):
//   L[t][n] = h^(-1-|n|) sum_d sum_k [h^-|k| M_k(t + d)] T_d[k][n]
// is a sum over (d, k) of rank-1 updates of the [512 x C] output. The
// reduction is taken four stencil offsets at a time for one moment
// component: one instruction multiplies a [16 cells x 4 offsets] slice of the
// shifted source window (A) by [4 offsets x 4 components] of the tables (B),
// for four groups of 4 cells at once. C = 20 splits into five column groups
// of 4, so no column padding is computed at p = 3.
//
// Data movement: the 20^3 reachable window of two moment components at a
// time ("round") is staged in LDS as double2 (128,000 bytes), zero on absent
// blocks and pre-scaled by h^-|k| (exact powers of two); every cell of it is
// then reused by all 892 offsets. Table operands stream from L2 (the packed
// tables are laid out in consumption order). The only HBM traffic is the
// window (read once) and L.
//
// Operand lane layouts of v_mfma_f64_4x4x4_4b (checked on gfx950):
//   A: lane l -> block (l%16)/4, row l%4, k l/16   (so: cell l%16 of a 16-cell tile)
//   B: lane l -> block (l%16)/4, col l%4, k l/16
//   D: lane l -> block (l%16)/4, col l%4, row l/16 (so: cell 4*((l%16)/4) + l/16)
#include <algorithm>
#include <functional>
#include <type_traits>

#include "kernels.h"
#include "m2l_mfma.h"
#include "p2m_common.h"

namespace fmm {

namespace {

constexpr int kWinCells = kWin * kWin * kWin;   // 8000

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__global__ void reset_counter_kernel(unsigned* counter) { *counter = 0u; }

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

template <int P, int WAVES, bool PF>
__device__ __forceinline__ void fwd_subgrid(const DevDesc& d, const double* __restrict__ M,
                                            double* __restrict__ L, const double* __restrict__ Bp,
                                            const int* __restrict__ lds_off,
                                            const uint32_t* __restrict__ touch, double2* smem) {
  constexpr int C = ncomp(P);
  constexpr int NG = (C + 3) / 4;        // output column groups of 4
  constexpr int ROUNDS = (C + 1) / 2;    // moment components staged two at a time
  constexpr int TPW = 32 / WAVES;        // 16-cell tiles per wave
  constexpr int NT = WAVES * 64;
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: keeps the per-quad table lookups on the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kk = lane >> 4;              // offset of the quad this lane feeds
  const int ci = lane & 15;              // cell of the tile this lane feeds

  // tile gt = wave*TPW + t: target plane gt/4, 4x4 patch ((gt&1)*4, ((gt>>1)&1)*4)
  int abase[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int gt = wave * TPW + t;
    const int z = gt >> 2, x = (gt & 1) * 4 + (ci & 3), y = ((gt >> 1) & 1) * 4 + (ci >> 2);
    // window coordinates of the target cell: frame (x+8, y+8, z+8) minus 2
    abase[t] = (x + 6) + kWin * (y + 6) + kWin * kWin * (z + 6);
  }
  const int zlo = (wave * TPW) >> 2, zhi = (wave * TPW + TPW - 1) >> 2;

  double acc[TPW][NG];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[t][g] = 0.0;

  const int l2 = d.log2_inv_h;
  const double* src = M + d.m_off;
  for (int r = 0; r < ROUNDS; ++r) {
    const int k0 = 2 * r, k1 = 2 * r + 1;
    const double s0 = ldexp(1.0, l2 * order_of(k0));
    const double s1 = k1 < C ? ldexp(1.0, l2 * order_of(k1)) : 0.0;
    const double* src0 = src + (size_t)k0 * kNCell;
    const double* src1 = src + (size_t)(k1 < C ? k1 : k0) * kNCell;
    // issue every load of this thread's share of the window before any LDS store,
    // so the HBM latency is paid once per round rather than once per cell
    constexpr int kStage = (kWinCells + NT - 1) / NT;
    double2 v[kStage];
#pragma unroll
    for (int i = 0; i < kStage; ++i) {
      const int c = tid + i * NT;
      v[i] = make_double2(0.0, 0.0);
      if (c < kWinCells) {
        const int wx = c % kWin, wy = (c / kWin) % kWin, wz = c / (kWin * kWin);
        const int jx = wx + kWin0, jy = wy + kWin0, jz = wz + kWin0;
        const int cell = jx + kFrame * jy + kFrame * kFrame * jz;
        if (block_present(d.mask, jx, jy, jz)) {
          v[i].x = src0[cell];
          v[i].y = src1[cell];
        }
      }
    }
    __syncthreads();   // previous round's reads of smem are done
#pragma unroll
    for (int i = 0; i < kStage; ++i) {
      const int c = tid + i * NT;
      if (c < kWinCells) smem[c] = make_double2(v[i].x * s0, v[i].y * s1);
    }
    __syncthreads();
    const double* Br = Bp + (size_t)r * kQuads * 2 * NG * 16 + kk * 4 + (lane & 3);
    // table operands of the next quad are loaded while this quad's products run
    double nb0[NG], nb1[NG];
    if (PF) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        nb0[g] = Br[g * 16];
        nb1[g] = Br[(NG + g) * 16];
      }
    }
    // per-quad scalars (blocks touched, LDS offsets) are fetched one quad ahead
    const int4* off4 = reinterpret_cast<const int4*>(lds_off);
    uint32_t tm_next = 0;
    for (int z = zlo; z <= zhi; ++z) tm_next |= touch[z * kQuads];
    int4 o_next = off4[0];
    for (int q = 0; q < kQuads; ++q) {
      const uint32_t tm = tm_next;
      const int4 o = o_next;
      if (q + 1 < kQuads) {
        tm_next = 0;
        for (int z = zlo; z <= zhi; ++z) tm_next |= touch[z * kQuads + q + 1];
        o_next = off4[q + 1];
      }
      double b0[NG], b1[NG];
      if (PF) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          b0[g] = nb0[g];
          b1[g] = nb1[g];
        }
        if (q + 1 < kQuads) {
          const double* Bn = Br + (size_t)(q + 1) * 2 * NG * 16;
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            nb0[g] = Bn[g * 16];
            nb1[g] = Bn[(NG + g) * 16];
          }
        }
      }
      if ((tm & d.mask) == 0) continue;   // every source of this quad is absent for this wave
      // each lane takes the offset of its k-slot (branch-free select of scalars)
      int doff = o.x;
      doff = kk == 1 ? o.y : doff;
      doff = kk == 2 ? o.z : doff;
      doff = kk == 3 ? o.w : doff;
      if (!PF) {
        const double* Bq = Br + (size_t)q * 2 * NG * 16;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          b0[g] = Bq[g * 16];
          b1[g] = Bq[(NG + g) * 16];
        }
      }
      double2 a[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) a[t] = smem[abase[t] + doff];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].x, b0[g], acc[t][g]);
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].y, b1[g], acc[t][g]);
      }
    }
  }

  // D layout: this lane holds cell (x = lane/16, y = (lane%16)/4) of each tile, column lane%4
  double* out = L + d.l_off;
  const int xi = lane >> 4, yi = (lane & 15) >> 2, j = lane & 3;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int gt = wave * TPW + t;
    const int z = gt >> 2, x = (gt & 1) * 4 + xi, y = ((gt >> 1) & 1) * 4 + yi;
    const int tcell = x + kBlock * y + kBlock * kBlock * z;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int n = 4 * g + j;
      if (n < C) out[(size_t)n * kNTarget + tcell] = ldexp(acc[t][g], l2 * (1 + order_of(n)));
    }
  }
}

template <int WAVES, bool PF>
__global__ void __launch_bounds__(WAVES * 64) m2l_fwd_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, const double* __restrict__ M, double* __restrict__ L,
    const double* __restrict__ B2, const double* __restrict__ B3, const double* __restrict__ B4,
    const int* __restrict__ lds_off, const uint32_t* __restrict__ touch) {
  __shared__ double2 smem[kWinCells];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= count) break;
    const DevDesc d = desc[items[item].sub];
    switch (d.p) {
      case 2: fwd_subgrid<2, WAVES, PF && (2 < 4 || WAVES == 4)>(d, M, L, B2, lds_off, touch, smem); break;
      case 3: fwd_subgrid<3, WAVES, PF && (3 < 4 || WAVES == 4)>(d, M, L, B3, lds_off, touch, smem); break;
      case 4: fwd_subgrid<4, WAVES, PF && (4 < 4 || WAVES == 4)>(d, M, L, B4, lds_off, touch, smem); break;
      default: break;
    }
    __syncthreads();   // s_item and smem are free for the next item
  }
}

// ---------------------------------------------------------------------------
// forward, table operands staged in LDS
// ---------------------------------------------------------------------------
//
// Same products and order as fwd_subgrid. Instead of every wave loading its
// table operands from L2 (16 distinct values per 64-lane load, replicated over
// the four MFMA blocks, which keeps the texture-address path ~70% busy), the
// workgroup copies the tables of a chunk of offset quads into the LDS left over
// by the window (double-buffered, one barrier per chunk) and each wave reads
// them with broadcast ds_read_b128 (both components of a column group at once).
// Table layout for this form: [round][quad][group][kk*4 + j][component].

constexpr int kBlChunkMax = 12 * 5 * 32;             // doubles per chunk buffer
// HARM: the harmonic form, (p+1)^2 folded components instead of C
// QDIV: chunks of 1/QDIV of the default length (an autotuner candidate)
template <int P, bool HARM = false, int QDIV = 1>
struct BlShape {
  static constexpr int CR = HARM ? (P + 1) * (P + 1) : ncomp(P);   // reduced components
  static constexpr int NG = (CR + 3) / 4;
  // quads per staged chunk (even: a full chunk ends on the second operand set)
  static constexpr int QC0 = HARM ? (kBlChunkMax / (NG * 32)) & ~1 : (P == 4 ? 6 : 12);
  static constexpr int QC = (QC0 / QDIV) & ~1;
  static constexpr int CHUNK = QC * NG * 32;         // doubles per chunk buffer
  static_assert(QC >= 2, "chunk length");
};
static_assert(BlShape<2>::CHUNK <= kBlChunkMax && BlShape<3>::CHUNK <= kBlChunkMax &&
              BlShape<4>::CHUNK <= kBlChunkMax && BlShape<2, true>::CHUNK <= kBlChunkMax &&
              BlShape<3, true>::CHUNK <= kBlChunkMax && BlShape<4, true>::CHUNK <= kBlChunkMax,
              "chunk buffer");
constexpr int kBlThreads = 512;

// PIPE: the inner loop reads only LDS (offsets staged once per workgroup, skip
// decisions as per-wave bitmasks), so the next quad's operand reads can be issued
// before this quad's products and waited for with partial counters.
// FULL: every neighbour block is present, so no quad is skipped and the quad
// loop carries no skip branches.
// HARM: the harmonic form. Each round stages two folded moment components
// (combinations of moment components of one order, per the round's plan), the
// products run over the (p+1)^2 harmonic columns, and L is expanded to all C
// components at the end through LDS.
// Hook: at the top of round r, when the window buffer and the table buffers are
// free (every wave is past the previous round's last barrier), hook.run() is
// called if hook.wants(r, ROUNDS) (uniform over the workgroup); it may use
// those buffers and must leave no LDS access in flight. Around it the sums so
// far are parked in the sub-grid's own L slots (written only at the end), so
// run() has the registers.
struct NoHook {
  __device__ bool wants(int, int) const { return false; }
  __device__ void run() const {}
  __device__ void run(double*) const {}
};
// the moments of the next item, at the top of round (workgroup index mod rounds)
template <class F>
struct MomentHook {
  int next, count;
  F moments;
  __device__ bool wants(int r, int rounds) const {
    return next < count && r == (int)(blockIdx.x % (unsigned)rounds);
  }
  __device__ void run() const { moments(next); }
};

// Rounds of one call: all of them, with L written; or one round, with the raw
// sums of its products (unscaled, before any expansion) written to `part`
// [column][target] for a later sum over rounds.
struct AllRounds {
  static constexpr bool kPartial = false;
  __device__ int begin() const { return 0; }
  __device__ int end(int rounds) const { return rounds; }
  __device__ double* partial() const { return nullptr; }
};
struct OneRound {
  static constexpr bool kPartial = true;
  int r;
  double* part;
  __device__ int begin() const { return r; }
  __device__ int end(int) const { return r + 1; }
  __device__ double* partial() const { return part; }
};

template <int P, bool PIPE, bool FULL = false, bool HARM = false, class Hook = NoHook, class Range = AllRounds,
          int QDIV = 1>
__device__ __forceinline__ void fwd_bl_subgrid(const DevDesc& d, const double* __restrict__ M,
                                               double* __restrict__ L,
                                               const double* __restrict__ Bl,
                                               const int* __restrict__ lds_off,
                                               const uint32_t* __restrict__ touch, double2* smem,
                                               double* sB, const int4* s_off,
                                               const HRound* __restrict__ hround = nullptr,
                                               const HExp* __restrict__ hexp = nullptr,
                                               Hook hook = Hook(), Range range = Range()) {
  constexpr int C = ncomp(P);
  constexpr int CR = BlShape<P, HARM, QDIV>::CR;
  constexpr int NG = BlShape<P, HARM, QDIV>::NG;
  constexpr int QC = BlShape<P, HARM, QDIV>::QC;
  constexpr int CH2 = BlShape<P, HARM, QDIV>::CHUNK / 2;    // double2 per chunk
  constexpr int ROUNDS = (CR + 1) / 2;
  constexpr int TPW = 4, NT = kBlThreads;
  constexpr int NCHUNK = (kQuads + QC - 1) / QC;
  static_assert((CH2 + NT - 1) / NT <= 2, "at most two staged table values per thread");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // target plane
  const int kk = lane >> 4, ci = lane & 15;
  int abase[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int x = (t & 1) * 4 + (ci & 3), y = (t >> 1) * 4 + (ci >> 2);
    abase[t] = (x + 6) + kWin * (y + 6) + kWin * kWin * (wave + 6);
  }
  double acc[TPW][NG];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[t][g] = 0.0;

  const int l2 = d.log2_inv_h;
  const double* src = M + d.m_off;
  const int4* off4 = reinterpret_cast<const int4*>(lds_off);
  const uint32_t* tw = touch + wave * kQuads;
  double2* sB2 = reinterpret_cast<double2*>(sB);
  const int boff = kk * 4 + (lane & 3);                // this lane's slot in a column group
  uint32_t cl0 = 0;                                    // live quads of chunk 0
  if constexpr (PIPE) {
    const bool on = lane < QC && (tw[min(lane, QC - 1)] & d.mask) != 0;
    cl0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(__ballot(on) & 0xffffffffu));
  }
  for (int r = range.begin(); r < range.end(ROUNDS); ++r) {
    if (hook.wants(r, ROUNDS)) {
      double* park = L + d.l_off;
      const int pxi = lane >> 4, pyi = (lane & 15) >> 2, pj = lane & 3;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tcell = ((t & 1) * 4 + pxi) + kBlock * ((t >> 1) * 4 + pyi) + kBlock * kBlock * wave;
#pragma unroll
        for (int g = 0; g < NG; ++g)
          if (4 * g + pj < CR) park[(size_t)(4 * g + pj) * kNTarget + tcell] = acc[t][g];
      }
      asm volatile("" ::: "memory");   // the sums are reloaded, not kept in registers
      hook.run();
      asm volatile("" ::: "memory");
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tcell = ((t & 1) * 4 + pxi) + kBlock * ((t >> 1) * 4 + pyi) + kBlock * kBlock * wave;
#pragma unroll
        for (int g = 0; g < NG; ++g)
          acc[t][g] = 4 * g + pj < CR ? park[(size_t)(4 * g + pj) * kNTarget + tcell] : 0.0;
      }
    }
    double s0, s1;
    const double *src0 = nullptr, *src1 = nullptr;
    if constexpr (HARM) {
      s0 = ldexp(1.0, l2 * hround[r].ord0);
      s1 = hround[r].ord1 >= 0 ? ldexp(1.0, l2 * hround[r].ord1) : 0.0;
    } else {
      const int k0 = 2 * r, k1 = 2 * r + 1;
      s0 = ldexp(1.0, l2 * order_of(k0));
      s1 = k1 < C ? ldexp(1.0, l2 * order_of(k1)) : 0.0;
      src0 = src + (size_t)k0 * kNCell;
      src1 = src + (size_t)(k1 < C ? k1 : k0) * kNCell;
    }
    // tables of chunk 0 (contiguous in this layout)
    const double2* gB = reinterpret_cast<const double2*>(Bl + (size_t)r * kQuads * NG * 32);
    // (clamped indices: every element is loaded, so the staging stays in registers;
    // slots past the chunk's quads are never read)
    double2 bst0 = gB[min(tid, CH2 - 1)], bst1 = gB[min(tid + NT, CH2 - 1)];
    // window: two halves of loads-then-stores keep the staging registers small
    constexpr int kStage = (kWinCells + NT - 1) / NT;
    constexpr int kHalf = (kStage + 1) / 2;
    // with a hook, the staging indices are recomputed each round from an opaque
    // copy of tid instead of being kept live across the rounds (and the hook)
    int stid = tid;
    if constexpr (!std::is_same_v<Hook, NoHook>) asm volatile("" : "+v"(stid));
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      double2 v[kHalf];
      if constexpr (HARM) {
        // folded components: sum over the round's moment components, in plan order
        int cell[kHalf];
        bool on[kHalf];
#pragma unroll
        for (int i = 0; i < kHalf; ++i) {
          const int c = stid + (hb * kHalf + i) * NT;
          v[i] = make_double2(0.0, 0.0);
          const int wx = c % kWin, wy = (c / kWin) % kWin, wz = c / (kWin * kWin);
          const int jx = wx + kWin0, jy = wy + kWin0, jz = wz + kWin0;
          cell[i] = jx + kFrame * jy + kFrame * kFrame * jz;
          on[i] = hb * kHalf + i < kStage && c < kWinCells && block_present(d.mask, jx, jy, jz);
        }
        const int nsup = hround[r].nsup;
        for (int u = 0; u < nsup; ++u) {
          const double* su = src + (size_t)hround[r].comp[u] * kNCell;
          const double f0 = hround[r].c0[u], f1 = hround[r].c1[u];
          double x[kHalf];
#pragma unroll
          for (int i = 0; i < kHalf; ++i) x[i] = on[i] ? su[cell[i]] : 0.0;
#pragma unroll
          for (int i = 0; i < kHalf; ++i) {
            v[i].x = __builtin_fma(f0, x[i], v[i].x);
            v[i].y = __builtin_fma(f1, x[i], v[i].y);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < kHalf; ++i) {
          const int c = stid + (hb * kHalf + i) * NT;
          v[i] = make_double2(0.0, 0.0);
          if (hb * kHalf + i < kStage && c < kWinCells) {
            const int wx = c % kWin, wy = (c / kWin) % kWin, wz = c / (kWin * kWin);
            const int jx = wx + kWin0, jy = wy + kWin0, jz = wz + kWin0;
            const int cell = jx + kFrame * jy + kFrame * kFrame * jz;
            if (block_present(d.mask, jx, jy, jz)) {
              v[i].x = src0[cell];
              v[i].y = src1[cell];
            }
          }
        }
      }
      if (hb == 0) __syncthreads();   // previous round's reads of smem and sB are done
#pragma unroll
      for (int i = 0; i < kHalf; ++i) {
        const int c = stid + (hb * kHalf + i) * NT;
        if (hb * kHalf + i < kStage && c < kWinCells) smem[c] = make_double2(v[i].x * s0, v[i].y * s1);
      }
    }
    sB2[tid] = bst0;
    if (tid + NT < CH2) sB2[tid + NT] = bst1;
    __syncthreads();
    // bit i of cl: quad q0 + i has a present source for this wave's plane (the
    // next chunk's touch words are loaded with its tables and reduced at its end)
    uint32_t cl = cl0;
    [[maybe_unused]] double2 a0[TPW], b0[NG], a1[TPW], b1[NG];   // operand sets (PIPE)
    [[maybe_unused]] int offn = 0;
    [[maybe_unused]] const int* so = reinterpret_cast<const int*>(s_off) + kk;
    static_assert(QC % 2 == 0, "a full chunk ends on the second operand set");
    for (int ch = 0; ch < NCHUNK; ++ch) {
      const int q0 = ch * QC;
      const int nq = min(QC, kQuads - q0);
      // next chunk's tables: global loads now, LDS stores after this chunk
      const bool more = ch + 1 < NCHUNK;
      const int nq2 = more ? min(QC, kQuads - q0 - QC) : 1;
      uint32_t tn = 0;
      if (more) {
        if constexpr (PIPE) tn = tw[q0 + QC + min(lane, nq2 - 1)];
        const int n2 = nq2 * NG * 16;
        const double2* gn = gB + (size_t)(q0 + QC) * NG * 16;
        bst0 = gn[min(tid, n2 - 1)];
        bst1 = gn[min(tid + NT, n2 - 1)];
      }
      const double2* bb = sB2 + (ch & 1) * CH2 + boff;
      if constexpr (PIPE) {
        // Two operand sets: the reads of quad qi + 1 are issued before the products
        // of quad qi, and the offset of qi + 2 one step further ahead. The reads
        // are unconditional, with table indices clamped into the chunk, so every
        // path into a product sees the same outstanding reads; operands read past
        // the chunk's last quad are never multiplied. Window offsets are not
        // clamped to the chunk, so a full chunk's last step leaves the window
        // operands of the next chunk's first quad in (a0, offn): after the
        // barrier only its table operands are read.
#define BL_LOADA(DA, OFF)                                                      \
  {                                                                            \
    const int doff_ = (OFF);                                                   \
    _Pragma("unroll") for (int t = 0; t < TPW; ++t) DA[t] = smem[abase[t] + doff_]; \
  }
#define BL_LOADB(DB, QI)                                                       \
  { _Pragma("unroll") for (int g = 0; g < NG; ++g) DB[g] = bb[((QI) * NG + g) * 16]; }
#define BL_LOAD(DA, DB, QI, OFF) \
  BL_LOADA(DA, OFF);             \
  BL_LOADB(DB, QI);
#define BL_MMA(SA, SB)                                                              \
  _Pragma("unroll") for (int t = 0; t < TPW; ++t) {                                 \
    _Pragma("unroll") for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(SA[t].x, SB[g].x, acc[t][g]); \
    _Pragma("unroll") for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(SA[t].y, SB[g].y, acc[t][g]); \
  }
// the reads for the next quad are spread through the first half of this quad's
// products, so no wave has a long stretch without matrix instructions (the two
// waves of a SIMD run in step between barriers and would otherwise leave the unit
// idle together), and the last read has half the products to complete
#define BL_INTERLEAVE()                                                             \
  {                                                                                 \
    constexpr int NLD = TPW + NG + 1, NMF = 2 * TPW * NG, PER = NMF / NLD > 2 ? 2 : 1; \
    _Pragma("unroll") for (int i_ = 0; i_ < NLD; ++i_) {                            \
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                            \
      __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);                          \
    }                                                                               \
    __builtin_amdgcn_sched_group_barrier(0x008, NMF - PER * NLD, 0);                \
  }
// product of quad QI from (SA, SB) while the reads of quad QN go into (DA, DB) and
// the offset of quad OQ into offn
#define BL_STEP(SA, SB, QI, DA, DB, QN, OQ)                                         \
  if (FULL || ((cl >> (QI)) & 1u)) {                                                \
    BL_LOAD(DA, DB, QN, offn);                                                      \
    offn = so[(OQ) * 4];                                                            \
    BL_MMA(SA, SB);                                                                 \
    BL_INTERLEAVE();                                                                \
  } else {                                                                          \
    __builtin_amdgcn_sched_barrier(0); /* keeps the reads in each branch's block */ \
    BL_LOAD(DA, DB, QN, offn);                                                      \
    offn = so[(OQ) * 4];                                                            \
  }
        if (ch == 0) {
          BL_LOADA(a0, so[q0 * 4]);
          offn = so[min(q0 + 1, kQuads - 1) * 4];
        }
        BL_LOADB(b0, 0);
#pragma unroll 1
        for (int qi = 0; qi < nq; qi += 2) {
          BL_STEP(a0, b0, qi, a1, b1, min(qi + 1, nq - 1), min(q0 + qi + 2, kQuads - 1));
          if (qi + 1 >= nq) break;
          BL_STEP(a1, b1, qi + 1, a0, b0, min(qi + 2, nq - 1), min(q0 + qi + 3, kQuads - 1));
          if (qi == 4 && more) {
            // next chunk's tables, stored mid-chunk (the buffer was freed by the
            // previous chunk's barrier) so the barrier does not wait on them
            double2* dst = sB2 + ((ch + 1) & 1) * CH2;
            dst[tid] = bst0;
            if (tid + NT < CH2) dst[tid + NT] = bst1;
          }
        }
#undef BL_LOADA
#undef BL_LOADB
#undef BL_LOAD
#undef BL_MMA
#undef BL_INTERLEAVE
#undef BL_STEP
      } else {
        uint32_t tm_next = tw[q0];
        int4 o_next = off4[q0];
        for (int qi = 0; qi < nq; ++qi) {
          const uint32_t tm = tm_next;
          const int4 o = o_next;
          if (qi + 1 < nq) {
            tm_next = tw[q0 + qi + 1];
            o_next = off4[q0 + qi + 1];
          }
          if ((tm & d.mask) == 0) continue;   // every source of this quad is absent for this wave
          int doff = o.x;
          doff = kk == 1 ? o.y : doff;
          doff = kk == 2 ? o.z : doff;
          doff = kk == 3 ? o.w : doff;
          double2 a[TPW];
#pragma unroll
          for (int t = 0; t < TPW; ++t) a[t] = smem[abase[t] + doff];
          double2 b[NG];
#pragma unroll
          for (int g = 0; g < NG; ++g) b[g] = bb[(qi * NG + g) * 16];
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
#pragma unroll
            for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].x, b[g].x, acc[t][g]);
#pragma unroll
            for (int g = 0; g < NG; ++g) acc[t][g] = mfma4(a[t].y, b[g].y, acc[t][g]);
          }
        }
      }
      if (more) {
        if constexpr (!PIPE || QC < 6) {
          double2* dst = sB2 + ((ch + 1) & 1) * CH2;
          dst[tid] = bst0;
          if (tid + NT < CH2) dst[tid + NT] = bst1;
        }
        if constexpr (PIPE) {
          const bool on = lane < nq2 && (tn & d.mask) != 0;
          cl = (uint32_t)__builtin_amdgcn_readfirstlane((int)(__ballot(on) & 0xffffffffu));
        }
      }
      __syncthreads();   // next chunk's tables visible; this chunk's buffer free
    }
  }

  const int xi = lane >> 4, yi = (lane & 15) >> 2, j = lane & 3;
  if constexpr (Range::kPartial) {
    double* part = range.partial();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tcell = ((t & 1) * 4 + xi) + kBlock * ((t >> 1) * 4 + yi) + kBlock * kBlock * wave;
#pragma unroll
      for (int g = 0; g < NG; ++g)
        if (4 * g + j < CR) part[(size_t)(4 * g + j) * kNTarget + tcell] = acc[t][g];
    }
    return;
  }
  double* out = L + d.l_off;
  if constexpr (HARM) {
    // harmonic columns to LDS ([n'][target], over the window, which every wave
    // has finished reading), then each thread expands one target to all C
    __syncthreads();
    double* lh = reinterpret_cast<double*>(smem);
    static_assert(CR * kNTarget <= 2 * kWinCells, "harmonic columns fit the window buffer");
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int x = (t & 1) * 4 + xi, y = (t >> 1) * 4 + yi;
      const int tcell = x + kBlock * y + kBlock * kBlock * wave;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int n = 4 * g + j;
        if (n < CR) lh[n * kNTarget + tcell] = acc[t][g];
      }
    }
    __syncthreads();
    static_assert(kBlThreads == kNTarget, "one target per thread");
#pragma unroll
    for (int n = 0; n < C; ++n) {
      const HExp& e = hexp[n];
      double v = 0.0;
      for (int u = 0; u < e.nterm; ++u) v = __builtin_fma(e.coef[u], lh[e.col[u] * kNTarget + tid], v);
      out[(size_t)n * kNTarget + tid] = ldexp(v, l2 * (1 + order_of(n)));
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int x = (t & 1) * 4 + xi, y = (t >> 1) * 4 + yi;
    const int tcell = x + kBlock * y + kBlock * kBlock * wave;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int n = 4 * g + j;
      if (n < C) out[(size_t)n * kNTarget + tcell] = ldexp(acc[t][g], l2 * (1 + order_of(n)));
    }
  }
}

// FUSE: the kernel computes each sub-grid's moments itself (the frame rows
// holding the reachable window, 8 particles per cell, written to M as the P2M
// kernel writes them) before that sub-grid's M2L reads them. A workgroup takes
// its next item when it starts an item and computes the next item's moments at
// the top of round (workgroup index mod rounds) of the current one, so at any
// time only about 1/rounds of the workgroups are in their HBM-bound moment
// phase while the others keep the matrix cores busy. Only the first item's
// moments are computed before any M2L. The moments are written and read by the
// same workgroup, with barriers between.
template <bool PIPE, bool HARM = false, bool FUSE = false, int QDIV = 1>
__global__ void __launch_bounds__(kBlThreads) m2l_fwd_bl_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, const double* M, double* __restrict__ L,
    const double* __restrict__ B2, const double* __restrict__ B3, const double* __restrict__ B4,
    const int* __restrict__ lds_off, const uint32_t* __restrict__ touch,
    const HRound* __restrict__ hr2, const HRound* __restrict__ hr3, const HRound* __restrict__ hr4,
    const HExp* __restrict__ he2, const HExp* __restrict__ he3, const HExp* __restrict__ he4,
    const double* __restrict__ pos = nullptr, const double* __restrict__ mass = nullptr,
    double* Mw = nullptr) {
  // (FUSE: Mw is M, writable; the moment phase writes through it)
  __shared__ double2 smem[kWinCells];
  __shared__ double sB[2 * kBlChunkMax];
  __shared__ int4 s_off[kQuads];
  __shared__ int s_item;
  static_assert(kP2MRowsLds <= 2 * kWinCells && kBlThreads == kP2MRowsThreads,
                "the moment phase fits the window buffer and the workgroup");
  if (PIPE) {
    const int4* off4 = reinterpret_cast<const int4*>(lds_off);
    for (int i = threadIdx.x; i < kQuads; i += blockDim.x) s_off[i] = off4[i];
  }
  // moments of item `it` into M (the window buffer is free whenever this runs)
  auto moments = [&](int it) __attribute__((always_inline)) {
    const DevDesc dn = desc[items[it].sub];
    double* lds = reinterpret_cast<double*>(smem);
    switch (dn.p) {
      case 2: p2m_window_rows<2>(dn, pos, mass, Mw, lds); break;
      case 3: p2m_window_rows<3>(dn, pos, mass, Mw, lds); break;
      case 4: p2m_window_rows<4>(dn, pos, mass, Mw, lds); break;
      default: break;
    }
  };
  int cur = 0;
  if constexpr (FUSE) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    cur = s_item;
    __syncthreads();   // every thread holds cur before s_item is written again
    if (cur < count) moments(cur);
  }
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    // FUSE: s_item is the next item, whose moments are computed during this one
    const int item = FUSE ? cur : s_item;
    const int next = s_item;
    if (item >= count) break;
    const DevDesc d = desc[items[item].sub];
    const bool full = d.mask == kFullMask;
    const auto hook = [&]() {
      if constexpr (FUSE) return MomentHook<decltype(moments)>{next, count, moments};
      else return NoHook{};
    }();
    switch (d.p) {
      case 2:
        if (PIPE && full)
          fwd_bl_subgrid<2, PIPE, true, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B2, lds_off, touch, smem, sB,
                                                                              s_off, hr2, he2, hook);
        else
          fwd_bl_subgrid<2, PIPE, false, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B2, lds_off, touch, smem, sB,
                                                                              s_off, hr2, he2, hook);
        break;
      case 3:
        if (PIPE && full)
          fwd_bl_subgrid<3, PIPE, true, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B3, lds_off, touch, smem, sB,
                                                                              s_off, hr3, he3, hook);
        else
          fwd_bl_subgrid<3, PIPE, false, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B3, lds_off, touch, smem, sB,
                                                                              s_off, hr3, he3, hook);
        break;
      case 4:
        // the dense p = 4 operand sets (9 column groups) do not fit the registers
        // of the pipelined loop; the harmonic ones (7) do
        if (HARM && PIPE && full)
          fwd_bl_subgrid<4, PIPE, true, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B4, lds_off, touch, smem, sB,
                                                                               s_off, hr4, he4, hook);
        else if (HARM && PIPE)
          fwd_bl_subgrid<4, PIPE, false, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B4, lds_off, touch, smem, sB,
                                                                                s_off, hr4, he4, hook);
        else
          fwd_bl_subgrid<4, false, false, HARM, std::remove_cv_t<decltype(hook)>, AllRounds, QDIV>(d, M, L, B4, lds_off, touch, smem, sB,
                                                                                s_off, hr4, he4, hook);
        break;
      default: break;
    }
    __syncthreads();   // every thread has read s_item; the item's LDS use is done
    cur = next;
  }
}

// ---------------------------------------------------------------------------
// split precision forward
// ---------------------------------------------------------------------------
//
// M = M_hi + M_lo and T = T_hi + T_lo (float32 parts of the float64 values;
// T_hi/T_lo are split from the float64 tables, M after its h-scaling). Per
// offset block the three products M_hi T_hi + M_hi T_lo + M_lo T_hi are
// summed in float32 on the matrix cores; each block sum is added to float64
// accumulators, and the h^(-1-|n|) scaling is applied in float64. One block
// is 16 offset quads (64 offsets) of one staged component pair.
//
// Columns n < 16 * NCT use v_mfma_f32_16x16x4 (A: lane -> cell l%16, offset
// slot l/16; B: lane -> offset slot l/16, column l%16; D: lane, v -> cell
// 4*(l/16)+v, column l%16). The remaining C - 16 * NCT columns use
// v_mfma_f32_4x4x1_16b on the same A register: block b = l/4 takes offset
// slot b/4 and cells 4*(b%4)..+3, so its D (lane, v -> cell 4*((l/4)%4)+v,
// column l%4) holds one partial sum per offset slot, added across slots
// at the end.

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma4x1(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

constexpr int kSplitBlockQuads = 16;   // 64 offsets per float32 block sum

// Columns handled in this call: 16-wide tiles [CT0, CT0 + NCTP) and, if WREM,
// the remainder columns (p = 4 runs two calls so its accumulators fit).
template <int P, int CT0, int NCTP, bool WREM>
__device__ __forceinline__ void fwd_split_subgrid(const DevDesc& d, const double* __restrict__ M,
                                                  double* __restrict__ L,
                                                  const float* __restrict__ Bhi,
                                                  const float* __restrict__ Blo,
                                                  const int* __restrict__ lds_off,
                                                  const uint32_t* __restrict__ touch, float4* smem) {
  constexpr int C = ncomp(P);
  constexpr int NG = (C + 3) / 4;                   // groups of 4 columns in the packed tables
  constexpr int ROUNDS = (C + 1) / 2;
  constexpr int NCT_ALL = C >= 16 ? C / 16 : 1;     // 16-wide column tiles in total
  constexpr int NCT = NCTP;                         // ... in this call
  constexpr int REM = WREM && C - 16 * NCT_ALL > 0 ? C - 16 * NCT_ALL : 0;   // 4x4x1 columns
  constexpr int WAVES = 8, TPW = 4, NT = WAVES * 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kk = lane >> 4, ci = lane & 15;
  int abase[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int gt = wave * TPW + t;
    const int z = gt >> 2, x = (gt & 1) * 4 + (ci & 3), y = ((gt >> 1) & 1) * 4 + (ci >> 2);
    abase[t] = (x + 6) + kWin * (y + 6) + kWin * kWin * (z + 6);
  }
  const int zp = wave;   // one target plane per wave

  double acc[TPW][NCT][4];
  double racc[TPW][4];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][c][v] = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) racc[t][v] = 0.0;
  }

  // lane offsets into one (round, quad, comp) chunk of the packed tables
  int boff[NCT];
  bool bvalid[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    const int g = 4 * (CT0 + c) + (ci >> 2);
    bvalid[c] = g < NG;
    boff[c] = (bvalid[c] ? g : 0) * 16 + kk * 4 + (lane & 3);
  }
  const int roff = 4 * NCT_ALL * 16 + kk * 4 + (lane & 3);   // remainder group

  const int l2 = d.log2_inv_h;
  const double* src = M + d.m_off;
  for (int r = 0; r < ROUNDS; ++r) {
    const int k0 = 2 * r, k1 = 2 * r + 1;
    const double s0 = ldexp(1.0, l2 * order_of(k0));
    const double s1 = k1 < C ? ldexp(1.0, l2 * order_of(k1)) : 0.0;
    const double* src0 = src + (size_t)k0 * kNCell;
    const double* src1 = src + (size_t)(k1 < C ? k1 : k0) * kNCell;
    // two halves of loads-then-stores keep the staging registers small
    constexpr int kStage = (kWinCells + NT - 1) / NT;
    constexpr int kHalf = (kStage + 1) / 2;
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      double2 v[kHalf];
#pragma unroll
      for (int i = 0; i < kHalf; ++i) {
        const int c = tid + (hb * kHalf + i) * NT;
        v[i] = make_double2(0.0, 0.0);
        if (hb * kHalf + i < kStage && c < kWinCells) {
          const int wx = c % kWin, wy = (c / kWin) % kWin, wz = c / (kWin * kWin);
          const int jx = wx + kWin0, jy = wy + kWin0, jz = wz + kWin0;
          const int cell = jx + kFrame * jy + kFrame * kFrame * jz;
          if (block_present(d.mask, jx, jy, jz)) {
            v[i].x = src0[cell];
            v[i].y = src1[cell];
          }
        }
      }
      if (hb == 0) __syncthreads();   // previous round's reads of smem are done
#pragma unroll
      for (int i = 0; i < kHalf; ++i) {
        const int c = tid + (hb * kHalf + i) * NT;
        if (hb * kHalf + i < kStage && c < kWinCells) {
          const double a0 = v[i].x * s0, a1 = v[i].y * s1;
          const float h0 = (float)a0, h1 = (float)a1;
          smem[c] = make_float4(h0, (float)(a0 - (double)h0), h1, (float)(a1 - (double)h1));
        }
      }
    }
    __syncthreads();

    const size_t chunk = (size_t)NG * 16;                     // one comp of one quad
    const float* Rh = Bhi + (size_t)r * kQuads * 2 * chunk;
    const float* Rl = Blo + (size_t)r * kQuads * 2 * chunk;
    const int4* off4 = reinterpret_cast<const int4*>(lds_off);
    uint32_t tm_next = touch[zp * kQuads];
    int4 o_next = off4[0];
    v4f f[TPW][NCT], fr[TPW];
    for (int q = 0; q < kQuads; ++q) {
      if (q % kSplitBlockQuads == 0) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
#pragma unroll
          for (int c = 0; c < NCT; ++c) f[t][c] = (v4f){0.f, 0.f, 0.f, 0.f};
          fr[t] = (v4f){0.f, 0.f, 0.f, 0.f};
        }
      }
      const uint32_t tm = tm_next;
      const int4 o = o_next;
      if (q + 1 < kQuads) {
        tm_next = touch[zp * kQuads + q + 1];
        o_next = off4[q + 1];
      }
      if ((tm & d.mask) != 0) {
        int doff = o.x;
        doff = kk == 1 ? o.y : doff;
        doff = kk == 2 ? o.z : doff;
        doff = kk == 3 ? o.w : doff;
        const float* Qh = Rh + (size_t)q * 2 * chunk;
        const float* Ql = Rl + (size_t)q * 2 * chunk;
        float bh[2][NCT], bl[2][NCT], rh[2], rl[2];
#pragma unroll
        for (int cp = 0; cp < 2; ++cp) {
#pragma unroll
          for (int c = 0; c < NCT; ++c) {
            bh[cp][c] = bvalid[c] ? Qh[cp * chunk + boff[c]] : 0.f;
            bl[cp][c] = bvalid[c] ? Ql[cp * chunk + boff[c]] : 0.f;
          }
          rh[cp] = REM ? Qh[cp * chunk + roff] : 0.f;
          rl[cp] = REM ? Ql[cp * chunk + roff] : 0.f;
        }
        float4 a[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) a[t] = smem[abase[t] + doff];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
#pragma unroll
          for (int cp = 0; cp < 2; ++cp) {
            const float ah = cp ? a[t].z : a[t].x, al = cp ? a[t].w : a[t].y;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
              f[t][c] = mfma16(ah, bh[cp][c], f[t][c]);
              f[t][c] = mfma16(ah, bl[cp][c], f[t][c]);
              f[t][c] = mfma16(al, bh[cp][c], f[t][c]);
            }
            if (REM) {
              fr[t] = mfma4x1(ah, rh[cp], fr[t]);
              fr[t] = mfma4x1(ah, rl[cp], fr[t]);
              fr[t] = mfma4x1(al, rh[cp], fr[t]);
            }
          }
        }
      }
      if (q % kSplitBlockQuads == kSplitBlockQuads - 1 || q == kQuads - 1) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
#pragma unroll
          for (int c = 0; c < NCT; ++c)
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) acc[t][c][v2] += (double)f[t][c][v2];
#pragma unroll
          for (int v2 = 0; v2 < 4; ++v2) racc[t][v2] += (double)fr[t][v2];
        }
      }
    }
  }

  double* out = L + d.l_off;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int gt = wave * TPW + t;
    const int z = gt >> 2, x0 = (gt & 1) * 4, y0 = ((gt >> 1) & 1) * 4;
    // 16x16 tiles: lane, v -> cell 4*(lane/16) + v (x = v, y = lane/16), column lane%16
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int n = 16 * (CT0 + c) + (lane & 15);
#pragma unroll
      for (int v2 = 0; v2 < 4; ++v2) {
        const int tcell = (x0 + v2) + kBlock * (y0 + (lane >> 4)) + kBlock * kBlock * z;
        if (n < C) out[(size_t)n * kNTarget + tcell] = ldexp(acc[t][c][v2], l2 * (1 + order_of(n)));
      }
    }
    if (REM) {
      // sum the four offset-slot partials (lanes l, l^16, l^32, l^48)
#pragma unroll
      for (int v2 = 0; v2 < 4; ++v2) {
        double s = racc[t][v2];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        const int cell = 4 * ((lane >> 2) & 3) + v2;          // x = v2, y = (lane/4)%4
        const int n = 16 * NCT_ALL + (lane & 3);
        const int tcell = (x0 + (cell & 3)) + kBlock * (y0 + (cell >> 2)) + kBlock * kBlock * z;
        if (lane < 16 && n < C) out[(size_t)n * kNTarget + tcell] = ldexp(s, l2 * (1 + order_of(n)));
      }
    }
  }
}

__global__ void __launch_bounds__(512) m2l_fwd_split_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, const double* __restrict__ M, double* __restrict__ L,
    const float* __restrict__ H2, const float* __restrict__ L2v, const float* __restrict__ H3,
    const float* __restrict__ L3v, const float* __restrict__ H4, const float* __restrict__ L4v,
    const int* __restrict__ lds_off, const uint32_t* __restrict__ touch) {
  __shared__ float4 smem[kWinCells];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= count) break;
    const DevDesc d = desc[items[item].sub];
    switch (d.p) {
      case 2: fwd_split_subgrid<2, 0, 1, true>(d, M, L, H2, L2v, lds_off, touch, smem); break;
      case 3: fwd_split_subgrid<3, 0, 1, true>(d, M, L, H3, L3v, lds_off, touch, smem); break;
      case 4:
        fwd_split_subgrid<4, 0, 1, false>(d, M, L, H4, L4v, lds_off, touch, smem);
        __syncthreads();
        fwd_split_subgrid<4, 1, 1, true>(d, M, L, H4, L4v, lds_off, touch, smem);
        break;
      default: break;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// adjoint: dM_k(s) = h^-|k| sum_{(t, d) : t + d = s} sum_n [h^(-1-|n|) dL_n(t)] T_d[k][n]
// ---------------------------------------------------------------------------
//
// Scatter form: every (target t, offset d) pair contributes to exactly one
// output cell s = t + d of the 20^3 window, so no product is wasted (a
// gather over output tiles would compute mostly zeros, since dL lives on
// the 8^3 block only). One workgroup owns one sub-grid; for each pair of
// output components ("round") the window's accumulators live in LDS. Wave w
// holds target plane w (its dL values stay in registers for the whole
// sub-grid) and applies the offsets of one group at a time (one dz, or two dz
// at least 8 apart), so within a group every output cell has one writing wave.
// One instruction multiplies [16 targets x 4 dL components] by [4 components
// x (2 output components x 2 offsets)]; the two offsets of a pair never map
// two cells of one 4x4 tile to the same output cell (|dx2 - dx1| >= 4 or
// |dy2 - dy1| >= 4, or different dz). Results
// are added with LDS atomic adds that return nothing; one wave's LDS
// operations execute in issue order, so each cell's sum is taken in pair
// order and the result is reproducible bit for bit.

constexpr int kBwdWaves = 8;
constexpr int kBwdThreads = kBwdWaves * 64;
// component stride of the LDS accumulators: odd, so that the two components a
// lane pair adds (lanes 2i and 2i + 1) fall in different banks; an even stride
// doubles the LDS cycles of every add (measured: 16.2 against 8.3 cycles for a
// 64-lane ds_add_f64 in this kernel's address pattern)
constexpr int kAccStride = kWinCells + 17;
constexpr int kMaxPairs = 512;
constexpr int kBwdGroups = 8;       // offset groups, between barriers (see build_pairs)

// FULL: every neighbour block is present, so no pair is skipped and the pair
// loop carries no branches.
// HARM: the harmonic form; dL is folded to the (p+1)^2 harmonic columns, the
// rounds accumulate folded output components and the write-out expands them.
// Hook: as for the forward kernel; here it runs after the barrier at the top of
// round r, with the accumulators all zero, may use them as scratch, and they
// are cleared again after it. The A operands are rebuilt from dL after it.
template <int P, bool FULL, bool HARM = false, class Hook = NoHook>
__device__ __forceinline__ void bwd_subgrid(const DevDesc& d, const double* __restrict__ dL,
                                            double* dM, const double* __restrict__ Bp,
                                            int npairs, const int* s_gs,
                                            const uint32_t* __restrict__ ptouch, double* smem,
                                            const int4* __restrict__ pairs, const HFold* __restrict__ hfold = nullptr,
                                            const HOut* __restrict__ hout = nullptr, Hook hook = Hook()) {
  constexpr int C = ncomp(P);
  constexpr int CR = HARM ? (P + 1) * (P + 1) : C;   // reduced components
  constexpr int KC = (CR + 3) / 4;    // dL component chunks of 4 (the reduction)
  constexpr int ROUNDS = (CR + 1) / 2;
  constexpr int TPW = 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // target plane
  const int kk = lane >> 4, ci = lane & 15, j = lane & 3;
  const int slot = j & 1, half = j >> 1;    // output component of the round, offset of the pair
  const int l2 = d.log2_inv_h;

  // A operands: dL of this wave's four 4x4 tiles, scaled by h^(-1-|n|)
  double a[TPW][KC];
  int obase[TPW];
  const double* src = dL + d.l_off;
  auto load_a = [&]() {
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int x0 = (t & 1) * 4, y0 = (t >> 1) * 4;
    const int tcell = x0 + (ci & 3) + kBlock * (y0 + (ci >> 2)) + kBlock * kBlock * wave;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int n = 4 * kc + kk;
      if constexpr (HARM) {
        // folded dL: the components that fold onto column n' (all of one order)
        double v = 0.0;
        if (n < CR) {
          const HFold& f = hfold[n];
          for (int u = 0; u < f.nterm; ++u)
            v = __builtin_fma(f.coef[u], src[(size_t)f.comp[u] * kNTarget + tcell], v);
          v = ldexp(v, l2 * (1 + order_of(f.comp[0])));
        }
        a[t][kc] = v;
      } else {
        a[t][kc] = n < C ? ldexp(src[(size_t)n * kNTarget + tcell], l2 * (1 + order_of(n))) : 0.0;
      }
    }
    // D layout: lane holds target cell (x = lane/16, y = (lane%16)/4) of the tile
    obase[t] = (x0 + (lane >> 4) + 6) + kWin * (y0 + ((lane & 15) >> 2) + 6) + kWin * kWin * (wave + 6) +
               slot * kAccStride;
  }
  };
  load_a();

  for (int i = tid; i < 2 * kAccStride; i += kBwdThreads) smem[i] = 0.0;

  // the pairs' output offsets (this lane's half) and, per target plane, the
  // blocks each pair writes, through buffer resources like the tables: waits for
  // them are waits on the vector memory counter, never on the LDS adds
  const __amdgpu_buffer_rsrc_t prs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int4*>(pairs), (short)0, npairs * 16, 0x00020000);
  const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint32_t*>(ptouch + wave * npairs), (short)0, npairs * 4, 0x00020000);
  double* out = dM + d.m_off;
  for (int r = 0; r < ROUNDS; ++r) {
    __syncthreads();
    if (hook.wants(r, ROUNDS)) {
      hook.run(smem);
      __syncthreads();
      for (int i = tid; i < 2 * kAccStride; i += kBwdThreads) smem[i] = 0.0;
      __syncthreads();
      load_a();
    }
    // tables through a buffer resource: a per-pair scalar offset and this lane's
    // fixed byte offset, so no per-pair address registers (reads past the end of
    // the tables would return zeros)
    const __amdgpu_buffer_rsrc_t brs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(Bp), (short)0, ROUNDS * npairs * KC * 16 * (int)sizeof(double), 0x00020000);
    const int sbase = r * npairs * KC * 16 * (int)sizeof(double);
    const int vboff = (kk * 4 + j) * (int)sizeof(double);
    // Three sets (tables, touch mask, products, output offset) rotate over the
    // pairs: at pair q the set of pair q - 1, whose products are issued, takes
    // the tables of pair q + 2 and the output offset of pair q - 1, and a set's
    // products are added into LDS (at that offset) just before the set is
    // multiplied again. Each offset is thus used two pairs after its load and
    // never copied, so no wait on a load younger than the tables in use. After
    // a barrier the sets hold zeros, so those adds change nothing.
    double b0[KC], b1[KC], b2[KC], acc0[TPW], acc1[TPW], acc2[TPW];
    int f0, f1, f2;              // this lane's output offset of the set's pending products
    uint32_t tm0 = 0, tm1 = 0, tm2 = 0;
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc0[t] = acc1[t] = acc2[t] = 0.0;
#define BW_OFFSET(Q) ((int)__builtin_amdgcn_raw_buffer_load_b32(prs, half * 4, max((Q), 0) * 16, 0))
#define BW_LOAD(BS, FS, TS, Q)                                                      \
  {                                                                                 \
    const int q_ = (Q);                                                             \
    const int so_ = sbase + q_ * KC * 16 * (int)sizeof(double);                     \
    _Pragma("unroll") for (int kc = 0; kc < KC; ++kc)                               \
      BS[kc] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(     \
                   brs, vboff + kc * 16 * (int)sizeof(double), so_, 0));            \
    if (!FULL) TS = __builtin_amdgcn_raw_buffer_load_b32(trs, 0, q_ * 4, 0);        \
    FS = BW_OFFSET(q_ - 3);                                                         \
  }
#define BW_FLUSH(AS, FS)                                                            \
  _Pragma("unroll") for (int t = 0; t < TPW; ++t)                                   \
    __hip_atomic_fetch_add(smem + obase[t] + (FS), AS[t], __ATOMIC_RELAXED,         \
                           __HIP_MEMORY_SCOPE_WORKGROUP);
#define BW_MMA(AS, BS)                                                              \
  {                                                                                 \
    _Pragma("unroll") for (int t = 0; t < TPW; ++t) AS[t] = 0.0;                    \
    _Pragma("unroll") for (int kc = 0; kc < KC; ++kc)                               \
      _Pragma("unroll") for (int t = 0; t < TPW; ++t) AS[t] = mfma4(a[t][kc], BS[kc], AS[t]); \
  }
// the loads and the adds are spread through the products
#define BW_INTERLEAVE()                                                             \
  {                                                                                 \
    constexpr int NMF = TPW * KC;                                                   \
    _Pragma("unroll") for (int i_ = 0; i_ < KC; ++i_) {                             \
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                            \
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    }                                                                               \
    _Pragma("unroll") for (int i_ = 0; i_ < TPW; ++i_) {                            \
      __builtin_amdgcn_sched_group_barrier(0x080, 1, 0);                            \
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    }                                                                               \
    __builtin_amdgcn_sched_group_barrier(0x008, NMF - TPW - KC, 0);                 \
  }
// pair Q from set S (products AS, pending products of pair Q - 3 at FS); set N
// (pair Q - 1) takes the tables of Q + 2 and the offset of pair Q - 1
#define BW_STEP(BS, FS, TS, AS, BN, FN, TN, Q)                                      \
  BW_LOAD(BN, FN, TN, min((Q) + 2, npairs - 1));                                    \
  BW_FLUSH(AS, FS);                                                                 \
  if (FULL || (__builtin_amdgcn_readfirstlane(TS) & d.mask) != 0) {                \
    BW_MMA(AS, BS);                                                                 \
    BW_INTERLEAVE();                                                                \
  } else {                                                                          \
    _Pragma("unroll") for (int t = 0; t < TPW; ++t) AS[t] = 0.0;                    \
  }
// at the end of an offset group: every set's products go in (the latest pair of
// each set below QN, whose offset is loaded here), then the barrier
#define BW_PENDING(X, QN) ((QN) - 1 - ((((QN) - 1 - (X)) % 3) + 3) % 3)
#define BW_GROUP_END(QN)                                                            \
  if (__builtin_expect((QN) == gend, 0)) {                                          \
    f0 = BW_OFFSET(BW_PENDING(0, QN));                                              \
    f1 = BW_OFFSET(BW_PENDING(1, QN));                                              \
    f2 = BW_OFFSET(BW_PENDING(2, QN));                                              \
    BW_FLUSH(acc0, f0);                                                             \
    BW_FLUSH(acc1, f1);                                                             \
    BW_FLUSH(acc2, f2);                                                             \
    _Pragma("unroll") for (int t = 0; t < TPW; ++t) acc0[t] = acc1[t] = acc2[t] = 0.0; \
    __syncthreads();   /* the next group writes other planes of other waves */      \
    ++g;                                                                            \
    gend = __builtin_amdgcn_readfirstlane(s_gs[g + 1]);                             \
  }
    BW_LOAD(b0, f0, tm0, 0);
    BW_LOAD(b1, f1, tm1, min(1, npairs - 1));
    int g = 0, gend = __builtin_amdgcn_readfirstlane(s_gs[1]);
#pragma unroll 1
    for (int q = 0; q < npairs; q += 3) {
      BW_STEP(b0, f0, tm0, acc0, b2, f2, tm2, q);
      BW_GROUP_END(q + 1);
      if (__builtin_expect(q + 1 >= npairs, 0)) break;
      BW_STEP(b1, f1, tm1, acc1, b0, f0, tm0, q + 1);
      BW_GROUP_END(q + 2);
      if (__builtin_expect(q + 2 >= npairs, 0)) break;
      BW_STEP(b2, f2, tm2, acc2, b1, f1, tm1, q + 2);
      BW_GROUP_END(q + 3);
    }
#undef BW_OFFSET
#undef BW_LOAD
#undef BW_FLUSH
#undef BW_MMA
#undef BW_INTERLEAVE
#undef BW_STEP
#undef BW_PENDING
#undef BW_GROUP_END
    // write the round's components of dM (whole frame) and clear the accumulators
    if constexpr (HARM) {
      const HOut& ho = hout[r];
      for (int c = tid; c < kNCell; c += kBwdThreads) {
        const int jx = c % kFrame, jy = (c / kFrame) % kFrame, jz = c / (kFrame * kFrame);
        const bool win = jx >= kWin0 && jx < kWin0 + kWin && jy >= kWin0 && jy < kWin0 + kWin &&
                         jz >= kWin0 && jz < kWin0 + kWin;
        const bool pres = win && block_present(d.mask, jx, jy, jz);
        const int wc = (jx - kWin0) + kWin * (jy - kWin0) + kWin * kWin * (jz - kWin0);
        double g0 = 0.0, g1 = 0.0;
        if (win) {
          g0 = smem[wc];
          g1 = smem[kAccStride + wc];
          smem[wc] = 0.0;
          smem[kAccStride + wc] = 0.0;
        }
        for (int e = 0; e < ho.nout; ++e) {
          const int k = ho.comp[e];
          double* o = out + (size_t)k * kNCell + c;
          double v = __builtin_fma(ho.c1[e], g1, ho.c0[e] * g0);
          v = pres ? ldexp(v, l2 * order_of(k)) : 0.0;
          *o = ho.add[e] ? *o + v : v;
        }
      }
      continue;
    }
    const double sc0 = ldexp(1.0, l2 * order_of(2 * r));
    const double sc1 = ldexp(1.0, l2 * order_of(2 * r + 1));
    for (int c = tid; c < kNCell; c += kBwdThreads) {
      const int jx = c % kFrame, jy = (c / kFrame) % kFrame, jz = c / (kFrame * kFrame);
      const bool win = jx >= kWin0 && jx < kWin0 + kWin && jy >= kWin0 && jy < kWin0 + kWin &&
                       jz >= kWin0 && jz < kWin0 + kWin;
      const bool pres = win && block_present(d.mask, jx, jy, jz);
      const int wc = (jx - kWin0) + kWin * (jy - kWin0) + kWin * kWin * (jz - kWin0);
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const int k = 2 * r + sl;
        double v = 0.0;
        if (win) {
          v = smem[sl * kAccStride + wc];
          smem[sl * kAccStride + wc] = 0.0;
        }
        if (k < C) out[(size_t)k * kNCell + c] = pres ? v * (sl ? sc1 : sc0) : 0.0;
      }
    }
  }
}

// the mass gradients of an earlier item, at the top of round (workgroup index
// mod rounds) of the current one
template <class F>
struct GradHook {
  int prev;
  F grads;
  __device__ bool wants(int r, int rounds) const {
    return prev >= 0 && r == (int)(blockIdx.x % (unsigned)rounds);
  }
  __device__ void run(double* lds) const { grads(prev, lds); }
};

// FUSE: the kernel also computes the mass gradients (the P2M adjoint of the
// sub-grid's dM, 8 particles per cell). A workgroup computes them for its
// previous item, whose dM it has written, at the top of round (workgroup index
// mod rounds) of its current item, so that HBM-bound work overlaps the matrix
// work of the other workgroups; its last item's follow after its loop.
template <bool HARM, bool FUSE = false>
__global__ void __launch_bounds__(kBwdThreads) m2l_bwd_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, const double* __restrict__ dL, double* dM,
    const double* __restrict__ B2, const double* __restrict__ B3, const double* __restrict__ B4,
    const int4* __restrict__ pairs, int npairs, const int* __restrict__ gstart,
    const uint32_t* __restrict__ ptouch, const HFold* __restrict__ hf2, const HFold* __restrict__ hf3,
    const HFold* __restrict__ hf4, const HOut* __restrict__ ho2, const HOut* __restrict__ ho3,
    const HOut* __restrict__ ho4, const double* __restrict__ pos = nullptr,
    double* __restrict__ dmass = nullptr) {
  __shared__ double smem[2 * kAccStride];
  __shared__ int s_gs[16];                // first pair of each offset group, and the end
  static_assert(kBwdGroups + 2 <= 16, "the group starts, the end and one read past it");
  __shared__ int s_item;
  static_assert(kP2MAdjRowsLds <= 2 * kAccStride && kBwdThreads == kP2MRowsThreads,
                "the gradient phase fits the accumulator buffer and the workgroup");
  if (threadIdx.x < kBwdGroups + 1) s_gs[threadIdx.x] = gstart[threadIdx.x];
  // the mass gradients of item `it` (its dM complete), with `lds` as staging
  auto grads = [&](int it, double* lds) __attribute__((always_inline)) {
    const DevDesc dp = desc[items[it].sub];
    switch (dp.p) {
      case 2: p2m_adjoint_rows<2>(dp, pos, dM, dmass, lds); break;
      case 3: p2m_adjoint_rows<3>(dp, pos, dM, dmass, lds); break;
      case 4: p2m_adjoint_rows<4>(dp, pos, dM, dmass, lds); break;
      default: break;
    }
  };
  int prev = -1;
  // (LDS operations complete in order; the staged values are read after the
  // barrier at the top of the item loop)
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= count) break;
    const DevDesc d = desc[items[item].sub];
    const bool full = d.mask == kFullMask;
    const auto hook = [&]() {
      if constexpr (FUSE) return GradHook<decltype(grads)>{prev, grads};
      else return NoHook{};
    }();
    switch (d.p) {
      case 2:
        if (full) bwd_subgrid<2, true, HARM>(d, dL, dM, B2, npairs, s_gs, ptouch, smem, pairs, hf2, ho2, hook);
        else bwd_subgrid<2, false, HARM>(d, dL, dM, B2, npairs, s_gs, ptouch, smem, pairs, hf2, ho2, hook);
        break;
      case 3:
        if (full) bwd_subgrid<3, true, HARM>(d, dL, dM, B3, npairs, s_gs, ptouch, smem, pairs, hf3, ho3, hook);
        else bwd_subgrid<3, false, HARM>(d, dL, dM, B3, npairs, s_gs, ptouch, smem, pairs, hf3, ho3, hook);
        break;
      case 4:
        if (full) bwd_subgrid<4, true, HARM>(d, dL, dM, B4, npairs, s_gs, ptouch, smem, pairs, hf4, ho4, hook);
        else bwd_subgrid<4, false, HARM>(d, dL, dM, B4, npairs, s_gs, ptouch, smem, pairs, hf4, ho4, hook);
        break;
      default: break;
    }
    __syncthreads();
    prev = item;
  }
  if constexpr (FUSE) {
    if (prev >= 0) {
      __syncthreads();
      grads(prev, smem);
    }
  }
}

// ---------------------------------------------------------------------------
// Round split, for batches too small to fill the GPU: work items are (sub-grid,
// round) pairs (WorkItem::cost holds the round), each writing its round's raw
// sums to its own slot of `part`; m2l_round_sum_kernel then adds a sub-grid's
// rounds in round order and scales (and, in the harmonic form, expands) them
// into L. Same products as the whole-sub-grid kernel, summed in another order.
// ---------------------------------------------------------------------------
constexpr int kPartStride = 35 * kNTarget;    // doubles per slot: C (p = 4) x 512

template <bool PIPE, bool HARM>
__global__ void __launch_bounds__(kBlThreads) m2l_fwd_round_kernel(
    const WorkItem* __restrict__ items, int count, unsigned* __restrict__ counter,
    const DevDesc* __restrict__ desc, const double* __restrict__ M, double* __restrict__ part,
    const double* __restrict__ B2, const double* __restrict__ B3, const double* __restrict__ B4,
    const int* __restrict__ lds_off, const uint32_t* __restrict__ touch,
    const HRound* __restrict__ hr2, const HRound* __restrict__ hr3, const HRound* __restrict__ hr4) {
  __shared__ double2 smem[kWinCells];
  __shared__ double sB[2 * kBlChunkMax];
  __shared__ int4 s_off[kQuads];
  __shared__ int s_item;
  if (PIPE) {
    const int4* off4 = reinterpret_cast<const int4*>(lds_off);
    for (int i = threadIdx.x; i < kQuads; i += blockDim.x) s_off[i] = off4[i];
  }
  const HExp* ne = nullptr;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= count) break;
    const DevDesc d = desc[items[item].sub];
    const bool full = d.mask == kFullMask;
    const OneRound rg{items[item].cost, part + (size_t)item * kPartStride};
    const NoHook nh;
    switch (d.p) {
      case 2:
        if (PIPE && full)
          fwd_bl_subgrid<2, PIPE, true, HARM>(d, M, nullptr, B2, lds_off, touch, smem, sB, s_off, hr2, ne, nh, rg);
        else
          fwd_bl_subgrid<2, PIPE, false, HARM>(d, M, nullptr, B2, lds_off, touch, smem, sB, s_off, hr2, ne, nh, rg);
        break;
      case 3:
        if (PIPE && full)
          fwd_bl_subgrid<3, PIPE, true, HARM>(d, M, nullptr, B3, lds_off, touch, smem, sB, s_off, hr3, ne, nh, rg);
        else
          fwd_bl_subgrid<3, PIPE, false, HARM>(d, M, nullptr, B3, lds_off, touch, smem, sB, s_off, hr3, ne, nh, rg);
        break;
      case 4:
        if (HARM && PIPE && full)
          fwd_bl_subgrid<4, PIPE, true, HARM>(d, M, nullptr, B4, lds_off, touch, smem, sB, s_off, hr4, ne, nh, rg);
        else if (HARM && PIPE)
          fwd_bl_subgrid<4, PIPE, false, HARM>(d, M, nullptr, B4, lds_off, touch, smem, sB, s_off, hr4, ne, nh, rg);
        else
          fwd_bl_subgrid<4, false, false, HARM>(d, M, nullptr, B4, lds_off, touch, smem, sB, s_off, hr4, ne, nh, rg);
        break;
      default: break;
    }
    __syncthreads();
  }
}

template <int P, bool HARM>
__device__ __forceinline__ void round_sum(const DevDesc& d, const double* __restrict__ part, int base,
                                          double* __restrict__ L, const HExp* __restrict__ hexp) {
  constexpr int C = ncomp(P);
  constexpr int CR = HARM ? (P + 1) * (P + 1) : C;
  constexpr int ROUNDS = (CR + 1) / 2;
  const int tid = threadIdx.x;
  const int l2 = d.log2_inv_h;
  double h[CR];
#pragma unroll
  for (int c = 0; c < CR; ++c) h[c] = 0.0;
  for (int r = 0; r < ROUNDS; ++r) {
    const double* src = part + (size_t)(base + r) * kPartStride + tid;
#pragma unroll
    for (int c = 0; c < CR; ++c) h[c] += src[(size_t)c * kNTarget];
  }
  double* out = L + d.l_off + tid;
#pragma unroll
  for (int n = 0; n < C; ++n) {
    double v;
    if constexpr (HARM) {
      const HExp& e = hexp[n];
      v = 0.0;
      for (int u = 0; u < e.nterm; ++u) {
        double hc = 0.0;
#pragma unroll
        for (int c = 0; c < CR; ++c) hc = c == e.col[u] ? h[c] : hc;
        v = __builtin_fma(e.coef[u], hc, v);
      }
    } else {
      v = h[n];
    }
    out[(size_t)n * kNTarget] = ldexp(v, l2 * (1 + order_of(n)));
  }
}

// one workgroup per sub-grid, one thread per target cell; base[b]: the slot of
// sub-grid b's first round (its rounds are consecutive slots)
template <bool HARM>
__global__ void __launch_bounds__(kNTarget) m2l_round_sum_kernel(
    const DevDesc* __restrict__ desc, const int* __restrict__ base, const double* __restrict__ part,
    double* __restrict__ L, const HExp* __restrict__ he2, const HExp* __restrict__ he3,
    const HExp* __restrict__ he4) {
  const int b = blockIdx.x;
  const DevDesc d = desc[b];
  switch (d.p) {
    case 2: round_sum<2, HARM>(d, part, base[b], L, he2); break;
    case 3: round_sum<3, HARM>(d, part, base[b], L, he3); break;
    case 4: round_sum<4, HARM>(d, part, base[b], L, he4); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// table packing
// ---------------------------------------------------------------------------

// forward: [r][q][c][g][kk*4 + j] = T_{4q+kk}[2r+c][4g+j]
// LDS-staged forward: [r][q][g][kk*4 + j][c], same values
__global__ void pack_fwd_kernel(const double* __restrict__ T, int p, double* __restrict__ out,
                                float* __restrict__ hi, float* __restrict__ lo,
                                double* __restrict__ outl) {
  const int C = ncomp(p), NG = (C + 3) / 4, ROUNDS = (C + 1) / 2;
  const int total = ROUNDS * kQuads * 2 * NG * 16;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = i & 3, kk = (i >> 2) & 3;
  int rest = i >> 4;
  const int g = rest % NG; rest /= NG;
  const int c = rest % 2; rest /= 2;
  const int q = rest % kQuads;
  const int r = rest / kQuads;
  const int k = 2 * r + c, n = 4 * g + j, s = 4 * q + kk;
  const double v = (k < C && n < C) ? T[((size_t)s * C + k) * C + n] : 0.0;
  out[i] = v;
  outl[((((size_t)r * kQuads + q) * NG + g) * 16 + kk * 4 + j) * 2 + c] = v;
  const float h = (float)v;
  hi[i] = h;
  lo[i] = (float)(v - (double)h);
}

// harmonic: [r][q][g][kk*4 + j][c] = T_{4q+kk}[rowk[2r + c]][colk[4g + j]] (0 where a map is -1)
struct HPackMaps {
  int rowk[32];   // full index of each round's folded components, or -1
  int colk[32];   // full index of each harmonic column, or -1 past (p+1)^2
};
__global__ void pack_fwdh_kernel(const double* __restrict__ T, int p, HPackMaps mp, int rounds, int ng,
                                 double* __restrict__ out) {
  const int C = ncomp(p);
  const int total = rounds * kQuads * ng * 32;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = i & 1;
  int rest = i >> 1;
  const int jj = rest & 15;
  rest >>= 4;
  const int g = rest % ng;
  rest /= ng;
  const int q = rest % kQuads;
  const int r = rest / kQuads;
  const int s = 4 * q + (jj >> 2);
  const int k = mp.rowk[2 * r + c], n = mp.colk[4 * g + (jj & 3)];
  out[i] = (k >= 0 && n >= 0) ? T[((size_t)s * C + k) * C + n] : 0.0;
}

// harmonic adjoint: [r][pair][kc][kk*4 + j] = T_{s_(j/2)}[rowk[2r + j%2]][colk[4kc + kk]]
__global__ void pack_bwdh_kernel(const double* __restrict__ T, int p, const int4* __restrict__ pairs,
                                 int npairs, HPackMaps mp, int rounds, int kcn, double* __restrict__ out) {
  const int C = ncomp(p);
  const int total = rounds * npairs * kcn * 16;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = i & 3, kk = (i >> 2) & 3;
  int rest = i >> 4;
  const int kc = rest % kcn;
  rest /= kcn;
  const int q = rest % npairs;
  const int r = rest / npairs;
  const int4 pr = pairs[q];
  const int so = (j >> 1) ? pr.w : pr.z;
  const int k = mp.rowk[2 * r + (j & 1)], n = mp.colk[4 * kc + kk];
  out[i] = (so >= 0 && k >= 0 && n >= 0) ? T[((size_t)so * C + k) * C + n] : 0.0;
}

// adjoint: [r][pair][kc][kk*4 + j] = T_{s_(j/2)}[2r + j%2][4kc + kk] (0 for a missing offset)
__global__ void pack_bwd_kernel(const double* __restrict__ T, int p, const int4* __restrict__ pairs,
                                int npairs, double* __restrict__ out) {
  const int C = ncomp(p), KC = (C + 3) / 4, ROUNDS = (C + 1) / 2;
  const int total = ROUNDS * npairs * KC * 16;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = i & 3, kk = (i >> 2) & 3;
  int rest = i >> 4;
  const int kc = rest % KC; rest /= KC;
  const int q = rest % npairs;
  const int r = rest / npairs;
  const int4 pr = pairs[q];
  const int so = (j >> 1) ? pr.w : pr.z;
  const int k = 2 * r + (j & 1), n = 4 * kc + kk;
  out[i] = (so >= 0 && k < C && n < C) ? T[((size_t)so * C + k) * C + n] : 0.0;
}

size_t fwd_pack_elems(int p) {
  const int C = ncomp(p), NG = (C + 3) / 4, ROUNDS = (C + 1) / 2;
  return (size_t)ROUNDS * kQuads * 2 * NG * 16;
}

size_t bwd_pack_elems(int p, int npairs) {
  const int C = ncomp(p), KC = (C + 3) / 4, ROUNDS = (C + 1) / 2;
  return (size_t)ROUNDS * npairs * KC * 16;
}

// Offset groups of the adjoint: wave w writes output plane w + 6 + dz, so two
// dz whose difference is at least 8 never make two of the 8 waves write one
// plane, and their offsets can run between the same two barriers. The 13 dz
// values make 8 groups (5 of two dz, 3 of one), 100 to 138 offsets each.
constexpr int kBwdGroupDz[kBwdGroups][2] = {{-6, 2}, {-5, 3}, {-4, 4}, {-3, 5}, {-2, 6},
                                            {-1, -1}, {0, 0}, {1, 1}};

// Offsets of one group paired so that the two never send two cells of a 4x4
// tile to the same output cell (4 cells apart in x or y, or different dz, so
// different planes). The lanes of a tile's add hold 4 x, 4 y, 2 components and
// the 2 offsets of the pair; with the accumulator rows 20 doubles apart and an
// odd component stride, the add takes the fewest LDS cycles when the two
// offsets' x differ by 2 mod 4 (measured: 8.2 cycles for a 64-lane ds_add_f64,
// 16 to 20 for any other difference). So the offsets are first paired by a
// maximum matching among such partners (a bipartite graph: x = 0, 1 mod 4
// against x = 2, 3 mod 4), the rest greedily with any partner 4 cells away,
// and what is left runs alone.
void build_pairs(const std::vector<int>& st, std::vector<int4>* pairs, std::vector<int>* gstart) {
  gstart->clear();
  for (int gi = 0; gi < kBwdGroups; ++gi) {
    gstart->push_back((int)pairs->size());
    std::vector<int> ids;
    for (int i = 0; i < kNStencil; ++i)
      if (st[3 * i + 2] == kBwdGroupDz[gi][0] || st[3 * i + 2] == kBwdGroupDz[gi][1]) ids.push_back(i);
    const int n = (int)ids.size();
    auto dx = [&](int a) { return st[3 * ids[a]]; };
    auto compatible = [&](int a, int b) {
      return st[3 * ids[a] + 2] != st[3 * ids[b] + 2] || std::abs(dx(a) - dx(b)) >= 4 ||
             std::abs(st[3 * ids[a] + 1] - st[3 * ids[b] + 1]) >= 4;
    };
    auto preferred = [&](int a, int b) { return compatible(a, b) && (((dx(a) - dx(b)) % 4) + 4) % 4 == 2; };
    std::vector<int> mate(n, -1);
    std::vector<char> seen(n);
    // augmenting paths from the x = 0, 1 (mod 4) side
    std::function<bool(int)> augment = [&](int a) {
      for (int b = 0; b < n; ++b)
        if (!seen[b] && preferred(a, b)) {
          seen[b] = 1;
          if (mate[b] < 0 || augment(mate[b])) {
            mate[b] = a;
            mate[a] = b;
            return true;
          }
        }
      return false;
    };
    for (int a = 0; a < n; ++a)
      if (((dx(a) % 4) + 4) % 4 < 2) {
        std::fill(seen.begin(), seen.end(), 0);
        augment(a);
      }
    for (int a = 0; a < n; ++a)
      if (mate[a] < 0)
        for (int b = n - 1; b > a; --b)
          if (mate[b] < 0 && compatible(a, b)) {
            mate[a] = b;
            mate[b] = a;
            break;
          }
    for (int a = 0; a < n; ++a) {
      if (mate[a] >= 0 && mate[a] < a) continue;   // listed with its partner
      const int s1 = ids[a], s2 = mate[a] >= 0 ? ids[mate[a]] : -1;
      const int o1 = st[3 * s1] + kWin * st[3 * s1 + 1] + kWin * kWin * st[3 * s1 + 2];
      // an offset without a partner: the second half's tables are zero, so its
      // lanes add zeros; they go to the cells 2 away in x (toward the centre, so
      // into the same row of the same wave's plane), where the add is as cheap
      // as a preferred pair's
      const int o2 = s2 >= 0 ? st[3 * s2] + kWin * st[3 * s2 + 1] + kWin * kWin * st[3 * s2 + 2]
                             : o1 + (st[3 * s1] >= 0 ? -2 : 2);
      pairs->push_back(make_int4(o1, o2, s1, s2));
    }
  }
  gstart->push_back((int)pairs->size());
}

int64_t block_pair_count(uint32_t mask, const std::vector<int>& st) {
  static int64_t per_block[27] = {-1};
  if (per_block[0] < 0) {
    int64_t v[27] = {};
    for (int t = 0; t < kNTarget; ++t) {
      const int jx = t % 8 + 8, jy = (t / 8) % 8 + 8, jz = t / 64 + 8;
      for (size_t i = 0; i < st.size(); i += 3)
        v[(jx + st[i]) / 8 + 3 * ((jy + st[i + 1]) / 8) + 9 * ((jz + st[i + 2]) / 8)]++;
    }
    for (int b = 0; b < 27; ++b) per_block[b] = v[b];
  }
  int64_t n = 0;
  for (int b = 0; b < 27; ++b)
    if ((mask >> b) & 1u) n += per_block[b];
  return n;
}

std::vector<int> host_stencil() {
  std::vector<int> s;
  for (int dz = -kRad; dz <= kRad; ++dz)
    for (int dy = -kRad; dy <= kRad; ++dy)
      for (int dx = -kRad; dx <= kRad; ++dx) {
        const int q = dx * dx + dy * dy + dz * dz;
        if (q >= 5 && q <= 36) {
          s.push_back(dx);
          s.push_back(dy);
          s.push_back(dz);
        }
      }
  return s;
}

// Configurations: forward waves per workgroup (tiles per wave = 32 / waves).
struct Config {
  int ldstab;       // table operands staged through LDS (8 waves): 1, or 2 with the
                    // next quad's operand reads issued ahead; 0: loaded per wave
  int waves;        // waves per workgroup (16-cell tiles per wave = 32 / waves)
  bool prefetch;    // table operands of the next offset quad loaded one quad ahead
                    // (not at p = 4 with 8 waves: the registers would spill)
  fmm_precision prec;
  int qdiv = 1;     // LDS-staged tables: chunks of 1/qdiv of the default length
};
constexpr Config kConfigs[] = {{2, 8, false, FMM_FP64}, {1, 8, false, FMM_FP64},
                               {0, 8, true, FMM_FP64},  {0, 8, false, FMM_FP64},
                               {0, 4, false, FMM_FP64}, {0, 4, true, FMM_FP64},
                               {0, 8, false, FMM_SPLIT_FP32}, {2, 8, false, FMM_FP64_HARMONIC},
                               {0, 4, false, FMM_EXACT_SLICE},
                               {1, 8, false, FMM_FP64_HARMONIC}, {2, 8, false, FMM_FP64_HARMONIC, 2}};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

}  // namespace

void fill_work_list(const fmm_subgrid* desc, int64_t nsub, bool harmonic, WorkItem* out) {
  static const std::vector<int> st = host_stencil();
  for (int64_t b = 0; b < nsub; ++b) {
    const int p = desc[b].p;
    const int64_t per_pair = harmonic ? (int64_t)(p + 1) * (p + 1) * (p + 1) * (p + 1)
                                      : (int64_t)ncomp(p) * ncomp(p);
    const int64_t pairs = block_pair_count(desc[b].mask, st);
    out[b].sub = (int32_t)b;
    out[b].cost = (int32_t)(per_pair * pairs / 4096);
  }
  std::sort(out, out + nsub, [](const WorkItem& a, const WorkItem& b) {
    return a.cost != b.cost ? a.cost > b.cost : a.sub < b.sub;
  });
}

std::vector<WorkItem> build_work_list(const fmm_subgrid* desc, int64_t nsub, bool harmonic) {
  std::vector<WorkItem> items((size_t)nsub);
  fill_work_list(desc, nsub, harmonic, items.data());
  return items;
}

namespace {
// blocks touched by the 8x8 target plane z shifted by offset o
uint32_t plane_blocks(const std::vector<int>& st, int z, int o) {
  const int dx = st[3 * o], dy = st[3 * o + 1], dz = st[3 * o + 2];
  const int bz = (8 + z + dz) / 8;
  uint32_t m = 0;
  for (int bx = (8 + dx) / 8; bx <= (15 + dx) / 8; ++bx)
    for (int by = (8 + dy) / 8; by <= (15 + dy) / 8; ++by) m |= 1u << (bx + 3 * by + 9 * bz);
  return m;
}
// ---- harmonic form: fold, round plan and expansion (host)

struct MI3 {
  int x, y, z;
};

std::vector<MI3> graded_indices(int p) {
  std::vector<MI3> v;
  for (int n = 0; n <= p; ++n)
    for (int kx = n; kx >= 0; --kx)
      for (int ky = n - kx; ky >= 0; --ky) v.push_back({kx, ky, n - kx - ky});
  return v;
}

int index_of(const std::vector<MI3>& v, int a, int b, int c) {
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].x == a && v[i].y == b && v[i].z == c) return (int)i;
  return -1;
}

// T(a,b,c) = -T(a+2,b,c-2) - T(a,b+2,c-2) for a family harmonic in its index,
// applied until the z-index is 0 or 1: coefficients over the kz <= 1 indices
void fold_into(const std::vector<MI3>& hs, int a, int b, int c, double coef, std::vector<double>* row) {
  if (c <= 1) {
    (*row)[index_of(hs, a, b, c)] += coef;
    return;
  }
  fold_into(hs, a + 2, b, c - 2, -coef, row);
  fold_into(hs, a, b + 2, c - 2, -coef, row);
}

struct HostHarmonic {
  std::vector<HRound> rounds;
  std::vector<HExp> exps;
  std::vector<HFold> folds;   // per harmonic column: the components folding onto it
  std::vector<HOut> outs;     // per round: the output components written from it
  HPackMaps maps;
  int ng = 0;
};

// The folded components are staged two per round; pairs that share moment
// components are formed first (largest overlap first), so each moment
// component is read as few times as possible.
bool build_harmonic(int p, HostHarmonic* out) {
  const std::vector<MI3> ks = graded_indices(p);
  std::vector<MI3> hs;
  for (const MI3& k : ks)
    if (k.z <= 1) hs.push_back(k);
  const int C = (int)ks.size(), CR = (int)hs.size();
  std::vector<std::vector<double>> F(C, std::vector<double>(CR, 0.0));   // F[k][k']
  for (int k = 0; k < C; ++k) fold_into(hs, ks[k].x, ks[k].y, ks[k].z, 1.0, &F[k]);
  std::vector<std::vector<int>> sup(CR);
  for (int h = 0; h < CR; ++h)
    for (int k = 0; k < C; ++k)
      if (F[k][h] != 0.0) sup[h].push_back(k);
  auto shared = [&](int a, int b) {
    int n = 0;
    for (int x : sup[a])
      for (int y : sup[b]) n += x == y;
    return n;
  };
  std::vector<std::pair<int, int>> pairs;
  std::vector<bool> used(CR, false);
  for (int best = CR; best >= 1; --best)
    for (int a = 0; a < CR; ++a)
      for (int b = a + 1; b < CR; ++b)
        if (!used[a] && !used[b] && shared(a, b) == best) {
          used[a] = used[b] = true;
          pairs.push_back({a, b});
        }
  std::vector<int> rest;
  for (int h = 0; h < CR; ++h)
    if (!used[h]) rest.push_back(h);
  for (size_t i = 0; i < rest.size(); i += 2)
    pairs.push_back({rest[i], i + 1 < rest.size() ? rest[i + 1] : -1});
  out->ng = (CR + 3) / 4;
  if ((int)pairs.size() * 2 > 32 || out->ng * 4 > 32) return false;
  for (int i = 0; i < 32; ++i) out->maps.rowk[i] = out->maps.colk[i] = -1;
  for (size_t r = 0; r < pairs.size(); ++r) {
    const int h0 = pairs[r].first, h1 = pairs[r].second;
    std::vector<int> u = sup[h0];
    if (h1 >= 0)
      for (int k : sup[h1])
        if (std::find(u.begin(), u.end(), k) == u.end()) u.push_back(k);
    std::sort(u.begin(), u.end());
    if ((int)u.size() > kHMaxSup) return false;
    HRound rd{};
    rd.nsup = (int)u.size();
    rd.ord0 = hs[h0].x + hs[h0].y + hs[h0].z;
    rd.ord1 = h1 >= 0 ? hs[h1].x + hs[h1].y + hs[h1].z : -1;
    for (size_t i = 0; i < u.size(); ++i) {
      rd.comp[i] = u[i];
      rd.c0[i] = F[u[i]][h0];
      rd.c1[i] = h1 >= 0 ? F[u[i]][h1] : 0.0;
    }
    out->rounds.push_back(rd);
    out->maps.rowk[2 * r] = index_of(ks, hs[h0].x, hs[h0].y, hs[h0].z);
    out->maps.rowk[2 * r + 1] = h1 >= 0 ? index_of(ks, hs[h1].x, hs[h1].y, hs[h1].z) : -1;
  }
  for (int h = 0; h < CR; ++h) out->maps.colk[h] = index_of(ks, hs[h].x, hs[h].y, hs[h].z);
  // adjoint: the fold of dL onto each harmonic column
  for (int h = 0; h < CR; ++h) {
    if ((int)sup[h].size() > kHMaxSup) return false;
    HFold f{};
    f.nterm = (int)sup[h].size();
    for (size_t i = 0; i < sup[h].size(); ++i) {
      f.comp[i] = sup[h][i];
      f.coef[i] = F[sup[h][i]][h];
    }
    out->folds.push_back(f);
  }
  // adjoint: dM_k = sum_k' F[k][k'] Gh_k', written from each round holding some k'
  std::vector<bool> written(C, false);
  out->outs.assign(pairs.size(), HOut{});
  for (size_t r = 0; r < pairs.size(); ++r) {
    const int h0 = pairs[r].first, h1 = pairs[r].second;
    HOut& o = out->outs[r];
    for (int k = 0; k < C; ++k) {
      const double c0 = F[k][h0], c1 = h1 >= 0 ? F[k][h1] : 0.0;
      if (c0 == 0.0 && c1 == 0.0) continue;
      if (o.nout == kHMaxOut) return false;
      o.comp[o.nout] = k;
      o.add[o.nout] = written[k] ? 1 : 0;
      o.c0[o.nout] = c0;
      o.c1[o.nout] = c1;
      ++o.nout;
      written[k] = true;
    }
  }
  for (int k = 0; k < C; ++k)
    if (!written[k]) return false;
  for (int k = 0; k < C; ++k) {
    HExp ex{};
    for (int h = 0; h < CR; ++h)
      if (F[k][h] != 0.0) {
        if (ex.nterm == kHMaxExp) return false;
        ex.col[ex.nterm] = h;
        ex.coef[ex.nterm] = F[k][h];
        ++ex.nterm;
      }
    out->exps.push_back(ex);
  }
  return true;
}

}  // namespace

bool harmonic_rounds_host(int p, std::vector<HRound>* rounds) {
  HostHarmonic hh;
  if (!build_harmonic(p, &hh)) return false;
  *rounds = hh.rounds;
  return true;
}

bool harmonic_plan_maps(int p, int32_t rowk[32], int32_t colk[32], int* nrounds) {
  HostHarmonic hh;
  if (!build_harmonic(p, &hh)) return false;
  for (int i = 0; i < 32; ++i) {
    rowk[i] = hh.maps.rowk[i];
    colk[i] = hh.maps.colk[i];
  }
  *nrounds = (int)hh.rounds.size();
  return true;
}

hipError_t mfma_tables_create(MfmaTables* t, double* const* d_T, const int* d_stencil,
                              hipStream_t s) {
  hipError_t e;
  t->stencil = d_stencil;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&t->num_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  const std::vector<int> st = host_stencil();
  // forward: LDS offsets of the offsets, blocks each quad touches per target plane
  std::vector<int> off(kNStencil);
  for (int i = 0; i < kNStencil; ++i) off[i] = st[3 * i] + kWin * st[3 * i + 1] + kWin * kWin * st[3 * i + 2];
  std::vector<uint32_t> touch(8 * kQuads, 0u);
  for (int z = 0; z < 8; ++z)
    for (int q = 0; q < kQuads; ++q)
      for (int o = 4 * q; o < 4 * q + 4; ++o) touch[z * kQuads + q] |= plane_blocks(st, z, o);
  // adjoint: offset pairs grouped by dz, blocks each pair writes per target plane
  std::vector<int4> pairs;
  std::vector<int> gstart;
  build_pairs(st, &pairs, &gstart);
  if ((int)pairs.size() > kMaxPairs || gstart.size() != kBwdGroups + 1) return hipErrorInvalidValue;
  t->npairs = (int)pairs.size();
  std::vector<uint32_t> ptouch(8 * pairs.size(), 0u);
  for (int z = 0; z < 8; ++z)
    for (size_t q = 0; q < pairs.size(); ++q) {
      uint32_t m = plane_blocks(st, z, pairs[q].z);
      if (pairs[q].w >= 0) m |= plane_blocks(st, z, pairs[q].w);
      ptouch[z * pairs.size() + q] = m;
    }
  if ((e = hipMalloc(&t->lds_off, off.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc(&t->touch, touch.size() * sizeof(uint32_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&t->pairs, pairs.size() * sizeof(int4))) != hipSuccess) return e;
  if ((e = hipMalloc(&t->gstart, gstart.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc(&t->ptouch, ptouch.size() * sizeof(uint32_t))) != hipSuccess) return e;
  // synchronous copies: the host vectors die at return
  if ((e = hipMemcpy(t->lds_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(t->touch, touch.data(), touch.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(t->pairs, pairs.data(), pairs.size() * sizeof(int4), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(t->gstart, gstart.data(), gstart.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(t->ptouch, ptouch.data(), ptouch.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  for (int p = 2; p <= kMaxP; ++p) {
    const size_t nf = fwd_pack_elems(p), nb = bwd_pack_elems(p, t->npairs);
    if ((e = hipMalloc(&t->fwd[p], nf * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->fwdl[p], nf * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->fwd_hi[p], nf * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->fwd_lo[p], nf * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->bwd[p], nb * sizeof(double))) != hipSuccess) return e;
    hipLaunchKernelGGL(pack_fwd_kernel, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, d_T[p], p,
                       t->fwd[p], t->fwd_hi[p], t->fwd_lo[p], t->fwdl[p]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(pack_bwd_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, d_T[p], p,
                       t->pairs, t->npairs, t->bwd[p]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    HostHarmonic hh;
    if (!build_harmonic(p, &hh)) return hipErrorInvalidValue;
    const size_t nh = hh.rounds.size() * (size_t)kQuads * hh.ng * 32;
    if ((e = hipMalloc(&t->fwdh[p], nh * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->hround[p], hh.rounds.size() * sizeof(HRound))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->hexp[p], hh.exps.size() * sizeof(HExp))) != hipSuccess) return e;
    if ((e = hipMemcpy(t->hround[p], hh.rounds.data(), hh.rounds.size() * sizeof(HRound),
                       hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(t->hexp[p], hh.exps.data(), hh.exps.size() * sizeof(HExp),
                       hipMemcpyHostToDevice)) != hipSuccess) return e;
    hipLaunchKernelGGL(pack_fwdh_kernel, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, d_T[p], p,
                       hh.maps, (int)hh.rounds.size(), hh.ng, t->fwdh[p]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t nbh = hh.rounds.size() * (size_t)t->npairs * hh.ng * 16;   // ng = n'-chunks of 4
    if ((e = hipMalloc(&t->bwdh[p], nbh * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->hfold[p], hh.folds.size() * sizeof(HFold))) != hipSuccess) return e;
    if ((e = hipMalloc(&t->hout[p], hh.outs.size() * sizeof(HOut))) != hipSuccess) return e;
    if ((e = hipMemcpy(t->hfold[p], hh.folds.data(), hh.folds.size() * sizeof(HFold),
                       hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(t->hout[p], hh.outs.data(), hh.outs.size() * sizeof(HOut),
                       hipMemcpyHostToDevice)) != hipSuccess) return e;
    hipLaunchKernelGGL(pack_bwdh_kernel, dim3((unsigned)((nbh + 255) / 256)), dim3(256), 0, s, d_T[p], p,
                       t->pairs, t->npairs, hh.maps, (int)hh.rounds.size(), hh.ng, t->bwdh[p]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

void mfma_tables_destroy(MfmaTables* t) {
  for (int p = 0; p <= kMaxP; ++p) {
    if (t->fwd[p]) (void)hipFree(t->fwd[p]);
    if (t->fwdl[p]) (void)hipFree(t->fwdl[p]);
    t->fwdl[p] = nullptr;
    if (t->fwd_hi[p]) (void)hipFree(t->fwd_hi[p]);
    if (t->fwd_lo[p]) (void)hipFree(t->fwd_lo[p]);
    if (t->bwd[p]) (void)hipFree(t->bwd[p]);
    if (t->fwdh[p]) (void)hipFree(t->fwdh[p]);
    if (t->hround[p]) (void)hipFree(t->hround[p]);
    if (t->hexp[p]) (void)hipFree(t->hexp[p]);
    if (t->bwdh[p]) (void)hipFree(t->bwdh[p]);
    if (t->hfold[p]) (void)hipFree(t->hfold[p]);
    if (t->hout[p]) (void)hipFree(t->hout[p]);
    t->bwdh[p] = nullptr;
    t->hfold[p] = nullptr;
    t->hout[p] = nullptr;
    t->fwdh[p] = nullptr;
    t->hround[p] = nullptr;
    t->hexp[p] = nullptr;
    t->fwd[p] = t->bwd[p] = nullptr;
    t->fwd_hi[p] = t->fwd_lo[p] = nullptr;
  }
  if (t->lds_off) (void)hipFree(t->lds_off);
  if (t->touch) (void)hipFree(t->touch);
  if (t->pairs) (void)hipFree(t->pairs);
  if (t->gstart) (void)hipFree(t->gstart);
  if (t->ptouch) (void)hipFree(t->ptouch);
  t->lds_off = nullptr;
  t->touch = nullptr;
  t->pairs = nullptr;
  t->gstart = nullptr;
  t->ptouch = nullptr;
}

int mfma_num_configs() { return kNumConfigs; }

bool mfma_config_supports(int cfg, fmm_precision prec) {
  return cfg >= 0 && cfg < kNumConfigs && kConfigs[cfg].prec == prec;
}

int mfma_default_config(fmm_precision prec) {
  for (int c = 0; c < kNumConfigs; ++c)
    if (kConfigs[c].prec == prec) return c;
  return 0;
}

bool mfma_config_fusable(int cfg) { return cfg >= 0 && cfg < kNumConfigs && kConfigs[cfg].ldstab > 0; }

hipError_t launch_m2l_mfma(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                           const double* M, double* L, fmm_precision prec, int cfg,
                           hipStream_t s, const double* pos, const double* mass, double* Mw) {
  if (w.count == 0) return hipSuccess;
  // (FMM_EXACT_SLICE runs through launch_m2l_slice)
  if (!mfma_config_supports(cfg, prec) || prec == FMM_EXACT_SLICE) return hipErrorInvalidValue;
  const bool fuse = pos != nullptr;
  if (fuse && (!mfma_config_fusable(cfg) || mass == nullptr || Mw != M)) return hipErrorInvalidValue;
  const int grid = std::min(t.num_cu, w.count);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, w.counter);
  const Config& c = kConfigs[cfg];
  const HRound* nr = nullptr;
  const HExp* ne = nullptr;
#define BL_LAUNCH(PIPEV, HARMV, FUSEV, B, HR, HE, ...)                                                    \
  hipLaunchKernelGGL((m2l_fwd_bl_kernel<PIPEV, HARMV, FUSEV, ##__VA_ARGS__>), dim3(grid), dim3(kBlThreads), 0, s,   \
                     w.items, w.count, w.counter, d_desc, M, L, B[2], B[3], B[4], t.lds_off, t.touch, \
                     HR[0], HR[1], HR[2], HE[0], HE[1], HE[2], pos, mass, Mw)
  const HRound* hr[3] = {t.hround[2], t.hround[3], t.hround[4]};
  const HExp* he[3] = {t.hexp[2], t.hexp[3], t.hexp[4]};
  const HRound* hr0[3] = {nr, nr, nr};
  const HExp* he0[3] = {ne, ne, ne};
  if (c.prec == FMM_FP64_HARMONIC) {
    if (c.ldstab == 1 && fuse) BL_LAUNCH(false, true, true, t.fwdh, hr, he);
    else if (c.ldstab == 1) BL_LAUNCH(false, true, false, t.fwdh, hr, he);
    else if (c.qdiv == 2 && fuse) BL_LAUNCH(true, true, true, t.fwdh, hr, he, 2);
    else if (c.qdiv == 2) BL_LAUNCH(true, true, false, t.fwdh, hr, he, 2);
    else if (fuse) BL_LAUNCH(true, true, true, t.fwdh, hr, he);
    else BL_LAUNCH(true, true, false, t.fwdh, hr, he);
    return hipGetLastError();
  }
  if (c.prec == FMM_SPLIT_FP32) {
    hipLaunchKernelGGL(m2l_fwd_split_kernel, dim3(grid), dim3(512), 0, s, w.items, w.count, w.counter,
                       d_desc, M, L, t.fwd_hi[2], t.fwd_lo[2], t.fwd_hi[3], t.fwd_lo[3], t.fwd_hi[4],
                       t.fwd_lo[4], t.lds_off, t.touch);
    return hipGetLastError();
  }
  if (c.ldstab) {
    if (c.ldstab == 2 && fuse) BL_LAUNCH(true, false, true, t.fwdl, hr0, he0);
    else if (c.ldstab == 2) BL_LAUNCH(true, false, false, t.fwdl, hr0, he0);
    else if (fuse) BL_LAUNCH(false, false, true, t.fwdl, hr0, he0);
    else BL_LAUNCH(false, false, false, t.fwdl, hr0, he0);
    return hipGetLastError();
  }
#undef BL_LAUNCH
#define FWD_LAUNCH(W, PFV)                                                                         \
  hipLaunchKernelGGL((m2l_fwd_kernel<W, PFV>), dim3(grid), dim3(W * 64), 0, s, w.items, w.count,   \
                     w.counter, d_desc, M, L, t.fwd[2], t.fwd[3], t.fwd[4], t.lds_off, t.touch)
  if (c.waves == 8 && c.prefetch) FWD_LAUNCH(8, true);
  else if (c.waves == 4 && c.prefetch) FWD_LAUNCH(4, true);
  else if (c.waves == 8) FWD_LAUNCH(8, false);
  else if (c.waves == 4) FWD_LAUNCH(4, false);
  else return hipErrorInvalidValue;
#undef FWD_LAUNCH
  return hipGetLastError();
}

int m2l_rounds(int p, bool harmonic) {
  const int cr = harmonic ? (p + 1) * (p + 1) : ncomp(p);
  return (cr + 1) / 2;
}

hipError_t launch_m2l_round_split(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                                  int64_t nsub, const int* d_base, const double* M, double* L,
                                  double* part, fmm_precision prec, int cfg, hipStream_t s) {
  if (w.count == 0) return hipSuccess;
  if (!mfma_config_supports(cfg, prec) || !mfma_config_fusable(cfg) ||
      w.count > kMaxSplitSlots || nsub > kMaxSplitSubgrids)
    return hipErrorInvalidValue;
  const int grid = std::min(t.num_cu, w.count);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, w.counter);
  const Config& c = kConfigs[cfg];
  const bool harm = c.prec == FMM_FP64_HARMONIC;
  if (harm)
    hipLaunchKernelGGL((m2l_fwd_round_kernel<true, true>), dim3(grid), dim3(kBlThreads), 0, s, w.items, w.count,
                       w.counter, d_desc, M, part, t.fwdh[2], t.fwdh[3], t.fwdh[4], t.lds_off, t.touch,
                       t.hround[2], t.hround[3], t.hround[4]);
  else if (c.ldstab == 2)
    hipLaunchKernelGGL((m2l_fwd_round_kernel<true, false>), dim3(grid), dim3(kBlThreads), 0, s, w.items, w.count,
                       w.counter, d_desc, M, part, t.fwdl[2], t.fwdl[3], t.fwdl[4], t.lds_off, t.touch,
                       nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((m2l_fwd_round_kernel<false, false>), dim3(grid), dim3(kBlThreads), 0, s, w.items, w.count,
                       w.counter, d_desc, M, part, t.fwdl[2], t.fwdl[3], t.fwdl[4], t.lds_off, t.touch,
                       nullptr, nullptr, nullptr);
  if (harm)
    hipLaunchKernelGGL((m2l_round_sum_kernel<true>), dim3((unsigned)nsub), dim3(kNTarget), 0, s, d_desc, d_base,
                       part, L, t.hexp[2], t.hexp[3], t.hexp[4]);
  else
    hipLaunchKernelGGL((m2l_round_sum_kernel<false>), dim3((unsigned)nsub), dim3(kNTarget), 0, s, d_desc, d_base,
                       part, L, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_m2l_mfma_backward(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                                    const double* dL, double* dM, bool harmonic, hipStream_t s,
                                    const double* pos, double* dmass) {
  if (w.count == 0) return hipSuccess;
  if ((pos == nullptr) != (dmass == nullptr)) return hipErrorInvalidValue;
  const int grid = std::min(t.num_cu, w.count);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, w.counter);
  const HFold* nf = nullptr;
  const HOut* no = nullptr;
#define BWD_LAUNCH(HARMV, FUSEV, B, HF0, HF1, HF2, HO0, HO1, HO2)                                  \
  hipLaunchKernelGGL((m2l_bwd_kernel<HARMV, FUSEV>), dim3(grid), dim3(kBwdThreads), 0, s, w.items,  \
                     w.count, w.counter, d_desc, dL, dM, B[2], B[3], B[4], t.pairs, t.npairs,       \
                     t.gstart, t.ptouch, HF0, HF1, HF2, HO0, HO1, HO2, pos, dmass)
  if (harmonic && pos)
    BWD_LAUNCH(true, true, t.bwdh, t.hfold[2], t.hfold[3], t.hfold[4], t.hout[2], t.hout[3], t.hout[4]);
  else if (harmonic)
    BWD_LAUNCH(true, false, t.bwdh, t.hfold[2], t.hfold[3], t.hfold[4], t.hout[2], t.hout[3], t.hout[4]);
  else if (pos)
    BWD_LAUNCH(false, true, t.bwd, nf, nf, nf, no, no, no);
  else
    BWD_LAUNCH(false, false, t.bwd, nf, nf, nf, no, no, no);
#undef BWD_LAUNCH
  return hipGetLastError();
}

}  // namespace fmm
