// Matrix-core M2L kernels (persistent, work-list driven) and their tables.
#pragma once

#include <vector>

#include "fmm_common.h"

namespace fmm {

// One work item: a sub-grid (forward and adjoint kernels both own whole
// sub-grids, so every output element has exactly one writer).
struct WorkItem {
  int32_t sub;    // descriptor index
  int32_t cost;   // relative cost used for the longest-first order
};

struct WorkList {
  const WorkItem* items = nullptr;   // device, longest first
  int count = 0;
  unsigned* counter = nullptr;       // device work counter, reset by every launch
  int64_t cost = 0;
};

// Host: items for the descriptors, longest first. The cost of an item is its
// products: C^2 x present pairs for the dense form, (p+1)^4 x present pairs for
// the harmonic form (harmonic = true), whose p = 4 : p = 3 ratio is 2.44, not 3.06.
std::vector<WorkItem> build_work_list(const fmm_subgrid* desc, int64_t nsub, bool harmonic = false);
// The same list written into out[0 .. nsub) and ordered in place (no allocation):
// longest first, equal costs by descriptor index.
void fill_work_list(const fmm_subgrid* desc, int64_t nsub, bool harmonic, WorkItem* out);

constexpr int kQuads = kNStencil / 4;   // offsets are consumed four at a time
static_assert(kNStencil % 4 == 0, "offset quads");

// Harmonic form (FMM_FP64_HARMONIC). The folded moments Mh_k' (k' with kz <= 1)
// are staged two per round; each is a combination of at most kHMaxSup moment
// components of its own order, with integer coefficients.
constexpr int kHMaxSup = 6;
struct HRound {
  int32_t nsup;            // moment components read in this round
  int32_t ord0, ord1;      // orders of the two folded components (ord1 < 0: only one)
  int32_t pad;
  int32_t comp[kHMaxSup];  // component indices in I_p
  double c0[kHMaxSup];     // fold coefficients of the round's first folded component
  double c1[kHMaxSup];     // and of its second
};
// One output component L_n as a combination of the harmonic ones L_n'.
constexpr int kHMaxExp = 3;
struct HExp {
  int32_t nterm;
  int32_t col[kHMaxExp];   // harmonic column indices n'
  double coef[kHMaxExp];
};

// Harmonic adjoint. dL folds to the harmonic columns like M (Wh_n' = sum over n
// of F[n][n'] W_n, one entry per n'); each round's two accumulators hold folded
// output components Gh_k', and dM_k = sum_k' F[k][k'] Gh_k' is written from
// them: a component whose folded terms span rounds is added to in each later
// round by the thread that wrote it.
struct HFold {
  int32_t nterm;
  int32_t comp[kHMaxSup];
  double coef[kHMaxSup];
};
constexpr int kHMaxOut = 6;
struct HOut {
  int32_t nout;
  int32_t comp[kHMaxOut];    // output component k
  int32_t add[kHMaxOut];     // 1: add to the value written in an earlier round
  double c0[kHMaxOut];       // coefficient of the round's first folded accumulator
  double c1[kHMaxOut];       // and of its second
};

struct MfmaTables {
  // forward, per order p: [rounds][quad][comp of pair][n-group][kk*4 + j] float64
  double* fwd[kMaxP + 1] = {};
  // forward with LDS-staged tables, per order p: [rounds][quad][n-group][kk*4 + j][comp of pair]
  double* fwdl[kMaxP + 1] = {};
  // split precision, per order p: the same layout, float32 hi and lo parts
  float* fwd_hi[kMaxP + 1] = {};
  float* fwd_lo[kMaxP + 1] = {};
  // adjoint, per order p: [rounds][offset pair][dL chunk][kk*4 + j] float64
  double* bwd[kMaxP + 1] = {};
  int4* pairs = nullptr;        // adjoint offset pairs: (LDS offset 1, LDS offset 2, stencil 1, stencil 2 or -1)
  int npairs = 0;
  int* gstart = nullptr;        // first pair of each dz (13 groups + end)
  uint32_t* ptouch = nullptr;   // [8][npairs] blocks a target plane writes per pair
  const int* stencil = nullptr;   // [892][3] offsets (owned by the context)
  int* lds_off = nullptr;     // [892] dx + 20 dy + 400 dz
  uint32_t* touch = nullptr;  // [8][quads] blocks touched by an 8x8 target plane per quad
  // harmonic form, per order p: tables [rounds][quad][n'-group][kk*4 + j][folded comp of pair]
  // (T_d restricted to kz <= 1 rows and columns), the rounds' fold plans and the
  // expansion of L
  double* fwdh[kMaxP + 1] = {};
  HRound* hround[kMaxP + 1] = {};
  HExp* hexp[kMaxP + 1] = {};
  // harmonic adjoint, per order p: tables [rounds][offset pair][n' chunk][kk*4 + j], the
  // fold of dL per harmonic column and the output plan per round
  double* bwdh[kMaxP + 1] = {};
  HFold* hfold[kMaxP + 1] = {};
  HOut* hout[kMaxP + 1] = {};
  int num_cu = 0;
};

hipError_t mfma_tables_create(MfmaTables* t, double* const* d_T, const int* d_stencil,
                              hipStream_t s);
// The harmonic form's plan for order p: full index (in I_p) of each round's two
// folded rows (rowk[2r], rowk[2r+1]; -1 if absent) and of each harmonic column
// (colk, -1 past (p+1)^2), and the number of rounds. The device copies of the
// rounds' fold plans and of L's expansion are MfmaTables::hround / hexp.
bool harmonic_plan_maps(int p, int32_t rowk[32], int32_t colk[32], int* nrounds);
void mfma_tables_destroy(MfmaTables* t);
// The harmonic form's round plan for order p (host copy of MfmaTables::hround[p]).
bool harmonic_rounds_host(int p, std::vector<HRound>* rounds);

// ---------------------------------------------------------------------------
// Exact-slice (int8) M2L, harmonic form, orders 2 and 3 (m2l_slice.hip).
//
// The folded moments of a sub-grid (the round plan's order, 16 bytes per cell,
// zero past (p+1)^2) are scaled by the fixed per-component prescale 2^f and
// one exponent e_A per sub-grid into (-1, 1) and cut into S signed 7-bit
// slices; the tables (restricted to the harmonic rows and columns, rows in
// the same order, columns in the expansion's order) are scaled by 2^-f per row
// and 2^-e_B(n') per column and cut likewise. Slice products with i + j <= S
// are summed exactly in int32 on the matrix cores (v_mfma_i32_16x16x64_i8),
// each round's sums added to float64 accumulators with their weights.
constexpr int kSliceMax = 8;            // slices per operand, at most
constexpr int kSliceMin = 6;
constexpr int kSliceBytes = 16;         // folded components per cell (padded)
constexpr int kSlicePlane = kWin * kWin * kWin * kSliceBytes;   // bytes per slice of one sub-grid
struct SliceTables {
  // per order p = 2, 3: [kSliceMax slices][quad][64 lanes][16 bytes]: lane l holds
  // column n' = l % 16 of offset 4 quad + l / 16, byte b = folded row b
  int8_t* B[kMaxP + 1] = {};
  int32_t eB[kMaxP + 1][16] = {};       // column exponents
  int32_t f[kMaxP + 1][16] = {};        // row (folded component) prescale, round-plan order
};
// Host: tables from the float64 tables d_T (copied to the host; synchronous).
hipError_t slice_tables_create(SliceTables* st, double* const* d_T, hipStream_t s);
void slice_tables_destroy(SliceTables* st);
// planes: nsub x S slice planes (S x kSlicePlane bytes per sub-grid, in descriptor
// order); expo: nsub ints. Every descriptor must have p <= 3. The first kernel
// slices each sub-grid's window, the second runs the persistent M2L over w.
hipError_t launch_m2l_slice(const MfmaTables& mt, const SliceTables& st, const WorkList& w,
                            const DevDesc* d_desc, int64_t nsub, const double* M, double* L,
                            int S, int8_t* planes, int32_t* expo, hipStream_t s);

int mfma_num_configs();
bool mfma_config_supports(int cfg, fmm_precision prec);
int mfma_default_config(fmm_precision prec);

// pos, mass, Mw (all or none; Mw == M): the fused form, for configurations
// where mfma_config_fusable(cfg). The kernel first computes each sub-grid's
// moments (frame rows holding the reachable window, 8 particles per cell,
// 16-byte aligned particle blocks) into M through Mw, as launch_p2m with
// window = true writes them, and then its M2L.
bool mfma_config_fusable(int cfg);
hipError_t launch_m2l_mfma(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                           const double* M, double* L, fmm_precision prec, int cfg,
                           hipStream_t s, const double* pos = nullptr,
                           const double* mass = nullptr, double* Mw = nullptr);
// Round split (small batches): w lists (sub-grid, round) pairs, sub-grid-major,
// WorkItem::cost holding the round; d_base[b] is the slot (list index) of
// sub-grid b's first round; part holds kMaxSplitSlots slots of 35 x 512
// doubles. The rounds' raw sums go to their slots, then each sub-grid's are
// added in round order into L. Configurations with LDS-staged tables only.
constexpr int kMaxSplitSubgrids = 256;
constexpr int kMaxSplitSlots = kMaxSplitSubgrids * 18;   // 18 rounds: dense p = 4
constexpr size_t kSplitPartBytes = (size_t)kMaxSplitSlots * 35 * 512 * sizeof(double);
int m2l_rounds(int p, bool harmonic);
hipError_t launch_m2l_round_split(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                                  int64_t nsub, const int* d_base, const double* M, double* L,
                                  double* part, fmm_precision prec, int cfg, hipStream_t s);
// harmonic: the harmonic form of the adjoint (equal to the dense one up to rounding)
// pos, dmass (both or neither): the kernel also computes the mass gradients of
// each sub-grid's dM (as launch_p2m_backward, 8 particles per cell, 16-byte
// aligned particle blocks) into dmass
hipError_t launch_m2l_mfma_backward(const MfmaTables& t, const WorkList& w, const DevDesc* d_desc,
                                    const double* dL, double* dM, bool harmonic, hipStream_t s,
                                    const double* pos = nullptr, double* dmass = nullptr);

}  // namespace fmm
