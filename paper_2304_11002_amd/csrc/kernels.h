// Host-side launchers of the device kernels (one translation unit each).
#pragma once

#include <vector>

#include "fmm_common.h"

namespace fmm {

// tables.hip
// Host: D_m(-d) for the ns offsets d of `stencil` ([ns][3]) and |m| <= order, [ns][ncomp(order)],
// each within one unit in the last place of the exact value.
std::vector<double> host_derivative_tables(const int* stencil, int ns, int order);
hipError_t launch_build_tensors(const double* d_D, int order_d, int p, double* d_T, hipStream_t s);

// p2m.hip
// d_ids[p], counts[p]: the sub-grids of order p; all_aligned: every descriptor's
// part_off is even (16-byte aligned particle blocks)
// window: only the reachable 20^3 window of each frame is read and written
hipError_t launch_p2m(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids, const int* counts,
                      const double* pos, const double* mass, int ppc, double* M, bool all_aligned,
                      bool window, hipStream_t s);
hipError_t launch_p2m_backward(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids,
                               const int* counts, const double* pos, int ppc, const double* dM,
                               double* dmass, bool all_aligned, hipStream_t s);

// evaluate.hip: near field + L2P at the particles of every target block;
// out [nsub][4][512][ppc]
hipError_t launch_evaluate(const DevDesc* d_desc, int64_t nsub, const double* pos,
                           const double* mass, int ppc, const double* L, double* out,
                           hipStream_t s);

// evaluate.hip: the same for the finest level of a uniform n^3 domain (n >= 8):
// pos/mass [n^3][ppc], L [C][n^3], out [4][n^3][ppc]
hipError_t launch_evaluate_grid(int p, int n, double h, const double* pos, const double* mass,
                                int ppc, const double* L, double* out, hipStream_t s);

// tree.hip: the multi-level iteration on a uniform octree (level arrays [C][n^3])
struct MfmaTables;
struct TreeTables {
  double* B[kMaxP + 1] = {};   // per order: interaction-list tables in consumption order
  double* Bh[kMaxP + 1] = {};  // the same for the harmonic form
  int* doff = nullptr;         // [8 parities][58 quads][4] offsets of the lists, packed
                               // (dx + 8) | (dy + 8) << 5 | (dz + 8) << 10
};
hipError_t tree_tables_create(TreeTables* tt, const double* const* d_T, const int* stencil_xyz,
                              int nstencil, hipStream_t s);
void tree_tables_destroy(TreeTables* tt);
hipError_t launch_tree_p2m(int p, const double* pos, const double* mass, int ppc, int n, double h,
                           double* M, hipStream_t s);
hipError_t launch_tree_m2m(int p, const double* Mc, double* Mp, int nc, double hc, hipStream_t s);
hipError_t launch_tree_l2l(int p, const double* Lp, double* Lc, int nc, double hc, hipStream_t s);
// every level in one launch: level l has n[l] cells per axis, spacing 2^lg[l],
// and sits at element offset off[l] of M and L
hipError_t launch_tree_m2l(int p, const TreeTables& tt, const MfmaTables& mt, bool harmonic,
                           const double* M, double* L, int nlev, const int* n, const int* lg,
                           const int64_t* off, hipStream_t s);

// m2l_ref.hip: sub-grids listed in d_ids (all of order p)
hipError_t launch_m2l_ref(int p, bool backward, const DevDesc* d_desc, const int* d_ids, int count,
                          const int* d_stencil, const double* d_T, const double* src, double* out,
                          hipStream_t s);

// m2l_mfma.hip: persistent matrix-core kernels over a work list
struct MfmaTables;   // device tables packed for the matrix-core kernels (per p)

}  // namespace fmm
