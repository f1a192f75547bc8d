// Host-side launchers of the device kernels (one translation unit each).
#pragma once

#include "fmm_common.h"

namespace fmm {

// tables.hip
hipError_t launch_gen_tables(const int* d_stencil, int order_d, double* d_D, hipStream_t s);
hipError_t launch_build_tensors(const double* d_D, int order_d, int p, double* d_T, hipStream_t s);

// p2m.hip
// d_ids[p], counts[p]: the sub-grids of order p; all_aligned: every descriptor's
// part_off is even (16-byte aligned particle blocks)
hipError_t launch_p2m(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids, const int* counts,
                      const double* pos, const double* mass, int ppc, double* M, bool all_aligned,
                      hipStream_t s);
hipError_t launch_p2m_backward(const DevDesc* d_desc, int64_t nsub, const int* const* d_ids,
                               const int* counts, const double* pos, int ppc, const double* dM,
                               double* dmass, bool all_aligned, hipStream_t s);

// evaluate.hip: near field + L2P at the particles of every target block;
// out [nsub][4][512][ppc]
hipError_t launch_evaluate(const DevDesc* d_desc, int64_t nsub, const double* pos,
                           const double* mass, int ppc, const double* L, double* out,
                           hipStream_t s);

// m2l_ref.hip: sub-grids listed in d_ids (all of order p)
hipError_t launch_m2l_ref(int p, bool backward, const DevDesc* d_desc, const int* d_ids, int count,
                          const int* d_stencil, const double* d_T, const double* src, double* out,
                          hipStream_t s);

// m2l_mfma.hip: persistent matrix-core kernels over a work list
struct MfmaTables;   // device tables packed for the matrix-core kernels (per p)

}  // namespace fmm
