/*
 * fmm.h -- C ABI of the MI355X (gfx950) same-level FMM interaction library.
 *
 * The operations are the steps of the gravity solver's cell-to-cell
 * interaction on N = 8 sub-grids (paper Sec. IV-C, "Octo-Tiger": FMM gravity
 * co-located with the 8^3 hydro sub-grids, cells carrying multipole moments;
 * Sec. VII-C, "Usage of multiple HPX tasks per Kokkos kernel invocation": the
 * three-step gravity iteration whose second step is the same-level
 * cell-to-cell "Multipole" interaction). The paper gives no formulas; the
 * definitions below are the Cartesian Taylor expansion of 1/|x - y|:
 *
 *   frame      one sub-grid = 24^3 cells j = (x, y, z), x fastest, linear
 *              index x + 24 y + 576 z: the 8^3 target block plus its 26
 *              neighbour blocks. Cell j spans [j h, (j+1) h), centre
 *              c_j = (j + 1/2) h. Block of cell j: j / 8 per axis, mask bit
 *              bx + 3 by + 9 bz; bit 13 (the centre block) must be set.
 *   I_p        multi-indices k = (kx, ky, kz), |k| <= p, graded order:
 *              order 0; x, y, z; xx, xy, xz, yy, yz, zz; xxx, ... C(p) =
 *              (p+1)(p+2)(p+3)/6 = 10, 20, 35 for p = 2, 3, 4.
 *   P2M        M_k(j) = sum_i m_i a_i^k / k!,  a_i = y_i - c_j.
 *   D_m(R)     the m-th Cartesian derivative of 1/|r| at R.
 *   T_d[k][n]  (-1)^|k| D_{k+n}(-d h): d = source cell - target cell, over
 *              the shell stencil S = {d in Z^3 : 5 <= |d|^2 <= 36}, |S| = 892.
 *   M2L        L_n(t) = sum_{d in S} sum_k M_k(t + d) T_d[k][n] for the 512
 *              target cells t (frame cells [8,16)^3); moments of absent
 *              blocks count as zero and their storage is never read.
 *              Phi(c_t + b) ~ sum_n L_n b^n / n! with Phi(x) = sum m / |x - y|.
 *
 * Memory layout (all float64, element offsets from the descriptor):
 *   pos   per sub-grid [13824][ppc][3]  absolute frame coordinates
 *   mass  per sub-grid [13824][ppc]
 *   M, dM per sub-grid [C][24][24][24]  (component-major, x fastest)
 *   L, dL per sub-grid [C][8][8][8]
 *
 * Conventions:
 *   - The caller owns every data buffer (device memory, 8-byte aligned);
 *     the library never frees caller memory and owns only what a context
 *     holds (stencil tables, work lists, captured graphs, tuning choices).
 *   - Compute calls are asynchronous on `stream` (a hipStream_t, NULL for
 *     the null stream). The host waits, and memory is allocated, only in
 *     these cases:
 *       * the first call with a descriptor set the context does not hold
 *         allocates device and pinned host memory for its copy and work
 *         lists (hipMalloc, hipHostMalloc);
 *       * when the context already holds 8 sets, that call first evicts the
 *         least recently used one: the host waits for that set's last launch
 *         and frees its memory and the graphs captured for it (graphs of the
 *         other sets are kept);
 *       * with FMM_OPT_USE_GRAPH, capturing a 17th graph first releases the
 *         least recently used graph, after the host has waited for that
 *         graph's last launch (on whatever stream it ran);
 *       * the first call on a set that runs the round split (FMM_OPT_ROUND_SPLIT,
 *         or fmm_autotune timing it) allocates its round list and round
 *         sums, held with the set;
 *       * the first FMM_EXACT_SLICE call on a set, or one with more slices
 *         than before, allocates the slice planes (after waiting for the
 *         set's last launch when it replaces them);
 *     fmm_create, fmm_destroy and fmm_autotune synchronise.
 *   - All argument checks run on the host before any HIP call: a call that
 *     returns FMM_EINVAL has touched neither the device nor the context's
 *     caches. HIP failures return FMM_EHIP; fmm_last_error() gives detail.
 *   - A context is not thread-safe: use one per host thread.
 *   - Calls with the same descriptor set are ordered even on different
 *     streams (each waits on the device for the previous one, since they
 *     share that set's work-list counters); calls with different sets, and
 *     the fmm_tree_* calls, may run concurrently.
 *   - Results are deterministic run to run: every output element is owned
 *     by one work item and summed in a fixed order.
 */
#ifndef FMM_H
#define FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_ctx fmm_ctx;

typedef int32_t fmm_status;
#define FMM_OK            0
#define FMM_EINVAL       -1  /* bad argument; nothing was enqueued */
#define FMM_ENOMEM       -2  /* a context-internal device/host allocation failed */
#define FMM_EHIP         -3  /* a HIP runtime call failed (detail in fmm_last_error) */
#define FMM_EUNSUPPORTED -4  /* valid request this context cannot run (e.g. host-only context) */

typedef int32_t fmm_precision;
#define FMM_FP64        0  /* float64 products and sums throughout */
#define FMM_SPLIT_FP32  1  /* hi/lo float32 products, float32 sums per offset block,
                              float64 across blocks, float64 tables and scaling */
#define FMM_FP64_HARMONIC 2 /* float64 in the harmonic (traceless) form: T_d is harmonic in k
                              and in n (1/r is harmonic), so the moments are folded to the
                              (p+1)^2 components with kz <= 1 (integer coefficients, within each
                              order), contracted with T_d restricted to those rows and columns,
                              and L is expanded back to all C components from its harmonic
                              ones (L_(a,b,c+2) = -L_(a+2,b,c) - L_(a,b+2,c)). Equal to
                              FMM_FP64 up to rounding; (p+1)^4 instead of C^2 products per pair */
#define FMM_EXACT_SLICE   3 /* the harmonic form on int8 matrix cores with exact integer sums (the
                              error-free splitting of Ozaki et al. with int8 slices): the folded
                              moments of a sub-grid are scaled by a fixed per-component power of two
                              (their geometric bound per unit cell mass) and one power of two for the
                              sub-grid into (-1, 1), the tables restricted to the harmonic rows and
                              columns by the inverse per-row factor and one power of two per column;
                              both are cut into S signed 7-bit slices (FMM_OPT_SLICES, 6 to 8), and
                              every slice product with i + j <= S is summed exactly in int32 over the
                              offsets and components, then weighted by 2^-7(i+j+2) in float64.
                              Error against the float64 M2L, relative to the absolute-value sum
                              Labs: below 1e-13 at S = 7, 1e-11 at S = 6 (about 1e-14 and 2e-12
                              measured). Orders 2 and 3 only (p = 4 returns FMM_EUNSUPPORTED);
                              needs 128,000 S bytes of device memory per sub-grid for the slices,
                              held with the descriptor set */

/* One descriptor per sub-grid (host memory). */
typedef struct {
    int32_t  p;           /* expansion order, 2, 3 or 4 */
    int32_t  log2_inv_h;  /* cell spacing h = 2^-log2_inv_h, 0 <= log2_inv_h <= 2 */
    uint32_t mask;        /* 27-bit present-block mask; bit 13 must be set */
    int32_t  reserved;    /* must be 0 */
    int64_t  m_off;       /* element offset of this sub-grid's M (or dM) block */
    int64_t  l_off;       /* element offset of this sub-grid's L (or dL) block */
    int64_t  part_off;    /* particle offset: pos at 3*part_off, mass at part_off */
} fmm_subgrid;

/* Library options (fmm_set_option). */
#define FMM_OPT_M2L_KERNEL  1  /* 0 auto (default), 1 reference VALU kernel, 2 MFMA kernel */
#define FMM_OPT_USE_GRAPH   2  /* 1 (default): replay cached hipGraphs for M2L; 0: plain launches */
#define FMM_OPT_TILE_CONFIG 3  /* -1 (default): autotuned/built-in choice; >= 0 forces a table entry */
#define FMM_OPT_P2M_WINDOW  5  /* fmm_p2m: 0 (default) writes every cell of the frame; 1 reads and writes
                                  only the frame rows (y, z) in [2,22)^2 (all 24 cells of each), which
                                  hold the reachable window [2,22)^3, the only cells fmm_m2l reads (the
                                  other cells of M keep their contents) */
#define FMM_OPT_ADJOINT_FORM 4 /* fmm_m2l_backward: 0 (default) dense form; 1 harmonic form (the
                                  transpose of the FMM_FP64_HARMONIC operator: dL folded to the
                                  (p+1)^2 harmonic columns, dM expanded from the folded components;
                                  equal to the dense adjoint up to rounding; MFMA kernel only) */
#define FMM_OPT_SLICES      7  /* FMM_EXACT_SLICE: slices per operand S, 6, 7 (default) or 8 */
#define FMM_OPT_ROUND_SPLIT 6  /* fmm_m2l (and the M2L of fmm_p2m_m2l when it runs as two
                                  launches) on batches of at most 256 sub-grids, with a configuration
                                  with LDS-staged tables: 0 one workgroup per sub-grid; 1 one
                                  workgroup per (sub-grid, round of two moment components), each
                                  round's sums added in round order by a second kernel; -1 (default)
                                  the choice fmm_autotune made for the descriptor set and precision
                                  (one workgroup per sub-grid until it has run). For batches that
                                  cannot fill the GPU, or whose longest sub-grid (p = 4) would set
                                  the time; equal up to rounding; 140 KB of device memory per
                                  (sub-grid, round) is held per descriptor set. */

/* Create a context on HIP device `device`, or a host-only context with
 * device = -1 (argument checking and host queries only; compute calls then
 * return FMM_EUNSUPPORTED after their checks pass). Computes the derivatives
 * of 1/r at the stencil offsets on the host (exact integer numerators, one
 * final rounding to float64: within one unit in the last place of every
 * entry), uploads them and forms the tables T_d for p = 2, 3, 4 and their
 * packed forms on the device, which makes this call synchronous. */
fmm_status fmm_create(fmm_ctx** out, int32_t device);

/* Release everything the context owns; NULL is accepted. Synchronises the device. */
fmm_status fmm_destroy(fmm_ctx* ctx);

/* Static strings; never NULL. */
const char* fmm_status_string(fmm_status s);
const char* fmm_last_error(const fmm_ctx* ctx);

fmm_status fmm_set_option(fmm_ctx* ctx, int32_t option, int64_t value);

/* Host queries (no device work). */
/* Number of stencil offsets (892) and the offsets (dx, dy, dz) in the
 * library's order, if `offsets` is not NULL (room for 3 * 892 int32). */
fmm_status fmm_stencil(int32_t* count, int32_t* offsets);
/* Number of (target cell, offset) pairs whose source block is present,
 * summed over the descriptors: the work unit of the throughput metric. */
fmm_status fmm_pair_count(const fmm_subgrid* desc, int64_t nsub, int64_t* pairs);

/* P2M (row "P2M": leaf moments about the cell centres; the paper's leaf
 * cells are the a = 0 special case). pos/mass as above, ppc particles per
 * cell (1..64). Writes all C * 13824 moments of each sub-grid (with
 * FMM_OPT_P2M_WINDOW = 1 only those of the rows holding the reachable
 * window, whose particles are then the only ones read); cells of absent
 * blocks get 0 and their particles are not read. */
fmm_status fmm_p2m(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                   const double* pos, const double* mass, int32_t ppc,
                   double* M, void* stream);

/* M2L (the same-level cell-to-cell interaction): writes L of every
 * sub-grid (overwrites, C * 512 values each). Mixed p, h and masks in one
 * call are handled by one persistent launch over a cost-sorted work list. */
fmm_status fmm_m2l(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                   const double* M, double* L, fmm_precision prec, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): fmm_m2l with the same
 * kernels and results (the configuration fmm_m2l uses for a descriptor set it
 * has not tuned: FMM_OPT_TILE_CONFIG, else the precision's default), with the
 * descriptor copy, the work list and the work counter in a statically
 * allocated device array instead of memory the context allocates per
 * descriptor set. The array holds FMM_NOALLOC_MAX_SUBGRIDS sub-grids (about
 * 0.8 MB) and exists once per device until the process ends. The call
 * allocates nothing: it waits on the host for the previous fmm_m2l_noalloc
 * call of this context to have copied its descriptors out of a pinned host
 * buffer that fmm_create allocated, writes this call's descriptors and
 * longest-first work list there, copies them to the array on `stream`, resets
 * the counter with a kernel and launches the persistent matrix-core kernel
 * (no graph). FMM_FP64, FMM_SPLIT_FP32 and FMM_FP64_HARMONIC; FMM_EXACT_SLICE
 * and FMM_OPT_M2L_KERNEL = 1 return FMM_EUNSUPPORTED, nsub above
 * FMM_NOALLOC_MAX_SUBGRIDS returns FMM_EINVAL. Every call on one device shares
 * that device's array, whatever its context: calls that can overlap on one
 * GPU (on other streams, or from other contexts) race and give wrong
 * results; calls ordered on one stream do not. */
#define FMM_NOALLOC_MAX_SUBGRIDS 16384
fmm_status fmm_m2l_noalloc(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                           const double* M, double* L, fmm_precision prec, void* stream);

/* P2M and M2L in one persistent launch. L is, bit for bit, what fmm_p2m
 * with FMM_OPT_P2M_WINDOW = 1 followed by fmm_m2l gives, and M receives
 * what that fmm_p2m writes: the moments of the frame rows holding the
 * reachable window (the other cells of M are not written), whatever
 * FMM_OPT_P2M_WINDOW is set to. Each workgroup computes a sub-grid's
 * moments itself, during the M2L of the sub-grid before it, so the
 * HBM-bound moment work of some workgroups overlaps the matrix work of the
 * others. The single launch is used for batches of more sub-grids than the
 * GPU has compute units, with ppc = 8, 16-byte aligned pos and mass, even
 * part_off and a configuration with LDS-staged tables (every
 * FMM_FP64_HARMONIC configuration; FMM_FP64 configurations 0 and 1);
 * otherwise, and with FMM_OPT_M2L_KERNEL = 1, the call runs the two steps
 * one after the other, with the same results. */
fmm_status fmm_p2m_m2l(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                       const double* pos, const double* mass, int32_t ppc,
                       double* M, double* L, fmm_precision prec, void* stream);

/* Adjoint of M2L with respect to M: dM_k(s) = sum over (t, d) with
 * s = t + d of sum_n dL_n(t) T_d[k][n]. dL laid out like L, dM like M;
 * dM is fully written (zero outside the reachable 20^3 window [2,22)^3
 * and on absent blocks). */
fmm_status fmm_m2l_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                            const double* dL, double* dM, void* stream);

/* Adjoint of P2M with respect to the masses: dmass_i = sum_k dM_k(j) a_i^k / k!
 * (positions held fixed). dmass laid out like mass, fully written (zero
 * for particles of absent blocks). */
fmm_status fmm_p2m_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                            const double* pos, int32_t ppc, const double* dM,
                            double* dmass, void* stream);

/* Both adjoints in one persistent launch: dM as fmm_m2l_backward writes it
 * and dmass as fmm_p2m_backward then computes from that dM, bit for bit.
 * Each workgroup computes a sub-grid's mass gradients itself, during the
 * M2L adjoint of the sub-grid after it, so the HBM-bound gradient work of
 * some workgroups overlaps the matrix work of the others. The single launch
 * is used for batches of more sub-grids than the GPU has compute units, with
 * ppc = 8, 16-byte aligned pos and dmass and even part_off; otherwise, and
 * with FMM_OPT_M2L_KERNEL = 1, the call runs the two adjoints one after the
 * other, with the same results. FMM_OPT_ADJOINT_FORM applies. */
fmm_status fmm_m2l_p2m_backward(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                                const double* pos, int32_t ppc, const double* dL,
                                double* dM, double* dmass, void* stream);

/* Evaluation at the particles (row "near field and L2P"; the leaf cells of
 * the paper's Sec. IV-C interact as point masses): for every particle i of
 * the 512 target cells t of each sub-grid, with b = y_i - c_t,
 *   phi_i  = sum_n L_n(t) b^n / n!  +  sum_{j != i} m_j / |y_i - y_j|
 *   grad_i = sum_{|m| <= p-1} L_{m+e}(t) b^m / m!
 *            - sum_{j != i} m_j (y_i - y_j) / |y_i - y_j|^3        (e = e_x, e_y, e_z)
 * where j runs over the particles of the 33 near cells t + d, |d|^2 <= 4
 * (the cells the shell S leaves out), in present blocks; grad_i is the
 * gradient of phi at y_i. L is laid out as fmm_m2l writes it (any
 * precision); pos/mass/ppc as for fmm_p2m (particles of absent blocks are
 * not read). out is dense in descriptor order, float64
 * [nsub][4][512][ppc]: phi, then the x, y and z components of grad, each
 * [512 target cells][ppc], fully written. Two different particles of the
 * near cells closer than about 1e-19 (in the units of pos), coincident ones
 * included, make that target's result inf or NaN: 1/r starts from a float32
 * estimate taken from r^2 rounded to float32, which underflows there.
 * nsub <= 2^21 per call. */
fmm_status fmm_evaluate(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                        const double* pos, const double* mass, int32_t ppc,
                        const double* L, double* out, void* stream);

/* ---------------------------------------------------------------------------
 * Multi-level iteration on a uniform octree (row "multi-level"; the paper's
 * three-step gravity iteration, Sec. VII-C: bottom-up traversal, the
 * cell-to-cell interactions on every level, top-down traversal; Sec. IV-C:
 * octree cells carry multipole moments, leaves act as point masses).
 *
 *   domain   n^3 finest cells of spacing h = 2^log2_h, cell j spans
 *            [j h, (j+1) h) per axis; particles pos [n^3][ppc][3] and mass
 *            [n^3][ppc], cell index x + n y + n^2 z (every particle inside its
 *            cell).
 *   levels   l = 0 (finest, n per axis) ... J (4 per axis); level l has n/2^l
 *            cells per axis of spacing 2^l h; parent of cell j is j/2.
 *   M, L     workspaces holding every level, finest first, each level
 *            [C][n_l][n_l][n_l] (x fastest): fmm_tree_size gives the total.
 *   P2M      level 0: M_k(j) = sum_i m_i (y_i - c_j)^k / k!.
 *   M2M      M_k(J) = sum_{children j} sum_{q <= k} M_q(j) s^(k-q)/(k-q)!,
 *            s = c_j - c_J.
 *   M2L      every level: L_n(t) = sum_{d in IL(t)} sum_k M_k(t+d) T_d[k][n]
 *            at the level's spacing, IL(t) = {d : |d|^2 > 4 and
 *            |floor((t mod 2 + d)/2)|^2 <= 4} (not near, parents near;
 *            231 offsets per parity of t); sources outside the domain absent.
 *   L2L      L_n(j) += sum_{m >= n} L_m(J) s^(m-n)/(m-n)!, coarsest first.
 *   evaluate the finest level's L2P plus the near field over |d|^2 <= 4, as
 *            fmm_evaluate; out [4][n^3][ppc] (phi, grad x, y, z).
 * Every pair of particles is then accounted for once (directly when their
 * cells are near, else on the one level where the cells' ancestors are not
 * near but the ancestors' parents are).
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t p;        /* expansion order, 2, 3 or 4 */
    int32_t n;        /* finest cells per axis: 8, 16, 32, 64 or 128 */
    int32_t ppc;      /* particles per finest cell, 1..64 */
    int32_t log2_h;   /* finest spacing h = 2^log2_h, -4 <= log2_h <= 4 */
    int32_t harmonic; /* M2L form: 0 dense C x C, 1 harmonic (as FMM_FP64_HARMONIC: equal up
                         to rounding, (p+1)^2 folded components) */
} fmm_tree;

/* Host query: number of levels (J + 1) and the float64 elements of one M or
 * L workspace (C * sum_l n_l^3). Either output may be NULL. */
fmm_status fmm_tree_size(const fmm_tree* tree, int32_t* levels, int64_t* elems);
/* P2M on level 0, then M2M up to the coarsest level: writes all of M. */
fmm_status fmm_tree_upward(fmm_ctx* ctx, const fmm_tree* tree, const double* pos,
                           const double* mass, double* M, void* stream);
/* The interaction-list M2L of every level: overwrites all of L. */
fmm_status fmm_tree_m2l(fmm_ctx* ctx, const fmm_tree* tree, const double* M, double* L,
                        void* stream);
/* L2L from the coarsest level down, in place: L_l += L2L(L_{l+1}). */
fmm_status fmm_tree_downward(fmm_ctx* ctx, const fmm_tree* tree, double* L, void* stream);
/* L2P of level 0 of L plus the near field; out [4][n^3][ppc], fully written. */
fmm_status fmm_tree_evaluate(fmm_ctx* ctx, const fmm_tree* tree, const double* pos,
                             const double* mass, const double* L, double* out, void* stream);
/* The whole iteration: upward, m2l, downward, evaluate (M and L are workspaces). */
fmm_status fmm_tree_solve(fmm_ctx* ctx, const fmm_tree* tree, const double* pos,
                          const double* mass, double* M, double* L, double* out, void* stream);

/* Copy the float64 stencil tables T_d[k][n] at unit spacing for order p to
 * device memory `out` ([892][C][C], offsets in fmm_stencil order). */
fmm_status fmm_stencil_tables(fmm_ctx* ctx, int32_t p, double* out, void* stream);

/* Autotuner: time every candidate M2L configuration (waves per workgroup,
 * operand prefetch) on these descriptors and buffers (M read, L
 * overwritten) and keep the fastest for later calls with the same
 * descriptor set and precision; `chosen` (may be NULL) receives its index.
 * On batches of at most 256 sub-grids whose chosen configuration stages its
 * tables in LDS it also times the round split (FMM_OPT_ROUND_SPLIT) with that
 * configuration, allocating its list as the option's first call does, and
 * keeps it for later calls if it is faster and the option is -1.
 * Synchronises the stream. FMM_OPT_TILE_CONFIG >= 0 overrides the choice. */
fmm_status fmm_autotune(fmm_ctx* ctx, const fmm_subgrid* desc, int64_t nsub,
                        const double* M, double* L, fmm_precision prec,
                        void* stream, int32_t* chosen);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
