// Evaluation at the particles of the target block: the far part from the
// local expansion (L2P) plus the direct sums over the near cells, the leaf
// (point-mass) interactions that the M2L shell leaves out (paper Sec. IV-C:
// leaf cells interact as monopoles). For a particle y_i of target cell t:
//
//   phi_i  = sum_n L_n(t) b^n / n!  +  sum_{j != i} m_j / |y_i - y_j|
//   grad_i = sum_{|m| <= p-1} L_{m+e}(t) b^m / m!  -  sum_{j != i} m_j (y_i - y_j) / |y_i - y_j|^3
//
// with b = y_i - c_t and j over the particles of the 33 cells t + d,
// |d|^2 <= 4, in present blocks. The near sums dominate (263 pairs per
// particle at 8 per cell) and are bound by FP64 VALU issue.
//
// Work decomposition: one workgroup per (sub-grid, target z-plane): 64 target
// cells, each thread owning R particles of one cell. The source planes
// z-2 .. z+2 pass through LDS one at a time (only the cells the plane's
// offsets reach: 12^2, 10^2 or 8^2), in chunks of 8 particles per cell.
// Absent blocks and particle slots beyond ppc are staged as zero mass far
// away, which adds exact zeros, so the inner loop has no tests. The eight
// planes of one sub-grid run on one XCD (workgroups are dealt round-robin
// over the 8 XCDs), so overlapping source planes are re-read from that
// XCD's L2.
#include "kernels.h"

namespace fmm {

constexpr int kEvThreads = 256;
constexpr int kEvKC = 8;                 // source particles per cell per staged chunk
constexpr int kEvW = 12;                 // staged plane width: frame cells [6, 18) per axis
constexpr int kEvR = 2;                  // target particles per thread (one cell)
constexpr double kEvFar = 1e100;         // coordinate of padding sources (zero mass)

// 1/sqrt(x) to float64 accuracy: the single-precision hardware estimate
// y0 (relative error below 2^-22 including the rounding of x to float)
// refined with the second-order step y = y0 (1 + e/2 + 3 e^2 / 8),
// e = 1 - x y0^2, whose error is of order e^3 (the binomial series of
// (1 - e)^{-1/2}). The float estimate costs half the issue slots of the
// double one. x beyond the float range (the far padding sources, x ~ 1e200)
// gives y0 = 0 and so y = 0; x below it (two particles closer than 1e-19)
// is not refined correctly.
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y0 = (double)__builtin_amdgcn_rsqf((float)x);
  const double e = __builtin_fma(-(x * y0), y0, 1.0);
  return __builtin_fma(y0 * e, __builtin_fma(0.375, e, 0.5), y0);
}

// Adds the local expansion's value and gradient at the thread's R targets
// (b relative to the cell centre) to acc. L of the target cell through a
// buffer resource: lane offset vo (the cell), component c at the scalar
// offset c * cstride bytes, so no per-load address registers; each component
// is read once for all R targets.
template <int P>
__device__ __forceinline__ void l2p_add(__amdgpu_buffer_rsrc_t Lr, int vo, int cstride,
                                        const double (&b)[kEvR][3], double (&acc)[kEvR][4]) {
  constexpr int C = ncomp(P);
  double pw[kEvR][3][P + 1];                    // b_axis^i / i!
#pragma unroll
  for (int r = 0; r < kEvR; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pw[r][a][0] = 1.0;
#pragma unroll
      for (int i = 1; i <= P; ++i) pw[r][a][i] = pw[r][a][i - 1] * b[r][a] * (1.0 / i);
    }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const MI k = mi_of(c);
    const double l = __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(Lr, vo, c * cstride, 0));
#pragma unroll
    for (int r = 0; r < kEvR; ++r) {
      const double(&x)[P + 1] = pw[r][0];
      const double(&y)[P + 1] = pw[r][1];
      const double(&z)[P + 1] = pw[r][2];
      // d/db_x (b^k / k!) = b^(k - e_x) / (k - e_x)!
      acc[r][0] = __builtin_fma(l, x[k.x] * y[k.y] * z[k.z], acc[r][0]);
      if (k.x > 0) acc[r][1] = __builtin_fma(l, x[k.x - 1] * y[k.y] * z[k.z], acc[r][1]);
      if (k.y > 0) acc[r][2] = __builtin_fma(l, x[k.x] * y[k.y - 1] * z[k.z], acc[r][2]);
      if (k.z > 0) acc[r][3] = __builtin_fma(l, x[k.x] * y[k.y] * z[k.z - 1], acc[r][3]);
    }
  }
}

// One source particle against the thread's R targets.
template <bool SELF>
__device__ __forceinline__ void near_pair(const double (&ty)[kEvR][3], double (&acc)[kEvR][4],
                                          const int (&tk)[kEvR], double sx, double sy, double sz,
                                          double sm, int k) {
#pragma unroll
  for (int r = 0; r < kEvR; ++r) {
    const double dx = ty[r][0] - sx, dy = ty[r][1] - sy, dz = ty[r][2] - sz;
    double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    double m = sm;
    if (SELF) {                       // the particle itself: no term
      const bool self = k == tk[r];
      r2 = self ? 1.0 : r2;
      m = self ? 0.0 : m;
    }
    const double ri = rsqrt_f64(r2);
    const double mr = m * ri;
    const double mr3 = mr * (ri * ri);
    acc[r][0] += mr;
    acc[r][1] = __builtin_fma(-mr3, dx, acc[r][1]);
    acc[r][2] = __builtin_fma(-mr3, dy, acc[r][2]);
    acc[r][3] = __builtin_fma(-mr3, dz, acc[r][3]);
  }
}

// Staged source plane in LDS: per particle slot kk (0..7) and cell (fx, fy)
// of the frame window [6, 18)^2 the four doubles x, y, z, m, at double index
// kk * kEvSlot + (fy - 6) * kEvRow + (fx - 6) * 4. Rows are padded by two
// doubles so that the two rows of cells one wave reads fall on disjoint LDS
// banks, and every read of a slot is a 16-byte (x, y) and (z, m) pair at a
// fixed immediate offset from one base address.
constexpr int kEvRow = kEvW * 4 + 2;           // 50 doubles
constexpr int kEvSlot = kEvW * kEvRow;         // 600 doubles
constexpr int kEvLds = kEvKC * kEvSlot;        // 4800 doubles = 38400 bytes

// Where the cells of one workgroup's neighbourhood live. Cells are named by
// frame coordinates f in [6, 18)^3 around the 8^3 target block [8, 16)^3.
//   FrameGeom: one sub-grid's 24^3 frame (descriptor: particle offset, mask,
//              L block of 512 targets, output [4][512][ppc] per sub-grid).
//   GridGeom:  an 8^3 block of a uniform n^3 domain (cell index x + n y + n^2 z,
//              L [C][n^3], output [4][n^3][ppc]); cells outside the domain are absent.
struct FrameGeom {
  DevDesc d;
  __device__ bool present(int fx, int fy, int fz) const { return block_present(d.mask, fx, fy, fz); }
  __device__ int64_t cell(int fx, int fy, int fz) const { return fx + kFrame * fy + kFrame * kFrame * fz; }
  __device__ int64_t part0() const { return d.part_off; }
  __device__ double coord(int f, int) const { return f; }
  __device__ int64_t lcell(int fx, int fy, int fz) const { return (fx - 8) + 8 * (fy - 8) + 64 * (fz - 8); }
  __device__ int64_t ncells_out() const { return kNTarget; }
};

struct GridGeom {
  int n, ox, oy, oz;     // frame coordinate f is global f + o (o = block origin - 8)
  __device__ bool present(int fx, int fy, int fz) const {
    const unsigned gx = fx + ox, gy = fy + oy, gz = fz + oz;
    return gx < (unsigned)n && gy < (unsigned)n && gz < (unsigned)n;
  }
  __device__ int64_t cell(int fx, int fy, int fz) const {
    return (fx + ox) + (int64_t)n * (fy + oy) + (int64_t)n * n * (fz + oz);
  }
  __device__ int64_t part0() const { return 0; }
  __device__ double coord(int f, int axis) const { return f + (axis == 0 ? ox : axis == 1 ? oy : oz); }
  __device__ int64_t lcell(int fx, int fy, int fz) const { return cell(fx, fy, fz); }
  __device__ int64_t ncells_out() const { return (int64_t)n * n * n; }
};

// Stages particle slots ch*8 .. ch*8+7 of the cells of frame plane fz that
// the offsets of reach RR (|dx|, |dy| <= RR) touch: (8 + 2 RR)^2 cells.
template <int RR, class Geom>
__device__ __forceinline__ void stage_plane(double* __restrict__ s, const Geom& geo,
                                            const double* __restrict__ pos,
                                            const double* __restrict__ mass, int ppc, int fz,
                                            int ch) {
  constexpr int WR = 8 + 2 * RR;
  constexpr int NITEMS = WR * WR * kEvKC;
  for (int it = threadIdx.x; it < NITEMS; it += kEvThreads) {
    const int kk = it % kEvKC;
    const int c = it / kEvKC;
    const int fx = 8 - RR + c % WR, fy = 8 - RR + c / WR;
    const int k = ch * kEvKC + kk;
    double2 xy = make_double2(kEvFar, kEvFar), zm = make_double2(kEvFar, 0.0);
    if (k < ppc && geo.present(fx, fy, fz)) {
      const int64_t pi = geo.part0() + geo.cell(fx, fy, fz) * ppc + k;
      xy.x = pos[3 * pi];
      xy.y = pos[3 * pi + 1];
      zm.x = pos[3 * pi + 2];
      zm.y = mass[pi];
    }
    double* o = s + kk * kEvSlot + (fy - 6) * kEvRow + (fx - 6) * 4;
    *reinterpret_cast<double2*>(o) = xy;
    *reinterpret_cast<double2*>(o + 2) = zm;
  }
}

// One target z-plane tz of one block: near sums over the staged source planes,
// then L2P, written for the block's 64 x ppc particles.
template <class Geom>
__device__ __forceinline__ void evaluate_plane(double* __restrict__ s_src, const Geom& geo, int p,
                                               double h, int tz, const double* __restrict__ pos,
                                               const double* __restrict__ mass, int ppc,
                                               const double* __restrict__ L, double* __restrict__ out) {
  const int64_t p0 = geo.part0();
  const int G = (ppc + kEvR - 1) / kEvR;       // threads per target cell
  const int nslot = 64 * G;
  const int nch = (ppc + kEvKC - 1) / kEvKC;
  const int64_t ncell = geo.ncells_out();

  for (int slot0 = 0; slot0 < nslot; slot0 += kEvThreads) {
    const int slot = slot0 + (int)threadIdx.x;
    const int q = slot / G;                    // target cell within the plane (>= 64: idle)
    const int g = slot - q * G;
    const bool active = q < 64;
    const int cx = q & 7, cy = (q >> 3) & 7;
    const int64_t tcell = geo.cell(8 + cx, 8 + cy, 8 + tz);
    double ty[kEvR][3], acc[kEvR][4];
    int tk[kEvR];
#pragma unroll
    for (int r = 0; r < kEvR; ++r) {
      tk[r] = g + r * G;
      // idle slots take a point outside the domain (their results are not written)
      ty[r][0] = ty[r][1] = ty[r][2] = -1e30;
      if (active && tk[r] < ppc) {
        const double* y = pos + 3 * (p0 + tcell * ppc + tk[r]);
        ty[r][0] = y[0];
        ty[r][1] = y[1];
        ty[r][2] = y[2];
      }
      acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
    }
    // this thread's cell in the staged window, offsets added per source cell
    const double* sbase = s_src + (cy + 2) * kEvRow + (cx + 2) * 4;

    for (int dz = -2; dz <= 2; ++dz) {
      const int rr = dz == 0 ? 2 : (dz == 1 || dz == -1 ? 1 : 0);   // in-plane reach
      const int fz = 8 + tz + dz;
      for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();                       // the previous chunk is consumed
        if (rr == 2) stage_plane<2>(s_src, geo, pos, mass, ppc, fz, ch);
        else if (rr == 1) stage_plane<1>(s_src, geo, pos, mass, ppc, fz, ch);
        else stage_plane<0>(s_src, geo, pos, mass, ppc, fz, ch);
        __syncthreads();
        for (int oy = -rr; oy <= rr; ++oy) {
          for (int ox = -rr; ox <= rr; ++ox) {
            if (ox * ox + oy * oy + dz * dz > 4) continue;
            const double* sc = sbase + oy * kEvRow + ox * 4;
            if (dz == 0 && ox == 0 && oy == 0) {
#pragma unroll
              for (int kk = 0; kk < kEvKC; ++kk) {
                const double2 xy = *reinterpret_cast<const double2*>(sc + kk * kEvSlot);
                const double2 zm = *reinterpret_cast<const double2*>(sc + kk * kEvSlot + 2);
                near_pair<true>(ty, acc, tk, xy.x, xy.y, zm.x, zm.y, ch * kEvKC + kk);
              }
            } else {
#pragma unroll
              for (int kk = 0; kk < kEvKC; ++kk) {
                const double2 xy = *reinterpret_cast<const double2*>(sc + kk * kEvSlot);
                const double2 zm = *reinterpret_cast<const double2*>(sc + kk * kEvSlot + 2);
                near_pair<false>(ty, acc, tk, xy.x, xy.y, zm.x, zm.y, 0);
              }
            }
          }
        }
      }
    }

    if (active) {
      const int64_t t = geo.lcell(8 + cx, 8 + cy, 8 + tz);
      const int cstride = (int)(ncell * (int64_t)sizeof(double));
      const __amdgpu_buffer_rsrc_t Lr = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<double*>(L), (short)0, ncomp(p) * cstride, 0x00020000);
      const int vo = (int)(t * (int64_t)sizeof(double));
      const double ccx = (geo.coord(8 + cx, 0) + 0.5) * h, ccy = (geo.coord(8 + cy, 1) + 0.5) * h,
                   ccz = (geo.coord(8 + tz, 2) + 0.5) * h;
      double* o = out + t * ppc;
      double bb[kEvR][3];
#pragma unroll
      for (int r = 0; r < kEvR; ++r) {
        bb[r][0] = ty[r][0] - ccx;
        bb[r][1] = ty[r][1] - ccy;
        bb[r][2] = ty[r][2] - ccz;
      }
      switch (p) {
        case 2: l2p_add<2>(Lr, vo, cstride, bb, acc); break;
        case 3: l2p_add<3>(Lr, vo, cstride, bb, acc); break;
        case 4: l2p_add<4>(Lr, vo, cstride, bb, acc); break;
        default: break;
      }
#pragma unroll
      for (int r = 0; r < kEvR; ++r) {
        if (tk[r] >= ppc) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) o[(int64_t)c * ncell * ppc + tk[r]] = acc[r][c];
      }
    }
  }
}

__global__ void __launch_bounds__(kEvThreads) __attribute__((amdgpu_waves_per_eu(4))) evaluate_kernel(
    const DevDesc* __restrict__ desc, int nsub, const double* __restrict__ pos,
    const double* __restrict__ mass, int ppc, const double* __restrict__ L,
    double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) double s_src[kEvLds];
  // block i -> XCD i % 8; the 8 planes of sub-grid b are blocks 8 apart
  const int i = blockIdx.x;
  const int b = (i / 64) * 8 + (i % 8);
  const int tz = (i / 8) % 8;
  if (b >= nsub) return;                       // whole workgroup: no barrier is skipped by part of it
  FrameGeom geo;
  geo.d = desc[b];
  evaluate_plane(s_src, geo, geo.d.p, ldexp(1.0, -geo.d.log2_inv_h), tz, pos, mass, ppc,
                 L + geo.d.l_off, out + (int64_t)b * 4 * kNTarget * ppc);
}

// The finest level of a uniform n^3 domain: (n/8)^3 blocks x 8 planes, the
// planes of one block dealt to one XCD as above.
__global__ void __launch_bounds__(kEvThreads) __attribute__((amdgpu_waves_per_eu(4))) evaluate_grid_kernel(
    int p, int n, double h, const double* __restrict__ pos, const double* __restrict__ mass, int ppc,
    const double* __restrict__ L, double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) double s_src[kEvLds];
  const int nb = n / 8;
  const int nblk = nb * nb * nb;
  const int i = blockIdx.x;
  const int b = (i / 64) * 8 + (i % 8);
  const int tz = (i / 8) % 8;
  if (b >= nblk) return;
  GridGeom geo;
  geo.n = n;
  geo.ox = 8 * (b % nb) - 8;
  geo.oy = 8 * ((b / nb) % nb) - 8;
  geo.oz = 8 * (b / (nb * nb)) - 8;
  evaluate_plane(s_src, geo, p, h, tz, pos, mass, ppc, L, out);
}

hipError_t launch_evaluate(const DevDesc* d_desc, int64_t nsub, const double* pos,
                           const double* mass, int ppc, const double* L, double* out,
                           hipStream_t s) {
  const int64_t groups = (nsub + 7) / 8 * 64;
  hipLaunchKernelGGL(evaluate_kernel, dim3((unsigned)groups), dim3(kEvThreads), 0, s, d_desc,
                     (int)nsub, pos, mass, ppc, L, out);
  return hipGetLastError();
}

hipError_t launch_evaluate_grid(int p, int n, double h, const double* pos, const double* mass,
                                int ppc, const double* L, double* out, hipStream_t s) {
  const int64_t nblk = (int64_t)(n / 8) * (n / 8) * (n / 8);
  const int64_t groups = (nblk + 7) / 8 * 64;
  hipLaunchKernelGGL(evaluate_grid_kernel, dim3((unsigned)groups), dim3(kEvThreads), 0, s, p, n, h,
                     pos, mass, ppc, L, out);
  return hipGetLastError();
}

}  // namespace fmm
