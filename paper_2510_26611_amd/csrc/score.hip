// Pose scoring kernels for gfx950 (wave64).
//
// Per pose (one wavefront):
//   A1  pose transform y_l = R(q) (x_l - c) + t about the geometric centre (eq. 3.14);
//   A2  long-range potential at every ligand atom from the rank-R canonical tensor
//       (Lemma 3.3, eq. 3.10): per mode the two factor rows around the point are
//       linearly interpolated and the R products are summed; lanes own columns, so
//       every factor-row load is one contiguous 512-byte segment;
//   A3  short-range potential (Def. 2.1): protein atoms within reach of the ligand
//       are taken from the cell list row by row; lanes own protein atoms, loop over
//       ligand atoms, and push the pairs with d^2 < r_c^2 into a per-wave LDS queue
//       that is drained 64 pairs at a time, so the Gaussians are evaluated by full
//       wavefronts however sparse the hits are;
//   A4  vdW flag (min d^2 >= sigma^2, eq. 3.14) and the pair count from the same
//       traversal;
//   A5  one wavefront reduction of the energy (and gradient) partials.
//
// Exactness.  The library is compiled with -ffp-contract=off: every a*b+c below
// rounds twice unless written as fma().  The transform, the grid coordinate and
// d^2 are written in one fixed operation order (see the comments), so the values
// that decide flags, counts and grid rows are reproducible bit for bit by any
// IEEE FP64 implementation that follows the same order.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"

namespace rsd {
namespace {

constexpr int kQueue = 128;   // per-wave ring of short-range pairs (two drains deep)

struct PairE {                // queued short-range pair (energy only)
  double d2, zz;
};
struct PairG {                // queued pair with what the gradient needs
  double d2, zz, dx, dy, dz;
  int l, pad;
};

static_assert(kPolyCoef == 8, "the short-range table lookup reads two double4 per interval");

struct ScoreParams {
  const double* __restrict__ F;
  int64_t mode_stride;        // nchunk * n * kChunk
  int64_t chunk_stride;       // n * kChunk
  int nchunk;
  double X0[3], smax[3];      // per mode: origin and last row (n_d - 1)
  int nm2[3];                 // per mode: last lerp row n_d - 2
  double inv_h;
  const double4* __restrict__ atoms;
  const int* __restrict__ cell_start;
  CellGrid cells;
  int64_t N;
  const double* __restrict__ t2;   // short-range t_k^2
  const double* __restrict__ w;    // short-range weights
  int S;
  const double* __restrict__ poly; // short-range polynomial table (energies only), or null
  double poly_x1, poly_inv_d1, poly_inv_d2;
  int poly_n1;
  double rc2, sig2, reach;          // reach = max(r_cut, vdw_min)
  const double4* __restrict__ lig;  // centred ligand (u_x, u_y, u_z, zeta)
  const double* __restrict__ rlig;  // max_l |u_l|
  int L;
  const double* __restrict__ quats;
  const double* __restrict__ trans;
  int64_t P;
  double* __restrict__ E;
  double* __restrict__ El;
  uint8_t* __restrict__ flags;
  int32_t* __restrict__ counts;
  double* __restrict__ grads;
  double* __restrict__ es;          // short-range energy per pose (split mode)
  double* __restrict__ gs;          // short-range gradient per pose (split mode)
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int lane_prefix(uint64_t mask) {   // set bits of mask below this lane
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ int lane_prefix_from(uint64_t mask, int base) {   // base + lane_prefix(mask)
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, (uint32_t)base));
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
// Cell coordinate floor(v) clamped to [0, dim-1]; clamping happens in FP64 so that huge or
// non-finite v never reaches an out-of-range float-to-int conversion.
__device__ __forceinline__ int cell_floor(double v, int dim) {
  if (!(v >= 0.0)) return 0;
  if (v >= (double)(dim - 1)) return dim - 1;
  return (int)v;
}

// Geometric centre c = (((0 + x_0) + x_1) + ...) / L and centred coordinates u_l = x_l - c;
// also max |u_l|.  One wavefront.
__device__ void ligand_prep(const double* __restrict__ pos, const double* __restrict__ zeta, int L,
                            double4* __restrict__ out, double* __restrict__ rlig) {
  __shared__ double c[3];
  const int lane = threadIdx.x;
  if (lane == 0) {
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int l = 0; l < L; ++l) {
      cx = cx + pos[3 * l + 0];
      cy = cy + pos[3 * l + 1];
      cz = cz + pos[3 * l + 2];
    }
    const double dl = (double)L;
    c[0] = cx / dl;
    c[1] = cy / dl;
    c[2] = cz / dl;
  }
  __syncthreads();
  double r2max = 0.0;
  for (int l = lane; l < L; l += 64) {
    const double ux = pos[3 * l + 0] - c[0];
    const double uy = pos[3 * l + 1] - c[1];
    const double uz = pos[3 * l + 2] - c[2];
    out[l] = make_double4(ux, uy, uz, zeta[l]);
    r2max = fmax(r2max, (ux * ux + uy * uy) + uz * uz);
  }
  r2max = wave_min(-r2max);
  if (lane == 0) rlig[0] = sqrt(-r2max);
}

__global__ __launch_bounds__(64) void k_ligand_prep(const double* __restrict__ pos,
                                                    const double* __restrict__ zeta, int L,
                                                    double4* __restrict__ out, double* __restrict__ rlig) {
  ligand_prep(pos, zeta, L, out, rlig);
}

// Rotation matrix of q = (w, x, y, z) in the fixed operation order shared by every kernel,
// after the validity test | ((w*w + x*x) + y*y) + z*z - 1 | <= 1e-12 with finite inputs.
__device__ __forceinline__ bool pose_frame(const double* __restrict__ q4, const double* __restrict__ t3,
                                           double R[9], double t[3]) {
  const double qw = q4[0], qx = q4[1], qy = q4[2], qz = q4[3];
  t[0] = t3[0];
  t[1] = t3[1];
  t[2] = t3[2];
  const double qq = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  const bool finite = isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz) && isfinite(t[0]) &&
                      isfinite(t[1]) && isfinite(t[2]);
  R[0] = 1.0 - 2.0 * (qy * qy + qz * qz); R[1] = 2.0 * (qx * qy - qw * qz); R[2] = 2.0 * (qx * qz + qw * qy);
  R[3] = 2.0 * (qx * qy + qw * qz); R[4] = 1.0 - 2.0 * (qx * qx + qz * qz); R[5] = 2.0 * (qy * qz - qw * qx);
  R[6] = 2.0 * (qx * qz - qw * qy); R[7] = 2.0 * (qy * qz + qw * qx); R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
  return finite && fabs(qq - 1.0) <= 1e-12;
}

// y_i = ((R_i0 u_0 + R_i1 u_1) + R_i2 u_2) + t_i
__device__ __forceinline__ double3 place(const double R[9], const double t[3], const double4 u) {
  return make_double3(((R[0] * u.x + R[1] * u.y) + R[2] * u.z) + t[0],
                      ((R[3] * u.x + R[4] * u.y) + R[5] * u.z) + t[1],
                      ((R[6] * u.x + R[7] * u.y) + R[8] * u.z) + t[2]);
}

// Grid coordinate s = (y - X0) * inv_h; in range iff 0 <= s <= n-1.
__device__ __forceinline__ bool in_grid(double y, double X0, double inv_h, double smax) {
  const double s = (y - X0) * inv_h;
  return s >= 0.0 && s <= smax;
}

// Two columns of one chunk for one atom: lerp each mode between rows i and i+1 (A, B),
// multiply the modes and accumulate the value (and the three one-sided derivative products).
template <bool GRAD>
__device__ __forceinline__ void long_pair(const double2 A0, const double2 B0, const double2 A1, const double2 B1,
                                          const double2 A2, const double2 B2, const double f0, const double f1,
                                          const double f2, double& part, double& g0, double& g1, double& g2) {
  const double dx0 = B0.x - A0.x, dx1 = B1.x - A1.x, dx2 = B2.x - A2.x;
  const double dy0 = B0.y - A0.y, dy1 = B1.y - A1.y, dy2 = B2.y - A2.y;
  const double lx0 = fma(f0, dx0, A0.x), lx1 = fma(f1, dx1, A1.x), lx2 = fma(f2, dx2, A2.x);
  const double ly0 = fma(f0, dy0, A0.y), ly1 = fma(f1, dy1, A1.y), ly2 = fma(f2, dy2, A2.y);
  const double lx01 = lx0 * lx1, ly01 = ly0 * ly1;
  part = fma(lx01, lx2, part);
  part = fma(ly01, ly2, part);
  if (GRAD) {
    g0 = fma(dx0 * lx1, lx2, g0);
    g0 = fma(dy0 * ly1, ly2, g0);
    g1 = fma(lx0 * dx1, lx2, g1);
    g1 = fma(ly0 * dy1, ly2, g1);
    g2 = fma(lx01, dx2, g2);
    g2 = fma(ly01, dy2, g2);
  }
}

template <bool GRAD>
struct PairT;
template <>
struct PairT<false> {
  using type = PairE;
};
template <>
struct PairT<true> {
  using type = PairG;
};

// LONG = true: the whole pose (A1-A5) in one wavefront.  LONG = false: A1, A3, A4 only;
// the short-range energy/gradient go to es/gs and k_combine adds the long-range partials.
template <bool GRAD, bool LONG>
__device__ void score_pose(const ScoreParams& a, const int64_t p, const double4* __restrict__ s_lig,
                           double4* __restrict__ s_y, typename PairT<GRAD>::type* __restrict__ q,
                           int* __restrict__ rowoff, int* __restrict__ rowstart, const double* __restrict__ s_tab,
                           const int lane);

// The short-range table (t_k^2 then w_k, kMaxTerms each) staged in LDS: the pair loop reads it
// once per term, and from global memory every read would be a full round trip (the compiler
// cannot prove the table is not written by the kernel, so it uses vector loads).
__device__ __forceinline__ void stage_short_table(const ScoreParams& a, double* __restrict__ s_tab) {
  for (int i = threadIdx.x; i < kMaxTerms; i += blockDim.x) {
    s_tab[i] = a.t2[i];
    s_tab[kMaxTerms + i] = a.w[i];
  }
}

template <bool GRAD, bool LONG>
__global__ __launch_bounds__(256) void k_score(const ScoreParams a) {
  using Pair = typename PairT<GRAD>::type;
  extern __shared__ double4 smem[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const int L = a.L;
  double4* s_lig = smem;
  double4* s_y = smem + L + (size_t)wv * L;                          // (y_0, y_1, y_2, zeta)
  char* tail = (char*)(smem + (size_t)L * (1 + W));
  Pair* q = (Pair*)(tail) + (size_t)wv * kQueue;
  int* rowoff = (int*)(tail + sizeof(Pair) * kQueue * W) + wv * 128;
  int* rowstart = rowoff + 64;
  double* s_tab = (double*)(tail + sizeof(Pair) * kQueue * W + sizeof(int) * 128 * W);

  for (int i = threadIdx.x; i < L; i += blockDim.x) s_lig[i] = a.lig[i];
  stage_short_table(a, s_tab);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * W + wv;
  if (p >= a.P) return;    // whole wavefront leaves; no block barrier follows
  score_pose<GRAD, LONG>(a, p, s_lig, s_y, q, rowoff, rowstart, s_tab, lane);
}

// One pose on one wavefront: A1, A3, A4 (and A2 when LONG), A5.
template <bool GRAD, bool LONG>
__device__ void score_pose(const ScoreParams& a, const int64_t p, const double4* __restrict__ s_lig,
                           double4* __restrict__ s_y, typename PairT<GRAD>::type* __restrict__ q,
                           int* __restrict__ rowoff, int* __restrict__ rowstart, const double* __restrict__ s_tab,
                           const int lane) {
  using Pair = typename PairT<GRAD>::type;
  const int L = a.L;
  // ---- A1: pose frame and atom positions
  double R[9], tv[3];
  const bool valid = pose_frame(a.quats + 4 * p, a.trans + 3 * p, R, tv);
  const double tx = tv[0], ty = tv[1], tz = tv[2];
  if (!valid) {
    if (lane == 0) {
      const double nan = __builtin_nan("");
      a.flags[p] = (uint8_t)RSD_FLAG_INVALID;
      a.counts[p] = 0;
      if (LONG) {
        a.E[p] = nan;
        if (a.El) a.El[p] = nan;
        if (GRAD) {
          for (int k = 0; k < 6; ++k) a.grads[6 * p + k] = nan;
        }
      }
    }
    return;
  }
  bool out_of_domain = false;
  for (int l = lane; l < L; l += 64) {
    const double4 u = s_lig[l];
    const double3 y = place(R, tv, u);
    s_y[l] = make_double4(y.x, y.y, y.z, u.w);
    const bool in = in_grid(y.x, a.X0[0], a.inv_h, a.smax[0]) && in_grid(y.y, a.X0[1], a.inv_h, a.smax[1]) &&
                    in_grid(y.z, a.X0[2], a.inv_h, a.smax[2]);
    out_of_domain |= !in;
  }
  const bool dom = __ballot(out_of_domain) == 0ull;
  wave_sync();

  double eL = 0.0, eS = 0.0;
  double gt0 = 0.0, gt1 = 0.0, gt2 = 0.0, gw0 = 0.0, gw1 = 0.0, gw2 = 0.0;

  // ---- A2: long-range.  The two half-wavefronts take two different atoms; lane j of a half
  // owns columns 2j and 2j+1 of every chunk and loads them from rows i and i+1 as 16-byte
  // loads (twice the bytes per lane of 8-byte loads through the same return path).
  if (LONG && dom && a.nchunk > 0) {
    const int64_t cs = a.chunk_stride / 2;                 // in double2
    const int half = lane >> 5, col2 = lane & 31;
    for (int l = 0; l < L; l += 2) {
      const int lx = l + half;
      const int la = lx < L ? lx : L - 1;                  // a missing partner repeats atom L-1 with no charge
      const double4 y = s_y[la];
      const double zeta = lx < L ? y.w : 0.0;
      const double s0 = (y.x - a.X0[0]) * a.inv_h, s1 = (y.y - a.X0[1]) * a.inv_h, s2 = (y.z - a.X0[2]) * a.inv_h;
      const int i0 = min((int)floor(s0), a.nm2[0]), i1 = min((int)floor(s1), a.nm2[1]);
      const int i2 = min((int)floor(s2), a.nm2[2]);
      const double f0 = s0 - (double)i0, f1 = s1 - (double)i1, f2 = s2 - (double)i2;
      const double2* p0 = (const double2*)(a.F + (int64_t)i0 * kChunk) + col2;
      const double2* p1 = (const double2*)(a.F + a.mode_stride + (int64_t)i1 * kChunk) + col2;
      const double2* p2 = (const double2*)(a.F + 2 * a.mode_stride + (int64_t)i2 * kChunk) + col2;
      double part = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
      int c = 0;
      for (; c + 2 <= a.nchunk; c += 2) {
        double2 A0[2], B0[2], A1[2], B1[2], A2[2], B2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          A0[u] = p0[u * cs]; B0[u] = p0[u * cs + kChunk / 2];
          A1[u] = p1[u * cs]; B1[u] = p1[u * cs + kChunk / 2];
          A2[u] = p2[u * cs]; B2[u] = p2[u * cs + kChunk / 2];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
          long_pair<GRAD>(A0[u], B0[u], A1[u], B1[u], A2[u], B2[u], f0, f1, f2, part, g0, g1, g2);
        p0 += 2 * cs; p1 += 2 * cs; p2 += 2 * cs;
      }
      for (; c < a.nchunk; ++c) {
        long_pair<GRAD>(p0[0], p0[kChunk / 2], p1[0], p1[kChunk / 2], p2[0], p2[kChunk / 2], f0, f1, f2, part, g0, g1, g2);
        p0 += cs; p1 += cs; p2 += cs;
      }
      eL = fma(zeta, part, eL);
      if (GRAD) {
        const double zh = zeta * a.inv_h;
        const double v0 = y.x - tx, v1 = y.y - ty, v2 = y.z - tz;   // R u_l
        const double G0 = zh * g0, G1 = zh * g1, G2 = zh * g2;
        gt0 += G0; gt1 += G1; gt2 += G2;
        gw0 += v1 * G2 - v2 * G1;
        gw1 += v2 * G0 - v0 * G2;
        gw2 += v0 * G1 - v1 * G0;
      }
    }
  }

  // ---- A3 + A4: short-range sum, pair count and minimum distance over the cell list
  int cnt = 0;
  double mind = __builtin_inf();
  if (a.N > 0) {
    const CellGrid g = a.cells;
    const double reach = a.rlig[0] + a.reach;
    const double Rc = reach * (1.0 + 1e-9) + 1e-9;     // conservative search radius about t
    const double Rc2 = Rc * Rc;
    const int cy0 = cell_floor((ty - Rc - g.origin) * g.inv_edge, g.dim);
    const int cy1 = cell_floor((ty + Rc - g.origin) * g.inv_edge, g.dim);
    const int cz0 = cell_floor((tz - Rc - g.origin) * g.inv_edge, g.dim);
    const int cz1 = cell_floor((tz + Rc - g.origin) * g.inv_edge, g.dim);
    const int ny = cy1 - cy0 + 1;
    // the same on every lane; readfirstlane tells the compiler so, which keeps the loops
    // below (and the queue counters they carry) uniform
    const int nrows = __builtin_amdgcn_readfirstlane(ny * (cz1 - cz0 + 1));
    // ring head / tail, wave-uniform: every update goes through readfirstlane so that the
    // compiler keeps them (and the drain test) in scalar registers
    int qh = 0, qt = 0;
    // The accept flag asks whether some pair is closer than sigma.  When sigma <= r_cut every
    // such pair is queued, so the minimum is taken over the queued pairs in the drain instead
    // of over every candidate test.
    const bool mind_in_drain = a.sig2 <= a.rc2;

    auto drain = [&](int m) {   // evaluate queued pairs [qh, qh + m), m <= 64
      wave_sync();
      if (lane < m) {
        const Pair e = q[(qh + lane) & (kQueue - 1)];
        if (mind_in_drain) mind = fmin(mind, e.d2);   // once per queued pair
        double gs = 0.0, dg = 0.0;
        if (!GRAD && a.poly) {
          // g(d^2) from the polynomial table: interval and position s in [-1, 1]
          const bool near = e.d2 < a.poly_x1;
          const double xs = near ? e.d2 * a.poly_inv_d1 : (e.d2 - a.poly_x1) * a.poly_inv_d2;
          const int ii = (int)xs;
          const double sv = 2.0 * (xs - (double)ii) - 1.0;
          const double4* c = reinterpret_cast<const double4*>(a.poly + (int64_t)(near ? ii : a.poly_n1 + ii) * kPolyCoef);
          const double4 c0 = c[0], c1 = c[1];
          double v = c1.w;
          v = fma(v, sv, c1.z);
          v = fma(v, sv, c1.y);
          v = fma(v, sv, c1.x);
          v = fma(v, sv, c0.w);
          v = fma(v, sv, c0.z);
          v = fma(v, sv, c0.y);
          gs = fma(v, sv, c0.x);
        } else {
#pragma unroll 2
          for (int k = 0; k < a.S; ++k) {
            const double t2 = s_tab[k], wk = s_tab[kMaxTerms + k];
            const double ex = exp(-(t2 * e.d2));
            gs = fma(wk, ex, gs);
            if (GRAD) dg = fma(wk * (-2.0 * t2), ex, dg);
          }
        }
        eS = fma(e.zz, gs, eS);
        if constexpr (GRAD) {
          const double cc = e.zz * dg;
          const double G0 = cc * e.dx, G1 = cc * e.dy, G2 = cc * e.dz;
          const double4 y = s_y[e.l];
          const double v0 = y.x - tx, v1 = y.y - ty, v2 = y.z - tz;
          gt0 += G0; gt1 += G1; gt2 += G2;
          gw0 += v1 * G2 - v2 * G1;
          gw1 += v2 * G0 - v0 * G2;
          gw2 += v0 * G1 - v1 * G0;
        }
      }
      qh = __builtin_amdgcn_readfirstlane(qh + m);
      wave_sync();
    };

    auto scan = [&](auto every) {   // every: the minimum over every test (sigma > r_cut)
      for (int rb = 0; rb < nrows; rb += 64) {
        const int r = rb + lane;
        int seg_start = 0, seg_len = 0;
        if (r < nrows) {
          const int cy = cy0 + r % ny, cz = cz0 + r / ny;
          const double ylo = g.origin + cy * g.edge, yhi = ylo + g.edge;
          const double zlo = g.origin + cz * g.edge, zhi = zlo + g.edge;
          const double dy = fmax(fmax(ylo - ty, ty - yhi), 0.0);
          const double dz = fmax(fmax(zlo - tz, tz - zhi), 0.0);
          const double rem = Rc2 - (dy * dy + dz * dz);
          if (rem >= 0.0) {
            const double hw = sqrt(rem);
            const int cx0 = cell_floor((tx - hw - g.origin) * g.inv_edge, g.dim);
            const int cx1 = cell_floor((tx + hw - g.origin) * g.inv_edge, g.dim);
            const int base = (cz * g.dim + cy) * g.dim;
            seg_start = a.cell_start[base + cx0];
            seg_len = a.cell_start[base + cx1 + 1] - seg_start;
          }
        }
        // inclusive scan of the segment lengths across the wavefront
        int incl = seg_len;
  #pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int v = __shfl_up(incl, off, 64);
          if (lane >= off) incl += v;
        }
        const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
        rowoff[lane] = incl - seg_len;
        rowstart[lane] = seg_start;
        wave_sync();
        for (int cb = 0; cb < total; cb += 64) {
          const int k = cb + lane;
          const bool act = k < total;
          // a lane without a candidate takes an atom so far away that every test fails
          double4 at = make_double4(1e300, 1e300, 1e300, 0.0);
          if (act) {
            int lo = 0, hi = 63;               // last row whose offset is <= k
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (rowoff[mid] <= k) lo = mid; else hi = mid - 1;
            }
            at = a.atoms[rowstart[lo] + (k - rowoff[lo])];
          }
          auto test = [&](const double4 y, const int l) {
            const double dx = y.x - at.x, dy = y.y - at.y, dz = y.z - at.z;
            const double d2 = (dx * dx + dy * dy) + dz * dz;     // ((dx^2 + dy^2) + dz^2), no fma
            const bool hit = d2 < a.rc2;                          // +inf for a lane without a candidate
            if constexpr (decltype(every)::value) mind = fmin(mind, d2);
            const uint64_t m = __ballot(hit);
            if (m != 0ull) {
              if (hit) {
                Pair& e = q[lane_prefix_from(m, qt) & (kQueue - 1)];
                e.d2 = d2;
                e.zz = at.w * y.w;
                if constexpr (GRAD) {
                  e.dx = dx; e.dy = dy; e.dz = dz; e.l = l;
                }
              }
              // the pair count is the wavefront's, like the queue tail
              cnt = __builtin_amdgcn_readfirstlane(cnt + (int)__popcll(m));
              qt = __builtin_amdgcn_readfirstlane(qt + (int)__popcll(m));
              if (qt - qh >= 64) drain(64);
            }
          };
          int l = 0;
          if constexpr (GRAD) {
            // two ligand atoms per step, both coordinate reads in flight together (faster with
            // gradients; without them the extra registers cost more than the overlap gains)
            for (; l + 2 <= L; l += 2) {
              const double4 y0 = s_y[l], y1 = s_y[l + 1];
              test(y0, l);
              test(y1, l + 1);
            }
          }
          for (; l < L; ++l) test(s_y[l], l);
        }
        wave_sync();
      }
    };
    if (mind_in_drain)
      scan(std::false_type{});
    else
      scan(std::true_type{});
    if (qt > qh) drain(qt - qh);
  }

  // ---- A5: reductions and output
  eL = wave_sum(eL);
  eS = wave_sum(eS);
  mind = wave_min(mind);   // cnt is already the wavefront's total
  if (GRAD) {
    gt0 = wave_sum(gt0); gt1 = wave_sum(gt1); gt2 = wave_sum(gt2);
    gw0 = wave_sum(gw0); gw1 = wave_sum(gw1); gw2 = wave_sum(gw2);
  }
  if (lane == 0) {
    const double nan = __builtin_nan("");
    a.flags[p] = (uint8_t)(dom ? (RSD_FLAG_IN_DOMAIN | (mind >= a.sig2 ? RSD_FLAG_ACCEPT : 0u)) : 0u);
    a.counts[p] = cnt;
    if (LONG) {
      a.E[p] = dom ? eL + eS : nan;
      if (a.El) a.El[p] = dom ? eL : nan;
      if (GRAD) {
        double* gp = a.grads + 6 * p;
        gp[0] = dom ? gt0 : nan; gp[1] = dom ? gt1 : nan; gp[2] = dom ? gt2 : nan;
        gp[3] = dom ? gw0 : nan; gp[4] = dom ? gw1 : nan; gp[5] = dom ? gw2 : nan;
      }
    } else {
      a.es[p] = eS;
      if (GRAD) {
        double* gp = a.gs + 6 * p;
        gp[0] = gt0; gp[1] = gt1; gp[2] = gt2; gp[3] = gw0; gp[4] = gw1; gp[5] = gw2;
      }
    }
  }
}

// ---------------------------------------------------------------- chunk-major long-range
// A2 reorganised for the 8 XCDs: a work item is (rank chunk c, block of poses), and the
// items are ordered chunk-major and dealt to XCDs in contiguous ranges (workgroup w runs
// on XCD w % 8), so each XCD streams all poses against one chunk of the factors
// (3 modes x n rows x 64 columns) while that chunk sits in its L2.  Every item writes,
// per pose, its chunk's share of sum_l zeta_l P_long(y_l) (and of the gradient).
struct LongParams {
  const double* __restrict__ F;
  int64_t mode_stride, chunk_stride;
  int nchunk;
  double X0[3], smax[3];         // per mode: origin and last row (n_d - 1)
  int nm2[3];                    // per mode: last lerp row n_d - 2
  double inv_h;
  const double4* __restrict__ lig;
  int L;
  const double* __restrict__ quats;
  const double* __restrict__ trans;
  int64_t P;
  int ppw;                       // poses per wavefront
  int cpi;                       // rank chunks per work item
  int64_t nblk;                  // pose blocks of 4 * ppw poses
  int64_t items, per_xcd;        // items = nblk * ceil(nchunk / cpi)
  double* __restrict__ part;     // [nchunk][P][S], S = 1 (energy) or 7 (energy, dE/dt, dE/domega)
  // tensors made by the canonical -> Tucker -> canonical step: column p of F_3 is column
  // slice[p] of U_3, so a chunk's mode-3 lerps take only a few distinct values per atom
  const double* __restrict__ U3; // rows x u3_ld, or null
  const int* __restrict__ slice; // [R]
  int u3_ld;
  int64_t R;
  // spatial order of the poses (or null): work slot i takes pose perm[i], and the partials
  // of slot i are stored at i; the combination writes each result back to its pose
  const int* __restrict__ perm;
};

constexpr int kSlots = kSharedSlots;   // distinct mode-3 columns per chunk served from LDS

struct GridPt {                  // one ligand atom of one pose: grid rows and weights
  double f0, f1, f2;
  int i0, i1, i2, pad;
};

template <bool GRAD, bool U3>
__device__ void long_item(const LongParams& a, const int c, const int64_t p0, double4* smem, bool reuse);

// The chunk's columns map to the U_3 columns clo .. clo + nsl - 1 (a contiguous range: the
// terms are grouped by core slice); with nsl <= kSlots the mode-3 lerps come from LDS.
__device__ __forceinline__ bool chunk_slices(const LongParams& a, int c, int* clo) {
  if (!a.U3) return false;
  const int64_t p_first = (int64_t)c * kChunk;
  const int64_t p_last = min(a.R, p_first + kChunk) - 1;
  *clo = a.slice[p_first];
  return a.slice[p_last] - *clo < kSlots;
}

// Work item `item`: rank chunks cpi * (item / nblk) .. + cpi - 1 for the pose block item % nblk.
// The pose transforms and grid rows are formed for the first chunk and kept in LDS for the
// others, which form only their mode-3 lerps; the chunks of an item follow one another, so the
// XCD's L2 holds the rows of about cpi chunks at once.  The whole workgroup calls it.
template <bool GRAD>
__device__ void long_work(const LongParams& a, const int64_t item, double4* smem) {
  const int c0 = a.cpi * (int)(item / a.nblk);
  const int64_t p0 = (item % a.nblk) * (4 * a.ppw);
  const int c1 = min(c0 + a.cpi, a.nchunk);
  for (int c = c0; c < c1; ++c) {
    int clo = 0;
    if (chunk_slices(a, c, &clo))
      long_item<GRAD, true>(a, c, p0, smem, c > c0);
    else
      long_item<GRAD, false>(a, c, p0, smem, c > c0);
  }
}

template <bool GRAD>
__global__ __launch_bounds__(256) void k_long(const LongParams a) {
  extern __shared__ double4 smem[];
  const int64_t j = blockIdx.x >> 3;
  if (j >= a.per_xcd) return;
  const int64_t item = (int64_t)(blockIdx.x & 7) * a.per_xcd + j;
  if (item >= a.items) return;
  long_work<GRAD>(a, item, smem);
}

// Chunk c of the long-range sum for the poses [p0, p0 + 4*ppw); the whole workgroup calls it.
// reuse: the ligand, the pose flags and the grid points (and their R u_l) in LDS are those of
// the previous call for the same poses; only the mode-3 lerps of this chunk are formed.  The
// barrier after the ligand load also separates this call's LDS writes from the previous
// call's final reads.
template <bool GRAD, bool U3>
__device__ void long_item(const LongParams& a, const int c, const int64_t p0, double4* smem, bool reuse) {
  constexpr int S = GRAD ? 7 : 1;
  const int L = a.L;
  const int PB = 4 * a.ppw;
  double4* s_lig = smem;
  GridPt* s_pt = (GridPt*)(smem + L);
  double4* s_v = (double4*)(s_pt + PB * L);    // GRAD: R u_l per point
  int* s_bad = (int*)(GRAD ? (void*)(s_v + PB * L) : (void*)s_v);
  double* s_out = (double*)(s_bad + PB);        // the block's PB x S results, stored together at the end
  double* s_l3 = s_out + PB * S;                // U3: per atom kSlots mode-3 lerps (GRAD: then their row differences)
  constexpr int L3 = GRAD ? 2 * kSlots : kSlots;
  int clo = 0;
  if (U3) chunk_slices(a, c, &clo);
  const int tid = threadIdx.x;
  if (!reuse) {
    for (int i = tid; i < L; i += 256) s_lig[i] = a.lig[i];
    for (int i = tid; i < PB; i += 256) s_bad[i] = 0;
  }
  __syncthreads();
  if (reuse) {
    if (U3) {   // this chunk's mode-3 lerps at the kept grid points (rejected poses are skipped later)
      for (int e = tid; e < PB * L; e += 256) {
        const GridPt g = s_pt[e];
        const double* r0 = a.U3 + (int64_t)g.i2 * a.u3_ld + clo;
        const double* r1 = r0 + a.u3_ld;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
          const int cq = clo + q < a.u3_ld ? q : 0;
          const double dq = r1[cq] - r0[cq];
          s_l3[e * L3 + q] = fma(g.f2, dq, r0[cq]);
          if (GRAD) s_l3[e * L3 + kSlots + q] = dq;
        }
      }
    }
  } else {
  for (int e = tid; e < PB * L; e += 256) {
    const int lp = e / L, l = e - lp * L;
    const int64_t p = p0 + lp;
    GridPt g{};
    bool ok = false;
    if (p < a.P) {
      double R[9], tv[3];
      const int64_t pi = a.perm ? (int64_t)a.perm[p] : p;
      if (pose_frame(a.quats + 4 * pi, a.trans + 3 * pi, R, tv)) {
        const double3 y = place(R, tv, s_lig[l]);
        if (in_grid(y.x, a.X0[0], a.inv_h, a.smax[0]) && in_grid(y.y, a.X0[1], a.inv_h, a.smax[1]) &&
            in_grid(y.z, a.X0[2], a.inv_h, a.smax[2])) {
          const double s0 = (y.x - a.X0[0]) * a.inv_h, s1 = (y.y - a.X0[1]) * a.inv_h;
          const double s2 = (y.z - a.X0[2]) * a.inv_h;
          g.i0 = min((int)floor(s0), a.nm2[0]);
          g.i1 = min((int)floor(s1), a.nm2[1]);
          g.i2 = min((int)floor(s2), a.nm2[2]);
          g.f0 = s0 - (double)g.i0;
          g.f1 = s1 - (double)g.i1;
          g.f2 = s2 - (double)g.i2;
          ok = true;
          if (GRAD) s_v[e] = make_double4(y.x - tv[0], y.y - tv[1], y.z - tv[2], 0.0);
          if (U3) {   // the mode-3 lerps (and differences) of the chunk's distinct U_3 columns, as F_3 would give
            const double* r0 = a.U3 + (int64_t)g.i2 * a.u3_ld + clo;
            const double* r1 = r0 + a.u3_ld;
#pragma unroll
            for (int q = 0; q < kSlots; ++q) {
              const int cq = clo + q < a.u3_ld ? q : 0;
              const double dq = r1[cq] - r0[cq];
              s_l3[e * L3 + q] = fma(g.f2, dq, r0[cq]);
              if (GRAD) s_l3[e * L3 + kSlots + q] = dq;
            }
          }
        }
      }
    }
    s_pt[e] = g;
    if (!ok) atomicOr(&s_bad[lp], 1);
  }
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  // U3: this lane's two columns as slots of the chunk's mode-3 columns
  int slot0 = 0, slot1 = 0;
  if (U3) {
    const int64_t pc = (int64_t)c * kChunk + 2 * (lane & 31);
    slot0 = pc < a.R ? a.slice[pc] - clo : 0;
    slot1 = pc + 1 < a.R ? a.slice[pc + 1] - clo : 0;
  }
  // The two half-wavefronts take two different atoms; lane j of a half owns columns 2j and
  // 2j+1 of the chunk and loads them from rows i and i+1 as 16-byte loads.  The return path
  // from L2 moves a fixed number of lanes per clock, so 16 instead of 8 bytes per lane nearly
  // halves the time of these gathers.  Atoms past L in the last group use atom L-1's rows with
  // a zero charge.
  const int half = lane >> 5;
  const double* F0 = a.F + (int64_t)c * a.chunk_stride + 2 * (lane & 31);
  const double* F1 = F0 + a.mode_stride;
  const double* F2 = F1 + a.mode_stride;
  for (int k = 0; k < a.ppw; ++k) {
    const int lp = wv * a.ppw + k;
    const int64_t p = p0 + lp;
    if (p >= a.P) break;
    double e = 0.0, gt0 = 0.0, gt1 = 0.0, gt2 = 0.0, gw0 = 0.0, gw1 = 0.0, gw2 = 0.0;
    if (!s_bad[lp]) {
      const GridPt* pts = s_pt + lp * L;
      for (int l0 = 0; l0 < L; l0 += 4) {
        double2 A0[2], B0[2], A1[2], B1[2], A2[2], B2[2];
        double f0[2], f1[2], f2[2], zeta[2], l3x[2], l3y[2], d3x[2], d3y[2];
        int la[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int lx = l0 + 2 * u + half;
          la[u] = lx < L ? lx : L - 1;
          zeta[u] = lx < L ? s_lig[la[u]].w : 0.0;
          const GridPt g = pts[la[u]];
          f0[u] = g.f0; f1[u] = g.f1; f2[u] = g.f2;
          const double2* q0 = (const double2*)(F0 + (int64_t)g.i0 * kChunk);
          const double2* q1 = (const double2*)(F1 + (int64_t)g.i1 * kChunk);
          A0[u] = q0[0]; B0[u] = q0[kChunk / 2];
          A1[u] = q1[0]; B1[u] = q1[kChunk / 2];
          if constexpr (U3) {
            const double* l3 = s_l3 + (lp * L + la[u]) * L3;
            l3x[u] = l3[slot0];
            l3y[u] = l3[slot1];
            if (GRAD) {
              d3x[u] = l3[kSlots + slot0];
              d3y[u] = l3[kSlots + slot1];
            }
          } else {
            const double2* q2 = (const double2*)(F2 + (int64_t)g.i2 * kChunk);
            A2[u] = q2[0]; B2[u] = q2[kChunk / 2];
          }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double dx0 = B0[u].x - A0[u].x, dx1 = B1[u].x - A1[u].x;
          const double dy0 = B0[u].y - A0[u].y, dy1 = B1[u].y - A1[u].y;
          const double dx2 = U3 ? (GRAD ? d3x[u] : 0.0) : B2[u].x - A2[u].x;
          const double dy2 = U3 ? (GRAD ? d3y[u] : 0.0) : B2[u].y - A2[u].y;
          const double lx0 = fma(f0[u], dx0, A0[u].x), lx1 = fma(f1[u], dx1, A1[u].x);
          const double lx2 = U3 ? l3x[u] : fma(f2[u], dx2, A2[u].x);
          const double ly0 = fma(f0[u], dy0, A0[u].y), ly1 = fma(f1[u], dy1, A1[u].y);
          const double ly2 = U3 ? l3y[u] : fma(f2[u], dy2, A2[u].y);
          const double lx01 = lx0 * lx1, ly01 = ly0 * ly1;
          e = fma(zeta[u], lx01 * lx2, e);
          e = fma(zeta[u], ly01 * ly2, e);
          if (GRAD) {
            const double zh = zeta[u] * a.inv_h;
            const double G0 = zh * (dx0 * lx1 * lx2 + dy0 * ly1 * ly2);
            const double G1 = zh * (lx0 * dx1 * lx2 + ly0 * dy1 * ly2);
            const double G2 = zh * (lx01 * dx2 + ly01 * dy2);
            const double4 v = s_v[lp * L + la[u]];
            gt0 += G0; gt1 += G1; gt2 += G2;
            gw0 += v.y * G2 - v.z * G1;
            gw1 += v.z * G0 - v.x * G2;
            gw2 += v.x * G1 - v.y * G0;
          }
        }
      }
    }
    e = wave_sum(e);
    if (GRAD) {
      gt0 = wave_sum(gt0); gt1 = wave_sum(gt1); gt2 = wave_sum(gt2);
      gw0 = wave_sum(gw0); gw1 = wave_sum(gw1); gw2 = wave_sum(gw2);
    }
    if (lane == 0) {
      double* o = s_out + lp * S;
      o[0] = e;
      if (GRAD) {
        o[1] = gt0; o[2] = gt1; o[3] = gt2; o[4] = gw0; o[5] = gw1; o[6] = gw2;
      }
    }
  }
  // One contiguous store of the block's results: single 8-byte stores from four wavefronts at
  // different times leave partial cache lines, each written back to HBM on its own.
  __syncthreads();
  const int np = (int)(a.P - p0 < PB ? a.P - p0 : PB);
  double* out = a.part + ((int64_t)c * a.P + p0) * S;
  for (int i = tid; i < np * S; i += 256) out[i] = s_out[i];
}

// E = sum_c part[c] + short part for poses in the grid; NaN otherwise (invalid poses keep
// the NaN energy they need, their flags already say why).
template <bool GRAD>
__device__ __forceinline__ void combine_pose(const double* __restrict__ part, int nchunk, int64_t P,
                                             const double* __restrict__ es, const double* __restrict__ gs,
                                             const uint8_t* __restrict__ flags, double* __restrict__ E,
                                             double* __restrict__ El, double* __restrict__ grads, int64_t slot,
                                             const int* __restrict__ perm) {
  constexpr int S = GRAD ? 7 : 1;
  const int64_t p = perm ? (int64_t)perm[slot] : slot;   // the pose whose partials are at slot
  const bool dom = (flags[p] & RSD_FLAG_IN_DOMAIN) != 0;
  double acc[S];
#pragma unroll
  for (int k = 0; k < S; ++k) acc[k] = 0.0;
  if (dom) {
    for (int c = 0; c < nchunk; ++c) {
      const double* o = part + ((int64_t)c * P + slot) * S;
#pragma unroll
      for (int k = 0; k < S; ++k) acc[k] += o[k];
    }
  }
  const double nan = __builtin_nan("");
  E[p] = dom ? acc[0] + es[p] : nan;
  if (El) El[p] = dom ? acc[0] : nan;
  if (GRAD) {
#pragma unroll
    for (int k = 0; k < 6; ++k) grads[6 * p + k] = dom ? acc[1 + k] + gs[6 * p + k] : nan;
  }
}

template <bool GRAD>
__global__ void k_combine(const double* __restrict__ part, int nchunk, int64_t P, const double* __restrict__ es,
                          const double* __restrict__ gs, const uint8_t* __restrict__ flags, double* __restrict__ E,
                          double* __restrict__ El, double* __restrict__ grads, const int* __restrict__ perm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    combine_pose<GRAD>(part, nchunk, P, es, gs, flags, E, El, grads, i, perm);
}

// ---------------------------------------------------------------- spatial order of the poses
// On a large grid one rank chunk's rows (3 x n x 512 bytes) exceed an XCD's L2, and poses in
// input order touch rows all over it.  Ordering the poses by a Morton code of their
// translation's cell (32 cells per axis over the box) makes the poses that an XCD works on
// together touch a narrow band of rows.  A counting sort on the device (histogram, scan,
// scatter; kernels only, so it can be captured in a HIP graph) gives the permutation; the
// order within a cell is that of the atomics, which no result depends on.
constexpr int kSortBits = 5;
constexpr int kSortCells = 1 << (3 * kSortBits);

__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {   // bit b of v to bit 3b
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < kSortBits; ++b) r |= ((v >> b) & 1u) << (3 * b);
  return r;
}

__device__ __forceinline__ int pose_cell(const double* __restrict__ t3, double lo, double inv_w) {
  uint32_t c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = (t3[d] - lo) * inv_w;   // NaN and out-of-box translations go to an edge cell
    c[d] = x >= (double)((1 << kSortBits) - 1) ? (uint32_t)((1 << kSortBits) - 1) : x > 0.0 ? (uint32_t)x : 0u;
  }
  return (int)(spread_bits(c[0]) | spread_bits(c[1]) << 1 | spread_bits(c[2]) << 2);
}

__global__ void k_fill_int(int* __restrict__ a, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_pose_hist(const double* __restrict__ trans, int64_t P, double lo, double inv_w,
                            int* __restrict__ cell_of, int* __restrict__ hist) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const int c = pose_cell(trans + 3 * p, lo, inv_w);
    cell_of[p] = c;
    atomicAdd(&hist[c], 1);
  }
}

// exclusive scan of the kSortCells counts in place, one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_cell_offsets(int* __restrict__ hist) {
  __shared__ int s_part[1024];
  constexpr int per = kSortCells / 1024;
  const int t = threadIdx.x;
  int sum = 0;
  for (int k = 0; k < per; ++k) sum += hist[t * per + k];
  s_part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan of the partial sums
    const int v = t >= off ? s_part[t - off] : 0;
    __syncthreads();
    s_part[t] += v;
    __syncthreads();
  }
  int run = s_part[t] - sum;
  for (int k = 0; k < per; ++k) {
    const int c = hist[t * per + k];
    hist[t * per + k] = run;
    run += c;
  }
}

__global__ void k_pose_scatter(const int* __restrict__ cell_of, int64_t P, int* __restrict__ next,
                               int* __restrict__ perm) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
    perm[atomicAdd(&next[cell_of[p]], 1)] = (int)p;
}

// The poses in the order perm (rsd_pose_order).
__global__ void k_pose_gather(const int* __restrict__ perm, int64_t P, const double* __restrict__ quats,
                              const double* __restrict__ trans, double* __restrict__ q_out, double* __restrict__ t_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[i];
    if (q_out)
      for (int k = 0; k < 4; ++k) q_out[4 * i + k] = quats[4 * p + k];
    if (t_out)
      for (int k = 0; k < 3; ++k) t_out[3 * i + k] = trans[3 * p + k];
  }
}

// ---------------------------------------------------------------- many requests per launch
// A batch scores requests with different tensors, ligands and pose counts in four launches
// (ligand frames, short-range, long-range, combine) for all of them.  Workgroups find their
// request by binary search over per-request prefix counts kept in the device table; the
// long-range work list is request-major, chunk-major and dealt to the XCDs in contiguous
// ranges exactly as for one request.  Every per-pose number is computed by the same
// device functions as rsd_score_poses in chunk-major mode, so a pose scores bit for bit the
// same alone and in a batch.
struct BatchDesc {
  ScoreParams sp;
  LongParams lp;
  const double* lig_pos;
  const double* lig_z;
  int64_t pose_base;    // first pose of the request in the combine launch
  int64_t short_base;   // first short-range block of the request within its ligand-size bucket
  int64_t xcd_base;     // first long-range slot of the request on every XCD, within its bucket
};

// Pointers read from the request table are generic to the compiler, which then emits flat
// loads and stores (slower, and they wait on the LDS counter too) for everything they reach.
// They point at device (global) memory or are null, and they are the same in every lane:
// passing the bits through an empty asm and back through the global address space keeps the
// compiler from folding the round trip away, so it emits global loads and stores as it does
// for pointers passed as kernel arguments.
template <class T>
__device__ __forceinline__ T* global_ptr(T* p) {
  uint64_t v = (uint64_t)(uintptr_t)p;
  asm("" : "+s"(v));
  return (T*)(__attribute__((address_space(1))) T*)v;
}

__device__ __forceinline__ void make_global(LongParams& a) {
  a.F = global_ptr(a.F);
  a.lig = global_ptr(a.lig);
  a.quats = global_ptr(a.quats);
  a.trans = global_ptr(a.trans);
  a.part = global_ptr(a.part);
  a.U3 = global_ptr(a.U3);
  a.slice = global_ptr(a.slice);
  a.perm = global_ptr(a.perm);
}

__device__ __forceinline__ void make_global(ScoreParams& a) {
  a.F = global_ptr(a.F);
  a.atoms = global_ptr(a.atoms);
  a.cell_start = global_ptr(a.cell_start);
  a.t2 = global_ptr(a.t2);
  a.w = global_ptr(a.w);
  a.poly = global_ptr(a.poly);
  a.lig = global_ptr(a.lig);
  a.rlig = global_ptr(a.rlig);
  a.quats = global_ptr(a.quats);
  a.trans = global_ptr(a.trans);
  a.E = global_ptr(a.E);
  a.El = global_ptr(a.El);
  a.flags = global_ptr(a.flags);
  a.counts = global_ptr(a.counts);
  a.grads = global_ptr(a.grads);
  a.es = global_ptr(a.es);
  a.gs = global_ptr(a.gs);
}

// last request r with key(r) <= x (requests with nothing to do share the next one's key)
template <class Key>
__device__ __forceinline__ int find_request(const BatchDesc* __restrict__ d, int nreq, int64_t x, Key key) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key(d[mid]) <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// find_request for a key that is the same in every lane (a workgroup index): the result is
// then made wave-uniform so that the request table is read with scalar loads
template <class Key>
__device__ __forceinline__ int find_request_uniform(const BatchDesc* __restrict__ d, int nreq, int64_t x, Key key) {
  return __builtin_amdgcn_readfirstlane(find_request(d, nreq, x, key));
}

__global__ __launch_bounds__(64) void k_batch_prep(const BatchDesc* __restrict__ d) {
  const BatchDesc& r = d[blockIdx.x];
  if (r.sp.P > 0) ligand_prep(r.lig_pos, r.lig_z, r.sp.L, const_cast<double4*>(r.sp.lig), const_cast<double*>(r.sp.rlig));
}

// Requests [first, first + nreq) of one ligand-size bucket (LDS sized for that bucket).
__global__ __launch_bounds__(256) void k_batch_short(const BatchDesc* __restrict__ dall, int first, int nreq) {
  extern __shared__ double4 smem[];
  const BatchDesc* d = dall + first;
  const int64_t blk = blockIdx.x;
  const int r = find_request_uniform(d, nreq, blk, [](const BatchDesc& x) { return x.short_base; });
  ScoreParams a = d[r].sp;   // by value: the fields then stay in registers inside the loops
  make_global(a);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const int L = a.L;
  double4* s_lig = smem;
  double4* s_y = smem + L + (size_t)wv * L;
  char* tail = (char*)(smem + (size_t)L * (1 + W));
  PairE* q = (PairE*)(tail) + (size_t)wv * kQueue;
  int* rowoff = (int*)(tail + sizeof(PairE) * kQueue * W) + wv * 128;
  int* rowstart = rowoff + 64;
  double* s_tab = (double*)(tail + sizeof(PairE) * kQueue * W + sizeof(int) * 128 * W);
  for (int i = threadIdx.x; i < L; i += blockDim.x) s_lig[i] = a.lig[i];
  stage_short_table(a, s_tab);
  __syncthreads();
  const int64_t p = (blk - d[r].short_base) * W + wv;
  if (p >= a.P) return;
  score_pose<false, false>(a, p, s_lig, s_y, q, rowoff, rowstart, s_tab, lane);
}

// Requests [first, first + nreq) of one ligand-size bucket (LDS sized for that bucket).  Each
// request's work list is split into 8 contiguous parts, part x running on XCD x, exactly as
// for a single request; XCD x walks its parts of the requests in order.
__global__ __launch_bounds__(256) void k_batch_long(const BatchDesc* __restrict__ dall, int first, int nreq) {
  extern __shared__ double4 smem[];
  const BatchDesc* d = dall + first;
  const int64_t j = blockIdx.x >> 3;
  const int r = find_request_uniform(d, nreq, j, [](const BatchDesc& x) { return x.xcd_base; });
  LongParams lp = d[r].lp;
  make_global(lp);
  const int64_t jl = j - d[r].xcd_base;
  if (jl >= lp.per_xcd) return;
  const int64_t item = (int64_t)(blockIdx.x & 7) * lp.per_xcd + jl;
  if (item >= lp.items) return;
  long_work<false>(lp, item, smem);
}

// Ligand frames of every request and, for the persistent launch, its eight work counters
// (zeroed here, in the same stream before it, so that a replayed graph starts from zero).
__global__ __launch_bounds__(64) void k_batch_prep_fused(const BatchDesc* __restrict__ d, int* __restrict__ next) {
  if (blockIdx.x == 0 && threadIdx.x < 8) next[threadIdx.x] = 0;
  const BatchDesc& r = d[blockIdx.x];
  if (r.sp.P > 0) ligand_prep(r.lig_pos, r.lig_z, r.sp.L, const_cast<double4*>(r.sp.lig), const_cast<double*>(r.sp.rlig));
}

// The whole batch's transform, short-range, vdW and long-range work in one persistent launch.
// Each XCD has a queue of work items: first its share of every request's long-range work list
// (request-major, then chunk-major, the part of XCD x exactly as in k_batch_long), then every
// eighth short-range block of four poses over all requests.  A workgroup on XCD x (workgroup
// w runs on XCD w mod 8) claims the next item of queue x with one atomic add and stops once
// the queue is exhausted, so every workgroup ends.  Requests find their items by binary search
// over prefix counts (xcd_base: long-range slots; short_base: short-range blocks, both over the
// whole table).  The per-pose arithmetic is that of rsd_score_poses in chunk-major mode.
__global__ __launch_bounds__(256) void k_batch_fused(const BatchDesc* __restrict__ d, int nreq, int64_t u_long,
                                                     int64_t u_short, int* __restrict__ next) {
  extern __shared__ double4 smem[];
  __shared__ int s_item;
  const int x = blockIdx.x & 7;
  const int64_t n_short = u_short > x ? (u_short - x + 7) / 8 : 0;
  const int64_t total = u_long + n_short;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    __syncthreads();   // the previous item is done with the LDS
    if (threadIdx.x == 0) s_item = atomicAdd(&next[x], 1);
    __syncthreads();
    const int64_t it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= total) break;
    if (it < u_long) {
      const int r = find_request_uniform(d, nreq, it, [](const BatchDesc& q) { return q.xcd_base; });
      LongParams lp = d[r].lp;
      make_global(lp);
      const int64_t jl = it - d[r].xcd_base;
      if (jl >= lp.per_xcd) continue;
      const int64_t item = (int64_t)x * lp.per_xcd + jl;
      if (item >= lp.items) continue;
      long_work<false>(lp, item, smem);
    } else {
      const int64_t g = (it - u_long) * 8 + x;
      const int r = find_request_uniform(d, nreq, g, [](const BatchDesc& q) { return q.short_base; });
      ScoreParams a = d[r].sp;
      make_global(a);
      const int L = a.L;
      double4* s_lig = smem;
      double4* s_y = smem + L + (size_t)wv * L;
      char* tail = (char*)(smem + (size_t)L * 5);
      PairE* q = (PairE*)(tail) + (size_t)wv * kQueue;
      int* rowoff = (int*)(tail + sizeof(PairE) * kQueue * 4) + wv * 128;
      int* rowstart = rowoff + 64;
      double* s_tab = (double*)(tail + sizeof(PairE) * kQueue * 4 + sizeof(int) * 128 * 4);
      for (int i = threadIdx.x; i < L; i += 256) s_lig[i] = a.lig[i];
      stage_short_table(a, s_tab);
      __syncthreads();
      const int64_t p = (g - d[r].short_base) * 4 + wv;
      if (p < a.P) score_pose<false, false>(a, p, s_lig, s_y, q, rowoff, rowstart, s_tab, lane);
    }
  }
}

__global__ void k_batch_combine(const BatchDesc* __restrict__ d, int nreq, int64_t poses) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < poses; g += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_request(d, nreq, g, [](const BatchDesc& x) { return x.pose_base; });
    const BatchDesc& x = d[r];
    combine_pose<false>(x.lp.part, x.lp.nchunk, x.sp.P, x.sp.es, nullptr, x.sp.flags, x.sp.E, x.sp.El, nullptr,
                        g - x.pose_base, x.lp.perm);
  }
}

}  // namespace

namespace {

// Scoring parameters of one request (both kernels' views); lig/rlig/es/gs/part are device scratch.
ScoreParams make_score_params(const Tensor* t, const ScoreIO& io, const double4* lig, const double* rlig, double* es,
                              double* gs) {
  ScoreParams a{};
  a.F = t->F;
  a.chunk_stride = (int64_t)t->n * kChunk;
  a.mode_stride = (int64_t)t->nchunk * a.chunk_stride;
  a.nchunk = t->nchunk;
  for (int d = 0; d < 3; ++d) {
    a.X0[d] = t->X0m[d];
    a.smax[d] = (double)(t->nm[d] - 1);
    a.nm2[d] = t->nm[d] - 2;
  }
  a.inv_h = t->inv_h;
  a.atoms = t->atoms;
  a.cell_start = t->cell_start;
  a.cells = t->cells;
  a.N = t->N;
  a.t2 = t->short_tab;
  a.w = t->short_tab + kMaxTerms;
  a.S = t->shrt.S;
  a.poly = t->short_poly;
  a.poly_x1 = t->poly_x1;
  a.poly_inv_d1 = t->poly_inv_d1;
  a.poly_inv_d2 = t->poly_inv_d2;
  a.poly_n1 = t->poly_n1;
  a.rc2 = t->sp.r_cut * t->sp.r_cut;
  a.sig2 = io.vdw_min * io.vdw_min;
  a.reach = t->sp.r_cut > io.vdw_min ? t->sp.r_cut : io.vdw_min;
  a.lig = lig;
  a.rlig = rlig;
  a.L = io.L;
  a.quats = io.quats;
  a.trans = io.trans;
  a.P = io.P;
  a.E = io.E;
  a.El = io.El;
  a.flags = io.flags;
  a.counts = io.counts;
  a.grads = io.grads;
  a.es = es;
  a.gs = gs;
  return a;
}

size_t short_lds(int L, int W, bool grad) {
  const size_t pair_bytes = grad ? sizeof(PairG) : sizeof(PairE);
  return sizeof(double4) * (size_t)L * (1 + W) + (size_t)W * (pair_bytes * kQueue + 128 * sizeof(int)) +
         2 * kMaxTerms * sizeof(double);
}

constexpr size_t kLdsDefault = 64 * 1024;   // dynamic LDS a kernel gets without asking
constexpr size_t kLdsMax = 160 * 1024;       // LDS of one gfx950 compute unit

// Dynamic LDS beyond the default must be allowed per kernel function (on the current device).
// The allowance only ever grows, so a launch prepared earlier (a batch built before another
// one with smaller needs) stays within it.
rsd_status allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= kLdsDefault) return RSD_OK;
  RSD_CHECK(bytes <= kLdsMax, RSD_E_UNSUPPORTED, "kernel needs %zu bytes of LDS", bytes);
  int dev = 0;
  RSD_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> allowed;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = allowed[{dev, kernel}];
  if (bytes <= cur) return RSD_OK;
  RSD_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  cur = bytes;
  return RSD_OK;
}

size_t long_lds(int L, int ppw, bool grad, bool u3) {
  const int PB = 4 * ppw;
  return sizeof(double4) * (size_t)L + (size_t)PB * L * (sizeof(GridPt) + (grad ? sizeof(double4) : 0)) +
         sizeof(int) * (size_t)PB + sizeof(double) * (size_t)PB * (grad ? 7 : 1) +
         (u3 ? sizeof(double) * (size_t)PB * L * kSlots * (grad ? 2 : 1) : 0);
}

int pick_ppw(int L, bool grad, bool u3, int want) {
  int ppw = want > 0 ? want : 4;
  while (ppw > 1 && long_lds(L, ppw, grad, u3) > 64 * 1024) --ppw;
  return ppw;
}

// Whether the chunk-major kernel serves the tensor's mode-3 lerps from LDS: the tensor keeps
// U_3, the option is on, and the extra LDS still fits at the poses per wavefront it gets.
// Rank chunks per long-range work item: option chunks_per_item, 0 automatic (2).  Two chunks
// share one pose transform per atom, and the two chunks' rows of modes 1-2 (2 x 2 x n x 512
// bytes, 4 MB at n = 2048) still fit an XCD's L2.
constexpr int kChunksPerItem = 2;
int chunks_per_item(const Context* ctx) { return ctx->opt_cpi > 0 ? ctx->opt_cpi : kChunksPerItem; }

bool use_u3(const Context* ctx, const Tensor* t, int L, bool grad, int ppw_want) {
  if (!t->U3 || !ctx->opt_shared_mode3) return false;
  return long_lds(L, pick_ppw(L, grad, true, ppw_want), grad, true) <= kLdsMax;
}

LongParams make_long_params(const Tensor* t, const ScoreIO& io, const double4* lig, int ppw, double* part,
                            bool shared_mode3, int cpi) {
  LongParams lp{};
  lp.F = t->F;
  lp.chunk_stride = (int64_t)t->n * kChunk;
  lp.mode_stride = (int64_t)t->nchunk * lp.chunk_stride;
  lp.nchunk = t->nchunk;
  for (int d = 0; d < 3; ++d) {
    lp.X0[d] = t->X0m[d];
    lp.smax[d] = (double)(t->nm[d] - 1);
    lp.nm2[d] = t->nm[d] - 2;
  }
  lp.inv_h = t->inv_h;
  lp.lig = lig;
  lp.L = io.L;
  lp.quats = io.quats;
  lp.trans = io.trans;
  lp.P = io.P;
  lp.ppw = ppw;
  lp.cpi = std::max(1, cpi);
  lp.nblk = (io.P + 4 * ppw - 1) / (4 * ppw);
  lp.items = lp.nblk * ((t->nchunk + lp.cpi - 1) / lp.cpi);
  lp.per_xcd = (lp.items + 7) / 8;
  lp.part = part;
  lp.U3 = shared_mode3 ? t->U3 : nullptr;
  lp.slice = t->slice;
  lp.u3_ld = t->u3_ld;
  lp.R = t->R;
  return lp;
}

// Whether a call's long-range gathers take its P poses in spatial order: option pose_order
// (0 automatic, 1 always, 2 never); automatically from kSortMinPoses poses on.  Neighbouring
// poses then share factor rows within a wavefront and workgroup (and, on grids whose rank
// chunk exceeds an XCD's L2, within the L2); the sort costs two passes over the translations.
constexpr int64_t kSortMinPoses = 16384;
bool sort_poses(const Context* ctx, const Tensor* t, int64_t P) {
  if (P < 2 || t->nchunk == 0) return false;
  if (ctx->opt_pose_order == 1) return true;
  if (ctx->opt_pose_order == 2) return false;
  return P >= kSortMinPoses;
}

// The permutation of P poses into spatial order (hist: kSortCells ints, cell_of and perm: P).
rsd_status launch_pose_sort(Context* ctx, hipStream_t s, const Tensor* t, const double* trans, int64_t P, int* hist,
                            int* cell_of, int* perm) {
  const double lo = -t->b, inv_w = (double)(1 << kSortBits) / (2.0 * t->b);
  const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 65536);
  hipStream_t saved = ctx->stream;
  ctx->stream = s;   // the timers record on the stream the sort runs on
  rsd_status st = RSD_OK;
  auto run = [&]() -> rsd_status {
    RSD_TIMED_LAUNCH(ctx, "sort", (k_fill_int<<<kSortCells / 256, 256, 0, s>>>(hist, kSortCells, 0)));
    RSD_TIMED_LAUNCH(ctx, "sort", (k_pose_hist<<<g, 256, 0, s>>>(trans, P, lo, inv_w, cell_of, hist)));
    RSD_TIMED_LAUNCH(ctx, "sort", (k_cell_offsets<<<1, 1024, 0, s>>>(hist)));
    RSD_TIMED_LAUNCH(ctx, "sort", (k_pose_scatter<<<g, 256, 0, s>>>(cell_of, P, hist, perm)));
    return RSD_OK;
  };
  st = run();
  ctx->stream = saved;
  return st;
}


}  // namespace

rsd_status pose_order(Context* ctx, const Tensor* t, const double* quats, const double* trans, int64_t P, int* perm,
                      double* q_out, double* t_out, int* sorted) {
  if (sorted) *sorted = sort_poses(ctx, t, P) ? 1 : 0;
  if (P == 0) return RSD_OK;
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(sizeof(int) * (size_t)(kSortCells + P), &ws));
  int* hist = (int*)ws;
  RSD_TRY(launch_pose_sort(ctx, ctx->stream, t, trans, P, hist, hist + kSortCells, perm));
  if (q_out || t_out) {
    const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 65536);
    RSD_TIMED_LAUNCH(ctx, "sort", (k_pose_gather<<<g, 256, 0, ctx->stream>>>(perm, P, quats, trans, q_out, t_out)));
  }
  return RSD_OK;
}

// Launch shape recorded by rsd_autotune for this workload, applied when the caller left all
// three shape options automatic.
void tuned_shape(const Context* ctx, const Tensor* t, int L, bool grad, int64_t P, int* mode, int* ppw, int* W) {
  if (!ctx->opt_use_tuning || *mode != 0 || *ppw != 0 || *W != 0 || P < 256) return;
  const auto it = ctx->tuned.find(std::make_tuple(t->n, t->nchunk, t->N, L, (int)grad));
  if (it == ctx->tuned.end()) return;
  *mode = it->second[0];
  *ppw = it->second[1];
  *W = it->second[2];
}

rsd_status launch_score(Context* ctx, const Tensor* t, const ScoreIO& io, void* ext_ws, size_t ext_bytes,
                        size_t* need) {
  if (io.P == 0) {
    if (need) *need = 0;
    return RSD_OK;
  }
  const bool grad = io.grads != nullptr;
  const int L = io.L;
  const int64_t P = io.P;
  hipStream_t s = ctx->stream;
  int mode = ctx->opt_score_mode, ppw_want = ctx->opt_poses_per_wave, W_want = ctx->opt_short_waves;
  tuned_shape(ctx, t, L, grad, P, &mode, &ppw_want, &W_want);

  // long-range mode: fused (one wavefront does the whole pose) or chunk-major (k_long)
  const int S = grad ? 7 : 1;
  const bool u3 = use_u3(ctx, t, L, grad, ppw_want);
  const int ppw = pick_ppw(L, grad, u3, ppw_want);
  bool split = t->nchunk > 0 && long_lds(L, ppw, grad, u3) <= kLdsMax;
  if (mode == 1) split = false;
  if (mode == 0 && (t->nchunk < 2 || P < 256)) split = false;

  // workspace: ligand (L double4) | radius | short energy (P) | short gradient (6P) | partials
  const size_t off_r = sizeof(double4) * (size_t)L;
  const size_t off_es = off_r + 256;
  const size_t off_gs = off_es + sizeof(double) * (size_t)(split ? P : 0);
  const size_t off_part = off_gs + sizeof(double) * (size_t)(split && grad ? 6 * P : 0);
  const bool sorted = split && sort_poses(ctx, t, P);
  // spatial order: cell histogram (kSortCells) | cell of each pose (P) | permutation (P)
  const size_t off_sort = off_part + sizeof(double) * (size_t)(split ? (int64_t)t->nchunk * P * S : 0);
  // the sorted poses' copies (quats then trans) after the sort's counts and permutation
  const size_t off_spose = (off_sort + sizeof(int) * (size_t)(kSortCells + 2 * P) + 255) / 256 * 256;
  const size_t total = sorted ? off_spose + sizeof(double) * 7 * (size_t)P : off_sort;
  if (need) {   // size query only
    *need = total;
    return RSD_OK;
  }
  void* ws = nullptr;
  if (ext_ws) {
    RSD_CHECK(total <= ext_bytes, RSD_E_UNSUPPORTED, "scoring needs %zu bytes of scratch, %zu available", total,
              ext_bytes);
    ws = ext_ws;
  } else {
    RSD_TRY(ctx->workspace(total, &ws));
  }
  char* w8 = (char*)ws;
  double4* lig = (double4*)w8;
  double* rlig = (double*)(w8 + off_r);
  RSD_TIMED_LAUNCH(ctx, "ligand_prep",
                   (k_ligand_prep<<<1, 64, 0, s>>>(io.lig_positions, io.lig_charges, L, lig, rlig)));
  const ScoreParams a = make_score_params(t, io, lig, rlig, (double*)(w8 + off_es), (double*)(w8 + off_gs));

  int W = W_want > 0 ? W_want : 4;
  if (W_want <= 0)
    while (W > 1 && short_lds(L, W, grad) > 64 * 1024) W >>= 1;
  RSD_CHECK(short_lds(L, W, grad) <= 64 * 1024, RSD_E_UNSUPPORTED, "ligand of %d atoms needs too much LDS", L);
  const int64_t blocks = (P + W - 1) / W;
  RSD_CHECK(blocks <= 0x7fffffffLL, RSD_E_UNSUPPORTED, "too many poses in one call");
  const dim3 g1((unsigned)blocks), b1(64 * W);
  const size_t lds1 = short_lds(L, W, grad);
  if (!split) {
    if (grad) {
      RSD_TIMED_LAUNCH(ctx, "score", (k_score<true, true><<<g1, b1, lds1, s>>>(a)));
    } else {
      RSD_TIMED_LAUNCH(ctx, "score", (k_score<false, true><<<g1, b1, lds1, s>>>(a)));
    }
    return RSD_OK;
  }
  LongParams lp = make_long_params(t, io, lig, ppw, (double*)(w8 + off_part), u3, chunks_per_item(ctx));
  RSD_CHECK(lp.per_xcd * 8 <= 0x7fffffffLL, RSD_E_UNSUPPORTED, "too many poses in one call");
  const int* comb_perm = nullptr;   // slot -> pose of the long-range partials, when sorted
  if (sorted) {
    int* hist = (int*)(w8 + off_sort);
    int* perm = hist + kSortCells + P;
    RSD_TRY(launch_pose_sort(ctx, s, t, io.trans, P, hist, hist + kSortCells, perm));
    // the long range reads the poses in sorted order from contiguous copies (one pass of
    // scattered reads here instead of one per rank chunk); the combination maps slots back
    double* q_sorted = (double*)(w8 + off_spose);
    double* t_sorted = q_sorted + 4 * P;
    const unsigned gs = (unsigned)std::min<int64_t>((P + 255) / 256, 65536);
    RSD_TIMED_LAUNCH(ctx, "sort", (k_pose_gather<<<gs, 256, 0, s>>>(perm, P, lp.quats, lp.trans, q_sorted, t_sorted)));
    lp.quats = q_sorted;
    lp.trans = t_sorted;
    comb_perm = perm;
  }
  const dim3 g2((unsigned)(lp.per_xcd * 8));
  const size_t lds2 = long_lds(L, ppw, grad, u3);
  const unsigned gc = (unsigned)std::min<int64_t>((P + 255) / 256, 65536);
  RSD_TRY(allow_lds(grad ? (const void*)k_long<true> : (const void*)k_long<false>, lds2));
  // The short-range kernel (FP64 ALU) and the long-range gathers (bound by the L2 return
  // path) use different units: with overlap on, the short range runs on a second stream
  // beside the long range, forked after the ligand preparation and joined before the
  // combine.
  hipStream_t s_short = s;
  if (ctx->opt_overlap && !ext_ws) {   // (the second stream's set-up allocates)
    RSD_TRY(ctx->aux_streams());
    if (!ctx->ev_fork) RSD_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    if (!ctx->ev_join) RSD_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    s_short = ctx->aux_stream[0];
    RSD_HIP(hipEventRecord(ctx->ev_fork, s));
    RSD_HIP(hipStreamWaitEvent(s_short, ctx->ev_fork, 0));
  }
  {
    struct StreamGuard {   // the timer of the short-range launch records on its stream
      Context* c;
      hipStream_t saved;
      ~StreamGuard() { c->stream = saved; }
    } sg{ctx, s};
    ctx->stream = s_short;
    if (grad) {
      RSD_TIMED_LAUNCH(ctx, "short", (k_score<true, false><<<g1, b1, lds1, s_short>>>(a)));
    } else {
      RSD_TIMED_LAUNCH(ctx, "short", (k_score<false, false><<<g1, b1, lds1, s_short>>>(a)));
    }
  }
  if (grad) {
    RSD_TIMED_LAUNCH(ctx, "long", (k_long<true><<<g2, 256, lds2, s>>>(lp)));
  } else {
    RSD_TIMED_LAUNCH(ctx, "long", (k_long<false><<<g2, 256, lds2, s>>>(lp)));
  }
  if (s_short != s) {
    RSD_HIP(hipEventRecord(ctx->ev_join, s_short));
    RSD_HIP(hipStreamWaitEvent(s, ctx->ev_join, 0));
  }
  if (grad) {
    RSD_TIMED_LAUNCH(ctx, "combine", (k_combine<true><<<gc, 256, 0, s>>>(lp.part, t->nchunk, P, a.es, a.gs, io.flags,
                                                                           io.E, io.El, io.grads, comb_perm)));
  } else {
    RSD_TIMED_LAUNCH(ctx, "combine", (k_combine<false><<<gc, 256, 0, s>>>(lp.part, t->nchunk, P, a.es, a.gs,
                                                                            io.flags, io.E, io.El, nullptr, comb_perm)));
  }
  return RSD_OK;
}

// ---------------------------------------------------------------- allocation-free scoring
// The scratch of rsd_score_poses_noalloc: one static array in the code object, so each GPU the
// library runs on holds its own copy from module load until the process ends.  In host code
// `scratch` only stands in for the symbol; its device address on each GPU is looked up once,
// with that GPU current, and every launch receives that address.
constexpr size_t kNoAllocBytes = (size_t)128 << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

rsd_status noalloc_scratch_init(int device) {
  RSD_CHECK(device >= 0 && device < kMaxDevices, RSD_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return RSD_OK;
  int cur = -1;
  RSD_HIP(hipGetDevice(&cur));
  RSD_CHECK(cur == device, RSD_E_INVALID, "device %d is not current", device);
  void* ptr = nullptr;
  RSD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  RSD_CHECK(ptr != nullptr, RSD_E_HIP, "no device address for the static scratch array");
  g_noalloc_ptr[device] = ptr;
  return RSD_OK;
}

// Scores io.P poses in equal slices whose scratch (the same layout launch_score uses) fits the
// static array; a pose's result does not depend on the slice it falls in.  Nothing here or in
// launch_score allocates when given the array: the second stream of the overlap option and the
// timing events are left out.  Nothing in the scratch needs to start at zero (the sort clears
// its own counts), so stale contents of an earlier call are harmless; calls that overlap on
// one GPU share the array and race.
rsd_status score_noalloc(Context* ctx, const Tensor* t, const ScoreIO& io) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_noalloc_ptr[ctx->device] : nullptr;
  }
  RSD_CHECK(base != nullptr, RSD_E_INVALID, "static scratch of device %d was not set up", ctx->device);
  if (io.P == 0) return RSD_OK;
  auto need_for = [&](int64_t P, size_t* bytes) -> rsd_status {
    ScoreIO q = io;
    q.P = P;
    return launch_score(ctx, t, q, base, kNoAllocBytes, bytes);
  };
  size_t one = 0;
  RSD_TRY(need_for(1, &one));
  RSD_CHECK(one <= kNoAllocBytes, RSD_E_UNSUPPORTED,
            "a single pose needs %zu bytes of scratch, more than the %zu of the static array", one, kNoAllocBytes);
  // largest slice that fits (the scratch grows with the slice), then equal slices of at most that
  int64_t lo = 1, hi = io.P;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    size_t b = 0;
    RSD_TRY(need_for(mid, &b));
    if (b <= kNoAllocBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t slices = (io.P + lo - 1) / lo;
  const int64_t per = (io.P + slices - 1) / slices;
  const bool saved_timing = ctx->timing;
  ctx->timing = false;
  rsd_status st = RSD_OK;
  for (int64_t p0 = 0; p0 < io.P && st == RSD_OK; p0 += per) {
    ScoreIO q = io;
    q.P = std::min<int64_t>(per, io.P - p0);
    q.quats = io.quats + 4 * p0;
    q.trans = io.trans + 3 * p0;
    q.E = io.E + p0;
    q.El = io.El ? io.El + p0 : nullptr;
    q.flags = io.flags + p0;
    q.counts = io.counts + p0;
    q.grads = io.grads ? io.grads + 6 * p0 : nullptr;
    st = launch_score(ctx, t, q, base, kNoAllocBytes, nullptr);
  }
  ctx->timing = saved_timing;
  return st;
}

// ---------------------------------------------------------------- gather-rate probe
// The long-range kernel's memory access without its arithmetic, for its roofline: a
// half-wavefront takes one row i of a 64-column chunk per step (a pseudo-random row, the same
// for its 32 lanes) and each lane loads 16 bytes of rows i and i+1 of two modes, two rows per
// half-wavefront in flight per step, as the kernel does for two atoms.  Workgroup w reads the
// chunk of XCD w mod 8 (2 * n * 512 bytes, L2-resident for n <= 2048).  The loaded values are
// summed and stored once per lane so that no load is dropped.
__global__ __launch_bounds__(256) void k_gather_probe(const double* __restrict__ F, int n, int64_t mode_stride,
                                                      int64_t chunk_stride, int iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double* F0 = F + (int64_t)(blockIdx.x & 7) * chunk_stride + 2 * (lane & 31);
  const double* F1 = F0 + mode_stride;
  uint32_t s = (uint32_t)(blockIdx.x * 8 + (threadIdx.x >> 5)) * 2654435761u + 12345u;
  const uint32_t mask = (uint32_t)n - 1u;   // n is a power of two
  double ax = 0.0, ay = 0.0;
  for (int it = 0; it < iters; ++it) {
    double2 A0[2], B0[2], A1[2], B1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      s = s * 1664525u + 1013904223u;
      uint32_t i0 = (s >> 7) & mask;
      s = s * 1664525u + 1013904223u;
      uint32_t i1 = (s >> 7) & mask;
      i0 = i0 == mask ? i0 - 1u : i0;
      i1 = i1 == mask ? i1 - 1u : i1;
      const double2* q0 = (const double2*)(F0 + (int64_t)i0 * kChunk);
      const double2* q1 = (const double2*)(F1 + (int64_t)i1 * kChunk);
      A0[u] = q0[0]; B0[u] = q0[kChunk / 2];
      A1[u] = q1[0]; B1[u] = q1[kChunk / 2];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ax += (A0[u].x + B0[u].x) + (A1[u].x + B1[u].x);
      ay += (A0[u].y + B0[u].y) + (A1[u].y + B1[u].y);
    }
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = ax + ay;
}

__global__ void k_fill_probe(double* __restrict__ x, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 1.0 + 1e-3 * (double)(i & 1023);
}

rsd_status probe_gather(Context* ctx, int n, int iters, double* ms, double* bytes) {
  RSD_CHECK(n >= 4 && n <= 16384 && (n & (n - 1)) == 0, RSD_E_INVALID, "n must be a power of two in [4, 16384]");
  RSD_CHECK(iters >= 1 && iters <= 4096, RSD_E_INVALID, "iters must be in [1, 4096]");
  constexpr int kBlocks = 8192;
  const int64_t chunk_stride = (int64_t)n * kChunk, mode_stride = 8 * chunk_stride;
  const int64_t count = 2 * mode_stride;
  hipStream_t s = ctx->stream;
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(sizeof(double) * (size_t)(count + (int64_t)kBlocks * 256), &ws));
  double* F = (double*)ws;
  double* out = F + count;
  k_fill_probe<<<1024, 256, 0, s>>>(F, count);
  RSD_HIP(hipGetLastError());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rsd_status st = RSD_OK;
  auto run = [&]() -> rsd_status {
    RSD_HIP(hipEventCreate(&e0));
    RSD_HIP(hipEventCreate(&e1));
    k_gather_probe<<<kBlocks, 256, 0, s>>>(F, n, mode_stride, chunk_stride, iters, out);   // warm-up
    RSD_HIP(hipGetLastError());
    double best = 1e300;
    for (int r = 0; r < 5; ++r) {
      RSD_HIP(hipEventRecord(e0, s));
      k_gather_probe<<<kBlocks, 256, 0, s>>>(F, n, mode_stride, chunk_stride, iters, out);
      RSD_HIP(hipGetLastError());
      RSD_HIP(hipEventRecord(e1, s));
      RSD_HIP(hipEventSynchronize(e1));
      float f = 0.0f;
      RSD_HIP(hipEventElapsedTime(&f, e0, e1));
      best = std::min(best, (double)f);
    }
    *ms = best;
    // per wavefront and step: two half-wavefronts x two rows in flight x (rows i, i+1 of two
    // modes) x 32 lanes x 16 bytes
    *bytes = (double)kBlocks * 4 * iters * 2 * 2 * 4 * 32 * 16;
    return RSD_OK;
  };
  st = run();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

// ---------------------------------------------------------------- launch-shape tuner
rsd_status autotune(Context* ctx, const Tensor* t, const ScoreIO& io, rsd_tune_report* rep) {
  const bool grad = io.grads != nullptr;
  const int L = io.L;
  hipStream_t s = ctx->stream;
  const int saved[4] = {ctx->opt_score_mode, ctx->opt_poses_per_wave, ctx->opt_short_waves, ctx->opt_use_tuning};
  const bool saved_timing = ctx->timing;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Shape {
    int mode, ppw, W;
    double ms;
  };
  std::vector<Shape> cand;
  double def_ms = 0.0;
  auto body = [&]() -> rsd_status {
    RSD_HIP(hipEventCreate(&e0));
    RSD_HIP(hipEventCreate(&e1));
    ctx->timing = false;
    ctx->opt_use_tuning = 0;
    auto time_shape = [&](int mode, int ppw, int W, double* ms) -> rsd_status {
      ctx->opt_score_mode = mode;
      ctx->opt_poses_per_wave = ppw;
      ctx->opt_short_waves = W;
      RSD_TRY(launch_score(ctx, t, io));   // untimed: code load, workspace growth
      double best = 1e300;
      for (int r = 0; r < 3; ++r) {
        RSD_HIP(hipEventRecord(e0, s));
        RSD_TRY(launch_score(ctx, t, io));
        RSD_HIP(hipEventRecord(e1, s));
        RSD_HIP(hipEventSynchronize(e1));
        float f = 0.0f;
        RSD_HIP(hipEventElapsedTime(&f, e0, e1));
        best = std::min(best, (double)f);
      }
      *ms = best;
      return RSD_OK;
    };
    RSD_TRY(time_shape(0, 0, 0, &def_ms));
    for (int W : {1, 2, 4}) {
      if (short_lds(L, W, grad) > 64 * 1024) continue;
      cand.push_back({1, 0, W, 0.0});
      if (t->nchunk == 0) continue;
      for (int ppw = 1; ppw <= 4; ++ppw)
        if (pick_ppw(L, grad, use_u3(ctx, t, L, grad, ppw), ppw) == ppw &&
            long_lds(L, ppw, grad, use_u3(ctx, t, L, grad, ppw)) <= kLdsMax)
          cand.push_back({2, ppw, W, 0.0});
    }
    for (auto& c : cand) RSD_TRY(time_shape(c.mode, c.ppw, c.W, &c.ms));
    return RSD_OK;
  };
  const rsd_status st = body();
  ctx->opt_score_mode = saved[0];
  ctx->opt_poses_per_wave = saved[1];
  ctx->opt_short_waves = saved[2];
  ctx->opt_use_tuning = saved[3];
  ctx->timing = saved_timing;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != RSD_OK) return st;
  RSD_CHECK(!cand.empty(), RSD_E_UNSUPPORTED, "no launch shape fits the LDS for L=%d", L);
  const Shape* best = &cand[0];
  for (const auto& c : cand)
    if (c.ms < best->ms) best = &c;
  ctx->tuned[std::make_tuple(t->n, t->nchunk, t->N, L, (int)grad)] = {best->mode, best->ppw, best->W};
  if (rep) {
    rep->score_mode = best->mode;
    rep->poses_per_wave = best->ppw;
    rep->short_waves = best->W;
    rep->candidates = (int32_t)cand.size();
    rep->best_ms = best->ms;
    rep->default_ms = def_ms;
  }
  return RSD_OK;
}

// Cell edge of the tensor's short-range cell list: scoring of the sample is timed (best of 3,
// HIP events on the context stream, the launch shapes the context would use) with the list
// rebuilt at edges r_cut / {3, 4, 5, 6}; the fastest stays.  ms[i]: time at divisor 3 + i.
rsd_status autotune_cells(Context* ctx, Tensor* t, const ScoreIO& io, int32_t* best_div, double* ms) {
  hipStream_t s = ctx->stream;
  const bool saved_timing = ctx->timing;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double t_div[4] = {0, 0, 0, 0};
  auto body = [&]() -> rsd_status {
    RSD_HIP(hipEventCreate(&e0));
    RSD_HIP(hipEventCreate(&e1));
    ctx->timing = false;
    for (int i = 0; i < 4; ++i) {
      RSD_TRY(rebuild_cells(ctx, t, 3 + i));
      RSD_TRY(launch_score(ctx, t, io));   // untimed: workspace growth
      double best = 1e300;
      for (int r = 0; r < 3; ++r) {
        RSD_HIP(hipEventRecord(e0, s));
        RSD_TRY(launch_score(ctx, t, io));
        RSD_HIP(hipEventRecord(e1, s));
        RSD_HIP(hipEventSynchronize(e1));
        float f = 0.0f;
        RSD_HIP(hipEventElapsedTime(&f, e0, e1));
        best = std::min(best, (double)f);
      }
      t_div[i] = best;
    }
    return RSD_OK;
  };
  rsd_status st = body();
  ctx->timing = saved_timing;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  int best = 1;   // r_cut / 4 unless another edge is faster
  for (int i = 0; i < 4; ++i)
    if (t_div[i] < t_div[best]) best = i;
  const rsd_status st2 = rebuild_cells(ctx, t, 3 + best);
  if (st == RSD_OK) st = st2;
  if (st != RSD_OK) return st;
  if (best_div) *best_div = 3 + best;
  if (ms)
    for (int i = 0; i < 4; ++i) ms[i] = t_div[i];
  return RSD_OK;
}

// ---------------------------------------------------------------- batches
struct Batch {
  Context* ctx = nullptr;
  int nreq = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  BatchDesc* d = nullptr;
  struct Launch {          // one launch over the table range [first, first + count)
    int first, count, W;   // W: wavefronts per workgroup (short range)
    size_t lds;
    int64_t units;         // workgroups (short range) or work-list slots per XCD (long range)
  };
  std::vector<Launch> shorts, longs;
  struct Sort {            // a request whose poses the long range takes in spatial order
    const Tensor* t;
    const double* trans;
    int64_t P;
    int* perm;
  };
  std::vector<Sort> sorts;
  int* sort_hist = nullptr;   // shared by the requests' sorts, which run one after another
  int* sort_cell = nullptr;
  int64_t poses = 0;
  // persistent mode: one launch of `groups` workgroups over u_long long-range slots per XCD and
  // u_short short-range blocks, with `lds` bytes of LDS; next: the eight queue counters
  bool fused = false;
  int64_t u_long = 0, u_short = 0;
  size_t lds = 0;
  int groups = 0;
  int* next = nullptr;
  std::vector<BatchDesc> host_table;   // source of the (asynchronous) table upload
  hipEvent_t uploaded = nullptr;       // recorded after the upload: host_table may go once it completes
};

// Work-group slots per CU that a launch's LDS leaves, capped by the wavefronts a CU holds.
// LDS goes to workgroups in granules of 1,280 bytes: a launch of 53,808 bytes per group fits
// two groups per CU, not three (measured as a 5 % slower batch when such a request set the
// launch's size for requests of 41-53 KB).
constexpr size_t kLdsGranule = 1280;
static int lds_occupancy(size_t lds, int waves_per_group) {
  const size_t g = (std::max<size_t>(lds, 1) + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
  return (int)std::min<size_t>(kLdsMax / g, (size_t)(32 / waves_per_group));
}

rsd_status batch_create(Context* ctx, const rsd_request* req_in, int32_t nreq, Batch** out) {
  *out = nullptr;
  RSD_CHECK(nreq >= 1 && nreq <= 65536, RSD_E_INVALID, "request count %d outside [1, 65536]", nreq);
  RSD_CHECK(req_in != nullptr, RSD_E_INVALID, "requests are NULL");
  for (int r = 0; r < nreq; ++r) {
    const rsd_request& q = req_in[r];
    RSD_CHECK(q.tensor != nullptr && static_cast<const Tensor*>(q.tensor)->ctx->device == ctx->device, RSD_E_INVALID,
              "request %d: tensor missing or on another device", r);
    RSD_CHECK(q.L >= 1 && q.L <= kMaxLigand, RSD_E_UNSUPPORTED, "request %d: L=%lld outside [1, %d]", r,
              (long long)q.L, kMaxLigand);
    RSD_CHECK(q.P >= 0 && q.P <= ((int64_t)1 << 31), RSD_E_INVALID, "request %d: P out of range", r);
    RSD_CHECK(std::isfinite(q.vdw_min) && q.vdw_min >= 0, RSD_E_INVALID, "request %d: bad vdw_min", r);
    RSD_CHECK(q.P == 0 || (q.lig_charges && q.lig_positions && q.quats && q.trans && q.energies && q.flags &&
                           q.counts),
              RSD_E_INVALID, "request %d: NULL pointer", r);
  }
  // Each request's launch shape as a call of its own would take it.  A launch's LDS is the
  // largest any of its requests needs, so requests are grouped by the occupancy their own LDS
  // allows: none then runs with fewer workgroups per CU than it would alone.
  struct Shape {
    int ppw, u3, W, occ_s, occ_l;
    size_t lds_s, lds_l;
  };
  std::vector<Shape> shp((size_t)nreq);
  for (int r = 0; r < nreq; ++r) {
    const rsd_request& q = req_in[r];
    const Tensor* t = static_cast<const Tensor*>(q.tensor);
    const int L = (int)q.L;
    int mode_k = ctx->opt_score_mode, ppw_k = ctx->opt_poses_per_wave, w_k = ctx->opt_short_waves;
    tuned_shape(ctx, t, L, false, q.P, &mode_k, &ppw_k, &w_k);
    Shape& x = shp[r];
    x.u3 = use_u3(ctx, t, L, false, ppw_k) ? 1 : 0;
    x.ppw = pick_ppw(L, false, x.u3 != 0, ppw_k);
    x.W = w_k > 0 ? std::min(w_k, 4) : 4;
    while (x.W > 1 && short_lds(L, x.W, false) > kLdsDefault) x.W >>= 1;
    x.lds_s = short_lds(L, x.W, false);
    x.lds_l = long_lds(L, x.ppw, false, x.u3 != 0);
    RSD_CHECK(x.lds_s <= kLdsDefault && x.lds_l <= kLdsMax, RSD_E_UNSUPPORTED,
              "request %d: ligand of %d atoms needs too much LDS", r, L);
    x.occ_s = lds_occupancy(x.lds_s, x.W);
    x.occ_l = lds_occupancy(x.lds_l, 4);
  }
  // persistent mode: one launch whose LDS is the largest any request's long-range items or
  // four-pose short-range blocks need (automatic: the grouped launches)
  bool fused = ctx->opt_batch_mode == 2;
  size_t lds_fused = 0;
  if (fused) {
    for (int r = 0; r < nreq; ++r) {
      lds_fused = std::max(lds_fused, std::max(shp[r].lds_l, short_lds((int)req_in[r].L, 4, false)));
    }
    if (lds_fused > kLdsMax) fused = false;
  }
  // table order: long-range occupancy, then the short-range shape (stable), so that every
  // launch covers a contiguous range and the heavier long-range kernel gets the fewest launches
  // (persistent mode: request order)
  std::vector<int> order((size_t)nreq);
  for (int r = 0; r < nreq; ++r) order[r] = r;
  if (!fused) std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const Shape &a = shp[x], &c = shp[y];
    if (a.occ_l != c.occ_l) return a.occ_l > c.occ_l;
    if (a.W != c.W) return a.W > c.W;
    return a.occ_s > c.occ_s;
  });
  Batch* b = new (std::nothrow) Batch();
  RSD_CHECK(b != nullptr, RSD_E_OOM, "host allocation failed");
  b->ctx = ctx;
  b->nreq = nreq;
  std::vector<int64_t> off_lig(nreq), off_es(nreq), off_part(nreq);
  std::vector<int64_t> off_perm(nreq, -1);
  int64_t nlig = 0, nes = 0, npart = 0, nperm = 0, maxsort = 0;
  for (int k = 0; k < nreq; ++k) {
    const rsd_request& q = req_in[order[k]];
    const Tensor* t = static_cast<const Tensor*>(q.tensor);
    off_lig[k] = nlig;
    nlig += q.L;
    off_es[k] = nes;
    nes += q.P;
    off_part[k] = npart;
    npart += (int64_t)t->nchunk * q.P;
    if (sort_poses(ctx, t, q.P)) {
      off_perm[k] = nperm;
      nperm += q.P;
      maxsort = std::max<int64_t>(maxsort, q.P);
    }
  }
  const size_t sz_desc = sizeof(BatchDesc) * (size_t)nreq;
  const size_t o_lig = (sz_desc + 255) / 256 * 256;
  const size_t o_r = o_lig + sizeof(double4) * (size_t)nlig;
  const size_t o_es = o_r + sizeof(double) * (size_t)nreq;
  const size_t o_part = o_es + sizeof(double) * (size_t)nes;
  // spatial order: the requests' permutations, then one histogram and cell array for all
  const size_t o_perm = o_part + sizeof(double) * (size_t)npart;
  const size_t o_hist = o_perm + sizeof(int) * (size_t)nperm;
  const size_t o_cell = o_hist + sizeof(int) * (size_t)(nperm ? kSortCells : 0);
  const size_t o_next = (o_cell + sizeof(int) * (size_t)maxsort + 255) / 256 * 256;
  b->bytes = o_next + 8 * sizeof(int);
  rsd_status st = ctx->block_alloc(&b->mem, &b->bytes);
  if (st != RSD_OK) {
    delete b;
    return st;
  }
  char* m = (char*)b->mem;
  std::vector<BatchDesc> h((size_t)nreq);
  int64_t pb = 0;
  for (int k = 0; k < nreq; ++k) {
    const rsd_request& q = req_in[order[k]];
    const Tensor* t = static_cast<const Tensor*>(q.tensor);
    ScoreIO io{};
    io.lig_charges = q.lig_charges;
    io.lig_positions = q.lig_positions;
    io.L = (int)q.L;
    io.quats = q.quats;
    io.trans = q.trans;
    io.P = q.P;
    io.vdw_min = q.vdw_min;
    io.E = q.energies;
    io.El = q.energies_long;
    io.flags = q.flags;
    io.counts = q.counts;
    io.grads = nullptr;
    double4* lig = (double4*)(m + o_lig) + off_lig[k];
    double* rlig = (double*)(m + o_r) + k;
    double* es = (double*)(m + o_es) + off_es[k];
    double* part = (double*)(m + o_part) + off_part[k];
    h[k].sp = make_score_params(t, io, lig, rlig, es, nullptr);
    h[k].lp = make_long_params(t, io, lig, shp[order[k]].ppw, part, shp[order[k]].u3 != 0, chunks_per_item(ctx));
    if (off_perm[k] >= 0) {
      int* perm = (int*)(m + o_perm) + off_perm[k];
      h[k].lp.perm = perm;
      b->sorts.push_back({t, q.trans, q.P, perm});
    }
    h[k].lig_pos = q.lig_positions;
    h[k].lig_z = q.lig_charges;
    h[k].pose_base = pb;
    pb += q.P;
  }
  rsd_status lst = RSD_OK;
  size_t lds_long_max = 0;
  if (fused) {
    // prefix counts over the whole table: long-range slots per XCD and four-pose short blocks
    for (int k = 0; k < nreq; ++k) {
      h[k].xcd_base = b->u_long;
      b->u_long += h[k].lp.per_xcd;
      h[k].short_base = b->u_short;
      b->u_short += (h[k].sp.P + 3) / 4;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 8)
      cus = 256;
    b->fused = true;
    b->lds = lds_fused;
    b->groups = 8 * (cus / 8) * lds_occupancy(lds_fused, 4);
    b->next = (int*)(m + o_next);
    if (b->u_long + (b->u_short + 7) / 8 > 0x7fffffffLL) {
      set_error("batch too large for one launch");
      lst = RSD_E_UNSUPPORTED;
    }
    if (lst == RSD_OK) lst = allow_lds((const void*)k_batch_fused, lds_fused);
  }
  // launches: maximal runs of the table with one short-range shape, and with one long-range
  // occupancy; each launch's LDS is the largest its requests need
  for (int k = 0; k < nreq && lst == RSD_OK && !fused;) {
    const Shape& s0 = shp[order[k]];
    Batch::Launch la{k, 0, s0.W, 0, 0};
    int e = k;
    for (; e < nreq && shp[order[e]].W == s0.W && shp[order[e]].occ_s == s0.occ_s; ++e) {
      h[e].short_base = la.units;
      la.units += (h[e].sp.P + la.W - 1) / la.W;
      la.lds = std::max(la.lds, shp[order[e]].lds_s);
    }
    la.count = e - k;
    if (la.units > 0x7fffffffLL) {
      set_error("batch too large for one launch");
      lst = RSD_E_UNSUPPORTED;
    }
    if (la.units > 0) b->shorts.push_back(la);
    k = e;
  }
  for (int k = 0; k < nreq && lst == RSD_OK && !fused;) {
    const int occ = shp[order[k]].occ_l;
    Batch::Launch la{k, 0, 4, 0, 0};
    int e = k;
    for (; e < nreq && shp[order[e]].occ_l == occ; ++e) {
      h[e].xcd_base = la.units;
      la.units += h[e].lp.per_xcd;
      la.lds = std::max(la.lds, shp[order[e]].lds_l);
    }
    la.count = e - k;
    if (la.units * 8 > 0x7fffffffLL) {
      set_error("batch too large for one launch");
      lst = RSD_E_UNSUPPORTED;
    }
    lds_long_max = std::max(lds_long_max, la.lds);
    if (la.units > 0) b->longs.push_back(la);
    k = e;
  }
  if (lst == RSD_OK && !fused) lst = allow_lds((const void*)k_batch_long, lds_long_max);
  if (lst != RSD_OK) {
    ctx->block_release(b->mem, b->bytes);
    delete b;
    return lst;
  }
  b->poses = pb;
  b->d = (BatchDesc*)m;
  if (nperm) {
    b->sort_hist = (int*)(m + o_hist);
    b->sort_cell = (int*)(m + o_cell);
  }
  b->host_table = std::move(h);
  hipError_t e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d, b->host_table.data(), sz_desc, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipEventRecord(b->uploaded, ctx->stream);
  if (e != hipSuccess) {
    if (b->uploaded) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipEventDestroy(b->uploaded);
    }
    ctx->block_release(b->mem, b->bytes);
    delete b;
    set_error("batch upload: %s", hipGetErrorString(e));
    return RSD_E_HIP;
  }
  *out = b;
  return RSD_OK;
}

rsd_status batch_run(Batch* b) {
  Context* ctx = b->ctx;
  hipStream_t s = ctx->stream;
  if (b->poses == 0) return RSD_OK;
  if (b->fused) {
    RSD_TIMED_LAUNCH(ctx, "ligand_prep", (k_batch_prep_fused<<<b->nreq, 64, 0, s>>>(b->d, b->next)));
  } else {
    RSD_TIMED_LAUNCH(ctx, "ligand_prep", (k_batch_prep<<<b->nreq, 64, 0, s>>>(b->d)));
  }
  for (const auto& so : b->sorts)
    RSD_TRY(launch_pose_sort(ctx, s, so.t, so.trans, so.P, b->sort_hist, b->sort_cell, so.perm));
  if (b->fused) {
    RSD_TIMED_LAUNCH(ctx, "fused", (k_batch_fused<<<(unsigned)b->groups, 256, b->lds, s>>>(
                                       b->d, b->nreq, b->u_long, b->u_short, b->next)));
  }
  for (const auto& la : b->shorts)
    RSD_TIMED_LAUNCH(ctx, "short", (k_batch_short<<<(unsigned)la.units, 64 * la.W, la.lds, s>>>(
                                       b->d, la.first, la.count)));
  for (const auto& la : b->longs)
    RSD_TIMED_LAUNCH(ctx, "long", (k_batch_long<<<(unsigned)(la.units * 8), 256, la.lds, s>>>(
                                      b->d, la.first, la.count)));
  const unsigned gc = (unsigned)std::min<int64_t>((b->poses + 255) / 256, 65536);
  RSD_TIMED_LAUNCH(ctx, "combine", (k_batch_combine<<<gc, 256, 0, s>>>(b->d, b->nreq, b->poses)));
  return RSD_OK;
}

// The scratch goes back to the context's block cache without waiting for the batch's queued
// launches: only later work on the same stream can receive it.
void batch_free(Batch* b) {
  if (!b) return;
  if (b->uploaded) {
    (void)hipEventSynchronize(b->uploaded);
    (void)hipEventDestroy(b->uploaded);
  }
  b->ctx->block_release(b->mem, b->bytes);
  delete b;
}

// ---------------------------------------------------------------- posing search (Algorithm PPIEM)
// Step A3, radial approach.  The ligand, rotated by q about its centre, has its centre at
// x_P + rho u.  For the pair (ligand atom l, protein atom m) with a = x_P + R(q) u_l and
// w = a - x_m, |rho u + w| = sigma at rho = -(u.w) +- sqrt((u.w)^2 - (|w|^2 - sigma^2)), and
// the pair is closer than sigma between the roots; the first contact when moving in from far
// away is rho* = the largest root over all pairs (-inf if no pair has a real root).
// One workgroup takes one orbit direction u and cpb orientations; tpc threads share each
// orientation's ligand atoms.  A pair has a real root only when the protein atom lies within
// sigma of the ligand atom's line y + rho u, i.e. when their projections onto the plane
// normal to u are within sigma.  Each tile of protein atoms is filtered against the cylinder
// of radius sigma + (ligand radius) about x_P + rho u (no ligand atom's line leaves it), and
// the survivors are sorted in LDS by a 2-D bin of their projection.  A thread then visits
// only the bins within sigma of its line's projection, row by row as contiguous ranges.
// Every pair with a real root is examined with the same arithmetic as without the bins, and
// the maximum does not depend on the order, so the radii are the same.  A root is taken
// (with its square root) only when it can beat the thread's best:
// -b + sqrt(disc) > best  <=>  disc >= 0 and (best + b < 0 or disc > (best + b)^2).
struct ContactParams {
  const double4* __restrict__ atoms;   // protein atoms (x, y, z, charge)
  int64_t N;
  const double4* __restrict__ lig;     // centred ligand (k_ligand_prep)
  const double* __restrict__ rlig;     // its radius
  int L;
  const double* __restrict__ dirs;
  const double* __restrict__ quats;
  int64_t U, Q;
  double xP[3];
  double sigma, gap;
  int tpc, cpb;
  int64_t qblocks;
  double* __restrict__ rho;
  double* __restrict__ pose_q;
  double* __restrict__ pose_t;
};

constexpr int kContactTile = 1024;   // protein atoms filtered per pass
constexpr int kContactBins = 32;     // at most this many bins per axis of the projection plane

__global__ __launch_bounds__(256) void k_contact(const ContactParams a) {
  __shared__ double4 s_at[kContactTile];                        // the tile's survivors, by bin
  __shared__ int s_key[kContactTile];                           // bin of each tile atom, -1 if filtered
  __shared__ int s_start[kContactBins * kContactBins + 1];      // first survivor of each bin
  __shared__ int s_fill[kContactBins * kContactBins];
  __shared__ double s_best[256];
  const int tid = threadIdx.x;
  const int64_t ui = (int64_t)blockIdx.x / a.qblocks;
  const int64_t qb = (int64_t)blockIdx.x % a.qblocks;
  const double ux = a.dirs[3 * ui], uy = a.dirs[3 * ui + 1], uz = a.dirs[3 * ui + 2];
  // an orthonormal basis (e1, e2) of the plane normal to u
  double e1x, e1y, e1z;
  {
    const double ax = fabs(ux), ay = fabs(uy), az = fabs(uz);
    // u x (the coordinate axis least aligned with u)
    if (ax <= ay && ax <= az) { e1x = 0.0; e1y = uz; e1z = -uy; }
    else if (ay <= az)        { e1x = -uz; e1y = 0.0; e1z = ux; }
    else                      { e1x = uy; e1y = -ux; e1z = 0.0; }
    const double inv = 1.0 / sqrt(fma(e1x, e1x, fma(e1y, e1y, e1z * e1z)));
    e1x *= inv; e1y *= inv; e1z *= inv;
  }
  const double e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
  const int j = tid / a.tpc, lt = tid - (tid / a.tpc) * a.tpc;
  const int64_t q = qb * a.cpb + j;
  const bool active = j < a.cpb && q < a.Q;
  double R[9], t[3];
  bool valid = false;
  if (active) valid = pose_frame(a.quats + 4 * q, a.xP, R, t);
  const double rc = a.sigma + a.rlig[0] + 1e-3;   // the cylinder radius, with a margin for rounding
  const double rc2 = rc * rc;
  const double s2 = a.sigma * a.sigma;
  // bins: the square [-rc, rc]^2 of the plane in nb x nb cells of edge eb (at least sigma / 2)
  const double eb = fmax(0.5 * a.sigma, 2.0 * rc / kContactBins);
  const int nb = min(kContactBins, max(1, (int)ceil(2.0 * rc / eb)));
  const double inv_eb = 1.0 / eb;
  const double rs = a.sigma * (1.0 + 1e-9) + 1e-6;   // query radius about a line, with a margin
  auto bin_of = [&](double c) { return min(nb - 1, max(0, (int)floor((c + rc) * inv_eb))); };
  double best = -INFINITY;
  const int nl = (a.L + a.tpc - 1) / a.tpc;
  for (int il = 0; il < nl; ++il) {
    const int l = lt + il * a.tpc;
    const bool has = active && valid && l < a.L;
    double3 y = make_double3(0.0, 0.0, 0.0);
    int bx0 = 0, bx1 = -1, by0 = 0, by1 = -1;
    if (has) {
      y = place(R, t, a.lig[l]);
      const double dx = y.x - a.xP[0], dy = y.y - a.xP[1], dz = y.z - a.xP[2];
      const double c1 = fma(e1x, dx, fma(e1y, dy, e1z * dz)), c2 = fma(e2x, dx, fma(e2y, dy, e2z * dz));
      bx0 = bin_of(c1 - rs); bx1 = bin_of(c1 + rs);
      by0 = bin_of(c2 - rs); by1 = bin_of(c2 + rs);
    }
    for (int64_t m0 = 0; m0 < a.N; m0 += kContactTile) {
      // bin of every atom of the tile within the cylinder
      for (int k = tid; k < nb * nb; k += 256) s_fill[k] = 0;
      __syncthreads();
      for (int k = tid; k < kContactTile; k += 256) {
        const int64_t m = m0 + k;
        int key = -1;
        if (m < a.N) {
          const double4 p = a.atoms[m];
          const double dx = p.x - a.xP[0], dy = p.y - a.xP[1], dz = p.z - a.xP[2];
          const double pr = fma(ux, dx, fma(uy, dy, uz * dz));
          const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
          if (d2 - pr * pr <= rc2) {
            const double c1 = fma(e1x, dx, fma(e1y, dy, e1z * dz)), c2 = fma(e2x, dx, fma(e2y, dy, e2z * dz));
            key = bin_of(c2) * nb + bin_of(c1);
            atomicAdd(&s_fill[key], 1);
          }
        }
        s_key[k] = key;
      }
      __syncthreads();
      if (tid < 64) {   // exclusive scan of the bin counts (one wavefront)
        int carry = 0;
        for (int b0 = 0; b0 < nb * nb; b0 += 64) {
          const int b = b0 + tid;
          const int v = b < nb * nb ? s_fill[b] : 0;
          int incl = v;
#pragma unroll
          for (int off = 1; off < 64; off <<= 1) {
            const int w = __shfl_up(incl, off, 64);
            if (tid >= off) incl += w;
          }
          if (b < nb * nb) {
            s_start[b] = carry + incl - v;
            s_fill[b] = carry + incl - v;
          }
          carry += __shfl(incl, 63, 64);
        }
        if (tid == 0) s_start[nb * nb] = carry;
      }
      __syncthreads();
      for (int k = tid; k < kContactTile; k += 256) {
        const int key = s_key[k];
        if (key >= 0) s_at[atomicAdd(&s_fill[key], 1)] = a.atoms[m0 + k];
      }
      __syncthreads();
      if (has) {
        for (int by = by0; by <= by1; ++by) {
          const int k1 = s_start[by * nb + bx1 + 1];
          for (int k = s_start[by * nb + bx0]; k < k1; ++k) {
            const double4 p = s_at[k];
            const double wx = y.x - p.x, wy = y.y - p.y, wz = y.z - p.z;
            const double bu = fma(ux, wx, fma(uy, wy, uz * wz));
            const double ww = fma(wx, wx, fma(wy, wy, wz * wz));
            const double disc = fma(bu, bu, s2 - ww);
            const double g = best + bu;
            if (disc >= 0.0 && (g < 0.0 || disc > g * g)) best = fmax(best, sqrt(disc) - bu);
          }
        }
      }
      __syncthreads();
    }
  }
  s_best[tid] = best;
  __syncthreads();
  if (active && lt == 0) {
    double r = -INFINITY;
    for (int k = 0; k < a.tpc; ++k) r = fmax(r, s_best[j * a.tpc + k]);
    const int64_t o = ui * a.Q + q;
    if (!valid) r = NAN;
    a.rho[o] = r;
    const bool placed = valid && r > -INFINITY;
    const double rr = r + a.gap;
    a.pose_t[3 * o + 0] = placed ? fma(rr, ux, a.xP[0]) : NAN;
    a.pose_t[3 * o + 1] = placed ? fma(rr, uy, a.xP[1]) : NAN;
    a.pose_t[3 * o + 2] = placed ? fma(rr, uz, a.xP[2]) : NAN;
    for (int c = 0; c < 4; ++c) a.pose_q[4 * o + c] = a.quats[4 * q + c];
  }
}

// Step A6, first half: for each orbit position the lowest energy over its accepted poses
// (lowest orientation index on ties); -1 / +inf when none is accepted.  One wavefront each.
__global__ __launch_bounds__(256) void k_orbit_best(const double* __restrict__ E, const uint8_t* __restrict__ flags,
                                                    int64_t U, int64_t Q, int32_t* __restrict__ best_q,
                                                    double* __restrict__ best_e) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= U) return;
  double be = INFINITY;
  int64_t bq = -1;
  for (int64_t q = lane; q < Q; q += 64) {
    const int64_t o = u * Q + q;
    const double e = E[o];
    if ((flags[o] & 1) && e < be) {   // lanes visit increasing q: strict < keeps the lowest index
      be = e;
      bq = q;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double oe = __shfl_xor(be, off, 64);
    const int64_t oq = __shfl_xor(bq, off, 64);
    if (oq >= 0 && (bq < 0 || oe < be || (oe == be && oq < bq))) {
      be = oe;
      bq = oq;
    }
  }
  if (lane == 0) {
    best_q[u] = (int32_t)bq;
    best_e[u] = be;
  }
}

// Step A6, second half: an orbit position with an accepted pose is a minimum when its value is
// not larger than any neighbour's (CSR neighbour lists over the orbit positions).
__global__ void k_orbit_local(const int32_t* __restrict__ best_q, const double* __restrict__ best_e, int64_t U,
                              const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
                              uint8_t* __restrict__ is_min) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < U; u += (int64_t)gridDim.x * blockDim.x) {
    bool m = best_q[u] >= 0;
    for (int32_t k = off[u]; m && k < off[u + 1]; ++k) m = best_e[u] <= best_e[idx[k]];
    is_min[u] = m ? 1 : 0;
  }
}

rsd_status launch_contact(Context* ctx, const Tensor* t, const double* lig_positions, int L, const double* dirs,
                          int64_t U, const double* quats, int64_t Q, const double xP[3], double sigma, double gap,
                          double* rho, double* pose_q, double* pose_t) {
  hipStream_t s = ctx->stream;
  void* ws = nullptr;
  const size_t bytes = sizeof(double4) * (size_t)L + 256 + sizeof(double) * (size_t)L;
  RSD_TRY(ctx->workspace(bytes, &ws));
  double4* lig = (double4*)ws;
  double* rl = (double*)((char*)ws + sizeof(double4) * (size_t)L);
  double* zero = rl + 32;   // charges are not needed here
  RSD_HIP(hipMemsetAsync(zero, 0, sizeof(double) * (size_t)L, s));
  RSD_TIMED_LAUNCH(ctx, "ligand_prep", (k_ligand_prep<<<1, 64, 0, s>>>(lig_positions, zero, L, lig, rl)));
  ContactParams a{};
  a.atoms = t->atoms;
  a.N = t->N;
  a.lig = lig;
  a.rlig = rl;
  a.L = L;
  a.dirs = dirs;
  a.quats = quats;
  a.U = U;
  a.Q = Q;
  for (int d = 0; d < 3; ++d) a.xP[d] = xP[d];
  a.sigma = sigma;
  a.gap = gap;
  a.tpc = L <= 256 ? L : 256;
  a.cpb = 256 / a.tpc;
  a.qblocks = (Q + a.cpb - 1) / a.cpb;
  a.rho = rho;
  a.pose_q = pose_q;
  a.pose_t = pose_t;
  const int64_t blocks = U * a.qblocks;
  RSD_CHECK(blocks <= 0x7fffffffLL, RSD_E_UNSUPPORTED, "too many orbit positions x orientations");
  RSD_TIMED_LAUNCH(ctx, "contact", (k_contact<<<(unsigned)blocks, 256, 0, s>>>(a)));
  return RSD_OK;
}

rsd_status launch_orbit_minima(Context* ctx, const double* E, const uint8_t* flags, int64_t U, int64_t Q,
                               const int32_t* off, const int32_t* idx, int32_t* best_q, double* best_e,
                               uint8_t* is_min) {
  hipStream_t s = ctx->stream;
  const int64_t b1 = (U + 3) / 4;
  RSD_CHECK(b1 <= 0x7fffffffLL, RSD_E_UNSUPPORTED, "too many orbit positions");
  RSD_TIMED_LAUNCH(ctx, "minima", (k_orbit_best<<<(unsigned)b1, 256, 0, s>>>(E, flags, U, Q, best_q, best_e)));
  const unsigned b2 = (unsigned)std::min<int64_t>((U + 255) / 256, 65536);
  RSD_TIMED_LAUNCH(ctx, "minima", (k_orbit_local<<<b2, 256, 0, s>>>(best_q, best_e, U, off, idx, is_min)));
  return RSD_OK;
}

// ---------------------------------------------------------------- a molecule's own energy (Prop. 3.2)
// E_long = 1/2 sum_j z_j (P_l(x_j) - z_j W0), W0 = sum_{k < K_long} w_k (the long-range reference
// kernel at distance zero: the atom's own long-range term), with P_l the trilinear value of the
// tensor at x_j; E_short = 1/2 sum_j z_j sum_{m != j, d^2 < r_c^2} z_m sum_{k >= K_long} w_k
// exp(-t_k^2 d^2).  Per-atom terms go to e_long[j], e_short[j] and are summed by one workgroup
// in a fixed order, so the result does not depend on scheduling.
struct SelfParams {
  const double* __restrict__ F;
  int64_t mode_stride, chunk_stride;
  int nchunk;
  double X0[3];
  int nm2[3];
  double inv_h, W0;
  const double4* __restrict__ atoms;
  int64_t N;
  const double* __restrict__ tab;     // short-range t_k^2 [kMaxTerms], then w_k [kMaxTerms]
  int S;
  double rc2;
  double* __restrict__ e_long;
  double* __restrict__ e_short;
};

// one wavefront per atom: lane l owns column l of every rank chunk
__global__ __launch_bounds__(256) void k_self_long(const SelfParams a) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= a.N) return;
  const double4 x = a.atoms[j];
  const double xs[3] = {x.x, x.y, x.z};
  int i[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    const double sd = (xs[d] - a.X0[d]) * a.inv_h;
    int id = (int)floor(sd);
    id = id < 0 ? 0 : (id > a.nm2[d] ? a.nm2[d] : id);
    i[d] = id;
    f[d] = sd - (double)id;
  }
  double v = 0.0;
  for (int c = 0; c < a.nchunk; ++c) {
    const double* base = a.F + (int64_t)c * a.chunk_stride + lane;
    double prod = 1.0;
    for (int d = 0; d < 3; ++d) {
      const double* row = base + d * a.mode_stride + (int64_t)i[d] * kChunk;
      const double lo = row[0], hi = row[kChunk];
      prod *= fma(f[d], hi - lo, lo);
    }
    v += prod;
  }
  v = wave_sum(v);
  if (lane == 0) a.e_long[j] = x.w * (v - x.w * a.W0);
}

// one thread per atom, protein atoms staged through LDS in tiles of 256
__global__ __launch_bounds__(256) void k_self_short(const SelfParams a) {
  __shared__ double4 s_at[256];
  __shared__ double s_tab[2 * kMaxTerms];
  const int tid = threadIdx.x;
  for (int k = tid; k < 2 * kMaxTerms; k += 256) s_tab[k] = a.tab[k];
  const int64_t j = (int64_t)blockIdx.x * 256 + tid;
  const double4 x = j < a.N ? a.atoms[j] : make_double4(0.0, 0.0, 0.0, 0.0);
  double acc = 0.0;
  for (int64_t m0 = 0; m0 < a.N; m0 += 256) {
    __syncthreads();
    if (m0 + tid < a.N) s_at[tid] = a.atoms[m0 + tid];
    __syncthreads();
    const int cnt = (int)(a.N - m0 < 256 ? a.N - m0 : 256);
    if (j < a.N) {
      for (int k = 0; k < cnt; ++k) {
        if (m0 + k == j) continue;
        const double4 p = s_at[k];
        const double dx = x.x - p.x, dy = x.y - p.y, dz = x.z - p.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < a.rc2) {
          double g = 0.0;
          for (int q = 0; q < a.S; ++q) g = fma(s_tab[kMaxTerms + q], exp(-(s_tab[q] * d2)), g);
          acc = fma(p.w, g, acc);
        }
      }
    }
  }
  if (j < a.N) a.e_short[j] = x.w * acc;
}

// out[0] = 1/2 sum e_long, out[1] = 1/2 sum e_short: strided partial sums, then a fixed tree
__global__ __launch_bounds__(1024) void k_self_sum(const double* __restrict__ e_long,
                                                   const double* __restrict__ e_short, int64_t N,
                                                   double* __restrict__ out) {
  __shared__ double s[2][1024];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t j = tid; j < N; j += 1024) {
    a += e_long[j];
    b += e_short[j];
  }
  s[0][tid] = a;
  s[1][tid] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
      s[0][tid] += s[0][tid + w];
      s[1][tid] += s[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = 0.5 * s[0][0];
    out[1] = 0.5 * s[1][0];
  }
}

rsd_status launch_self_energy(Context* ctx, const Tensor* t, double* E_long, double* E_short) {
  hipStream_t s = ctx->stream;
  const int64_t N = t->N;
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(sizeof(double) * (size_t)(2 * N + 2), &ws));
  double* e = (double*)ws;
  SelfParams a{};
  a.F = t->F;
  a.chunk_stride = (int64_t)t->n * kChunk;
  a.mode_stride = (int64_t)t->nchunk * a.chunk_stride;
  a.nchunk = t->nchunk;
  for (int d = 0; d < 3; ++d) {
    a.X0[d] = t->X0m[d];
    a.nm2[d] = t->nm[d] - 2;
  }
  a.inv_h = t->inv_h;
  double tk[kMaxTerms], wk[kMaxTerms];
  sinc_table(t->sp, tk, wk);
  double W0 = 0.0;
  for (int k = 0; k < t->sp.K_long; ++k) W0 += wk[k];
  a.W0 = W0;
  a.atoms = t->atoms;
  a.N = N;
  a.tab = t->short_tab;
  a.S = t->shrt.S;
  a.rc2 = t->sp.r_cut * t->sp.r_cut;
  a.e_long = e;
  a.e_short = e + N;
  RSD_CHECK((N + 3) / 4 <= 0x7fffffffLL, RSD_E_UNSUPPORTED, "too many atoms");
  if (t->nchunk > 0) {
    RSD_TIMED_LAUNCH(ctx, "self", (k_self_long<<<(unsigned)((N + 3) / 4), 256, 0, s>>>(a)));
  } else {
    RSD_HIP(hipMemsetAsync(a.e_long, 0, sizeof(double) * (size_t)N, s));
  }
  RSD_TIMED_LAUNCH(ctx, "self", (k_self_short<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(a)));
  RSD_TIMED_LAUNCH(ctx, "self", (k_self_sum<<<1, 1024, 0, s>>>(a.e_long, a.e_short, N, e + 2 * N)));
  double out[2];
  RSD_HIP(hipMemcpyAsync(out, e + 2 * N, sizeof(out), hipMemcpyDeviceToHost, s));
  RSD_HIP(hipStreamSynchronize(s));
  *E_long = out[0];
  *E_short = out[1];
  return RSD_OK;
}

}  // namespace rsd
