// Rank reduction of the long-range sum on the device (Algorithm TEP, steps 3-5).
//
// The collective long-range potential of eq. 2.6 is a canonical tensor of rank
// N*K_long whose mode-d factor columns are the 1-D Gaussians
// g_{k,m,d}[j] = exp(-t_k^2 (X_j - x_{m,d})^2).  Its rank is cut by the
// canonical -> Tucker -> canonical transform with the reduced HOSVD (RHOSVD):
//   1. per mode, the side matrix A_d (n x N*K_long) with unit-norm columns,
//      weights xi_{m,k} = z_m w_k prod_d ||g_{k,m,d}||;
//   2. the Gram matrix A_d A_d^T (n x n), by default from its Toeplitz-times-Hankel
//      structure on the uniform grid (optionally as a dense FP64 matrix-core product),
//      its dominant eigenvectors U_d (eigenvalues >= eps^2 * largest, i.e. singular
//      values >= eps * largest);
//   3. the projections B_d = U_d^T A_d and the Tucker core
//      beta = sum_c xi_c B_1[:,c] x B_2[:,c] x B_3[:,c], as one matrix product whose
//      left operand is the Khatri-Rao product of B_1 and B_2 formed in LDS;
//   4. a batched SVD of the core's mode-3 slices; kept terms (singular value >= eps
//      times the largest over all slices) become canonical terms, assembled as
//      F_d = U_d V_d directly into the column-chunked layout the scorer reads.
// Library calls: rocSOLVER for the symmetric eigenproblem and the small slice SVDs.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rsd {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int TM = 64;       // output tile rows
constexpr int TN = 64;       // output tile cols
constexpr int TK = 32;       // contraction depth per LDS stage
constexpr int TNW = 80;      // the wide product's single column tile
// LDS rows of a stage.  (k, m)-ordered stages use rows of 80 doubles (160 words, half the
// 64 banks): the four 16-lane groups of an MFMA operand read (16 consecutive m of rows
// k .. k+3) then fall in disjoint banks per 32-lane half.  (m, k)-ordered stages use rows of
// TK + 2 doubles (68 words): lane (m, k) of a read starts at bank 4m + 2k, again disjoint.
constexpr int LDT = 80;
constexpr int LDK = TK + 2;
constexpr int kStage = TNW * LDK;   // doubles per operand stage: max(TK * LDT, TNW * LDK)

// ----------------------------------------------------------------- operand loaders
// A loader moves one TK x W stage of its operand (element (k0 + kk, m0 + mm), zero outside
// [k0, k1) x [0, dim)) into LDS in two steps:
//   fetch: global loads (or generated values) into registers, with no condition, the row
//          index clamped into [.., k1 - 1] and the column to a valid one, so the loads of the
//          next stage stay in flight while the matrix cores work on this one;
//   store: the mask for rows and columns outside the operand, any arithmetic on the fetched
//          values, and the LDS write.
// at(s, k, m) reads element (k, m) of a stored stage.  256 threads; W = 64 or TNW.
// (k, m)-ordered stages: element e = j * 256 + t of the stage (j < TK * W / 256) is row e / W,
// column e % W, so the lanes of one load and one LDS write run along memory.
struct OpKM {                 // element (k, m) = p[k * ld + m]
  const double* __restrict__ p;
  int64_t ld;
  int dim;
  template <int W> static constexpr int regs() { return TK * W / 256; }
  __device__ void setup(int) {}
  template <int W>
  __device__ void fetch(double* r, int m0, int64_t kb, int64_t k1) const {
#pragma unroll
    for (int j = 0; j < regs<W>(); ++j) {
      const int e = j * 256 + (int)threadIdx.x, kk = e / W, m = m0 + e - kk * W;
      const int64_t k = min(kb + kk, k1 - 1);
      r[j] = p[k * ld + (m < dim ? m : 0)];
    }
  }
  template <int W>
  __device__ void store(double* s, const double* r, int m0, int64_t kb, int64_t k1) const {
#pragma unroll
    for (int j = 0; j < regs<W>(); ++j) {
      const int e = j * 256 + (int)threadIdx.x, kk = e / W, mm = e - kk * W;
      s[kk * LDT + mm] = (kb + kk < k1 && m0 + mm < dim) ? r[j] : 0.0;
    }
  }
  static __device__ double at(const double* s, int k, int m) { return s[k * LDT + m]; }
};

// (m, k)-ordered stages: thread t takes contraction index t % 32 of the columns
// t / 32 + 8 j, so the lanes of one load run along an m-row of the operand.
struct OpMK {                 // element (k, m) = p[m * ld + k]  (each m-row contiguous along k)
  const double* __restrict__ p;
  int64_t ld;
  int dim;
  template <int W> static constexpr int regs() { return W / 8; }
  __device__ void setup(int) {}
  template <int W>
  __device__ void fetch(double* r, int m0, int64_t kb, int64_t k1) const {
    const int kk = threadIdx.x & 31, mg = threadIdx.x >> 5;
    const int64_t k = min(kb + kk, k1 - 1);
#pragma unroll
    for (int j = 0; j < regs<W>(); ++j) {
      const int m = m0 + mg + 8 * j;
      r[j] = p[(int64_t)(m < dim ? m : 0) * ld + k];
    }
  }
  template <int W>
  __device__ void store(double* s, const double* r, int m0, int64_t kb, int64_t k1) const {
    const int kk = threadIdx.x & 31, mg = threadIdx.x >> 5;
#pragma unroll
    for (int j = 0; j < regs<W>(); ++j) {
      const int mm = mg + 8 * j;
      s[mm * LDK + kk] = (kb + kk < k1 && m0 + mm < dim) ? r[j] : 0.0;
    }
  }
  static __device__ double at(const double* s, int k, int m) { return s[m * LDK + k]; }
};

// The generated left operands fill 64-wide (k, m)-ordered stages only: thread t owns column
// t % 64 and rows t / 64 + 4 j.
struct OpKhatriRao {          // element (k, m = a*r2 + b) = P1[k*ld1 + a] * P2[k*ld2 + b]
  const double* __restrict__ P1;
  const double* __restrict__ P2;
  int64_t ld1, ld2;
  int r2;
  int dim;                    // r1 * r2
  int a_, b_;
  template <int W> static constexpr int regs() { return 16; }   // both factors of 8 entries
  __device__ void setup(int m0) {
    const int m = m0 + (threadIdx.x & 63);
    a_ = m < dim ? m / r2 : 0;
    b_ = m < dim ? m % r2 : 0;
  }
  template <int W>
  __device__ void fetch(double* r, int, int64_t kb, int64_t k1) const {
    static_assert(W == TM, "generated operands fill 64-wide stages");
    const int kq = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = min(kb + kq + 4 * j, k1 - 1);
      r[2 * j] = P1[k * ld1 + a_];
      r[2 * j + 1] = P2[k * ld2 + b_];
    }
  }
  template <int W>
  __device__ void store(double* s, const double* r, int m0, int64_t kb, int64_t k1) const {
    const int mm = threadIdx.x & 63, kq = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      s[(kq + 4 * j) * LDT + mm] = (kb + kq + 4 * j < k1 && m0 + mm < dim) ? r[2 * j] * r[2 * j + 1] : 0.0;
  }
  static __device__ double at(const double* s, int k, int m) { return s[k * LDT + m]; }
};

// One entry of a 1-D factor column at offset dx = X_i - x_m from the atom: the collocated
// Gaussian exp(-t^2 dx^2), or with gal != 0 its average over the cell [X_i - h/2, X_i + h/2]
// (eq. 2.1's piecewise-constant projection):
//   sqrt(pi) / (2 t h) (erf(t (dx + h/2)) - erf(t (dx - h/2))),
// with the difference taken of erfc values where both arguments share a sign.  For t h < 0.01
// the erf difference would cancel most of its digits; there the average is the series
// f + f2 (t h)^2 / 24 + f4 (t h)^4 / 1920 in a = t dx, with f = exp(-a^2) and f2, f4 its second
// and fourth derivatives; the next term is below 4e-16 relative.
__device__ __forceinline__ double gauss_entry(double t2, double dx, double h, int gal) {
  if (!gal) return exp(-(t2 * (dx * dx)));
  const double t = sqrt(t2);
  const double th = t * h;
  if (th < 0.01) {
    const double a = t * dx, a2 = a * a;
    const double e = exp(-a2);
    const double f2 = (4.0 * a2 - 2.0) * e;
    const double f4 = ((16.0 * a2 - 48.0) * a2 + 12.0) * e;
    const double s2 = th * th;
    return e + s2 * (f2 / 24.0 + s2 * (f4 / 1920.0));
  }
  const double u1 = t * (dx - 0.5 * h), u2 = t * (dx + 0.5 * h);
  double d;
  if (u1 >= 0.0) {
    d = erfc(u1) - erfc(u2);
  } else if (u2 <= 0.0) {
    d = erfc(-u2) - erfc(-u1);
  } else {
    d = erf(u2) - erf(u1);
  }
  return 0.886226925452758 / th * d;   // sqrt(pi) / 2 = 0.886226925452758...
}

// GAL selects the cell-average entries at compile time: their erf code would otherwise set the
// register budget of the projection for the collocated entries too.  REC (collocated only) makes
// the entries of a thread's rows by a recurrence; the caller picks it when every column's ratio
// r below stays within [e^-5, e^5] over the whole box.
template <bool GAL, bool REC = false>
struct OpGauss {              // element (k = grid row i, m = column c) = g_c(X_i - x_c) / nu_c (gauss_entry)
  const double* __restrict__ pos;    // N x 3
  const double* __restrict__ t2;     // K_long
  const double* __restrict__ inv_nu; // columns
  int K, d, n;
  double b, h;
  int dim;                           // number of columns
  double x_, t2_, s_, q_;
  template <int W> static constexpr int regs() { return 8; }
  __device__ void setup(int m0) {
    const int col = m0 + (threadIdx.x & 63);
    if (col < dim) {
      x_ = pos[3 * (col / K) + d];
      t2_ = t2[col % K];
      s_ = inv_nu[col];
    } else {
      x_ = 0.0; t2_ = 0.0; s_ = 0.0;
    }
    q_ = exp(-(32.0 * t2_ * (h * h)));
  }
  template <int W>
  __device__ void fetch(double* r, int, int64_t kb, int64_t) const {
    static_assert(W == TM, "generated operands fill 64-wide stages");
    const int kq = threadIdx.x >> 6;
    const double dx = (-b + (double)(kb + kq + 1) * h) - x_;
    // collocated entries of the thread's rows (four apart) by the recurrence
    // g(d + 4h) = g(d) r(d), r(d) = exp(-t^2 (8 h d + 16 h^2)), r(d + 4h) = r(d) q, q = exp(-32 t^2 h^2),
    // anchored by two exponentials per stage
    if constexpr (!GAL && REC) {
      double g = exp(-(t2_ * (dx * dx))), rr = exp(-(t2_ * (8.0 * h * dx + 16.0 * (h * h))));
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        r[j] = g * s_;
        g *= rr;
        rr *= q_;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double X = -b + (double)(kb + kq + 4 * j + 1) * h;
        r[j] = gauss_entry(t2_, X - x_, h, GAL ? 1 : 0) * s_;
      }
    }
  }
  template <int W>
  __device__ void store(double* s, const double* r, int, int64_t kb, int64_t k1) const {
    const int mm = threadIdx.x & 63, kq = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 8; ++j) s[(kq + 4 * j) * LDT + mm] = (kb + kq + 4 * j < k1) ? r[j] : 0.0;
  }
  static __device__ double at(const double* s, int k, int m) { return s[k * LDT + m]; }
};

// ----------------------------------------------------------------- rank reduction of explicit factors
// Rows i0 .. i0 + rows - 1 of one mode of a chunked factor table (R columns) as columns
// col0 .. col0 + R - 1 of a row-major matrix with ldA columns:
// A[i * ldA + col0 + p] = F[chunk p / kChunk][row i0 + i][p % kChunk].
__global__ void k_take_rows(const double* __restrict__ F, int n_src, int64_t R, int i0, int rows,
                            double* __restrict__ A, int64_t ldA, int64_t col0) {
  const int64_t total = (int64_t)rows * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / R);
    const int64_t p = e % R;
    A[(int64_t)i * ldA + col0 + p] = F[((p / kChunk) * n_src + i0 + i) * kChunk + p % kChunk];
  }
}

// Column norms nu[p] = ||A[:, p]|| of a row-major rows x R matrix, one thread per column.
__global__ void k_row_colnorms(const double* __restrict__ A, int rows, int64_t R, double* __restrict__ nu) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < R; p += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < rows; ++i) {
      const double v = A[(int64_t)i * R + p];
      s = fma(v, v, s);
    }
    nu[p] = sqrt(s);
  }
}

// Term weights xi[p] = nu1 nu2 nu3; a term with a zero column in any mode is zero (xi = 0).
__global__ void k_local_weights(const double* __restrict__ nu0, const double* __restrict__ nu1,
                                const double* __restrict__ nu2, int64_t R, double* __restrict__ xi) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < R; p += (int64_t)gridDim.x * blockDim.x) {
    const bool live = nu0[p] > 0.0 && nu1[p] > 0.0 && nu2[p] > 0.0;
    xi[p] = live ? nu0[p] * nu1[p] * nu2[p] : 0.0;
  }
}

// Unit-norm columns: A[i][p] /= nu[p]; the columns of zero terms are set to zero in every mode.
__global__ void k_normalize_cols(double* __restrict__ A, int rows, int64_t R, const double* __restrict__ nu,
                                 const double* __restrict__ xi) {
  const int64_t total = (int64_t)rows * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e % R;
    A[e] = xi[p] != 0.0 ? A[e] / nu[p] : 0.0;
  }
}

// ----------------------------------------------------------------- FP64 MFMA GEMM
// C[split][m][n] (+)= sum_{k in split} A(k, m) * B(k, n) for one 64 x 64 tile per workgroup.
// Four wavefronts, each a 32 x 32 sub-tile of 2 x 2 v_mfma_f64_16x16x4 blocks.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator item v of lane l is
// D[4v + l/16][l%16].
struct GemmShape {
  int M, N;
  int64_t K, kper;            // contraction length and per-split chunk
  double* C;
  int64_t ldc;
  int64_t split_stride;       // elements between split slices of C
  int accumulate;             // add into C instead of overwriting
  int tri;                    // enumerate only tiles with m-block <= n-block
  int tiles_n;                // number of n tiles (for tri)
  int64_t chunk_rows;         // nonzero: C is in the factors' chunked layout, element (m, n) at
                              // C[((n / kChunk) * chunk_rows + m) * kChunk + n % kChunk]
};

template <class AOp, class BOp>
__global__ __launch_bounds__(256) void k_gemm(AOp A, BOp B, const GemmShape g) {
  __shared__ double sA[kStage];
  __shared__ double sB[kStage];
  int bm, bn;
  if (g.tri) {
    int idx = blockIdx.x, row = 0, len = g.tiles_n;
    while (idx >= len) { idx -= len; ++row; --len; }
    bm = row;
    bn = row + idx;
  } else {
    bm = blockIdx.x;   // the long dimension (side-matrix columns) in x, which allows 2^31 - 1 tiles
    bn = blockIdx.y;
  }
  const int m0 = bm * TM, n0 = bn * TN;
  const int64_t k0 = (int64_t)blockIdx.z * g.kper;
  const int64_t k1 = min(g.K, k0 + g.kper);
  A.setup(m0);
  B.setup(n0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  d4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
  double ra[AOp::template regs<TM>()], rb[BOp::template regs<TN>()];
  if (k0 < k1) {
    A.template fetch<TM>(ra, m0, k0, k1);
    B.template fetch<TN>(rb, n0, k0, k1);
  }
  for (int64_t kb = k0; kb < k1; kb += TK) {
    A.template store<TM>(sA, ra, m0, kb, k1);
    B.template store<TN>(sB, rb, n0, kb, k1);
    __syncthreads();
    // the next stage (after the last one: rows clamped to k1 - 1, never stored)
    A.template fetch<TM>(ra, m0, kb + TK, k1);
    B.template fetch<TN>(rb, n0, kb + TK, k1);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const double a0 = AOp::at(sA, kk + lk, wm + lr);
      const double a1 = AOp::at(sA, kk + lk, wm + 16 + lr);
      const double b0 = BOp::at(sB, kk + lk, wn + lr);
      const double b1 = BOp::at(sB, kk + lk, wn + 16 + lr);
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* C = g.C + (int64_t)blockIdx.z * g.split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * v + lk;
        const int n = n0 + wn + 16 * j + lr;
        if (m < g.M && n < g.N) {
          double* c = g.chunk_rows ? C + ((int64_t)(n / kChunk) * g.chunk_rows + m) * kChunk + n % kChunk
                                   : C + (int64_t)m * g.ldc + n;
          *c = g.accumulate ? *c + acc[i][j][v] : acc[i][j][v];
        }
      }
}

// The same product for N <= 80 in one 64 x 80 tile per workgroup.  Wavefront w takes rows
// 16w .. 16w+15 against all five 16-column blocks, so a narrow product (N = a Tucker rank)
// is not split over two 64-column tiles of which the second is mostly padding, and an A tile
// that is generated rather than loaded (the Gaussians) is made once instead of once per
// column tile.  Each output element sums the same products in the same order as k_gemm.
// Workgroups per compute unit the wide product is compiled for: three for the two large
// contractions of the build (projection, Tucker core), whose registers fit in a third of the
// file; two elsewhere, where the wider fetches would otherwise spill.
template <class AOp, class BOp>
struct WideOcc {
  static constexpr int value = 2;
};
template <>
struct WideOcc<OpGauss<false>, OpKM> {
  static constexpr int value = 3;
};
template <>
struct WideOcc<OpGauss<false, true>, OpKM> {
  static constexpr int value = 3;
};
template <>
struct WideOcc<OpKhatriRao, OpKM> {
  static constexpr int value = 3;
};

template <class AOp, class BOp>
__global__ __launch_bounds__(256, (WideOcc<AOp, BOp>::value)) void k_gemm_w(AOp A, BOp B, const GemmShape g) {
  __shared__ double sA[kStage];
  __shared__ double sB[kStage];
  const int m0 = blockIdx.x * TM;
  const int64_t k0 = (int64_t)blockIdx.z * g.kper;
  const int64_t k1 = min(g.K, k0 + g.kper);
  A.setup(m0);
  B.setup(0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  d4v acc[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) acc[j] = d4v{0.0, 0.0, 0.0, 0.0};
  double ra[AOp::template regs<TM>()], rb[BOp::template regs<TNW>()];
  if (k0 < k1) {
    A.template fetch<TM>(ra, m0, k0, k1);
    B.template fetch<TNW>(rb, 0, k0, k1);
  }
  for (int64_t kb = k0; kb < k1; kb += TK) {
    A.template store<TM>(sA, ra, m0, kb, k1);
    B.template store<TNW>(sB, rb, 0, kb, k1);
    __syncthreads();
    A.template fetch<TM>(ra, m0, kb + TK, k1);
    B.template fetch<TNW>(rb, 0, kb + TK, k1);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const double a = AOp::at(sA, kk + lk, 16 * w + lr);
#pragma unroll
      for (int j = 0; j < 5; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, BOp::at(sB, kk + lk, 16 * j + lr), acc[j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* C = g.C + (int64_t)blockIdx.z * g.split_stride;
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + 16 * w + 4 * v + lk;
      const int n = 16 * j + lr;
      if (m < g.M && n < g.N) {
        double* c = g.chunk_rows ? C + ((int64_t)(n / kChunk) * g.chunk_rows + m) * kChunk + n % kChunk
                                 : C + (int64_t)m * g.ldc + n;
        *c = g.accumulate ? *c + acc[j][v] : acc[j][v];
      }
    }
}

// Rows of a row-major matrix scaled in place: p[r * ld + c] *= scale[r] for c < cols.
__global__ void k_scale_rows(double* __restrict__ p, int64_t ld, int64_t rows, int cols,
                             const double* __restrict__ scale) {
  const int64_t total = rows * ld;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ld;
    if (e - r * ld < cols) p[e] = p[e] * scale[r];
  }
}

// Sum split slices: out[m*ldo + n] = sum_s part[s*stride + m*ldp + n].
__global__ void k_reduce_splits(const double* __restrict__ part, int splits, int64_t stride, int M, int N,
                                int64_t ldp, double* __restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / N, nn = e % N;
    double s = 0.0;
    for (int q = 0; q < splits; ++q) s += part[q * stride + m * ldp + nn];
    out[m * ldo + nn] = s;
  }
}

// ----------------------------------------------------------------- small kernels
// Column norms nu_c = ||g_c|| of columns c in [c0, c1) of mode d (one wavefront per column).
__global__ void k_col_norms(const double* __restrict__ pos, const double* __restrict__ t2, int K, int d, int n,
                            double b, double h, int64_t c0, int64_t c1, double* __restrict__ nu,
                            double* __restrict__ inv_nu, int gal) {
  const int lane = threadIdx.x & 63;
  const int64_t c = c0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (c >= c1) return;
  const double x = pos[3 * (c / K) + d];
  const double tt = t2[c % K];
  double s = 0.0;
  if (gal) {
    for (int i = lane; i < n; i += 64) {
      const double dx = (-b + (double)(i + 1) * h) - x;
      const double g = gauss_entry(tt, dx, h, gal);
      s = fma(g, g, s);
    }
  } else {
    // g_i^2 = exp(-2 t^2 dx_i^2) over runs of 8 rows per lane, by the recurrence
    // g_{i+1}^2 = g_i^2 r_i, r_i = exp(-2 t^2 (2 h dx_i + h^2)), r_{i+1} = r_i q, q = exp(-4 t^2 h^2),
    // anchored by two exponentials per run (the long-range Gaussians are wide on the grid,
    // t h << 1, so r stays near 1; a run where r could leave [e^-40, e^40] takes one exponential
    // per entry); the norms only scale the columns, which the weights undo
    const double q = exp(-4.0 * tt * (h * h));
    for (int i0 = 8 * lane; i0 < n; i0 += 8 * 64) {
      const double dx = (-b + (double)(i0 + 1) * h) - x;
      const double ar = -2.0 * tt * (2.0 * h * dx + h * h);
      const int m = min(8, n - i0);
      if (fabs(ar) * 8.0 < 40.0) {
        double e = exp(-2.0 * tt * (dx * dx));
        double r = exp(ar);
        for (int u = 0; u < m; ++u) {
          s += e;
          e *= r;
          r *= q;
        }
      } else {   // a narrow Gaussian: each entry on its own
        for (int u = 0; u < m; ++u) {
          const double du = dx + (double)u * h;
          s += exp(-2.0 * tt * (du * du));
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    const double r = sqrt(s);
    nu[c] = r;
    inv_nu[c] = r > 0.0 ? 1.0 / r : 0.0;
  }
}

// Normalised side-matrix chunk: A[(c - c0) * n + i] = g_c[i] / nu_c  (column-contiguous).
__global__ void k_gen_columns(const double* __restrict__ pos, const double* __restrict__ t2, int K, int d, int n,
                              double b, double h, int64_t c0, int64_t c1, const double* __restrict__ inv_nu,
                              double* __restrict__ A, int gal) {
  const int64_t total = (c1 - c0) * (int64_t)n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + e / n;
    const int i = (int)(e % n);
    const double x = pos[3 * (c / K) + d];
    const double dx = (-b + (double)(i + 1) * h) - x;
    A[e] = gauss_entry(t2[c % K], dx, h, gal) * inv_nu[c];
  }
}

// ----------------------------------------------------------------- Gram matrix on a uniform grid
// With nodes X_i = -b + (i+1) h, the product of two samples of one Gaussian column splits as
//   g(X_i) g(X_j) = exp(-t^2 (X_i - X_j)^2 / 2) * exp(-2 t^2 (x - (X_i + X_j)/2)^2),
// a factor that depends on i - j only (Toeplitz) times one that depends on i + j only (Hankel).
// Summed over the unit-norm columns c = (m, k) of a mode,
//   G[i][j] = sum_k T_k[|i - j|] * H_k[i + j],
//   T_k[e] = exp(-t_k^2 (e h)^2 / 2),  H_k[s] = sum_m exp(-2 t_k^2 (x_m - (-b + (s/2 + 1) h))^2) / nu_{m,k}^2,
// the same matrix as A_d A_d^T up to rounding, for O(K (2n-1) N + K n^2) work instead of O(n^2 N K).

// H_k[s] for s in [0, 2n-1), one thread per s, one k per grid row; atoms staged through LDS.
__global__ __launch_bounds__(256) void k_gram_hankel(const double* __restrict__ pos, const double* __restrict__ t2,
                                                     const double* __restrict__ inv_nu, int K, int d, int n, double b,
                                                     double h, int64_t N, double* __restrict__ H) {
  __shared__ double sx[256], sc[256];
  const int k = blockIdx.y;
  const int64_t ns = 2 * (int64_t)n - 1;
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double mid = -b + (0.5 * (double)s + 1.0) * h;
  const double a = 2.0 * t2[k];
  double acc = 0.0;
  for (int64_t m0 = 0; m0 < N; m0 += 256) {
    __syncthreads();
    const int64_t m = m0 + threadIdx.x;
    if (m < N) {
      const double v = inv_nu[m * K + k];
      sx[threadIdx.x] = pos[3 * m + d];
      sc[threadIdx.x] = v * v;
    }
    __syncthreads();
    const int cnt = (int)(N - m0 < 256 ? N - m0 : 256);
    for (int j = 0; j < cnt; ++j) {
      const double dx = sx[j] - mid;
      acc = fma(sc[j], exp(-(a * (dx * dx))), acc);
    }
  }
  if (s < ns) H[(int64_t)k * ns + s] = acc;
}

// T_k[e] for e in [0, n).
__global__ void k_gram_toeplitz(const double* __restrict__ t2, int K, int n, double h, double* __restrict__ T) {
  const int64_t total = (int64_t)K * n;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(x / n);
    const double e = (double)(x % n) * h;
    T[x] = exp(-(0.5 * t2[k] * (e * e)));
  }
}

// G[i][j] = sum_k T_k[|i-j|] H_k[i+j] for one 64 x 64 tile per workgroup.  A tile needs 127
// consecutive entries of each table per term (i - j and i + j each span 127 values), staged
// in LDS eight terms at a time.  Every entry is formed from (|i-j|, i+j) only, so G is exactly
// symmetric.
__global__ __launch_bounds__(256) void k_gram_assemble(const double* __restrict__ T, const double* __restrict__ H,
                                                       int K, int n, double* __restrict__ G) {
  constexpr int KG = 8;
  __shared__ double sT[KG][128], sH[KG][128];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int dbase = i0 - j0 - 63;    // i - j - dbase in [0, 126]
  const int sbase = i0 + j0;         // i + j - sbase in [0, 126]
  const int64_t ns = 2 * (int64_t)n - 1;
  const int jj = threadIdx.x & 63, ib = threadIdx.x >> 6;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < K; k0 += KG) {
    __syncthreads();
    for (int x = threadIdx.x; x < KG * 128; x += 256) {
      const int kk = x >> 7, e = x & 127, k = k0 + kk;
      const int dlt = abs(dbase + e);
      const int64_t sidx = (int64_t)sbase + e;
      sT[kk][e] = (k < K && dlt < n) ? T[(int64_t)k * n + dlt] : 0.0;
      sH[kk][e] = (k < K && sidx < ns) ? H[(int64_t)k * ns + sidx] : 0.0;
    }
    __syncthreads();
    const int kn = K - k0 < KG ? K - k0 : KG;
    for (int kk = 0; kk < kn; ++kk) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int ii = ib + 4 * q;
        acc[q] = fma(sT[kk][ii - jj + 63], sH[kk][ii + jj], acc[q]);
      }
    }
  }
  const int j = j0 + jj;
  if (j >= n) return;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = i0 + ib + 4 * q;
    if (i < n) G[(int64_t)i * n + j] = acc[q];
  }
}

// Top-r eigenvectors (eigenvalues ascending in Z, column-major n x n) -> U[i * ldu + a], descending.
__global__ void k_take_eigvecs(const double* __restrict__ Z, int n, int r, double* __restrict__ U, int ldu) {
  const int64_t total = (int64_t)n * ldu;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ldu), a = (int)(e % ldu);
    U[e] = a < r ? Z[(int64_t)(n - 1 - a) * n + i] : 0.0;
  }
}

// The upper triangle of the leading k x k block of a column-major matrix (ld lda) into a
// column-major k x k matrix, zeros below the diagonal.
__global__ void k_upper_copy(const double* __restrict__ X, int64_t lda, int k, double* __restrict__ Rb) {
  const int64_t total = (int64_t)k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % k), j = (int)(e / k);
    Rb[e] = a <= j ? X[(int64_t)j * lda + a] : 0.0;
  }
}

// Mirror the computed upper tiles of a row-major symmetric matrix onto its lower part.
__global__ void k_symmetrize(double* __restrict__ G, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (i > j) G[e] = G[(int64_t)j * n + i];
  }
}

// Deterministic test vectors in [-1, 1): splitmix64 of (seed, index).
__global__ void k_random_fill(double* __restrict__ X, int64_t count, uint64_t seed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    X[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// ----------------------------------------------------------------- small factorizations
// Orthonormal bases of the eigensolver's n x k panels without a long chain of library launches:
// the randomized Cholesky QR (a Householder QR of a small random sketch Theta Y gives R_s, and
// Y R_s^{-1} is well conditioned whatever the condition of Y), followed by Cholesky QR passes.
// Both factorizations run in one workgroup of 256 lanes with the matrix in registers: a group
// of eight lanes holds four adjacent columns, each lane a contiguous block of their rows.  A
// step puts what every lane needs (the QR's reflector, the Cholesky's next four rows) into LDS,
// double-buffered so that a step has one barrier; each lane reads only its own rows of it, and
// a column's sum over its rows takes three lane exchanges.  The step loops are unrolled so that
// the slot of the step's column (and in the Cholesky the registers holding its rows) are
// compile-time constants.  The triangular inverse then works by 16 x 16 blocks in LDS.
constexpr int kSmallRows = 144;          // sketch rows (k <= 128 columns): a k + 16 embedding
constexpr int kSmallCols = 128;
constexpr int kQrRowsPerLane = kSmallRows / 8;   // 18
constexpr int kChRowsPerLane = kSmallCols / 8;   // 16
constexpr int kInvBlock = 16;

// Sum over aligned groups of eight lanes by DPP moves, which do not go through LDS: partners
// one and two lanes apart within each quad, then the mirror within each half-row (lane i and
// 7 - i).  Every stage adds two values in either order, so all eight lanes end with the same
// bits.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double group8_sum(double x) {
  x += dpp_move<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_move<0x141>(x);   // row_half_mirror
  return x;
}

// LDS of the two kernels (doubles): the k x (k + 1) triangle, then the double-buffered step
// vector (and, for the QR, the two taus).
constexpr size_t qr_lds_doubles(int k) { return (size_t)k * (k + 1) + 2 * kSmallRows + 2; }
constexpr size_t chol_lds_doubles(int k) { return (size_t)k * (k + 1) + 8 * kSmallCols; }

// The inverse of the upper triangular k x k matrix in LDS (row-major, leading dimension ld), in
// place, by blocks of 16 rows and columns.  First the diagonal blocks, one lane per column of a
// block: the reciprocals of the diagonal, then the substitution up the column with the partial
// sums of the rows above updated as each entry is found (a chain of one product and one fused
// multiply-add per entry).  Then, from the second last block row I up, the matrix cores form
// X_IJ = -D_I^{-1} sum_{I < L <= J} R_IL X_LJ for every J > I at once, one wavefront per J, the
// blocks below already holding X (only upper triangles are read: the rest of the diagonal
// blocks is never written).  A diagonal entry below floor in magnitude is raised to it (a
// direction the panel does not resolve; its basis column is then noise that the later passes
// normalise).  All four wavefronts of the workgroup call it.
__device__ void upper_inverse_blocked(double* A, int k, int ld, double floor) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = (k + kInvBlock - 1) / kInvBlock;
  {
    const int ib = tid / kInvBlock, cc = tid % kInvBlock;   // diagonal block and column in it
    const int o = ib * kInvBlock;
    const bool act = ib < nb && o + cc < k;
    double x[kInvBlock], acc[kInvBlock], rinv[kInvBlock];
#pragma unroll
    for (int i = 0; i < kInvBlock; ++i) {
      x[i] = 0.0;
      acc[i] = i == cc ? 1.0 : 0.0;
      rinv[i] = 1.0;
      if (act && i <= cc) {
        double rii = A[(o + i) * ld + o + i];
        rii = fabs(rii) < floor ? (rii < 0.0 ? -floor : floor) : rii;
        rinv[i] = 1.0 / rii;
      }
    }
#pragma unroll
    for (int l = kInvBlock - 1; l >= 0; --l) {
      if (act && l <= cc) {   // column cc of the block's inverse is zero below row cc
        x[l] = acc[l] * rinv[l];
#pragma unroll
        for (int i = 0; i < l; ++i) acc[i] = fma(-A[(o + i) * ld + o + l], x[l], acc[i]);
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < kInvBlock; ++i)
        if (i <= cc) A[(o + i) * ld + o + cc] = x[i];
    }
    __syncthreads();
  }
  // v_mfma_f64_16x16x4: lane (lk, lr) = (lane / 16, lane % 16) gives A[lr][lk] and B[lk][lr] of
  // a 4-wide slice of the inner index and holds D[4v + lk][lr], v = 0..3
  const int lr = lane & 15, lk = lane >> 4;
  for (int I = nb - 2; I >= 0; --I) {
    const int r0 = I * kInvBlock;
    d4v t[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int J = I + 1 + wv + 4 * h;   // at most seven blocks right of I over four wavefronts
      t[h] = d4v{0.0, 0.0, 0.0, 0.0};
      if (J < nb) {
        const int cJ = J * kInvBlock + lr;
        for (int L = I + 1; L <= J; ++L) {
#pragma unroll
          for (int kq = 0; kq < 4; ++kq) {
            const int l = L * kInvBlock + 4 * kq + lk;
            const double a = l < k ? A[(r0 + lr) * ld + l] : 0.0;
            const double b = (l < k && cJ < k && l <= cJ) ? A[l * ld + cJ] : 0.0;
            t[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, t[h], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();   // every block of row I of R has been read
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int J = I + 1 + wv + 4 * h;
      if (J < nb) {
        // X_IJ = -D_I^{-1} T: T's slice kq is this lane's accumulator entry kq
        d4v xb = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const int q = 4 * kq + lk;
          const double a = q >= lr ? A[(r0 + lr) * ld + r0 + q] : 0.0;
          xb = __builtin_amdgcn_mfma_f64_16x16x4f64(a, t[h][kq], xb, 0, 0, 0);
        }
        const int cJ = J * kInvBlock + lr;
        if (cJ < k) {
#pragma unroll
          for (int v = 0; v < 4; ++v) A[(r0 + 4 * v + lk) * ld + cJ] = -xb[v];
        }
      }
    }
    __syncthreads();
  }
}

// Householder QR of the s x k matrix S (row-major, k <= s <= kSmallRows, k <= kSmallCols) and
// the inverse of its triangular factor R: Rinv (k x k row-major, zeros below the diagonal).
// Reflector j (LAPACK's convention): beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta,
// v = x / (alpha - beta) below the diagonal; none where the column below is already zero.
// Lanes: group G = tid / 8 holds columns 4G .. 4G+3, lane g = tid % 8 rows 18g .. 18g+17.  At
// step j the group of column j forms v (1 on row j, zeros above) and puts it in LDS; every
// lane then applies the reflector to all four of its columns: in those left of j it changes
// only rows below their diagonal, which are not read again, and in those right of j it leaves
// row j final.  The registers thus end holding R above the diagonal; beta goes to LDS at once.
__global__ __launch_bounds__(256) void k_qr_rinv(const double* __restrict__ S, int s, int k,
                                                 double* __restrict__ Rinv) {
  constexpr int RL = kQrRowsPerLane;
  extern __shared__ double sm[];
  const int ld = k + 1;
  double* Rm = sm;                          // k rows of k + 1: R, then its inverse
  double* vb = Rm + (size_t)k * ld;         // 2 x kSmallRows
  double* tb = vb + 2 * kSmallRows;         // 2
  const int tid = threadIdx.x, G = tid >> 3, g = tid & 7;
  const int row0 = g * RL, col0 = 4 * G;
  double a[RL][4];
#pragma unroll
  for (int rr = 0; rr < RL; ++rr)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = row0 + rr, c = col0 + q;
      a[rr][q] = (i < s && c < k) ? S[i * k + c] : 0.0;
    }
  // steps in blocks of four: within a block the column slot (j mod 4) and the buffer (j mod 2)
  // are fixed by t
  for (int jb = 0; jb < k; jb += 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = jb + t;
      if (j >= k) continue;   // uniform; no early exit, so that the loop unrolls fully
      double* v = vb + (t & 1) * kSmallRows;
      if (G == (j >> 2)) {
        double part = 0.0, alpha = 0.0;
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) {
          const int i = row0 + rr;
          const double x = a[rr][t];
          part = fma(i > j ? x : 0.0, x, part);
          alpha += i == j ? x : 0.0;
        }
        part = group8_sum(part);
        alpha = group8_sum(alpha);
        double beta = alpha, tau = 0.0, scale = 0.0;
        if (part > 0.0) {
          const double nrm = sqrt(alpha * alpha + part);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) {
          const int i = row0 + rr;
          v[i] = i > j ? a[rr][t] * scale : (i == j ? 1.0 : 0.0);
        }
        if (g == 0) {
          tb[t & 1] = tau;
          Rm[j * ld + j] = beta;
        }
      }
      __syncthreads();
      const double tau = tb[t & 1];
      double vr[RL];
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) vr[rr] = v[row0 + rr];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double w = 0.0;
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) w = fma(vr[rr], a[rr][c], w);
        w = group8_sum(w) * tau;
#pragma unroll
        for (int rr = 0; rr < RL; ++rr) a[rr][c] = fma(-vr[rr], w, a[rr][c]);
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < RL; ++rr)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = row0 + rr, c = col0 + q;
      if (i < c && c < k) Rm[i * ld + c] = a[rr][q];
    }
  __syncthreads();
  double dmax = 0.0;
  for (int j = 0; j < k; ++j) dmax = fmax(dmax, fabs(Rm[j * ld + j]));
  upper_inverse_blocked(Rm, k, ld, dmax * 0x1p-63);
  for (int e = tid; e < k * k; e += 256) {
    const int i = e / k, c = e % k;
    Rinv[e] = c >= i ? Rm[i * ld + c] : 0.0;
  }
}

// Upper Cholesky factor C of the symmetric part of M (k x k row-major, C^T C = (M + M^T)/2)
// and its inverse Cinv (row-major, zeros below).  A pivot that is not positive (the panel lost
// rank) sets *bad = 1 and is replaced by the smallest positive one seen, so the launch ends
// normally; the caller reads *bad.  Lanes as in the QR, with rows 16g .. 16g+15, and the
// matrix padded with the identity to a multiple of four.  Four rows at a time: the lanes
// holding rows j .. j+3 put them in LDS; every lane factors their 4 x 4 diagonal block D
// (D = C_D^T C_D), forms rows j .. j+3 of C at its own rows and columns by substitution with
// C_D^T, and subtracts their products from its entries (those in rows and columns already done
// are not read again).
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ M, int k, double* __restrict__ Cinv,
                                                  int* __restrict__ bad) {
  constexpr int RL = kChRowsPerLane;
  extern __shared__ double sm[];
  const int ld = k + 1;
  double* Cm = sm;                          // k rows of k + 1: C, then its inverse
  double* rb = Cm + (size_t)k * ld;         // 2 x 4 rows of kSmallCols: rows j .. j+3, double-buffered
  const int tid = threadIdx.x, G = tid >> 3, g = tid & 7;
  const int row0 = g * RL, col0 = 4 * G;
  const int kp = (k + 3) & ~3;
  double a[RL][4];
#pragma unroll
  for (int rr = 0; rr < RL; ++rr)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = row0 + rr, c = col0 + q;
      a[rr][q] = (i < k && c < k) ? 0.5 * (M[i * k + c] + M[c * k + i]) : (i == c ? 1.0 : 0.0);
    }
  double dmin = 1e300;
  int badv = 0;
  for (int jb = 0; jb < kp; jb += RL) {
#pragma unroll
    for (int u = 0; u < RL / 4; ++u) {
      const int j = jb + 4 * u;
      if (j >= kp) continue;   // uniform; no early exit, so that the loop unrolls fully
      double* r = rb + (u & 1) * 4 * kSmallCols;
      if (g == jb / RL) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) r[t * kSmallCols + col0 + q] = a[4 * u + t][q];
      }
      __syncthreads();
      // C_D, upper: c[t][s] for s >= t, iv[t] = 1 / c[t][t]
      double c[4][4], iv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double p = r[t * kSmallCols + j + t];
#pragma unroll
        for (int m = 0; m < t; ++m) p = fma(-c[m][t], c[m][t], p);
        if (!(p > 0.0)) {
          badv = 1;
          p = dmin < 1e300 ? dmin * dmin : 1.0;
        }
        c[t][t] = sqrt(p);
        dmin = fmin(dmin, c[t][t]);
        iv[t] = 1.0 / c[t][t];
#pragma unroll
        for (int s2 = t + 1; s2 < 4; ++s2) {
          double x = r[t * kSmallCols + j + s2];
#pragma unroll
          for (int m = 0; m < t; ++m) x = fma(-c[m][t], c[m][s2], x);
          c[t][s2] = x * iv[t];
        }
      }
      // rows j .. j+3 of C at column x: the solution y of C_D^T y = (A_jx .. A_j+3,x)
      auto solve = [&](int x, double y[4]) {
        double b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = r[t * kSmallCols + x];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          double v = b[t];
#pragma unroll
          for (int m = 0; m < t; ++m) v = fma(-c[m][t], y[m], v);
          y[t] = v * iv[t];
        }
      };
      double yc[4][4];   // [column q][row t]
#pragma unroll
      for (int q = 0; q < 4; ++q) solve(col0 + q, yc[q]);
      if (g == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = j + t, col = col0 + q;
            if (row < k && col >= row && col < k) Cm[row * ld + col] = col == row ? c[t][t] : yc[q][t];
          }
      }
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) {
        double y[4];
        solve(row0 + rr, y);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int t = 0; t < 4; ++t) a[rr][q] = fma(-y[t], yc[q][t], a[rr][q]);
      }
    }
  }
  if (tid == 0 && badv) *bad = 1;
  __syncthreads();
  upper_inverse_blocked(Cm, k, ld, 0.0);
  for (int e = tid; e < k * k; e += 256) {
    const int i = e / k, c = e % k;
    Cinv[e] = c >= i ? Cm[i * ld + c] : 0.0;
  }
}

// xi_c = z_m w_k nu1_c nu2_c nu3_c for column c = m*K + k.
__global__ void k_weights(const double* __restrict__ z, const double* __restrict__ w, int K, int64_t C,
                          const double* __restrict__ nu1, const double* __restrict__ nu2,
                          const double* __restrict__ nu3, double* __restrict__ xi) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x)
    xi[c] = z[c / K] * w[c % K] * nu1[c] * nu2[c] * nu3[c];
}

// Core beta[(a*r2 + b) * ldb + c] -> column-major slices S[c][b][a] (r1 x r2, lda = r1).
__global__ void k_core_slices(const double* __restrict__ beta, int r1, int r2, int r3, int64_t ldb,
                              double* __restrict__ S) {
  const int64_t total = (int64_t)r1 * r2 * r3;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % r1);
    const int64_t rest = e / r1;
    const int bb = (int)(rest % r2);
    const int c = (int)(rest / r2);
    S[e] = beta[((int64_t)a * r2 + bb) * ldb + c];
  }
}

// Kept canonical terms of the slice SVDs, chosen on the device: term (c, q) is kept when
// sv[c * ns + q] >= eps * (the largest over all slices) and > 0, and the kept terms are numbered
// p = 0, 1, ... in (c, q) order.  One workgroup: pos[c * ns + q] = p or -1, slice[p] = c,
// out[0] = R and out[1] = the number of kChunk-column chunks whose columns come from fewer than
// kSharedSlots slices (the chunks the scoring kernels serve from U_3).
constexpr int kSelThreads = 1024;
__global__ __launch_bounds__(kSelThreads) void k_t2c_select(const double* __restrict__ sv, int total, int ns,
                                                            double eps, int* __restrict__ pos,
                                                            int* __restrict__ slice, int* __restrict__ out) {
  __shared__ double s_max[kSelThreads / 64];
  __shared__ int s_scan[2][kSelThreads];
  __shared__ int s_u3[kSelThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double mx = 0.0;
  for (int e = tid; e < total; e += kSelThreads) mx = fmax(mx, sv[e]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) s_max[wv] = mx;
  __syncthreads();
  double smax = 0.0;
  for (int w = 0; w < kSelThreads / 64; ++w) smax = fmax(smax, s_max[w]);
  const double cut = eps * smax;
  // each thread takes a contiguous run of the (c, q) order
  const int per = (total + kSelThreads - 1) / kSelThreads;
  const int e0 = min(total, tid * per), e1 = min(total, e0 + per);
  int cnt = 0;
  for (int e = e0; e < e1; ++e) cnt += (sv[e] >= cut && sv[e] > 0.0) ? 1 : 0;
  // inclusive scan of the counts (Hillis-Steele, two LDS buffers)
  int cur = 0;
  s_scan[0][tid] = cnt;
  __syncthreads();
  for (int off = 1; off < kSelThreads; off <<= 1) {
    const int v = s_scan[cur][tid] + (tid >= off ? s_scan[cur][tid - off] : 0);
    s_scan[cur ^ 1][tid] = v;
    cur ^= 1;
    __syncthreads();
  }
  int p = s_scan[cur][tid] - cnt;
  for (int e = e0; e < e1; ++e) {
    if (sv[e] >= cut && sv[e] > 0.0) {
      pos[e] = p;
      slice[p] = e / ns;
      ++p;
    } else {
      pos[e] = -1;
    }
  }
  const int R = s_scan[cur][kSelThreads - 1];
  __syncthreads();   // slice[] is complete
  const int nchunk = (R + kChunk - 1) / kChunk;
  int u3 = 0;
  for (int ch = tid; ch < nchunk; ch += kSelThreads) {
    const int p0 = ch * kChunk, p1 = min(R, p0 + kChunk) - 1;
    u3 += (slice[p1] - slice[p0] < kSharedSlots) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) u3 += __shfl_xor(u3, off, 64);
  if (lane == 0) s_u3[wv] = u3;
  __syncthreads();
  if (tid == 0) {
    int t3 = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) t3 += s_u3[w];
    out[0] = R;
    out[1] = t3;
  }
}

// The kept terms as columns p of V_1 (r1 x R: s_q u_q), V_2 (r2 x R: v_q) and V_3 (r3 x R: e_c),
// from the slice SVDs in the layout sv[c*ns + q], uv[c*r1*ns + q*r1 + a], vv[c*ns*r2 + b*ns + q].
__global__ void k_t2c_factors(const double* __restrict__ sv, const double* __restrict__ uv,
                              const double* __restrict__ vv, const int* __restrict__ pos, int total, int ns,
                              int r1, int r2, int r3, int64_t R, double* __restrict__ V1, double* __restrict__ V2,
                              double* __restrict__ V3) {
  const int rows = r1 + r2 + r3;
  const int64_t work = (int64_t)total * rows;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < work; w += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(w / rows), row = (int)(w - (int64_t)e * rows);
    const int64_t p = pos[e];
    if (p < 0) continue;
    const int c = e / ns, q = e - c * ns;
    if (row < r1) {
      V1[(int64_t)row * R + p] = sv[e] * uv[((int64_t)c * ns + q) * r1 + row];
    } else if (row < r1 + r2) {
      const int b = row - r1;
      V2[(int64_t)b * R + p] = vv[((int64_t)c * r2 + b) * ns + q];
    } else {
      const int c3 = row - r1 - r2;
      V3[(int64_t)c3 * R + p] = c3 == c ? 1.0 : 0.0;
    }
  }
}

// One-sided (Hestenes) Jacobi SVD of the mode-3 slices of the core, one workgroup per
// slice held in LDS.  Column pairs are orthogonalised in the round-robin order (n/2
// disjoint pairs per round, eight lanes per pair); a sweep is n-1 rounds; sweeps
// stop when no pair needed a rotation.  Then column q of the rotated slice is
// s_q u_q, and v_q = S^T u_q / s_q is taken from the original slice (v_q enters the
// tensor only multiplied by s_q, so the division loses nothing that matters).
// Output layout matches a thin LAPACK-style SVD with ns = n values per slice:
// sv[c*n + q], u[c*m*n + q*m + a], vt[c*n*n + q + b*n].
constexpr int kJacobiMaxElems = 18432;   // m * n doubles of one slice (144 KB of LDS)
constexpr int kJacobiMaxSweeps = 80;

__device__ __forceinline__ int rr_player(int pos, int round, int np) {
  int x = pos - 1 + round;                // < 2 (np - 1): one conditional subtraction
  x -= x >= np - 1 ? np - 1 : 0;
  return pos == 0 ? 0 : 1 + x;
}

constexpr int kJacobiThreads = 512;   // eight lanes per column pair, up to 64 pairs per round
constexpr int kJacobiLanes = 8;

// The rotation of one column pair from its sums al = |a_p|^2, be = |a_q|^2, ga = a_p . a_q
// (over the eight lanes of the pair, an aligned group); false when the pair is left alone: its
// cosine is below the rounding level of the dot product, or a column is below the skip level.
// Rutishauser's tangent sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (be - al) / (2 ga),
// is written over the common denominator: two square roots and one division in the chain.
__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double skip, double tol,
                                                double& cs, double& sn) {
  al = group8_sum(al);
  be = group8_sum(be);
  ga = group8_sum(ga);
  if (!(ga != 0.0 && fmin(al, be) > skip && fabs(ga) > tol * sqrt(al * be))) return false;
  const double D = be - al, G2 = 2.0 * ga;
  const double den = fabs(D) + sqrt(fma(D, D, G2 * G2));
  const double rs = 1.0 / sqrt(fma(den, den, G2 * G2));
  cs = den * rs;
  sn = (D >= 0.0 ? G2 : -G2) * rs;
  return true;
}

// The sweeps of one-sided Jacobi over the nc columns (mr rows each, column-major in LDS at sM):
// column pairs in the round-robin order, eight lanes per pair, each over every eighth row
// (loads unrolled so that several are in flight), the three sums combined within the group
// (a 64-lane reduction per pair, or one lane per pair, leaves each round waiting on LDS
// latency).  ACCV: every rotation is also applied to the columns of the nv x nc matrix at sV.
// Pairs with a column whose squared norm is at most skip are left alone, and a pair is rotated
// only when its cosine exceeds the rounding level of an mr-term dot product; the sweeps stop
// when none was rotated.  Returns the number of sweeps.  All lanes of the workgroup call it.
template <bool ACCV>
__device__ int jacobi_sweeps(double* sM, int mr, int nc, double* sV, int nv, double skip, int* s_rot) {
  const int tid = threadIdx.x;
  const int np = nc + (nc & 1);
  const double tol = fmax(1e-14, 4.0 * mr * 1.1102230246251565e-16);
  int sweep = 0;
  for (; sweep < kJacobiMaxSweeps && nc > 1; ++sweep) {
    if (tid == 0) *s_rot = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      for (int k8 = tid; k8 < (np / 2) * kJacobiLanes; k8 += kJacobiThreads) {
        const int k = k8 / kJacobiLanes, part = k8 % kJacobiLanes;
        const int pa = rr_player(k, round, np), pb = rr_player(np - 1 - k, round, np);
        const int p = min(pa, pb), q = max(pa, pb);
        if (q >= nc) continue;
        double* ap = sM + p * mr;
        double* aq = sM + q * mr;
        double cs, sn, al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 4
        for (int row = part; row < mr; row += kJacobiLanes) {
          const double x = ap[row], y = aq[row];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        if (!jacobi_rotation(al, be, ga, skip, tol, cs, sn)) continue;
#pragma unroll 4
        for (int row = part; row < mr; row += kJacobiLanes) {
          const double x = ap[row], y = aq[row];
          ap[row] = cs * x - sn * y;
          aq[row] = sn * x + cs * y;
        }
        if (ACCV) {
          double* vp = sV + p * nv;
          double* vq = sV + q * nv;
#pragma unroll 4
          for (int row = part; row < nv; row += kJacobiLanes) {
            const double x = vp[row], y = vq[row];
            vp[row] = cs * x - sn * y;
            vq[row] = sn * x + cs * y;
          }
        }
        *s_rot = 1;
      }
      __syncthreads();
    }
    const int rot = *s_rot;
    __syncthreads();
    if (!rot) break;
  }
  return sweep;
}

// The Frobenius norm squared of the m x n slice at Sc, copied into LDS at sA on the way.
__device__ double load_slice(const double* __restrict__ Sc, int m, int n, double* sA, double* s_part) {
  constexpr int kWaves = kJacobiThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double fro = 0.0;
  for (int e = tid; e < m * n; e += kJacobiThreads) {
    const double x = Sc[e];
    sA[e] = x;
    fro = fma(x, x, fro);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) fro += __shfl_xor(fro, off, 64);
  if (lane == 0) s_part[wv] = fro;
  __syncthreads();
  double fro_all = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) fro_all += s_part[w];
  return fro_all;
}

// ACCV: the rotations are also applied to V (n x n, from the identity, in LDS after the slice),
// and vt returns V itself: orthogonal to working precision, so the right vectors of small
// singular values are as accurate as the large ones' (v = S^T u / s is not, and serves only
// where v enters multiplied by s).
template <bool ACCV>
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_svd(const double* __restrict__ S, int m, int n,
                                                               double skip_rel2, double* __restrict__ sv,
                                                               double* __restrict__ uv, double* __restrict__ vt,
                                                               int* __restrict__ sweeps) {
  extern __shared__ double sA[];
  double* sV = sA + (size_t)m * n;       // ACCV: column q of V at sV[q * n .. q * n + n - 1]
  constexpr int kWaves = kJacobiThreads / 64;
  __shared__ int s_rot;
  __shared__ double s_part[kWaves];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* Sc = S + (int64_t)c * m * n;
  if (ACCV)
    for (int e = tid; e < n * n; e += kJacobiThreads) sV[e] = (e / n == e % n) ? 1.0 : 0.0;
  // columns below sqrt(skip_rel2) of the slice norm hold nothing above the truncation level;
  // pairs involving them are left alone (rotating them only churns rounding noise)
  const double skip = skip_rel2 * load_slice(Sc, m, n, sA, s_part);
  const int sweep = jacobi_sweeps<ACCV>(sA, m, n, sV, n, skip, &s_rot);
  if (tid == 0) sweeps[c] = sweep;
  // singular values and normalised left vectors
  for (int q = wv; q < n; q += kWaves) {
    double s2 = 0.0;
    for (int row = lane; row < m; row += 64) s2 = fma(sA[q * m + row], sA[q * m + row], s2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
    const double sq = sqrt(s2);
    const double inv = sq > 0.0 ? 1.0 / sq : 0.0;
    for (int row = lane; row < m; row += 64) {
      const double u = sA[q * m + row] * inv;
      sA[q * m + row] = u;
      uv[(int64_t)c * m * n + (int64_t)q * m + row] = u;
    }
    if (lane == 0) sv[(int64_t)c * n + q] = sq;
  }
  __syncthreads();
  if (ACCV) {   // vt[q + b n] = V[b][q]
    for (int e = tid; e < n * n; e += kJacobiThreads) {
      const int q = e % n, b = e / n;
      vt[(int64_t)c * n * n + e] = sV[q * n + b];
    }
    return;
  }
  // v_q = S^T u_q / s_q
  for (int e = tid; e < n * n; e += kJacobiThreads) {
    const int q = e % n, bcol = e / n;
    const double* scol = Sc + (int64_t)bcol * m;
    const double* u = sA + q * m;
    double w = 0.0;
#pragma unroll 8
    for (int a = 0; a < m; ++a) w = fma(scol[a], u[a], w);
    const double sq = sv[(int64_t)c * n + q];
    vt[(int64_t)c * n * n + q + (int64_t)bcol * n] = sq > 0.0 ? w / sq : 0.0;
  }
}

// The same slice SVDs, with the slice first reduced by a Householder QR (A = Q R, in place in
// LDS: R on and above the diagonal, the reflectors below it): one-sided Jacobi then runs on the
// p = min(m, n) columns of X = R^T (n rows each), whose rows are the rows of R, with the rotations
// accumulated in W (p x p, from the identity).  On the core slices, whose singular values are
// strongly graded, this takes 5 to 7 sweeps where the slice itself takes 14 to 17.  With
// X W = Z: A = (Q W) Z^T, so s_q = |z_q|, v_q = z_q / s_q and u_q = Q w_q (the reflectors applied
// to w_q padded with zeros).  Singular values q >= p are zero, with zero vectors.  Output layout
// as k_jacobi_svd's; LDS: m n + max(m, n) p + p^2 + p doubles.
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_svd_qr(const double* __restrict__ S, int m, int n,
                                                                  double skip_rel2, double* __restrict__ sv,
                                                                  double* __restrict__ uv, double* __restrict__ vt,
                                                                  int* __restrict__ sweeps) {
  extern __shared__ double sA[];                     // m x n, column-major
  constexpr int kWaves = kJacobiThreads / 64;
  const int p = min(m, n), mx = max(m, n);
  double* sX = sA + (size_t)m * n;                   // X = R^T (n x p), later U (m x p)
  double* sW = sX + (size_t)mx * p;                  // W (p x p)
  double* tau = sW + (size_t)p * p;                  // p
  __shared__ int s_rot;
  __shared__ double s_part[kWaves];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* Sc = S + (int64_t)c * m * n;
  const double skip = skip_rel2 * load_slice(Sc, m, n, sA, s_part);
  // Householder QR (LAPACK's convention, as in k_qr_rinv); wavefront 0 forms reflector j, then
  // eight lanes per column apply it to the columns right of j
  for (int j = 0; j < p; ++j) {
    double* aj = sA + (size_t)j * m;
    if (wv == 0) {
      double part = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) part = fma(aj[i], aj[i], part);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      const double alpha = aj[j];
      double beta = alpha, tj = 0.0, scale = 0.0;
      if (part > 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, part));
        beta = alpha >= 0.0 ? -nrm : nrm;
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = j + 1 + lane; i < m; i += 64) aj[i] *= scale;
      if (lane == 0) {
        aj[j] = beta;
        tau[j] = tj;
      }
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      for (int k8 = tid; k8 < (n - j - 1) * kJacobiLanes; k8 += kJacobiThreads) {
        double* ac = sA + (size_t)(j + 1 + k8 / kJacobiLanes) * m;
        const int part = k8 % kJacobiLanes;
        double w = 0.0;
        for (int i = j + 1 + part; i < m; i += kJacobiLanes) w = fma(aj[i], ac[i], w);
        w = tj * (group8_sum(w) + ac[j]);
        if (part == 0) ac[j] -= w;
        for (int i = j + 1 + part; i < m; i += kJacobiLanes) ac[i] = fma(-aj[i], w, ac[i]);
      }
    }
    __syncthreads();
  }
  // X: column a holds row a of R; W = I
  for (int e = tid; e < n * p; e += kJacobiThreads) {
    const int a = e / n, b = e % n;
    sX[e] = b >= a ? sA[a + (size_t)b * m] : 0.0;
  }
  for (int e = tid; e < p * p; e += kJacobiThreads) sW[e] = (e / p == e % p) ? 1.0 : 0.0;
  __syncthreads();
  const int sweep = jacobi_sweeps<true>(sX, n, p, sW, p, skip, &s_rot);
  if (tid == 0) sweeps[c] = sweep;
  // s_q and v_q = z_q / s_q; zeros for q >= p
  for (int q = wv; q < n; q += kWaves) {
    const double* z = sX + (size_t)q * n;
    double s2 = 0.0;
    if (q < p)
      for (int row = lane; row < n; row += 64) s2 = fma(z[row], z[row], s2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
    const double sq = sqrt(s2);
    const double inv = sq > 0.0 ? 1.0 / sq : 0.0;
    for (int b = lane; b < n; b += 64) vt[(int64_t)c * n * n + q + (int64_t)b * n] = q < p ? z[b] * inv : 0.0;
    if (lane == 0) sv[(int64_t)c * n + q] = sq;
  }
  __syncthreads();
  // U = Q [W; 0] in place of X: the reflectors from the last to the first
  double* sU = sX;
  for (int e = tid; e < m * p; e += kJacobiThreads) {
    const int q = e / m, a = e % m;
    sU[e] = a < p ? sW[(size_t)q * p + a] : 0.0;
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;   // uniform
    const double* aj = sA + (size_t)j * m;
    for (int k8 = tid; k8 < p * kJacobiLanes; k8 += kJacobiThreads) {
      double* uq = sU + (size_t)(k8 / kJacobiLanes) * m;
      const int part = k8 % kJacobiLanes;
      double w = 0.0;
      for (int i = j + 1 + part; i < m; i += kJacobiLanes) w = fma(aj[i], uq[i], w);
      w = tj * (group8_sum(w) + uq[j]);
      if (part == 0) uq[j] -= w;
      for (int i = j + 1 + part; i < m; i += kJacobiLanes) uq[i] = fma(-aj[i], w, uq[i]);
    }
    __syncthreads();
  }
  for (int e = tid; e < m * n; e += kJacobiThreads) {
    const int q = e / m;
    uv[(int64_t)c * m * n + e] = q < p ? sU[e] : 0.0;
  }
}

// LDS of k_jacobi_svd_qr for an m x n slice, in doubles, and the most it may take (160 KB per
// workgroup, less the kernel's own few bytes).
constexpr size_t jacobi_qr_lds_doubles(int m, int n) {
  return (size_t)m * n + (size_t)(m > n ? m : n) * (m < n ? m : n) + (size_t)(m < n ? m : n) * (m < n ? m : n) +
         (m < n ? m : n);
}
constexpr size_t kJacobiQrMaxLds = 20400;

// Singular values of a k x k Jacobi SVD (unsorted) into decreasing order, with the rows of the
// LAPACK-style VT layout vt[q + b k] (right vector q, component b) moved along; ties keep their
// index order.  info = 0, or 1 when the sweeps hit their limit, 2 when a value is not a number.
__global__ __launch_bounds__(256) void k_svd_sort(const double* __restrict__ sv_in, const double* __restrict__ vt_in,
                                                  int k, const int* __restrict__ sweeps, double* __restrict__ sv_out,
                                                  double* __restrict__ vt_out, rocblas_int* __restrict__ info) {
  __shared__ int s_nan;
  if (threadIdx.x == 0) s_nan = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < k; q += blockDim.x) {
    const double v = sv_in[q];
    if (!(v == v)) {
      s_nan = 1;
      continue;
    }
    int rank = 0;
    for (int p = 0; p < k; ++p) {
      const double w = sv_in[p];
      rank += (w > v || (w == v && p < q)) ? 1 : 0;
    }
    sv_out[rank] = v;
    for (int b = 0; b < k; ++b) vt_out[rank + (int64_t)b * k] = vt_in[q + (int64_t)b * k];
  }
  __syncthreads();
  if (threadIdx.x == 0) *info = s_nan ? 2 : (*sweeps < kJacobiMaxSweeps ? 0 : 1);
}

// ----------------------------------------------------------------- host helpers
// A scratch buffer of a build or rank reduction, drawn from the context's scratch cache.  Its
// block stays with the call (queued work may still use it) and returns to the cache when
// the call's ScratchScope ends; releasing a DevBuf only forgets the pointer.
struct DevBuf {
  double* p = nullptr;
  size_t bytes = 0;
  rsd_status alloc(Context* c, size_t n) {
    bytes = sizeof(double) * (n ? n : 1);
    return c->scratch_get((void**)&p, bytes);
  }
};

// Declared first in an entry function, so that it ends last: one wait for the context
// stream, then every scratch block of the call goes back to the cache.
struct ScratchScope {
  Context* c;
  ~ScratchScope() { c->scratch_end(); }
};

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline unsigned grid1d(int64_t total) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (total + 255) / 256), 65536); }

// Issues f(d, stream) for the three modes d on the context stream and the two auxiliary
// streams, each after the work already queued on the context stream, with the context stream
// current while f(d) issues; the context stream then waits for all three (also when an f fails).
// With per-launch timing on, all three go to the context stream, so that each launch's events
// time that launch alone.
template <class F>
rsd_status on_three_streams(Context* ctx, F&& f) {
  const hipStream_t main = ctx->stream;
  RSD_TRY(ctx->aux_streams());
  const bool serial = ctx->timing;
  const hipStream_t st[3] = {main, serial ? main : ctx->aux_stream[0], serial ? main : ctx->aux_stream[1]};
  struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  for (auto& x : ev.e) RSD_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  RSD_HIP(hipEventRecord(ev.e[0], main));
  RSD_HIP(hipStreamWaitEvent(st[1], ev.e[0], 0));
  RSD_HIP(hipStreamWaitEvent(st[2], ev.e[0], 0));
  rsd_status rs = RSD_OK;
  for (int d = 0; d < 3 && rs == RSD_OK; ++d) {
    ctx->stream = st[d];
    rs = f(d, st[d]);
    ctx->stream = main;
  }
  for (int i = 1; i < 3; ++i) {
    RSD_HIP(hipEventRecord(ev.e[i], st[i]));
    RSD_HIP(hipStreamWaitEvent(main, ev.e[i], 0));
  }
  return rs;
}

template <class AOp, class BOp>
rsd_status gemm(Context* ctx, const char* name, const AOp& A, const BOp& B, GemmShape g, int splits) {
  dim3 grid;
  if (g.tri) {
    g.tiles_n = div_up(g.N, TN);
    grid = dim3((unsigned)(g.tiles_n * (g.tiles_n + 1) / 2), 1, (unsigned)splits);
  } else {
    RSD_CHECK(div_up(g.N, TN) <= 65535 && splits <= 65535, RSD_E_UNSUPPORTED, "%s: product shape exceeds the launch grid",
              name);
    grid = dim3((unsigned)div_up(g.M, TM), (unsigned)div_up(g.N, TN), (unsigned)splits);
    if (g.N <= TNW) {   // one column tile
      grid.y = 1;
      RSD_TIMED_LAUNCH(ctx, name, (k_gemm_w<AOp, BOp><<<grid, 256, 0, ctx->stream>>>(A, B, g)));
      return RSD_OK;
    }
  }
  RSD_TIMED_LAUNCH(ctx, name, (k_gemm<AOp, BOp><<<grid, 256, 0, ctx->stream>>>(A, B, g)));
  return RSD_OK;
}

rsd_status check_info(Context* ctx, rocblas_int* d_info, int count, const char* what) {
  std::vector<rocblas_int> info((size_t)count);
  RSD_HIP(hipMemcpyAsync(info.data(), d_info, sizeof(rocblas_int) * count, hipMemcpyDeviceToHost, ctx->stream));
  RSD_HIP(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < count; ++i)
    RSD_CHECK(info[i] == 0, RSD_E_NUMERIC, "%s did not converge (info %d at %d)", what, (int)info[i], i);
  return RSD_OK;
}

// Dynamic LDS beyond 64 KB for the two small-factorization kernels (once per device).
rsd_status allow_small_lds() {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  RSD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return RSD_OK;
  RSD_HIP(hipFuncSetAttribute((const void*)k_qr_rinv, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * qr_lds_doubles(kSmallCols))));
  RSD_HIP(hipFuncSetAttribute((const void*)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * chol_lds_doubles(kSmallCols))));
  done.push_back(dev);
  return RSD_OK;
}

// Scratch of one mode's orthonormalizations (k <= kSmallCols).
struct OrthBufs {
  DevBuf theta, sk, part, w, rinv, tmp;
  int splits = 1;
  rsd_status alloc(Context* c, int n, int k) {
    splits = std::max(1, std::min(32, n / 128));
    RSD_TRY(theta.alloc(c, (size_t)kSmallRows * n));
    RSD_TRY(sk.alloc(c, (size_t)kSmallRows * k));
    RSD_TRY(part.alloc(c, (size_t)splits * kSmallRows * k));
    RSD_TRY(w.alloc(c, (size_t)k * k));
    RSD_TRY(rinv.alloc(c, (size_t)k * k));
    RSD_TRY(tmp.alloc(c, (size_t)k * n));
    return RSD_OK;
  }
};

// C (M x N, ld N) = sum over the K rows of A(k, m) B(k, n), split over the contraction and summed.
template <class AOp, class BOp>
rsd_status gemm_split(Context* ctx, const AOp& A, const BOp& B, int M, int N, int64_t K, double* part, int splits,
                      double* C, const char* name = "eig") {
  GemmShape g{};
  g.M = M; g.N = N; g.K = K;
  g.kper = (int64_t)div_up(K, (int64_t)splits * TK) * TK;
  g.C = part; g.ldc = N; g.split_stride = (int64_t)M * N; g.accumulate = 0; g.tri = 0;
  RSD_TRY(gemm(ctx, name, A, B, g, splits));
  RSD_TIMED_LAUNCH(ctx, name, (k_reduce_splits<<<grid1d((int64_t)M * N), 256, 0, ctx->stream>>>(
                                  part, splits, (int64_t)M * N, M, N, N, C, N)));
  return RSD_OK;
}

// A basis of the k columns of the n x k panel Y, stored transposed (Yt: k x n, row-major, i.e. Y
// column-major): the randomized Cholesky QR -- the Householder QR of the sketch Theta Y
// (kSmallRows x k, Theta uniform random) gives R_s, and Q1 = Y R_s^{-1} has a condition number
// near that of Theta on the range of Y, independent of Y's -- then `passes` Cholesky QR passes,
// Q <- Q C^{-1} with C^T C = Q^T Q (two make it orthonormal to rounding; none leaves the well
// conditioned Q1, enough for a power step).  The result (transposed, k x n) goes to out (passes
// even); *bad is set when a Cholesky pivot was not positive.  Y and out must differ.
rsd_status orth_rchol(Context* ctx, const double* Yt, int k, int n, OrthBufs& b, double* out, int* bad,
                      int passes, const char* name = "eig") {
  hipStream_t s = ctx->stream;
  const int sr = kSmallRows;
  RSD_TRY(gemm_split(ctx, OpMK{b.theta.p, n, sr}, OpMK{Yt, n, k}, sr, k, n, b.part.p, b.splits, b.sk.p, name));
  RSD_TIMED_LAUNCH(ctx, name, (k_qr_rinv<<<1, 256, sizeof(double) * qr_lds_doubles(k), s>>>(
                                  b.sk.p, sr, k, b.rinv.p)));
  GemmShape g{};
  g.M = k; g.N = n; g.K = k; g.kper = ((int64_t)k + TK - 1) / TK * TK; g.ldc = n;
  g.split_stride = 0; g.accumulate = 0; g.tri = 0;
  g.C = out;
  RSD_TRY(gemm(ctx, name, OpKM{b.rinv.p, k, k}, OpKM{Yt, n, n}, g, 1));      // out = (Y R_s^{-1})^T
  double* bufs[2] = {out, b.tmp.p};   // pass 0: out -> tmp, pass 1: tmp -> out
  for (int pass = 0; pass < passes; ++pass) {
    const double* src = bufs[pass];
    RSD_TRY(gemm_split(ctx, OpMK{src, n, k}, OpMK{src, n, k}, k, k, n, b.part.p, b.splits, b.w.p, name));
    RSD_TIMED_LAUNCH(ctx, name, (k_chol_inv<<<1, 256, sizeof(double) * chol_lds_doubles(k), s>>>(
                                    b.w.p, k, b.rinv.p, bad)));
    g.C = bufs[1 - pass];
    RSD_TRY(gemm(ctx, name, OpKM{b.rinv.p, k, k}, OpKM{src, n, n}, g, 1));
  }
  return RSD_OK;
}

// Dominant eigenvectors of the three modes' symmetric PSD Gram matrices G_d (n x n, row-major
// and exactly symmetric), by randomized subspace iteration: Y = G Omega with k deterministic
// test vectors, an orthonormal basis Q of Y (Householder QR), one power step Q <- orth(G Q),
// then Rayleigh-Ritz on Q^T G Q (k x k).  Eigenvalues >= eps^2 * the largest are kept; if
// fewer than 16 of the k Ritz values fall below that cut, k is doubled and the mode is redone.
// The three modes run on three streams (the context stream and two auxiliary ones, each with
// its own rocBLAS handle): their QR and small eigensolver calls are chains of short launches,
// which then overlap.  The host synchronises once per pass to read the Ritz values.
rsd_status subspace_eigvecs3(Context* ctx, rocblas_handle hb, double* G3, int n, double eps, rocblas_int* d_info,
                             DevBuf U[3], int r_out[3], int ldu_out[3]) {
  hipStream_t main = ctx->stream;
  RSD_TRY(ctx->aux_streams());
  hipStream_t st[3] = {main, ctx->aux_stream[0], ctx->aux_stream[1]};
  rocblas_handle hbs[3] = {hb, (rocblas_handle)ctx->aux_blas[0], (rocblas_handle)ctx->aux_blas[1]};
  const int64_t nn = (int64_t)n * n;
  for (int d = 0; d < 3; ++d)
    RSD_TIMED_LAUNCH(ctx, "eig", (k_symmetrize<<<grid1d(nn), 256, 0, main>>>(G3 + d * nn, n)));
  hipEvent_t ready = nullptr, done[2] = {nullptr, nullptr};
  struct Events {
    hipEvent_t* e[3];
    ~Events() {
      for (auto* x : e)
        if (*x) (void)hipEventDestroy(*x);
    }
  } evguard{{&ready, &done[0], &done[1]}};
  RSD_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  RSD_HIP(hipEventCreateWithFlags(&done[0], hipEventDisableTiming));
  RSD_HIP(hipEventCreateWithFlags(&done[1], hipEventDisableTiming));
  RSD_HIP(hipEventRecord(ready, main));
  RSD_HIP(hipStreamWaitEvent(st[1], ready, 0));
  RSD_HIP(hipStreamWaitEvent(st[2], ready, 0));
  struct Mode {
    int k = 0;
    bool finished = false;
    bool lib = false;          // orthonormalize with rocSOLVER's Householder QR
    DevBuf Om, Y, Z, T, W, E, tau, Q, flag, part;
    OrthBufs ob;
  } m[3];
  RSD_TRY(allow_small_lds());
  for (int d = 0; d < 3; ++d) m[d].k = std::min(n, 128);
  struct StreamGuard {   // issue a mode's work on its stream; the context stream comes back afterwards
    Context* c;
    hipStream_t saved;
    ~StreamGuard() { c->stream = saved; }
  } sg{ctx, main};
  rsd_status st_all = RSD_OK;
  for (int pass = 0; pass < 8 && st_all == RSD_OK; ++pass) {
    bool any = false;
    for (int d = 0; d < 3; ++d) {
      Mode& md = m[d];
      if (md.finished) continue;
      any = true;
      ctx->stream = st[d];
      const int k = md.k;
      md.lib = md.lib || ctx->opt_qr == 1 || k > kSmallCols;
      auto issue = [&]() -> rsd_status {
        RSD_TRY(md.Om.alloc(ctx, (size_t)n * k));
        RSD_TRY(md.Y.alloc(ctx, (size_t)n * k));
        RSD_TRY(md.Z.alloc(ctx, (size_t)n * k));
        RSD_TRY(md.T.alloc(ctx, (size_t)k * k));
        RSD_TRY(md.W.alloc(ctx, k));
        RSD_TRY(md.E.alloc(ctx, k));
        RSD_TRY(md.tau.alloc(ctx, k));
        // the k x n and k x k products have only 2 x (n / 64) and 4 output tiles: their
        // contraction over n is split for about 256 workgroups, and the slices summed
        const int sp_kn = std::max(1, std::min(n / 256, div_up(256, div_up(k, TM) * div_up(n, TN))));
        const int sp_kk = std::max(1, std::min(n / 64, div_up(256, div_up(k, TM) * div_up(k, TN))));
        RSD_TRY(md.part.alloc(ctx, std::max((size_t)sp_kn * k * n, (size_t)sp_kk * k * k)));
        double* G = G3 + d * nn;
        RSD_TIMED_LAUNCH(ctx, "eig", (k_random_fill<<<grid1d((int64_t)n * k), 256, 0, st[d]>>>(
                                         md.Om.p, (int64_t)n * k, 0x5EEDull + (uint64_t)d)));
        if (!md.lib) {
          RSD_TRY(md.ob.alloc(ctx, n, k));
          RSD_TRY(md.Q.alloc(ctx, (size_t)n * k));
          RSD_TRY(md.flag.alloc(ctx, 1));
          RSD_HIP(hipMemsetAsync(md.flag.p, 0, sizeof(double), st[d]));
          RSD_TIMED_LAUNCH(ctx, "eig", (k_random_fill<<<grid1d((int64_t)kSmallRows * n), 256, 0, st[d]>>>(
                                           md.ob.theta.p, (int64_t)kSmallRows * n, 0x7E7Aull + (uint64_t)d)));
        }
        // P: column-major n x k -> a basis of its columns in P: orthonormal (full), or only well
        // conditioned (before the power step, which needs just the span)
        auto qr = [&](DevBuf& P, bool full) -> rsd_status {
          if (!md.lib) {
            RSD_TRY(orth_rchol(ctx, P.p, k, n, md.ob, md.Q.p, (int*)md.flag.p, full ? 2 : 0));
            std::swap(P.p, md.Q.p);
            return RSD_OK;
          }
          double* A = P.p;
          KernelTimer kt;
          if (ctx->timing) RSD_TRY(ctx->timer_begin("eig", &kt));
          RSD_CHECK(rocsolver_dgeqrf(hbs[d], n, k, A, n, md.tau.p) == rocblas_status_success, RSD_E_HIP,
                    "rocsolver_dgeqrf failed");
          RSD_CHECK(rocsolver_dorgqr(hbs[d], n, k, k, A, n, md.tau.p) == rocblas_status_success, RSD_E_HIP,
                    "rocsolver_dorgqr failed");
          if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
          return RSD_OK;
        };
        // Y^T = Omega^T G  (k x n row-major = n x k column-major)
        RSD_TRY(gemm_split(ctx, OpKM{md.Om.p, k, k}, OpKM{G, n, n}, k, n, n, md.part.p, sp_kn, md.Y.p));
        RSD_TRY(qr(md.Y, false));
        // one power step: Z^T = Q^T G, orthonormalise
        RSD_TRY(gemm_split(ctx, OpMK{md.Y.p, n, k}, OpKM{G, n, n}, k, n, n, md.part.p, sp_kn, md.Z.p));
        RSD_TRY(qr(md.Z, true));
        // Rayleigh-Ritz: Y^T = Q^T G (k x n), T = Q^T G Q (k x k)
        RSD_TRY(gemm_split(ctx, OpMK{md.Z.p, n, k}, OpKM{G, n, n}, k, n, n, md.part.p, sp_kn, md.Y.p));
        RSD_TRY(gemm_split(ctx, OpMK{md.Z.p, n, k}, OpMK{md.Y.p, n, k}, k, k, n, md.part.p, sp_kk, md.T.p));
        return RSD_OK;
      };
      st_all = issue();
      ctx->stream = main;
      if (st_all != RSD_OK) break;
    }
    // the small eigensolver calls last: a call may wait on the host for its own stream, and
    // the other modes' products are queued by then
    for (int d = 0; d < 3 && any && st_all == RSD_OK; ++d) {
      Mode& md = m[d];
      if (md.finished) continue;
      ctx->stream = st[d];
      auto eig = [&]() -> rsd_status {
        KernelTimer kt;
        if (ctx->timing) RSD_TRY(ctx->timer_begin("eig", &kt));
        const rocblas_status rs = rocsolver_dsyevd(hbs[d], rocblas_evect_original, rocblas_fill_upper, md.k, md.T.p,
                                                   md.k, md.W.p, md.E.p, d_info + d);
        RSD_CHECK(rs == rocblas_status_success, RSD_E_HIP, "rocsolver_dsyevd failed (%d)", (int)rs);
        if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
        return RSD_OK;
      };
      st_all = eig();
      ctx->stream = main;
    }
    if (!any || st_all != RSD_OK) break;
    // read every unfinished mode's Ritz values; finish the modes whose subspace was large enough
    for (int d = 0; d < 3 && st_all == RSD_OK; ++d) {
      Mode& md = m[d];
      if (md.finished) continue;
      const int k = md.k;
      std::vector<double> w((size_t)k);
      rocblas_int info = 0;
      int bad = 0;
      hipError_t e = hipMemcpyAsync(&info, d_info + d, sizeof(info), hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess) e = hipMemcpyAsync(w.data(), md.W.p, sizeof(double) * k, hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess && !md.lib) e = hipMemcpyAsync(&bad, md.flag.p, sizeof(int), hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess) e = hipStreamSynchronize(st[d]);
      if (e != hipSuccess) {
        set_error("Ritz values: %s", hipGetErrorString(e));
        st_all = RSD_E_HIP;
        break;
      }
      if (bad) {   // a Cholesky pass lost rank (its Rayleigh-Ritz input is then meaningless): redo with Householder QR
        md.lib = true;
        continue;
      }
      if (info != 0) {
        set_error("Ritz eigensolver of mode %d did not converge (info %d)", d, (int)info);
        st_all = RSD_E_NUMERIC;
        break;
      }
      const double lmax = w[k - 1];
      if (!(lmax > 0.0 && std::isfinite(lmax))) {
        set_error("Gram matrix of mode %d has no positive eigenvalue", d);
        st_all = RSD_E_NUMERIC;
        break;
      }
      int r = 0;
      for (int i = k - 1; i >= 0 && w[i] >= eps * eps * lmax; --i) ++r;
      if (r > k - 16 && k < n) {
        md.k = std::min(n, 2 * k);   // redo this mode with a larger subspace on the next pass
        continue;
      }
      if (r < 1 || r > 1024) {
        set_error("mode-%d rank %d outside [1, 1024]", d, r);
        st_all = RSD_E_UNSUPPORTED;
        break;
      }
      const int ldu = ((r + 7) / 8) * 8;
      ctx->stream = st[d];
      auto finish = [&]() -> rsd_status {
        DevBuf Vsel;
        RSD_TRY(Vsel.alloc(ctx, (size_t)k * ldu));
        RSD_TIMED_LAUNCH(ctx, "eig", (k_take_eigvecs<<<grid1d((int64_t)k * ldu), 256, 0, st[d]>>>(md.T.p, k, r,
                                                                                                   Vsel.p, ldu)));
        RSD_TRY(U[d].alloc(ctx, (size_t)n * ldu));
        GemmShape gu{};
        gu.split_stride = 0; gu.accumulate = 0; gu.tri = 0;
        gu.M = n; gu.N = r; gu.K = k; gu.kper = ((int64_t)k + TK - 1) / TK * TK; gu.C = U[d].p; gu.ldc = ldu;
        return gemm(ctx, "eig", OpKM{md.Z.p, n, n}, OpKM{Vsel.p, ldu, r}, gu, 1);
      };
      st_all = finish();
      ctx->stream = main;
      r_out[d] = r;
      ldu_out[d] = ldu;
      md.finished = true;
    }
  }
  // the context stream continues after the auxiliary streams' work
  (void)hipEventRecord(done[0], st[1]);
  (void)hipEventRecord(done[1], st[2]);
  (void)hipStreamWaitEvent(main, done[0], 0);
  (void)hipStreamWaitEvent(main, done[1], 0);
  if (st_all != RSD_OK) {
    (void)hipStreamSynchronize(st[1]);
    (void)hipStreamSynchronize(st[2]);
    return st_all;
  }
  for (int d = 0; d < 3; ++d)
    RSD_CHECK(m[d].finished, RSD_E_NUMERIC, "subspace iteration of mode %d did not settle", d);
  return RSD_OK;
}

}  // namespace

// Steps 4-5 shared by the build and the restriction to a sub-box: the Tucker core
// beta[(a*r2 + b)][c] = sum_col xi_col B1[col][a] B2[col][b] B3[col][c] (Bt_d = B_d^T, C columns),
// the slice SVDs, and the canonical factors F_d = U_d V_d written into t's chunked layout
// (mode d has t->nm[d] rows; rows beyond it, up to t->n, are zero).
rsd_status tucker_canonical(Context* ctx, Tensor* t, DevBuf Bt[3], DevBuf U[3], const int r[3], const int ldu[3],
                            const double* xi, int64_t C, rocblas_handle hb, rocblas_int* d_info) {
  hipStream_t s = ctx->stream;
  const double eps = t->sp.eps;
  const int n = t->n;
  const int M12 = r[0] * r[1];
  // output tiles (one column tile when r3 <= TNW, the wide kernel), and enough contraction
  // splits for about eight workgroups per compute unit
  const int tiles = div_up(M12, TM) * (r[2] <= TNW ? 1 : div_up(r[2], TN));
  const int csplit = std::max(1, std::min(64, div_up(2048, tiles)));
  DevBuf Cpart, beta;
  RSD_TRY(Cpart.alloc(ctx, (size_t)csplit * M12 * r[2]));
  RSD_TRY(beta.alloc(ctx, (size_t)M12 * r[2]));
  OpKhatriRao kr{Bt[0].p, Bt[1].p, ldu[0], ldu[1], r[1], M12, 0, 0};
  // the weights go into the mode-3 side matrix (each entry the same rounded product the
  // contraction would form), which is not read again
  RSD_TIMED_LAUNCH(ctx, "core", (k_scale_rows<<<grid1d(C * ldu[2]), 256, 0, s>>>(Bt[2].p, ldu[2], C, r[2], xi)));
  OpKM b3{Bt[2].p, ldu[2], r[2]};
  {
    GemmShape g{};
    g.M = M12; g.N = r[2]; g.K = C;
    g.kper = (int64_t)div_up(C, (int64_t)csplit * TK) * TK;
    g.C = Cpart.p; g.ldc = r[2]; g.split_stride = (int64_t)M12 * r[2]; g.accumulate = 0; g.tri = 0;
    RSD_TRY(gemm(ctx, "core", kr, b3, g, csplit));
    RSD_TIMED_LAUNCH(ctx, "core", (k_reduce_splits<<<grid1d((int64_t)M12 * r[2]), 256, 0, s>>>(
                                      Cpart.p, csplit, (int64_t)M12 * r[2], M12, r[2], r[2], beta.p, r[2])));
  }

  // 5. Tucker -> canonical: SVD of the mode-3 slices (r1 x r2, column-major)
  const int r1 = r[0], r2 = r[1], r3 = r[2];
  // 0 automatic: the QR-preconditioned Jacobi where its LDS fits, else the plain one, else rocSOLVER
  const size_t qr_lds = jacobi_qr_lds_doubles(r1, r2);
  const bool jacobi_qr = ctx->opt_t2c == 3 || (ctx->opt_t2c == 0 && qr_lds <= kJacobiQrMaxLds);
  const bool jacobi = jacobi_qr || ctx->opt_t2c == 1 || (ctx->opt_t2c == 0 && (int64_t)r1 * r2 <= kJacobiMaxElems);
  RSD_CHECK(!jacobi_qr || qr_lds <= kJacobiQrMaxLds, RSD_E_UNSUPPORTED, "core slice too large for LDS");
  RSD_CHECK(!jacobi || jacobi_qr || (int64_t)r1 * r2 <= kJacobiMaxElems, RSD_E_UNSUPPORTED,
            "core slice too large for LDS");
  const int ns = jacobi ? r2 : std::min(r1, r2);      // singular values per slice
  DevBuf S, Sv, Uv, Vv, Ev;
  RSD_TRY(S.alloc(ctx, (size_t)r1 * r2 * r3));
  RSD_TRY(Sv.alloc(ctx, (size_t)ns * r3));
  RSD_TRY(Uv.alloc(ctx, (size_t)r1 * ns * r3));
  RSD_TRY(Vv.alloc(ctx, (size_t)ns * r2 * r3));
  RSD_TRY(Ev.alloc(ctx, (size_t)ns * r3));
  RSD_TIMED_LAUNCH(ctx, "t2c", (k_core_slices<<<grid1d((int64_t)r1 * r2 * r3), 256, 0, s>>>(beta.p, r1, r2, r3,
                                                                                            r3, S.p)));
  RSD_CHECK(r3 <= 1024, RSD_E_UNSUPPORTED, "too many core slices");
  const double skip_rel2 = std::max(1e-3 * eps * 1e-3 * eps, 1e-30);
  if (jacobi_qr) {
    RSD_HIP(hipFuncSetAttribute((const void*)k_jacobi_svd_qr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(double) * qr_lds)));
    RSD_TIMED_LAUNCH(ctx, "t2c", (k_jacobi_svd_qr<<<r3, kJacobiThreads, sizeof(double) * qr_lds, s>>>(
                                     S.p, r1, r2, skip_rel2, Sv.p, Uv.p, Vv.p, (int*)d_info)));
  } else if (jacobi) {
    RSD_HIP(hipFuncSetAttribute((const void*)k_jacobi_svd<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(sizeof(double) * (size_t)r1 * r2)));
    RSD_TIMED_LAUNCH(ctx, "t2c", (k_jacobi_svd<false><<<r3, kJacobiThreads, sizeof(double) * (size_t)r1 * r2, s>>>(
                                     S.p, r1, r2, skip_rel2, Sv.p, Uv.p, Vv.p, (int*)d_info)));
  } else {
    KernelTimer kt;
    if (ctx->timing) RSD_TRY(ctx->timer_begin("t2c", &kt));
    rocblas_status rs = rocsolver_dgesvd_strided_batched(
        hb, rocblas_svect_singular, rocblas_svect_singular, r1, r2, S.p, r1, (rocblas_stride)r1 * r2, Sv.p,
        (rocblas_stride)ns, Uv.p, r1, (rocblas_stride)r1 * ns, Vv.p, ns, (rocblas_stride)ns * r2, Ev.p,
        (rocblas_stride)ns, rocblas_outofplace, d_info, r3);
    RSD_CHECK(rs == rocblas_status_success, RSD_E_HIP, "rocsolver_dgesvd_strided_batched failed (%d)", (int)rs);
    if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
  }
  // the kept terms, chosen and numbered on the device; the host reads R, the count of chunks
  // served from U_3 and the solver's status (Jacobi sweeps or gesvd info) in one copy
  const int total = ns * r3;
  DevBuf Pos, Sl, Out;
  RSD_TRY(Pos.alloc(ctx, (size_t)total));   // ints, in double-sized scratch
  RSD_TRY(Sl.alloc(ctx, (size_t)total));
  RSD_TRY(Out.alloc(ctx, 1));
  int* pos = (int*)Pos.p;
  int* sl = (int*)Sl.p;
  int* out2 = (int*)Out.p;
  RSD_TIMED_LAUNCH(ctx, "assemble", (k_t2c_select<<<1, kSelThreads, 0, s>>>(Sv.p, total, ns, eps, pos, sl, out2)));
  std::vector<int> info((size_t)r3 + 2);
  RSD_HIP(hipMemcpyAsync(info.data(), d_info, sizeof(int) * r3, hipMemcpyDeviceToHost, s));
  RSD_HIP(hipMemcpyAsync(info.data() + r3, out2, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  RSD_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < r3; ++c) {
    if (jacobi)
      RSD_CHECK(info[c] < kJacobiMaxSweeps, RSD_E_NUMERIC, "Jacobi SVD of core slice %d did not converge", c);
    else
      RSD_CHECK(info[c] == 0, RSD_E_NUMERIC, "slice SVD did not converge (info %d at %d)", info[c], c);
  }
  const int64_t R = info[r3];
  RSD_CHECK(R <= ((int64_t)1 << 20), RSD_E_UNSUPPORTED, "canonical rank %lld too large", (long long)R);
  RSD_TRY(alloc_factors(ctx, t, R));
  if (R == 0) return RSD_OK;
  // keep U_3 and the column -> slice map: the scoring kernels lerp a chunk's few distinct
  // mode-3 columns once per atom instead of gathering all of them
  t->u3_chunks = info[r3 + 1];
  RSD_TRY(ctx->dev_alloc((void**)&t->U3, sizeof(double) * (size_t)t->nm[2] * ldu[2]));
  RSD_TRY(ctx->dev_alloc((void**)&t->slice, sizeof(int) * (size_t)R));
  t->u3_ld = ldu[2];
  RSD_HIP(hipMemcpyAsync(t->U3, U[2].p, sizeof(double) * (size_t)t->nm[2] * ldu[2], hipMemcpyDeviceToDevice, s));
  RSD_HIP(hipMemcpyAsync(t->slice, sl, sizeof(int) * (size_t)R, hipMemcpyDeviceToDevice, s));
  // V_d (r_d x R): columns p = s*u (mode 1), v (mode 2), e_c (mode 3)
  DevBuf V[3];
  for (int d = 0; d < 3; ++d) RSD_TRY(V[d].alloc(ctx, (size_t)r[d] * R));
  RSD_TIMED_LAUNCH(ctx, "assemble", (k_t2c_factors<<<grid1d((int64_t)total * (r1 + r2 + r3)), 256, 0, s>>>(
                                        Sv.p, Uv.p, Vv.p, pos, total, ns, r1, r2, r3, R, V[0].p, V[1].p, V[2].p)));
  const int64_t mode = (int64_t)t->nchunk * n * kChunk;
  for (int d = 0; d < 3; ++d) {
    // F_d = U_d V_d on the matrix cores, written straight into the chunked layout: rows of the
    // layout beyond U_d's and columns beyond R come out zero (both operands are masked there).
    // Mode 3's V is one-hot, so its columns are U_3's columns exactly.
    GemmShape g{};
    g.M = n; g.N = t->nchunk * kChunk; g.K = r[d]; g.kper = (int64_t)div_up(r[d], TK) * TK;
    g.C = t->F + d * mode; g.ldc = kChunk; g.split_stride = 0; g.accumulate = 0; g.tri = 0; g.chunk_rows = n;
    RSD_TRY(gemm(ctx, "assemble", OpMK{U[d].p, ldu[d], t->nm[d]}, OpKM{V[d].p, R, (int)R}, g, 1));
  }
  return RSD_OK;
}

// Dominant left singular vectors of explicit rows x R matrices A_d (row-major, one per mode),
// with the singular values computed from A itself rather than from A A^T: the Gram matrix
// squares the spectrum, and at eps = 1e-8 its eigenvalue cut eps^2 lies at the rounding level
// of FP64, where the exactly low-rank modes of canonical factors (mode 3 of a factor set made
// by the canonical -> Tucker -> canonical step has only r3 distinct columns) pass noise as rank.
//   rows <= R and rows <= 96: B = A itself (Q = I): A^T = Q_b R_b (Householder QR of the
//     column-major R x rows view of A), the SVD of the rows x rows factor R_b, whose right
//     singular vectors are A's left ones.
//   otherwise a randomized range finder: Q = orth(A Omega) with k = 64 test vectors (128 above
//     1024 rows) and one power step Q <- orth(A (A^T Q)) (skipped when k = min(rows, R)
//     captures the range exactly), B = Q^T A, B^T = Q_b R_b, the SVD of R_b, U = Q V.  If
//     fewer than 16 of the k singular values fall below the cut and k < min(rows, R), k is
//     doubled and the mode is redone.
// The orthonormal bases come from the randomized Cholesky QR (orth_rchol; B^T's triangular
// factor is replaced by R' = Q_b^T B^T, which has the same singular values and right singular
// vectors), or, when a Cholesky pass loses rank or k > kSmallCols, from rocSOLVER's Householder
// QR.  Singular values >= eps * the largest are kept.  The three modes run on three streams (the
// context stream and two auxiliary ones with their own rocBLAS handles), since their QR and
// SVD calls are chains of short launches; the host synchronises once per pass to read the
// singular values.  U_d is rows_d x ldu_d, row-major, zero beyond column r_d.
__global__ void k_vt_rows(const double* __restrict__ VT, int k, int rows, int r, double* __restrict__ U, int ldu) {
  const int64_t total = (int64_t)rows * ldu;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ldu), a = (int)(e % ldu);
    U[e] = a < r ? VT[(int64_t)i * k + a] : 0.0;   // U[i][a] = V[i][a] = VT[a + i k]
  }
}

static rsd_status left_basis3(Context* ctx, rocblas_handle hb, double* const A[3], const int rows[3], int64_t R,
                              double eps, rocblas_int* d_info, DevBuf U[3], int r_out[3], int ldu_out[3]) {
  hipStream_t main = ctx->stream;
  RSD_TRY(ctx->aux_streams());
  hipStream_t st[3] = {main, ctx->aux_stream[0], ctx->aux_stream[1]};
  rocblas_handle hbs[3] = {hb, (rocblas_handle)ctx->aux_blas[0], (rocblas_handle)ctx->aux_blas[1]};
  hipEvent_t ready = nullptr, done[2] = {nullptr, nullptr};
  struct Events {
    hipEvent_t* e[3];
    ~Events() {
      for (auto* x : e)
        if (*x) (void)hipEventDestroy(*x);
    }
  } evguard{{&ready, &done[0], &done[1]}};
  RSD_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  RSD_HIP(hipEventCreateWithFlags(&done[0], hipEventDisableTiming));
  RSD_HIP(hipEventCreateWithFlags(&done[1], hipEventDisableTiming));
  RSD_HIP(hipEventRecord(ready, main));
  RSD_HIP(hipStreamWaitEvent(st[1], ready, 0));
  RSD_HIP(hipStreamWaitEvent(st[2], ready, 0));
  struct Mode {
    int k = 0, kmax = 0;
    bool direct = false, finished = false;
    bool lib = false;            // orthonormalize with rocSOLVER's Householder QR
    DevBuf Om, Y, W, Rb, Sv, VT, E, tau, Ul, Qa, Qb, flag, part, Vj, Sj;
    OrthBufs ob;
    double* q = nullptr;         // the range basis Q (rows x k column-major) of the last pass
  } m[3];
  RSD_TRY(allow_small_lds());
  for (int d = 0; d < 3; ++d) {
    m[d].kmax = (int)std::min<int64_t>(rows[d], R);
    m[d].direct = rows[d] <= R && rows[d] <= 96;
    m[d].k = m[d].kmax <= 96 ? m[d].kmax : std::min(m[d].kmax, rows[d] > 1024 ? 128 : 64);
  }
  struct StreamGuard {   // a mode's work is issued on its stream; the context stream comes back afterwards
    Context* c;
    hipStream_t saved;
    ~StreamGuard() { c->stream = saved; }
  } sg{ctx, main};
  const int solver_opt = ctx->opt_svd == 0 ? 4 : ctx->opt_svd;
  auto issue = [&](int d) -> rsd_status {
    Mode& md = m[d];
    const int k = md.k, nr = rows[d];
    const bool exact = k == md.kmax;
    hipStream_t s = st[d];
    md.lib = md.lib || ctx->opt_qr == 1 || k > kSmallCols;
    RSD_TRY(md.W.alloc(ctx, (size_t)R * k));
    RSD_TRY(md.Rb.alloc(ctx, (size_t)k * k));
    RSD_TRY(md.Sv.alloc(ctx, (size_t)k));
    RSD_TRY(md.VT.alloc(ctx, (size_t)k * k));
    RSD_TRY(md.E.alloc(ctx, (size_t)k));
    RSD_TRY(md.tau.alloc(ctx, (size_t)k));
    const int nmax = (int)std::max<int64_t>(nr, R);
    if (!md.lib) {
      // randomized Cholesky QR (orth_rchol): sketch matrix, two output panels, the pivot flag
      RSD_TRY(md.ob.alloc(ctx, nmax, k));
      RSD_TRY(md.Qa.alloc(ctx, (size_t)nmax * k));
      RSD_TRY(md.Qb.alloc(ctx, (size_t)nmax * k));
      RSD_TRY(md.flag.alloc(ctx, 1));
      const int sk_split = std::max(1, std::min(64, (int)(R / 64)));
      RSD_TRY(md.part.alloc(ctx, (size_t)sk_split * k * k));
      RSD_HIP(hipMemsetAsync(md.flag.p, 0, sizeof(double), s));
      RSD_TIMED_LAUNCH(ctx, "restrict", (k_random_fill<<<grid1d((int64_t)kSmallRows * nmax), 256, 0, s>>>(
                                            md.ob.theta.p, (int64_t)kSmallRows * nmax, 0x7E7Aull + (uint64_t)d)));
    }
    // an orthonormal basis of the columns of the mrows x k column-major panel X (k x mrows
    // row-major): in place with rocSOLVER, else into `out`; returns where the basis is
    auto orth = [&](double* X, int mrows, double* out, double** basis) -> rsd_status {
      if (!md.lib) {
        RSD_TRY(orth_rchol(ctx, X, k, mrows, md.ob, out, (int*)md.flag.p, 2, "qr"));
        *basis = out;
        return RSD_OK;
      }
      KernelTimer kt;
      if (ctx->timing) RSD_TRY(ctx->timer_begin("qr", &kt));
      RSD_CHECK(rocsolver_dgeqrf(hbs[d], mrows, k, X, (rocblas_int)mrows, md.tau.p) == rocblas_status_success,
                RSD_E_HIP, "rocsolver_dgeqrf failed");
      RSD_CHECK(rocsolver_dorgqr(hbs[d], mrows, k, k, X, (rocblas_int)mrows, md.tau.p) == rocblas_status_success,
                RSD_E_HIP, "rocsolver_dorgqr failed");
      if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
      *basis = X;
      return RSD_OK;
    };
    GemmShape g{};
    g.split_stride = 0; g.accumulate = 0; g.tri = 0;
    if (md.direct) {
      // B^T = A^T: the column-major R x rows view of A, copied (A is needed for the projection)
      RSD_HIP(hipMemcpyAsync(md.W.p, A[d], sizeof(double) * (size_t)R * nr, hipMemcpyDeviceToDevice, s));
    } else {
      RSD_TRY(md.Om.alloc(ctx, (size_t)R * k));
      RSD_TRY(md.Y.alloc(ctx, (size_t)nr * k));
      RSD_TIMED_LAUNCH(ctx, "restrict", (k_random_fill<<<grid1d(R * k), 256, 0, s>>>(md.Om.p, R * k,
                                                                                      0x5EEDull + (uint64_t)d)));
      // Y = A Omega as Y^T (k x rows row-major = rows x k column-major)
      g.M = k; g.N = nr; g.K = R; g.kper = (R + TK - 1) / TK * TK; g.C = md.Y.p; g.ldc = nr;
      RSD_TRY(gemm(ctx, "restrict", OpKM{md.Om.p, k, k}, OpMK{A[d], R, nr}, g, 1));
      double* q = nullptr;
      RSD_TRY(orth(md.Y.p, nr, md.Qa.p, &q));
      if (!exact) {
        // W = A^T Q (R x k row-major), then Y^T = W^T A^T and orthonormalise again
        g.M = (int)R; g.N = k; g.K = nr; g.kper = ((int64_t)nr + TK - 1) / TK * TK; g.C = md.W.p; g.ldc = k;
        RSD_TRY(gemm(ctx, "restrict", OpKM{A[d], R, (int)R}, OpMK{q, nr, k}, g, 1));
        g.M = k; g.N = nr; g.K = R; g.kper = (R + TK - 1) / TK * TK; g.C = md.Y.p; g.ldc = nr;
        RSD_TRY(gemm(ctx, "restrict", OpKM{md.W.p, k, k}, OpMK{A[d], R, nr}, g, 1));
        RSD_TRY(orth(md.Y.p, nr, md.Qa.p, &q));
      }
      md.q = q;
      // B^T = A^T Q as a column-major R x k matrix (k x R row-major)
      RSD_CHECK(div_up(R, TN) <= 65535, RSD_E_UNSUPPORTED, "too many columns (%lld) for the projection",
                (long long)R);
      g.M = k; g.N = (int)R; g.K = nr; g.kper = ((int64_t)nr + TK - 1) / TK * TK; g.C = md.W.p; g.ldc = R;
      RSD_TRY(gemm(ctx, "restrict", OpMK{q, nr, k}, OpKM{A[d], R, (int)R}, g, 1));
    }
    if (!md.lib) {
      // B^T = Q_b R' with Q_b orthonormal: R' = Q_b^T B^T (k x k) has B^T's singular values and
      // right singular vectors; it is formed transposed (row-major R'^T = column-major R'), the
      // layout the SVD below reads
      double* qb = nullptr;
      RSD_TRY(orth(md.W.p, (int)R, md.Qb.p, &qb));
      const int sk_split = std::max(1, std::min(64, (int)(R / 64)));
      RSD_TRY(gemm_split(ctx, OpMK{md.W.p, R, k}, OpMK{qb, R, k}, k, k, R, md.part.p, sk_split, md.Rb.p, "qr"));
    } else {
      RSD_CHECK(rocsolver_dgeqrf(hbs[d], (rocblas_int)R, k, md.W.p, (rocblas_int)R, md.tau.p) == rocblas_status_success,
                RSD_E_HIP, "rocsolver_dgeqrf failed");
      RSD_TIMED_LAUNCH(ctx, "restrict", (k_upper_copy<<<grid1d((int64_t)k * k), 256, 0, s>>>(md.W.p, R, k, md.Rb.p)));
    }
    KernelTimer kt;
    if (ctx->timing) RSD_TRY(ctx->timer_begin("svd", &kt));
    rocblas_status rs = rocblas_status_success;
    // the Jacobi kernel holds R' and its accumulated rotations in LDS: k <= 96
    const int solver = solver_opt == 4 && 2 * (int64_t)k * k > kJacobiMaxElems ? 3 : solver_opt;
    if (solver == 1) {
      rs = rocsolver_dgesvd(hbs[d], rocblas_svect_none, rocblas_svect_singular, k, k, md.Rb.p, k, md.Sv.p, nullptr, 1,
                            md.VT.p, k, md.E.p, rocblas_outofplace, d_info + d);
    } else if (solver == 2) {
      RSD_TRY(md.Ul.alloc(ctx, (size_t)k * k));
      rs = rocsolver_dgesdd(hbs[d], rocblas_svect_singular, rocblas_svect_singular, k, k, md.Rb.p, k, md.Sv.p,
                            md.Ul.p, k, md.VT.p, k, d_info + d);
    } else if (solver == 3) {
      rs = rocsolver_dgesvdj(hbs[d], rocblas_svect_none, rocblas_svect_singular, k, k, md.Rb.p, k, 0.0, md.E.p, 100,
                             d_info + 3 + d, md.Sv.p, nullptr, 1, md.VT.p, k, d_info + d);
    } else {
      // one-sided Jacobi in one workgroup (no host wait, so the three modes overlap), then sorted
      RSD_TRY(md.Ul.alloc(ctx, (size_t)k * k));
      RSD_TRY(md.Vj.alloc(ctx, (size_t)k * k));
      RSD_TRY(md.Sj.alloc(ctx, (size_t)k));
      RSD_HIP(hipFuncSetAttribute((const void*)k_jacobi_svd<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * 2 * (size_t)k * k)));
      const double skip_rel2 = std::max(1e-3 * eps * 1e-3 * eps, 1e-30);
      // (timed by the bracket around the whole solver)
      k_jacobi_svd<true><<<1, kJacobiThreads, sizeof(double) * 2 * (size_t)k * k, s>>>(
          md.Rb.p, k, k, skip_rel2, md.Sj.p, md.Ul.p, md.Vj.p, (int*)(d_info + 8 + d));
      RSD_HIP(hipGetLastError());
      k_svd_sort<<<1, 256, 0, s>>>(md.Sj.p, md.Vj.p, k, (const int*)(d_info + 8 + d), md.Sv.p, md.VT.p, d_info + d);
      RSD_HIP(hipGetLastError());
    }
    RSD_CHECK(rs == rocblas_status_success, RSD_E_HIP, "rocSOLVER SVD (%d) failed (%d)", solver, (int)rs);
    if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
    return RSD_OK;
  };
  auto finish = [&](int d, int r, int ldu) -> rsd_status {
    Mode& md = m[d];
    const int k = md.k, nr = rows[d];
    hipStream_t s = st[d];
    RSD_TRY(U[d].alloc(ctx, (size_t)nr * ldu));
    if (md.direct) {
      RSD_TIMED_LAUNCH(ctx, "restrict", (k_vt_rows<<<grid1d((int64_t)nr * ldu), 256, 0, s>>>(md.VT.p, k, nr, r,
                                                                                                U[d].p, ldu)));
    } else {
      RSD_HIP(hipMemsetAsync(U[d].p, 0, U[d].bytes, s));   // columns r .. ldu - 1 stay zero
      // U[i][a] = sum_j Q[i][j] V[j][a],  V[j][a] = VT[a + j k]
      GemmShape g{};
      g.split_stride = 0; g.accumulate = 0; g.tri = 0;
      g.M = nr; g.N = r; g.K = k; g.kper = ((int64_t)k + TK - 1) / TK * TK; g.C = U[d].p; g.ldc = ldu;
      RSD_TRY(gemm(ctx, "restrict", OpKM{md.q, nr, nr}, OpKM{md.VT.p, k, r}, g, 1));
    }
    return RSD_OK;
  };
  rsd_status st_all = RSD_OK;
  for (int pass = 0; pass < 8 && st_all == RSD_OK; ++pass) {
    bool any = false;
    for (int d = 0; d < 3 && st_all == RSD_OK; ++d) {
      if (m[d].finished) continue;
      any = true;
      ctx->stream = st[d];
      st_all = issue(d);
      ctx->stream = main;
    }
    if (!any || st_all != RSD_OK) break;
    for (int d = 0; d < 3 && st_all == RSD_OK; ++d) {
      Mode& md = m[d];
      if (md.finished) continue;
      const int k = md.k;
      std::vector<double> sv((size_t)k);
      rocblas_int info = 0;
      int bad = 0;
      hipError_t e = hipMemcpyAsync(&info, d_info + d, sizeof(info), hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess) e = hipMemcpyAsync(sv.data(), md.Sv.p, sizeof(double) * k, hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess && !md.lib) e = hipMemcpyAsync(&bad, md.flag.p, sizeof(int), hipMemcpyDeviceToHost, st[d]);
      if (e == hipSuccess) e = hipStreamSynchronize(st[d]);
      if (e != hipSuccess) {
        set_error("singular values: %s", hipGetErrorString(e));
        st_all = RSD_E_HIP;
        break;
      }
      if (bad) {   // a Cholesky pass lost rank (its SVD input is then meaningless): redo with Householder QR
        md.lib = true;
        continue;
      }
      if (info != 0) {
        set_error("SVD of mode %d did not converge (info %d)", d, (int)info);
        st_all = RSD_E_NUMERIC;
        break;
      }
      // rocSOLVER returns the singular values in decreasing order
      if (!(sv[0] > 0.0 && std::isfinite(sv[0]))) {
        set_error("factor matrix of mode %d has no positive singular value", d);
        st_all = RSD_E_NUMERIC;
        break;
      }
      int r = 0;
      while (r < k && sv[r] >= eps * sv[0]) ++r;
      if (r > k - 16 && k < md.kmax) {
        md.k = std::min(md.kmax, 2 * k);   // redo this mode with more test vectors on the next pass
        continue;
      }
      if (r < 1 || r > 1024) {
        set_error("mode-%d rank %d outside [1, 1024]", d, r);
        st_all = RSD_E_UNSUPPORTED;
        break;
      }
      const int ldu = ((r + 7) / 8) * 8;
      ctx->stream = st[d];
      st_all = finish(d, r, ldu);
      ctx->stream = main;
      r_out[d] = r;
      ldu_out[d] = ldu;
      md.finished = true;
    }
  }
  // the context stream continues after the auxiliary streams' work; the modes' buffers are
  // released on return, after every stream has finished with them
  (void)hipEventRecord(done[0], st[1]);
  (void)hipEventRecord(done[1], st[2]);
  (void)hipStreamWaitEvent(main, done[0], 0);
  (void)hipStreamWaitEvent(main, done[1], 0);
  for (int d = 0; d < 3; ++d) (void)hipStreamSynchronize(st[d]);
  RSD_TRY(st_all);
  for (int d = 0; d < 3; ++d)
    RSD_CHECK(m[d].finished, RSD_E_NUMERIC, "rank reduction of mode %d did not settle", d);
  return RSD_OK;
}

// Rank reduction of a canonical tensor given by explicit factors: the rows i_lo[d] ..
// i_lo[d] + t->nm[d] - 1 of the factors of src[0..nsrc-1], side by side (the sum of those
// canonical tensors), reduced by the same RHOSVD steps as the build.  With one source and a
// sub-box this is the restriction of scheme (C) in Sec. 3.3; with several sources on one grid
// it is the sum of their potentials (eq. 5.1) followed by the rank reduction (the
// add-and-compress of Algorithm TEP, step 4).  Steps: unit-norm columns with the products of
// the norms as weights, the Gram matrix of each mode (rows x rows), its eigenvectors above
// eps^2 times the largest eigenvalue (dense solver for small grids, the build's subspace
// iteration for large ones), the projection, then steps 4-5 (tucker_canonical).
rsd_status reduce_factors(Context* ctx, const Tensor* const* src, int nsrc, Tensor* t, const int i_lo[3]) {
  ScratchScope scope{ctx};
  int64_t R = 0;
  for (int k = 0; k < nsrc; ++k) R += src[k]->R;
  if (R == 0) return alloc_factors(ctx, t, 0);
  RSD_CHECK(R < ((int64_t)1 << 31), RSD_E_UNSUPPORTED, "too many columns (%lld) to reduce", (long long)R);
  hipStream_t s = ctx->stream;
  const double eps = t->sp.eps;
  if (!ctx->blas) {
    rocblas_handle hnew = nullptr;
    RSD_CHECK(rocblas_create_handle(&hnew) == rocblas_status_success, RSD_E_HIP, "rocblas_create_handle failed");
    ctx->blas = hnew;
  }
  rocblas_handle hb = (rocblas_handle)ctx->blas;
  RSD_CHECK(rocblas_set_stream(hb, s) == rocblas_status_success, RSD_E_HIP, "rocblas_set_stream failed");
  rocblas_int* d_info = nullptr;
  RSD_TRY(ctx->scratch_get((void**)&d_info, 4096));
  DevBuf A[3], nu[3], xi, U[3], Bt[3];
  for (int d = 0; d < 3; ++d) {
    const int rows = t->nm[d];
    RSD_TRY(A[d].alloc(ctx, (size_t)rows * R));
    RSD_TRY(nu[d].alloc(ctx, (size_t)R));
    int64_t col0 = 0;
    for (int k = 0; k < nsrc; ++k) {
      const Tensor* sk = src[k];
      if (sk->R == 0) continue;
      const int64_t sm = (int64_t)sk->nchunk * sk->n * kChunk;
      RSD_TIMED_LAUNCH(ctx, "restrict", (k_take_rows<<<grid1d((int64_t)rows * sk->R), 256, 0, s>>>(
                                            sk->F + d * sm, sk->n, sk->R, i_lo[d], rows, A[d].p, R, col0)));
      col0 += sk->R;
    }
    RSD_TIMED_LAUNCH(ctx, "restrict", (k_row_colnorms<<<grid1d(R), 256, 0, s>>>(A[d].p, rows, R, nu[d].p)));
  }
  RSD_TRY(xi.alloc(ctx, (size_t)R));
  RSD_TIMED_LAUNCH(ctx, "restrict", (k_local_weights<<<grid1d(R), 256, 0, s>>>(nu[0].p, nu[1].p, nu[2].p, R, xi.p)));
  for (int d = 0; d < 3; ++d)
    RSD_TIMED_LAUNCH(ctx, "restrict", (k_normalize_cols<<<grid1d((int64_t)t->nm[d] * R), 256, 0, s>>>(
                                          A[d].p, t->nm[d], R, nu[d].p, xi.p)));
  int r[3] = {0, 0, 0}, ldu[3] = {0, 0, 0};
  double* const Ap[3] = {A[0].p, A[1].p, A[2].p};
  RSD_TRY(left_basis3(ctx, hb, Ap, t->nm, R, eps, d_info, U, r, ldu));
  for (int d = 0; d < 3; ++d) {
    // B_d^T[p][a] = sum_i A[i][p] U[i][a]
    const int rows = t->nm[d];
    RSD_TRY(Bt[d].alloc(ctx, (size_t)R * ldu[d]));
    GemmShape gp{};
    gp.M = (int)R; gp.N = r[d]; gp.K = rows; gp.kper = ((rows + TK - 1) / TK) * TK;
    gp.C = Bt[d].p; gp.ldc = ldu[d]; gp.split_stride = 0; gp.accumulate = 0; gp.tri = 0;
    RSD_TRY(gemm(ctx, "restrict", OpKM{A[d].p, (int)R, (int)R}, OpKM{U[d].p, ldu[d], r[d]}, gp, 1));
  }
  t->ranks[0] = r[0];
  t->ranks[1] = r[1];
  t->ranks[2] = r[2];
  return tucker_canonical(ctx, t, Bt, U, r, ldu, xi.p, R, hb, d_info);
}

rsd_status build_factors(Context* ctx, Tensor* t, const double* d_z, const double* d_pos) {
  ScratchScope scope{ctx};
  const int n = t->n;
  const int K = t->sp.K_long;
  const int64_t N = t->N;
  const int64_t C = N * K;                    // columns of each side matrix
  const double eps = t->sp.eps;
  hipStream_t s = ctx->stream;
  RSD_CHECK(C < ((int64_t)1 << 30), RSD_E_UNSUPPORTED, "too many side-matrix columns (N*K_long)");
  if (C == 0) return alloc_factors(ctx, t, 0);

  // long-range nodes and weights
  double tk[kMaxTerms], wk[kMaxTerms];
  sinc_table(t->sp, tk, wk);
  std::vector<double> t2h((size_t)K), wh((size_t)K);
  for (int k = 0; k < K; ++k) {
    t2h[k] = tk[k] * tk[k];
    wh[k] = wk[k];
  }
  DevBuf t2d, wd;
  RSD_TRY(t2d.alloc(ctx, K));
  RSD_TRY(wd.alloc(ctx, K));
  RSD_HIP(hipMemcpyAsync(t2d.p, t2h.data(), sizeof(double) * K, hipMemcpyHostToDevice, s));
  RSD_HIP(hipMemcpyAsync(wd.p, wh.data(), sizeof(double) * K, hipMemcpyHostToDevice, s));

  if (!ctx->blas) {
    rocblas_handle hnew = nullptr;
    RSD_CHECK(rocblas_create_handle(&hnew) == rocblas_status_success, RSD_E_HIP, "rocblas_create_handle failed");
    ctx->blas = hnew;
  }
  rocblas_handle hb = (rocblas_handle)ctx->blas;
  RSD_CHECK(rocblas_set_stream(hb, s) == rocblas_status_success, RSD_E_HIP, "rocblas_set_stream failed");

  // Galerkin factors have no Toeplitz-times-Hankel Gram: they take the dense product
  const int gal = t->galerkin ? 1 : 0;
  const bool dense_gram = ctx->opt_gram == 2 || gal;
  // dense form: column chunks of the side matrix, at most ~1 GiB each
  const int64_t max_cols = std::max<int64_t>(TK, ((int64_t)1 << 27) / n / TK * TK);
  const int64_t chunk_cols = std::min<int64_t>(C, max_cols);
  DevBuf Abuf, nu[3], inv_nu[3], G3, Gpart, W3, E3, Ttab, Htab;
  for (int d = 0; d < 3; ++d) {
    RSD_TRY(nu[d].alloc(ctx, (size_t)C));
    RSD_TRY(inv_nu[d].alloc(ctx, (size_t)C));
  }
  const int64_t nn = (int64_t)n * n;
  RSD_TRY(G3.alloc(ctx, (size_t)(3 * nn)));
  const int Tn = div_up(n, TN);
  const int tri_tiles = Tn * (Tn + 1) / 2;
  const int gsplit = std::max(1, std::min(16, div_up(1024, tri_tiles)));
  if (dense_gram) {
    RSD_TRY(Abuf.alloc(ctx, (size_t)chunk_cols * n));
    RSD_TRY(Gpart.alloc(ctx, (size_t)gsplit * nn));
  } else {
    RSD_TRY(Ttab.alloc(ctx, (size_t)K * n));
    RSD_TRY(Htab.alloc(ctx, 3 * (size_t)K * (2 * (size_t)n - 1)));
  }
  RSD_TRY(W3.alloc(ctx, 3 * (size_t)n));
  RSD_TRY(E3.alloc(ctx, 3 * (size_t)n));
  rocblas_int* d_info = nullptr;
  RSD_TRY(ctx->scratch_get((void**)&d_info, 4096));

  int r[3] = {0, 0, 0};
  int ldu[3] = {0, 0, 0};
  DevBuf U[3], Bt[3];
  const double h = t->h, b = t->b;
  // 1. column norms and the Gram matrix of every mode, chunk by chunk
  if (!dense_gram)
    RSD_TIMED_LAUNCH(ctx, "gram", (k_gram_toeplitz<<<grid1d((int64_t)K * n), 256, 0, s>>>(t2d.p, K, n, h, Ttab.p)));
  if (!dense_gram) {
    // the modes are independent, and the Hankel sums of one mode fill only a few hundred
    // workgroups: the three run side by side
    RSD_TRY(on_three_streams(ctx, [&](int d, hipStream_t sd) -> rsd_status {
      RSD_TIMED_LAUNCH(ctx, "gen", (k_col_norms<<<div_up(C, 4), 256, 0, sd>>>(d_pos, t2d.p, K, d, n, b, h, 0, C,
                                                                                nu[d].p, inv_nu[d].p, gal)));
      double* Hd = Htab.p + (size_t)d * K * (2 * (size_t)n - 1);
      const dim3 gh((unsigned)div_up(2 * (int64_t)n - 1, 256), (unsigned)K);
      RSD_TIMED_LAUNCH(ctx, "gram", (k_gram_hankel<<<gh, 256, 0, sd>>>(d_pos, t2d.p, inv_nu[d].p, K, d, n, b, h, N,
                                                                       Hd)));
      const dim3 ga((unsigned)Tn, (unsigned)Tn);
      RSD_TIMED_LAUNCH(ctx, "gram", (k_gram_assemble<<<ga, 256, 0, sd>>>(Ttab.p, Hd, K, n, G3.p + d * nn)));
      return RSD_OK;
    }));
  }
  for (int d = 0; d < 3 && dense_gram; ++d) {
    RSD_TIMED_LAUNCH(ctx, "gen", (k_col_norms<<<div_up(C, 4), 256, 0, s>>>(d_pos, t2d.p, K, d, n, b, h, 0, C,
                                                                             nu[d].p, inv_nu[d].p, gal)));
    RSD_HIP(hipMemsetAsync(Gpart.p, 0, Gpart.bytes, s));
    for (int64_t c0 = 0; c0 < C; c0 += chunk_cols) {
      const int64_t c1 = std::min(C, c0 + chunk_cols);
      RSD_TIMED_LAUNCH(ctx, "gen", (k_gen_columns<<<grid1d((c1 - c0) * n), 256, 0, s>>>(
                                       d_pos, t2d.p, K, d, n, b, h, c0, c1, inv_nu[d].p, Abuf.p, gal)));
      OpKM op{Abuf.p, n, n};
      GemmShape g{};
      g.M = n; g.N = n; g.K = c1 - c0;
      g.kper = (int64_t)div_up(g.K, (int64_t)gsplit * TK) * TK;
      g.C = Gpart.p; g.ldc = n; g.split_stride = nn;
      g.accumulate = 1; g.tri = 1;
      RSD_TRY(gemm(ctx, "gram", op, op, g, gsplit));
    }
    RSD_TIMED_LAUNCH(ctx, "gram", (k_reduce_splits<<<grid1d(nn), 256, 0, s>>>(Gpart.p, gsplit, nn, n, n, n,
                                                                                G3.p + d * nn, n)));
  }
  // 2. eigenvectors: randomized subspace iteration (large n) or one batched dense call
  //    (row-major upper tiles = column-major lower triangle)
  const bool subspace = ctx->opt_eig == 2 || (ctx->opt_eig == 0 && n >= 1024);
  std::vector<double> lam3(3 * (size_t)n, 0.0);
  if (!subspace) {
    KernelTimer kt;
    if (ctx->timing) RSD_TRY(ctx->timer_begin("eig", &kt));
    rocblas_status rs = rocsolver_dsyevd_strided_batched(hb, rocblas_evect_original, rocblas_fill_lower, n, G3.p, n,
                                                         (rocblas_stride)nn, W3.p, (rocblas_stride)n, E3.p,
                                                         (rocblas_stride)n, d_info, 3);
    RSD_CHECK(rs == rocblas_status_success, RSD_E_HIP, "rocsolver_dsyevd_strided_batched failed (%d)", (int)rs);
    if (ctx->timing) RSD_TRY(ctx->timer_end(&kt));
    RSD_TRY(check_info(ctx, d_info, 3, "symmetric eigensolver"));
    RSD_HIP(hipMemcpy(lam3.data(), W3.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
  }
  if (subspace) RSD_TRY(subspace_eigvecs3(ctx, hb, G3.p, n, eps, d_info, U, r, ldu));
  for (int d = 0; d < 3 && !subspace; ++d) {
    {
      const double* lam = lam3.data() + (size_t)d * n;
      const double lmax = lam[n - 1];
      RSD_CHECK(lmax > 0.0 && std::isfinite(lmax), RSD_E_NUMERIC, "Gram matrix of mode %d has no positive eigenvalue",
                d);
      int rd = 0;
      for (int i = n - 1; i >= 0 && lam[i] >= eps * eps * lmax; --i) ++rd;
      RSD_CHECK(rd >= 1 && rd <= 1024, RSD_E_UNSUPPORTED, "mode-%d rank %d outside [1, 1024]", d, rd);
      r[d] = rd;
      ldu[d] = ((rd + 7) / 8) * 8;
      RSD_TRY(U[d].alloc(ctx, (size_t)n * ldu[d]));
      RSD_TIMED_LAUNCH(ctx, "eig", (k_take_eigvecs<<<grid1d((int64_t)n * ldu[d]), 256, 0, s>>>(G3.p + d * nn, n, rd,
                                                                                              U[d].p, ldu[d])));
    }
  }
  // 3. projections B_d^T[c][a] = sum_i A(i, c) U[i][a], side-matrix columns regenerated in LDS;
  //    the three modes side by side, so that the last wave of workgroups of one overlaps the next.
  //    The collocated Gaussians come by a recurrence when its ratio exp(-t^2 (8 h d + 16 h^2))
  //    stays within [e^-5, e^5] for every term and every offset |d| <= 2b in the box.
  double t2max = 0.0;
  for (double v : t2h) t2max = std::max(t2max, v);
  const bool rec = t2max * (8.0 * h * 2.0 * b + 16.0 * h * h) < 5.0;
  RSD_TRY(on_three_streams(ctx, [&](int d, hipStream_t) -> rsd_status {
    const int rd = r[d];
    RSD_TRY(Bt[d].alloc(ctx, (size_t)C * ldu[d]));
    auto project = [&](auto ga) -> rsd_status {
      ga.pos = d_pos; ga.t2 = t2d.p; ga.inv_nu = inv_nu[d].p; ga.K = K; ga.d = d; ga.n = n; ga.b = b; ga.h = h;
      ga.dim = (int)C;
      OpKM ub{U[d].p, ldu[d], rd};
      GemmShape g{};
      g.M = (int)C; g.N = rd; g.K = n; g.kper = ((n + TK - 1) / TK) * TK;
      g.C = Bt[d].p; g.ldc = ldu[d]; g.split_stride = 0; g.accumulate = 0; g.tri = 0;
      return gemm(ctx, "project", ga, ub, g, 1);
    };
    return gal ? project(OpGauss<true>{}) : rec ? project(OpGauss<false, true>{}) : project(OpGauss<false>{});
  }));
  t->ranks[0] = r[0];
  t->ranks[1] = r[1];
  t->ranks[2] = r[2];

  // 4. Tucker core beta[(a*r2 + b)][c] = sum_col xi_col B1[col][a] B2[col][b] B3[col][c]
  DevBuf xi;
  RSD_TRY(xi.alloc(ctx, (size_t)C));
  RSD_TIMED_LAUNCH(ctx, "core", (k_weights<<<grid1d(C), 256, 0, s>>>(d_z, wd.p, K, C, nu[0].p, nu[1].p, nu[2].p,
                                                                     xi.p)));
  return tucker_canonical(ctx, t, Bt, U, r, ldu, xi.p, C, hb, d_info);
}

}  // namespace rsd
