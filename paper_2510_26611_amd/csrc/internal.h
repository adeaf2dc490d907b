// Internal declarations of librsdock (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <array>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "rsdock.h"

namespace rsd {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define RSD_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t rsd_e_ = (call);                                                         \
    if (rsd_e_ != hipSuccess) {                                                         \
      ::rsd::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(rsd_e_),       \
                       __FILE__, __LINE__);                                             \
      return RSD_E_HIP;                                                                 \
    }                                                                                   \
  } while (0)

#define RSD_CHECK(cond, code, ...)     \
  do {                                 \
    if (!(cond)) {                     \
      ::rsd::set_error(__VA_ARGS__);   \
      return (code);                   \
    }                                  \
  } while (0)

#define RSD_TRY(expr)                  \
  do {                                 \
    rsd_status rsd_s_ = (expr);        \
    if (rsd_s_ != RSD_OK) return rsd_s_; \
  } while (0)

// ---------------------------------------------------------------- layout constants
// Factor matrices are stored column-chunked: for mode d and chunk c the block
// F[d][c] is an n x kChunk row-major array (row i at offset i*kChunk), so the
// kChunk doubles of one row are one contiguous 512-byte segment and rows i and
// i+1 of a chunk are adjacent.  Columns beyond R are zero.
constexpr int kChunk = 64;
constexpr int kPolyCoef = 8;       // coefficients per interval of the short-range polynomial table
constexpr int kMaxTerms = 64;   // M + 1 <= 64
constexpr int kMaxLigand = 896;   // keeps one wave's LDS within 64 KB

struct ShortTable {            // short-range Gaussians (terms k >= K_long)
  int S;
  double t2[kMaxTerms];        // t_k^2
  double w[kMaxTerms];         // folded weights
};

struct CellGrid {              // uniform cells over the box [-b, b]^3, x fastest
  double origin;               // -b (same on every axis)
  double edge;
  double inv_edge;
  int dim;                     // cells per axis
  int ncells;                  // dim^3
};

// ---------------------------------------------------------------- context
struct KernelTimer {
  std::string name;
  hipEvent_t start, stop;
};

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;           // 0 = unlimited
  size_t in_use = 0;
  // growable scratch owned by the context
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* blas = nullptr;        // rocblas_handle for the eigen/SVD steps of the build (lazy)
  // two more streams (default priority) and their rocblas handles: the build runs the three
  // modes' eigensolvers concurrently on the context stream and these (lazy)
  hipStream_t aux_stream[2] = {nullptr, nullptr};
  void* aux_blas[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // scoring: short range on aux_stream[0] (lazy)
  int live_tensors = 0;        // tensors made with this context and not yet freed
  bool closing = false;        // rsd_context_free was called; released with the last tensor
  // tuning options (rsd_context_set_option)
  int opt_score_mode = 0;      // 0 auto, 1 fused per-pose kernel, 2 chunk-major long-range kernel
  int opt_poses_per_wave = 0;  // chunk-major kernel: poses per wavefront (0 = automatic)
  int opt_t2c = 0;             // core slice SVDs: 0 auto, 1 Jacobi in LDS, 2 rocSOLVER, 3 QR then Jacobi
  int opt_eig = 0;             // Gram eigenvectors: 0 auto, 1 dense batched eigensolver, 2 subspace iteration
  int opt_qr = 0;              // subspace-iteration bases: 0 auto (randomized Cholesky QR, k <= 128), 1 rocSOLVER QR
  int opt_cpi = 0;             // rank chunks per long-range work item: 0 auto (2), 1..4
  int opt_svd = 0;             // small SVD of explicit-factor rank reduction: 0 auto, 1 gesvd, 2 gesdd, 3 Jacobi
  int opt_factors = 0;         // build factors: bit 0 Galerkin cell averages (else collocation at the
                               // nodes), bit 1 charges snapped to their nearest nodes (eq. 2.5)
  int opt_gram = 0;            // Gram matrices: 0 auto, 1 Toeplitz x Hankel form, 2 dense matrix-core product
  int opt_short_waves = 0;     // short-range kernel: wavefronts per workgroup (0 = automatic)
  int opt_use_tuning = 1;      // apply shapes recorded by rsd_autotune to automatic calls
  int opt_overlap = 0;         // chunk-major scoring: short range on a second stream beside the long range
  int opt_batch_mode = 0;      // batches: 0 automatic (grouped), 1 grouped launches, 2 one persistent launch
  int opt_pose_order = 0;      // chunk-major scoring: poses in spatial order (0 automatic, 1 always, 2 never)
  int opt_short_poly = 1;      // tensors made with this context carry the short-range polynomial table
  int opt_shared_mode3 = 1;    // chunk-major scoring lerps a chunk's distinct U_3 columns once per atom
  // launch shapes recorded by rsd_autotune: (n, nchunk, N, L, grad) -> (mode, ppw, short waves)
  std::map<std::tuple<int, int, int64_t, int, int>, std::array<int, 3>> tuned;
  bool timing = false;
  std::vector<KernelTimer> pending;
  std::map<std::string, std::pair<int64_t, double>> ktime;

  // Released batch scratch kept for reuse.  A cached block is handed only to later work on
  // this context's stream, which stream order makes safe (set_stream drains the old stream
  // first), so releasing needs no device-wide wait as hipFree would.  Cached blocks count as
  // in use and are freed when an allocation would exceed the budget or fail.
  std::vector<std::pair<void*, size_t>> block_cache;

  // Scratch of the tensor builds and rank reductions (dozens of buffers per call).  Blocks
  // handed out by scratch_get stay with the call until scratch_end, which waits for the
  // context stream once and keeps them for the next call: no allocation, free or wait
  // inside the call.  Cached blocks count as in use and go when the budget needs room.
  std::vector<std::pair<void*, size_t>> scratch_cache, scratch_live;

  // short-range polynomial tables by (M, K_long, h_M, L_s, r_cut), shared by the tensors
  struct Poly {
    double* p = nullptr;
    size_t bytes = 0;
    int n1 = 0;
    double x1 = 0.0, inv_d1 = 0.0, inv_d2 = 0.0;
  };
  std::map<std::tuple<int, int, double, double, double>, Poly> poly_cache;

  rsd_status dev_alloc(void** p, size_t bytes);
  void dev_free(void* p, size_t bytes);
  rsd_status block_alloc(void** p, size_t* bytes);   // in: bytes wanted; out: size of the block handed out
  void block_release(void* p, size_t bytes);
  void block_trim();
  rsd_status scratch_get(void** p, size_t bytes);
  void scratch_end();
  rsd_status workspace(size_t bytes, void** out);
  rsd_status aux_streams();
  rsd_status timer_begin(const char* name, KernelTimer* t);
  rsd_status timer_end(KernelTimer* t);
  rsd_status collect_timers();
};

// RAII-free helper to bracket a kernel launch with timing events.
#define RSD_TIMED_LAUNCH(ctx, name, launch)                        \
  do {                                                             \
    ::rsd::KernelTimer rsd_kt_;                                    \
    if ((ctx)->timing) RSD_TRY((ctx)->timer_begin((name), &rsd_kt_)); \
    launch;                                                        \
    RSD_HIP(hipGetLastError());                                    \
    if ((ctx)->timing) RSD_TRY((ctx)->timer_end(&rsd_kt_));        \
  } while (0)

// ---------------------------------------------------------------- tensor
struct Tensor {
  Context* ctx = nullptr;
  int n = 0;                   // factor rows in the layout (the largest of nm[])
  double b = 0, h = 0, X0 = 0, inv_h = 0;
  // per-mode grid: origin and row count (all X0 and n, except for a tensor restricted to a
  // sub-box, whose modes start at different nodes and may have different lengths)
  double X0m[3] = {0, 0, 0};
  int nm[3] = {0, 0, 0};
  bool restricted = false;
  bool galerkin = false;       // built from cell-average (Galerkin) factors
  bool snapped = false;        // long-range factors of the charges moved to their nearest nodes
  int64_t R = 0;
  int nchunk = 0;              // ceil(R / kChunk); the kernels handle nchunk == 0
  int ranks[3] = {0, 0, 0};
  rsd_sinc_params sp{};
  double* F = nullptr;         // 3 * nchunk * n * kChunk doubles
  size_t F_bytes = 0;
  int64_t N = 0;
  double4* atoms = nullptr;    // cell-sorted (x, y, z, charge)
  int* cell_start = nullptr;   // ncells + 1
  size_t cell_bytes = 0;
  CellGrid cells{};
  int cell_div = 0;            // cell edge r_cut / cell_div (0: 4), chosen by the cell tuner
  double* short_tab = nullptr; // device copy of ShortTable t2[], w[] (2 * kMaxTerms)
  ShortTable shrt{};
  // made by the canonical -> Tucker -> canonical step: column p of F_3 is column slice[p] of
  // U_3 (nm[2] rows, leading dimension u3_ld); null for imported or loaded tensors
  double* U3 = nullptr;
  int* slice = nullptr;
  int u3_ld = 0;
  int u3_chunks = 0;           // rank chunks whose columns use at most kSlots columns of U_3
  // the short-range kernel g(x) = sum_k w_k exp(-t_k^2 x) as piecewise polynomials in x = d^2
  // (kPolyCoef monomial coefficients per interval on [-1, 1]); owned by the context's cache,
  // null when not built
  double* short_poly = nullptr;
  int poly_n1 = 0;             // intervals of width poly_d1 on [0, poly_x1), then of width poly_d2
  double poly_x1 = 0.0, poly_inv_d1 = 0.0, poly_inv_d2 = 0.0;
  std::vector<double> host_charges;    // kept for save/load
  std::vector<double> host_positions;
  size_t bytes() const;
};

// sinc table (host): t_k and folded w_k, k = 0..M
void sinc_table(const rsd_sinc_params& sp, double* t, double* w);

// host-side argument checks and tables (api.hip), also exercised by the sanitizer build
rsd_status check_sinc(const rsd_sinc_params* sp);
rsd_status check_grid(int32_t n, double b);
rsd_status check_protein(const std::vector<double>& z, const std::vector<double>& pos, int32_t n, double b);
bool build_short_poly(const ShortTable& st, double rc2, std::vector<double>* coef, int* n1, double* x1,
                      double* d1, double* d2);

// grid constants with the fixed operation order shared by every component
inline void grid_constants(int n, double b, double* h, double* X0, double* inv_h) {
  *h = (2.0 * b) / (double)n;
  *X0 = -b + *h;
  *inv_h = 1.0 / *h;
}

// ---------------------------------------------------------------- launchers (device work)
rsd_status build_cells(Context* ctx, Tensor* t, const double* d_charges, const double* d_positions);
// the tensor's cell list again with edge r_cut / div (cells.hip)
rsd_status rebuild_cells(Context* ctx, Tensor* t, int div);

struct ScoreIO {
  const double* lig_charges;   // device
  const double* lig_positions; // device
  int L;
  const double* quats;         // device
  const double* trans;         // device
  int64_t P;
  double vdw_min;
  double* E;
  double* El;                  // may be null
  uint8_t* flags;
  int32_t* counts;
  double* grads;               // may be null
};
// Enqueues the scoring of io.P poses.  Scratch comes from the context's growable workspace, or
// from ext_ws (ext_bytes long, RSD_E_UNSUPPORTED if too small) when given; with need != nullptr
// nothing is launched and *need receives the scratch bytes the call would use.
rsd_status launch_score(Context* ctx, const Tensor* t, const ScoreIO& io, void* ext_ws = nullptr,
                        size_t ext_bytes = 0, size_t* need = nullptr);
// rsd_score_poses_noalloc (score.hip): launch_score over pose slices whose scratch fits the
// library's static per-device array; no device memory is allocated.
rsd_status score_noalloc(Context* ctx, const Tensor* t, const ScoreIO& io);
// Looks up (once per device, with that device current) the device address of the static
// scratch array of score_noalloc.
rsd_status noalloc_scratch_init(int device);
// rsd_probe_gather (score.hip): time the long-range kernel's gather pattern alone
rsd_status probe_gather(Context* ctx, int n, int iters, double* ms, double* bytes);
constexpr int kSharedSlots = 4;   // distinct U_3 columns a chunk may use to take mode 3 from LDS
// rsd_pose_order (score.hip): the spatial order of the long-range kernels and the poses in it;
// *sorted: whether automatic scoring of t sorts poses itself
rsd_status pose_order(Context* ctx, const Tensor* t, const double* quats, const double* trans, int64_t P, int* perm,
                      double* q_out, double* t_out, int* sorted);
rsd_status autotune(Context* ctx, const Tensor* t, const ScoreIO& io, rsd_tune_report* rep);
// rsd_autotune_cells (score.hip): times scoring with cell edges r_cut / {3, 4, 5, 6}, keeps the fastest
rsd_status autotune_cells(Context* ctx, Tensor* t, const ScoreIO& io, int32_t* best_div, double* ms);
// a molecule's own energy (score.hip)
rsd_status launch_self_energy(Context* ctx, const Tensor* t, double* E_long, double* E_short);
// posing search (score.hip)
rsd_status launch_contact(Context* ctx, const Tensor* t, const double* lig_positions, int L, const double* dirs,
                          int64_t U, const double* quats, int64_t Q, const double xP[3], double sigma, double gap,
                          double* rho, double* pose_q, double* pose_t);
rsd_status launch_orbit_minima(Context* ctx, const double* E, const uint8_t* flags, int64_t U, int64_t Q,
                               const int32_t* off, const int32_t* idx, int32_t* best_q, double* best_e,
                               uint8_t* is_min);

// many requests per launch (score.hip)
struct Batch;
rsd_status batch_create(Context* ctx, const rsd_request* req, int32_t nreq, Batch** out);
rsd_status batch_run(Batch* b);
void batch_free(Batch* b);

// factor storage of a tensor with canonical rank R (api.hip)
rsd_status alloc_factors(Context* ctx, Tensor* t, int64_t R);
// rank reduction on the device (build.hip)
rsd_status build_factors(Context* ctx, Tensor* t, const double* d_charges, const double* d_positions);
rsd_status reduce_factors(Context* ctx, const Tensor* const* src, int nsrc, Tensor* t, const int i_lo[3]);

}  // namespace rsd

struct rsd_context : rsd::Context {};
struct rsd_tensor : rsd::Tensor {};
