/*
 * rsdock.h -- C ABI of librsdock, an MI355X (gfx950) library that scores rigid
 * protein-ligand poses by the electrostatic binding energy computed from the
 * range-separated (RS) tensor representation of the protein potential.
 *
 * Method: Benner, Khoromskij, Khoromskaia, Stein, "Fast tensor-based electrostatic
 * energy calculations in the perspective of protein-ligand docking problem",
 * arXiv 2510.26611.
 *   - Algorithm TEP (Sec. 3.4): the long-range part of the protein potential as a
 *     rank-R canonical tensor on an n x n x n grid, rank-reduced by
 *     canonical -> Tucker (RHOSVD) -> canonical          -> rsd_build_rs_tensor
 *   - Algorithm PLIE (Sec. 3.4) with Lemma 3.3 (eq. 3.10): per-pose binding energy
 *     E = sum_l zeta_l P(y_l), plus the short-range part of the RS format
 *     (Def. 2.1) and the van der Waals constraint of eq. 3.14  -> rsd_score_poses
 *
 * Units: Angstrom, elementary charge, Coulomb constant 1 (energies in e^2/A).
 * Floating point is IEEE FP64 throughout.
 *
 * Memory.  Unless a call's mem_flags holds RSD_DEVICE_PTRS, every array argument
 * is a host pointer: the call copies inputs in, runs, copies outputs back and
 * returns when the outputs are written.  With RSD_DEVICE_PTRS every array
 * argument is a device pointer on the context's device; the call enqueues its
 * work on the context's stream and returns before completion (outputs are valid
 * after the stream has been synchronised).  The caller owns every argument
 * array; the library owns tensors until rsd_tensor_free.
 *
 * Errors.  Every call returns rsd_status; on failure nothing is written to the
 * outputs and rsd_last_error() (thread-local) describes the cause.
 * Per-pose geometry is not an error: see RSD_FLAG_*.
 *
 * Threads.  A context and the tensors made with it may be used from one host
 * thread at a time.  A tensor may be scored through any context on its device (for
 * example one context per stream); it must outlive every call and batch that uses it.
 */
#ifndef RSDOCK_H
#define RSDOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSD_OK = 0,
  RSD_E_INVALID = -1,     /* bad argument (null pointer, size, non-finite input, ...) */
  RSD_E_OOM = -2,         /* device allocation failed or the context's HBM budget is exceeded */
  RSD_E_HIP = -3,         /* a HIP runtime call failed */
  RSD_E_NUMERIC = -4,     /* the rank reduction did not converge */
  RSD_E_UNSUPPORTED = -5, /* a size, or a combination of inputs, the library does not support */
  RSD_E_IO = -6           /* file could not be read or written, or is not a tensor file */
} rsd_status;

/* mem_flags bits */
#define RSD_DEVICE_PTRS 1u

/* per-pose flag bits written by rsd_score_poses */
#define RSD_FLAG_ACCEPT 1u     /* in the grid and min over atom pairs of d^2 >= vdw_min^2 (eq. 3.14) */
#define RSD_FLAG_IN_DOMAIN 2u  /* every ligand atom inside the grid's node range */
#define RSD_FLAG_INVALID 4u    /* non-finite pose input or | |q|^2 - 1 | > 1e-12 */

typedef struct rsd_context rsd_context;
typedef struct rsd_tensor rsd_tensor;

/* Sinc-quadrature Gaussian sum for 1/r (Sec. 2, eq. 2.2) and its range separation (eq. 2.4).
 * Nodes t_k = sinh(k h_M)/L_s, weights w_0 = a_0, w_k = 2 a_k with
 * a_k = h_M cosh(k h_M)/(sqrt(pi) L_s), k = 0..M (the +-k terms folded, widest first).
 * Terms k < K_long are long-range (held in the tensor), k >= K_long short-range
 * (summed exactly over protein atoms with d^2 < r_cut^2).  eps is the relative
 * truncation of the rank reduction (singular values below eps * largest are dropped). */
typedef struct {
  int32_t M;       /* 0 <= M <= 63 */
  int32_t K_long;  /* 0 <= K_long <= M+1 */
  double h_M;      /* > 0 */
  double L_s;      /* > 0, Angstrom */
  double r_cut;    /* >= 0, Angstrom */
  double eps;      /* 0 <= eps < 1 */
} rsd_sinc_params;

/* Library version (major, minor). */
rsd_status rsd_version(int32_t* major, int32_t* minor);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* rsd_last_error(void);

/* Context: device id, the hipStream_t all work is enqueued on (NULL = the null
 * stream; the caller keeps ownership of the stream) and an HBM budget in bytes
 * for resident tensors plus library workspace (0 = no limit beyond the device). */
rsd_status rsd_context_create(int32_t device, void* hip_stream, size_t hbm_budget_bytes,
                              rsd_context** out);
rsd_status rsd_context_set_stream(rsd_context* ctx, void* hip_stream);
/* Bytes currently held by the context (tensors + workspace). */
rsd_status rsd_context_memory(const rsd_context* ctx, size_t* bytes_in_use, size_t* budget);
/* Free a context.  If tensors made with it are still alive the context stops accepting
 * work and is released together with the last of them (rsd_tensor_free). */
void rsd_context_free(rsd_context* ctx);

/* Build the RS tensor of a protein (Algorithm TEP).
 *   charges   [N]     protein charges z_m
 *   positions [N*3]   protein atom coordinates (x, y, z) per atom, row-major; every
 *                     coordinate must lie in the node range [-b + 2b/n, b]
 *   n         grid points per axis, even, 4 <= n <= 32768; mesh h = 2b/n; nodes
 *             X_j = -b + (j+1) h, j = 0..n-1 (Sec. 2, eq. 2.1, origin at node n/2)
 *   b         half-width of the box [-b, b]^3, > 0
 *   sp        quadrature, range split, cutoff and truncation (see rsd_sinc_params)
 * Steps: long-range factor columns exp(-t_k^2 (X_j - x_{m,d})^2) collocated at the true
 * atom positions (eq. 2.6); per mode the Gram matrix of the column-normalised factor
 * matrix on FP64 matrix cores, its dominant eigenvectors, projection, Tucker core,
 * and slice-wise SVD of the core into canonical terms (TEP step 4); and a cell list of
 * the protein atoms for the short-range sum.  Synchronous: returns when the tensor
 * is resident.  Errors: RSD_E_INVALID (sizes, non-finite or out-of-box input),
 * RSD_E_OOM, RSD_E_NUMERIC, RSD_E_HIP. */
rsd_status rsd_build_rs_tensor(rsd_context* ctx, const double* charges, const double* positions,
                               int64_t N, int32_t n, double b, const rsd_sinc_params* sp,
                               uint32_t mem_flags, rsd_tensor** out);

/* Make a resident tensor from given canonical factors (e.g. ones built elsewhere).
 *   F1, F2, F3 [n*R]  factor matrices, row-major n x R (entry (i, p) at i*R + p); the
 *                     tensor is sum_p F1[:,p] (x) F2[:,p] (x) F3[:,p] (weights folded in)
 *   R >= 0; charges/positions/N as in rsd_build_rs_tensor (for the short-range part).
 * Synchronous. */
rsd_status rsd_tensor_import(rsd_context* ctx, const double* F1, const double* F2, const double* F3,
                             int64_t R, int32_t n, double b, const rsd_sinc_params* sp,
                             const double* charges, const double* positions, int64_t N,
                             uint32_t mem_flags, rsd_tensor** out);

/* Score P poses of a rigid ligand (Algorithm PLIE, Lemma 3.3 with the short-range
 * term of Def. 2.1, and the constraint of eq. 3.14).
 *   lig_charges   [L]    ligand charges zeta_l
 *   lig_positions [L*3]  ligand atom coordinates in its own frame; the pose rotates
 *                        them about their geometric centre c = (sum_l x_l)/L
 *   quats [P*4]  unit quaternions (w, x, y, z), used as given (q and -q score the same)
 *   trans [P*3]  position of the ligand centre: y_l = R(q)(x_l - c) + t
 *   vdw_min      van der Waals distance sigma >= 0
 * Outputs (caller-allocated, P entries each):
 *   energies       E = sum_l zeta_l (P_long(y_l) + P_short(y_l)); NaN unless in domain
 *   energies_long  sum_l zeta_l P_long(y_l) (may be NULL)
 *   flags          RSD_FLAG_* bits
 *   counts         number of (ligand, protein) atom pairs with d^2 < r_cut^2
 *   grads [P*6]    (dE/dt, dE/domega): translation gradient and the derivative with
 *                  respect to a rotation vector omega applied as q' = quat(omega) q about
 *                  the centre (the rigid-body force reduction of Sec. 5.2); may be NULL
 * Long-range values are the trilinear interpolant of the tensor: per mode, the two
 * factor rows around the point are linearly interpolated; the gradient is the exact
 * derivative of that interpolant (the one-sided difference of eq. 3.12 inside the cell).
 * Limits: 1 <= L <= 896.  P = 0 is a no-op.  Errors: RSD_E_INVALID (with host
 * pointers also for an invalid pose), RSD_E_UNSUPPORTED, RSD_E_OOM, RSD_E_HIP. */
rsd_status rsd_score_poses(rsd_context* ctx, const rsd_tensor* tensor,
                           const double* lig_charges, const double* lig_positions, int64_t L,
                           const double* quats, const double* trans, int64_t P, double vdw_min,
                           uint32_t mem_flags, double* energies, double* energies_long,
                           uint8_t* flags, int32_t* counts, double* grads);

/* rsd_score_poses for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * validation as rsd_score_poses with RSD_DEVICE_PTRS (mem_flags must hold it: host arrays
 * would need staging memory, RSD_E_INVALID otherwise).  The call allocates nothing: its
 * scratch (ligand frame, short-range partial sums, per-chunk long-range partials, the pose
 * sort) lives in one static 128 MiB array per GPU that the library holds from its first use
 * on that GPU until the process ends.  The poses are scored in equal slices whose scratch
 * fits the array (each pose's result does not depend on the slicing); a call whose single
 * pose would not fit returns RSD_E_UNSUPPORTED.  Enqueues on the context stream and returns
 * before completion; the context's timing option is ignored, and the short range always runs
 * on the context stream (option overlap ignored).  Every call on one GPU shares its array:
 * calls that can overlap on one GPU (contexts on different streams) race and must be ordered
 * by the caller.  Errors: as rsd_score_poses. */
rsd_status rsd_score_poses_noalloc(rsd_context* ctx, const rsd_tensor* tensor,
                                   const double* lig_charges, const double* lig_positions, int64_t L,
                                   const double* quats, const double* trans, int64_t P, double vdw_min,
                                   uint32_t mem_flags, double* energies, double* energies_long,
                                   uint8_t* flags, int32_t* counts, double* grads);

/* Many requests per launch.  A request is one rsd_score_poses call with device pointers
 * and no gradients; the tensors may differ between requests but belong to one context.
 * rsd_batch_create validates the requests, allocates the batch's device scratch (per-request
 * ligand frames, short-range energies, long-range partials) and enqueues the upload of a
 * request table on the context stream (it returns without waiting for the device).  rsd_batch_run enqueues the launches on the context stream that score
 * every request (ligand frames; short-range, vdW and counts; long-range in rank-chunk-major
 * order over all requests; combine), grouped by LDS occupancy or as one persistent launch
 * (option batch_mode); it allocates nothing and does not synchronise, so it
 * may be captured in a HIP graph and replayed.  The request arrays are read at run time:
 * new poses written into the same buffers are scored by the next run.  Each pose scores
 * bit for bit as in rsd_score_poses with option score_mode = 2.  The tensors may come from
 * any context on the same device and must stay alive until the batch is freed.
 * Errors: RSD_E_INVALID, RSD_E_UNSUPPORTED (sizes), RSD_E_OOM, RSD_E_HIP. */
typedef struct {
  const rsd_tensor* tensor;
  const double* lig_charges;    /* [L] */
  const double* lig_positions;  /* [L*3] */
  int64_t L;
  const double* quats;          /* [P*4] */
  const double* trans;          /* [P*3] */
  int64_t P;                    /* >= 0 */
  double vdw_min;
  double* energies;             /* [P] */
  double* energies_long;        /* [P] or NULL */
  uint8_t* flags;               /* [P] */
  int32_t* counts;              /* [P] */
} rsd_request;

typedef struct rsd_batch rsd_batch;
rsd_status rsd_batch_create(rsd_context* ctx, const rsd_request* requests, int32_t n_requests, rsd_batch** out);
rsd_status rsd_batch_run(rsd_batch* batch);
void rsd_batch_free(rsd_batch* batch);

/* The long-range tensor restricted to a sub-box and rank-reduced (Sec. 3.3, scheme (C), the
 * hybrid: the global tensor is computed once and its rank is reduced separately in each box
 * that accompanies the ligand; Table 3.1 shows ranks far below the global ones).
 * The new tensor keeps the grid rows of `src` that trilinear evaluation inside the box
 * [lo, hi] (Angstrom, per axis) can reach: rows floor((lo_d - X0)/h) .. floor((hi_d - X0)/h) + 1
 * of mode d, clipped to the grid, so its modes have their own origin and row count (see
 * rsd_tensor_grid) and the same mesh h.  The restricted canonical tensor is exact there; its
 * rank is then reduced by the build's RHOSVD steps at relative accuracy `eps` (explicit
 * unit-norm factor columns, weights = products of the column norms).  The protein atoms,
 * cell list and short-range table are copied, so scoring works as with any tensor; poses
 * with an atom outside the kept rows are flagged out of domain.  The result belongs to
 * `ctx` and is independent of `src` (which may be freed).  Restricted tensors cannot be
 * saved.  Errors: RSD_E_INVALID for a NULL argument, lo >= hi, non-finite bounds, a box that
 * misses the grid, or eps outside (0, 1); RSD_E_OOM beyond the budget. */
rsd_status rsd_tensor_restrict(rsd_context* ctx, const rsd_tensor* src, const double lo[3], const double hi[3],
                               double eps, rsd_tensor** out);

/* The potential of a complex of molecules M_1..M_m (eq. 5.1: a molecule of the complex, or a
 * ligand, is scored against the sum of the other molecules' potentials), built by the
 * add-and-compress of Algorithm TEP, step 4: the canonical factors of `count` tensors on one
 * grid are put side by side (the canonical tensor of the sum has all their terms) and that
 * sum's rank is reduced by the build's RHOSVD steps at relative accuracy `eps`, exactly as in
 * rsd_tensor_restrict.  The short-range part and the van der Waals test use the union of the
 * molecules' atoms (the sources' atoms in order).  The long-range error is at most the sum of
 * the sources' errors plus the truncation at eps.  The same call builds one large molecule in
 * pieces (rsd_build_rs_tensor on chunks of its atoms, then one combine).
 * Requirements: 1 <= count <= 4096; every source on ctx's device, with the same grid (n, b,
 * per-mode origins and row counts: all from the build/import, or all restrictions to the same
 * box) and the same sinc parameters apart from eps.  The result belongs to `ctx` and does not
 * reference the sources.  Errors: RSD_E_INVALID for a NULL argument, a bad count or eps
 * outside (0, 1); RSD_E_UNSUPPORTED for sources on different grids or quadratures; RSD_E_OOM
 * beyond the budget. */
rsd_status rsd_tensor_combine(rsd_context* ctx, const rsd_tensor* const* tensors, int32_t count, double eps,
                              rsd_tensor** out);

/* The electrostatic energy of the molecule itself from its own tensor (Prop. 3.2, eqs. 3.8-3.9):
 *   E_long  = 1/2 sum_j z_j (P_l(x_j) - z_j sum_{k < K_long} w_k),
 * the long-range potential at each atom (trilinear, as in scoring) minus the atom's own
 * long-range term (its charge times the long-range reference kernel at distance zero), and
 *   E_short = 1/2 sum_j z_j sum_{m != j, d^2 < r_c^2} z_m sum_{k >= K_long} w_k exp(-t_k^2 d^2),
 * the short-range pairs, which the proposition assumes to vanish (all pair distances beyond
 * the short-range support); E_long + E_short approximates 1/2 sum_{j != m} z_j z_m / d_jm.
 * Host outputs; synchronises the context stream.  The short-range sum runs over all atom
 * pairs (O(N^2), no cell list).  Errors: RSD_E_INVALID (NULL), RSD_E_UNSUPPORTED for a
 * restricted tensor. */
rsd_status rsd_self_energy(rsd_context* ctx, const rsd_tensor* t, double* E_long, double* E_short);

/* ---- posing search (Algorithm PPIEM, steps A2-A6) ----
 * The search scans a grid of orbit directions u_i (positions of the ligand centre around the
 * protein centre x_P) times orientations q_k of the ligand about its own centre; each pose
 * sits at first contact (step A3) and is scored by rsd_score_poses (steps A4-A5); the lowest
 * energy per orbit position and the local minima over the orbit grid follow (step A6).  The
 * arrays of these calls are DEVICE pointers (HBM), laid out orbit-major: entry u * Q + q. */

/* Step A2: the protein's geometric centre x_P, the unweighted mean of its atom positions,
 * summed in index order and divided by N.  RSD_E_INVALID for a tensor without atoms. */
rsd_status rsd_tensor_centre(const rsd_tensor* t, double centre[3]);

/* Step A3, radial approach.  For orbit direction u (unit, dirs[3u..3u+2]) and orientation q
 * (unit quaternion, quats[4q..4q+3]) the ligand centre moves along x_P + rho u; coming in from
 * far away, the first contact with the van der Waals distance is at
 *   rho* = max over protein-ligand pairs of the larger root of |rho u + w|^2 = sigma^2,
 *   w = centre + R(q) (x_l - c) - x_m,
 * after which every larger rho keeps all pairs at >= sigma (the root formula is exact; the
 * device evaluates it in FP64).  Outputs, for entry o = u * Q + q:
 *   rho[o]            rho*; -inf if the line never comes within sigma of the protein; NaN
 *                     for an invalid quaternion (| |q|^2 - 1 | > 1e-12 or non-finite);
 *   pose_quats[4o..]  q (copied);
 *   pose_trans[3o..]  centre + (rho* + gap) u, NaN where rho* is not finite -- ready for
 *                     rsd_score_poses with RSD_MEM_DEVICE (NaN poses are flagged invalid).
 * Inputs: lig_positions [L*3], dirs [U*3], quats [Q*4] on the device; centre[3] on the host
 * (normally rsd_tensor_centre); sigma > 0, gap >= 0 (a gap of 1e-6 A keeps the contact poses
 * strictly admissible).  Enqueued on the context stream, not synchronised.  Errors:
 * RSD_E_INVALID (NULL, sizes, non-finite sigma/gap/centre), RSD_E_UNSUPPORTED (L). */
rsd_status rsd_contact_poses(rsd_context* ctx, const rsd_tensor* t, const double* lig_positions, int64_t L,
                             const double* dirs, int64_t U, const double* quats, int64_t Q, const double centre[3],
                             double sigma, double gap, double* rho, double* pose_quats, double* pose_trans);

/* Step A6.  For each orbit position u: best_rotation[u] = the orientation q with the lowest
 * energies[u*Q + q] among poses with the accept bit (flags & 1; the lowest q on ties), -1 if
 * none, and best_energy[u] its energy (+inf if none); is_minimum[u] = 1 when u has an
 * accepted pose and best_energy[u] <= best_energy[v] for every neighbour v, listed in CSR
 * form: nbr_index[nbr_offsets[u] .. nbr_offsets[u+1]-1] (indices in [0, U)).  All arrays on
 * the device.  The neighbour lists are read back and checked first (one synchronisation);
 * the kernels are then enqueued on the context stream.  Errors: RSD_E_INVALID (NULL, sizes,
 * offsets not starting at 0 or decreasing, an index outside [0, U)). */
rsd_status rsd_orbit_minima(rsd_context* ctx, const double* energies, const uint8_t* flags, int64_t U, int64_t Q,
                            const int32_t* nbr_offsets, const int32_t* nbr_index, int32_t* best_rotation,
                            double* best_energy, uint8_t* is_minimum);

/* Per-mode grid of a tensor: origin X0[d] (Angstrom), row count rows[d] and the mesh h.
 * For tensors from rsd_build_rs_tensor / rsd_tensor_import every mode has X0 = -b + h and
 * rows = n.  Any output pointer may be NULL. */
rsd_status rsd_tensor_grid(const rsd_tensor* t, double X0[3], int32_t rows[3], double* h);

/* Tensor metadata: grid size, canonical rank R, Tucker ranks (0 for imported tensors)
 * and resident device bytes.  Any output pointer may be NULL.  For a restricted tensor, n
 * is the largest row count of its modes (the factor layout's rows). */
rsd_status rsd_tensor_query(const rsd_tensor* t, int32_t* n, int64_t* R, int32_t ranks[3],
                            size_t* bytes);

/* Factor layout of a tensor, for accounting the bytes the long-range gathers move
 * (Lemma 3.3: two rows per mode per ligand atom):
 *   nchunk          number of 64-column rank chunks (R padded to a multiple of 64)
 *   shared_mode3    chunks whose 64 columns use at most 4 distinct mode-3 columns of the
 *                   Tucker basis U_3; for them scoring reads the mode-3 rows of the U_3
 *                   columns once per atom instead of gathering the factor rows (tensors made
 *                   by the canonical -> Tucker -> canonical step; 0 for imported ones). */
rsd_status rsd_tensor_layout(const rsd_tensor* t, int32_t* nchunk, int32_t* shared_mode3);

/* Measurement helper: times (best of 5 launches, HIP events on the context stream) a kernel
 * that performs only the long-range scoring kernel's gathers: per half-wavefront one row i
 * of a 64-column chunk per step, 16-byte loads of rows i and i+1 of two modes per lane, on a
 * 2 * n * 512-byte working set per XCD.  Its rate is the ceiling of the L2 -> compute-unit
 * return path for that pattern, against which the scoring kernel's gathers are reported.
 *   n      rows per chunk (power of two, 4..16384); iters: steps per wavefront (1..4096)
 *   ms     best launch time; bytes: bytes loaded per launch.
 * Synchronous.  Uses the context's workspace.  Errors: RSD_E_INVALID, RSD_E_OOM, RSD_E_HIP. */
rsd_status rsd_probe_gather(rsd_context* ctx, int32_t n, int32_t iters, double* ms, double* bytes);

/* Copy the factors to host arrays F1, F2, F3 of n*R doubles each (row-major n x R).
 * Synchronous. */
rsd_status rsd_tensor_export(const rsd_tensor* t, double* F1, double* F2, double* F3);

/* Versioned binary file: header (magic, version, n, b, R, ranks, sinc params, N),
 * factors, protein atoms and a checksum.  Load rebuilds the cell list. */
rsd_status rsd_tensor_save(const rsd_tensor* t, const char* path);
rsd_status rsd_tensor_load(rsd_context* ctx, const char* path, rsd_tensor** out);

void rsd_tensor_free(rsd_tensor* t);

/* Tuning options of a context (the autotuner sets these):
 *   "score_mode"      0 automatic, 1 one wavefront per pose for the whole pose,
 *                     2 long-range part in rank-chunk-major order across the XCDs
 *   "poses_per_wave"  poses per wavefront in mode 2 (0 automatic, 1..4)
 *   "chunks_per_item" rank chunks per work item of the mode-2 long-range kernel (also in
 *                     batches, fixed when the batch is created): 0 automatic (2), 1..4; the
 *                     pose transforms and grid rows of an item are formed once for its chunks
 *   "eig_solver"      eigenvectors of the Gram matrices in the build: 0 automatic (subspace
 *                     iteration for n >= 1024), 1 dense batched eigensolver, 2 subspace iteration
 *   "qr_solver"       bases of the subspace iteration in the build and of the range panels in
 *                     the rank reduction: 0 automatic (randomized Cholesky QR in one workgroup for
 *                     k <= 128 columns, Householder QR where a Cholesky pass loses rank),
 *                     1 rocSOLVER's Householder QR
 *   "t2c_solver"      SVD of the Tucker core slices in the build: 0 automatic (3 where its LDS
 *                     fits, else 1, else 2), 1 one-sided Jacobi with the slice in LDS,
 *                     2 rocSOLVER gesvd, 3 one-sided Jacobi on the transposed triangle of a
 *                     Householder QR of the slice (fewer sweeps on graded slices)
 *   "factors"         1-D factors of rsd_build_rs_tensor: 0 (default) the Gaussians collocated
 *                     at the grid nodes; 1 their averages over the grid cells, i.e. the
 *                     projection onto piecewise-constant basis functions of eq. 2.1 (the Gram
 *                     matrices are then formed densely on the matrix cores); 2 (3) the
 *                     shift-and-window construction of eq. 2.5: every charge is moved to its
 *                     nearest grid node (j = floor((x - X_0)/h + 1/2), clipped to the grid) and
 *                     the single-charge reference Gaussians (cell averages) are centred there and
 *                     windowed onto the grid; the long range then errs to first order in h
 *                     (Table 3.2), while the short range and the vdW test keep the true positions
 *   "svd_solver"      the k x k SVD inside the rank reduction of explicit factors
 *                     (rsd_tensor_restrict, rsd_tensor_combine): 0 automatic (4), 1 rocSOLVER gesvd,
 *                     2 rocSOLVER gesdd (divide and conquer), 3 rocSOLVER gesvdj (Jacobi),
 *                     4 the library's one-sided Jacobi kernel (one workgroup per mode)
 *   "gram_solver"     Gram matrices of the side matrices in the build: 0 automatic (1),
 *                     1 Toeplitz-times-Hankel form of the uniform grid (O(n N K + n^2 K)),
 *                     2 dense product of the generated side matrix on matrix cores (O(n^2 N K))
 *   "batch_mode"      launches of rsd_batch_run (fixed when the batch is created): 0 automatic
 *                     (currently 1), 1 requests grouped by LDS occupancy, one short-range and one
 *                     long-range launch per group; 2 one persistent launch for the transform,
 *                     short range, vdW test and long range of every request, its workgroups
 *                     claiming work items from one queue per XCD (requests whose ligands need more
 *                     than 160 KB of LDS in that form fall back to 1); both add a ligand-frame
 *                     launch before and a combine launch after, and give the same bits
 *   "short_waves"     wavefronts (poses) per workgroup of the short-range kernel: 0 automatic,
 *                     1, 2 or 4 (must fit 64 KB of LDS for the ligand)
 *   "shared_mode3"    1 (default): for tensors made by the build, a restriction or a combine,
 *                     whose mode-3 factor columns are copies of the r_3 columns of U_3, the
 *                     chunk-major energy kernel lerps each chunk's few distinct U_3 columns once
 *                     per atom (same values, fewer gathers); 0: gather every mode-3 column
 *   "short_poly"      1 (default): tensors made afterwards with this context evaluate the
 *                     short-range Gaussian sum of energy-only scoring from a table of degree-7
 *                     Chebyshev interpolants in d^2 (one per quadrature and cutoff, kept by the
 *                     context; checked on the host to 1e-11 relative, else not used); gradient
 *                     calls and 0 evaluate the exponentials
 *   "pose_order"      chunk-major long range: 0 automatic (calls and batch requests of at least
 *                     16384 poses), 1 always, 2 never take the poses in spatial order (a
 *                     counting sort of their translations by a Morton code of 32^3 cells over
 *                     the box, on the device).  Neighbouring poses then share factor rows within
 *                     a workgroup and, on grids whose rank chunk (3 x n x 512 bytes) exceeds the
 *                     4 MiB L2 of an XCD, within the L2; the results are those of input order
 *                     bit for bit, each written to its own pose
 *   "overlap"         1: in chunk-major scoring the short-range kernel runs on a second stream
 *                     of the context beside the long-range kernel (joined before the results
 *                     are combined); 0 (default): one stream.  The long-range gathers slow
 *                     down by about as much as the short range saves, so the default is off
 *   "use_tuning"      1 (default): calls whose three launch-shape options above are automatic
 *                     take the shape rsd_autotune recorded for their workload; 0: ignore it
 * Errors: RSD_E_INVALID for an unknown name or value. */
rsd_status rsd_context_set_option(rsd_context* ctx, const char* name, int64_t value);

/* The spatial order in which the chunk-major long-range kernels take poses on large grids
 * (option "pose_order"), for a caller that splits a large request into parts scored at
 * different times (a serving loop): parts cut from the ordered poses each cover a compact
 * region, so their factor rows stay in the L2 (Algorithm PLIE's sum over poses is
 * unchanged; each pose's result does not depend on the order).
 *   t          the tensor the poses will be scored against (its box sets the cells)
 *   quats [P*4] (may be NULL when quats_out is NULL), trans [P*3]   device arrays
 *   perm [P]   out, device: perm[i] = the input index of the pose at position i; the order
 *              sorts the poses by a Morton code of their translation's cell (32^3 cells over
 *              the box; coordinates outside it or NaN clamp to the edge cells), poses of one
 *              cell in no particular order
 *   quats_out [P*4], trans_out [P*3]   out, device (or NULL): the poses in that order
 *   sorted     out (or NULL): 1 if scoring these P poses on this context would sort them itself
 * Asynchronous on the context stream (which it synchronises only when the context's
 * workspace must grow to 4 * (32768 + P) bytes).  Errors: RSD_E_INVALID (NULL arrays, P out
 * of range, a tensor of another device); RSD_E_OOM. */
rsd_status rsd_pose_order(rsd_context* ctx, const rsd_tensor* t, const double* quats,
                          const double* trans, int64_t P, int32_t* perm, double* quats_out,
                          double* trans_out, int32_t* sorted);

/* Launch-shape tuner (the scoring kernels' tile parameters: poses per wavefront of the
 * rank-chunk-major long-range kernel, wavefronts per workgroup of the short-range kernel, and
 * chunk-major versus fused per-pose long-range evaluation).  Every candidate shape whose LDS
 * fits is timed on the given poses with HIP events on the context stream (one untimed call,
 * then the best of three), and the fastest is recorded in the context for the workload key
 * (grid n, rank chunks of 64 columns, protein atoms, ligand atoms, gradients or not).
 * Later rsd_score_poses calls and batch requests on this context with matching key, at least
 * 256 poses and automatic launch-shape options use it.  Pass a representative sample of the
 * workload (same tensor, ligand and pose distribution; ~1e4 poses is plenty).  Inputs are
 * device pointers with the layout of rsd_score_poses; the scores go to library scratch and
 * are discarded.  Per-pose results do not depend on the shape except that the fused and the
 * chunk-major evaluation sum the ranks in different orders (both within the parity
 * tolerance).  Synchronises the context stream.  `report` may be NULL.
 * Errors: as rsd_score_poses; RSD_E_OOM if the scratch does not fit the budget. */

typedef struct rsd_tune_report {
  int32_t score_mode;      /* chosen: 1 fused, 2 chunk-major */
  int32_t poses_per_wave;  /* chosen (chunk-major) */
  int32_t short_waves;     /* chosen */
  int32_t candidates;      /* shapes timed */
  double best_ms;          /* per call on the sample, chosen shape */
  double default_ms;       /* per call on the sample, untuned automatic shape */
} rsd_tune_report;

rsd_status rsd_autotune(rsd_context* ctx, const rsd_tensor* t, const double* lig_charges,
                        const double* lig_positions, int64_t L, const double* quats, const double* trans,
                        int64_t P, double vdw_min, int32_t grads, rsd_tune_report* report);

/* The cell size of the tensor's short-range cell list, tuned on a sample of a workload
 * (device pointers, as rsd_autotune): the list is rebuilt with cell edges r_cut / div for
 * div = 3, 4, 5, 6 (at most 128 cells per axis), scoring of the sample is timed for each
 * (best of 3 calls, the launch shapes the context would pick), and the fastest edge stays
 * with the tensor.  ms[4] (may be NULL): milliseconds per call for div = 3..6; *best_div:
 * the divisor kept.  Pair counts and flags do not depend on the cell size; energies change
 * only by the order in which the short range adds its pairs.  The tensor must not be in use
 * by queued work of other streams.  Synchronous.  Errors: as rsd_autotune. */
rsd_status rsd_autotune_cells(rsd_context* ctx, rsd_tensor* t, const double* lig_charges,
                              const double* lig_positions, int64_t L, const double* quats,
                              const double* trans, int64_t P, double vdw_min, int32_t grads,
                              int32_t* best_div, double* ms);

/* Kernel timing with HIP events on the context stream (off by default).  When on,
 * every library kernel launch is bracketed by events and its duration is added to
 * a per-kernel total once the stream reaches it; rsd_kernel_time synchronises the
 * stream and reports the number of launches and total milliseconds of the named
 * kernel ("score", "cells", "gram", ...) since timing was switched on. */
rsd_status rsd_context_set_timing(rsd_context* ctx, int32_t enable);
rsd_status rsd_kernel_time(rsd_context* ctx, const char* kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* RSDOCK_H */
