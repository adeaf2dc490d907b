// Cell list of the protein atoms for the short-range sum and the vdW check.
//
// The RS format keeps the short-range part as per-atom terms of small support
// (Def. 2.1, "list of weights and centres"); summing them "locally" needs the
// atoms near a point.  Atoms are counting-sorted into uniform cubic cells over
// the box [-b, b]^3 (x fastest), so the cells of one (y, z) row form one
// contiguous range of the sorted atom array.  Within a cell atoms keep their
// input order, which makes the sorted array, and every sum over it, identical
// from run to run.
#include "internal.h"

namespace rsd {
namespace {

__device__ __forceinline__ int cell_coord(double x, double origin, double inv_edge, int dim) {
  int c = (int)floor((x - origin) * inv_edge);
  return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

__global__ void k_cell_count(const double* __restrict__ pos, int64_t N, CellGrid g,
                             int* __restrict__ cell_of, int* __restrict__ count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int cx = cell_coord(pos[3 * i + 0], g.origin, g.inv_edge, g.dim);
  int cy = cell_coord(pos[3 * i + 1], g.origin, g.inv_edge, g.dim);
  int cz = cell_coord(pos[3 * i + 2], g.origin, g.inv_edge, g.dim);
  int c = (cz * g.dim + cy) * g.dim + cx;
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of count[0..n) into start[0..n] by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_single(const int* __restrict__ count, int n,
                                                      int* __restrict__ start) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, tid * per), hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += count[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan of the partial sums
    int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;  // exclusive prefix of this thread's range
  for (int i = lo; i < hi; ++i) {
    start[i] = run;
    run += count[i];
  }
  if (tid == 1023) start[n] = part[1023];
}

__global__ void k_cell_scatter(const int* __restrict__ cell_of, int64_t N, const int* __restrict__ start,
                               int* __restrict__ cursor, int* __restrict__ order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int c = cell_of[i];
  int slot = start[c] + atomicAdd(&cursor[c], 1);
  order[slot] = (int)i;
}

// Restore input order inside every cell (insertion sort; cells hold few atoms).
__global__ void k_cell_sort(int ncells, const int* __restrict__ start, int* __restrict__ order) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int lo = start[c], hi = start[c + 1];
  for (int i = lo + 1; i < hi; ++i) {
    int v = order[i];
    int j = i - 1;
    while (j >= lo && order[j] > v) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
}

__global__ void k_cell_gather(const int* __restrict__ order, int64_t N, const double* __restrict__ pos,
                              const double* __restrict__ z, double4* __restrict__ atoms) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  int64_t i = order[s];
  atoms[s] = make_double4(pos[3 * i + 0], pos[3 * i + 1], pos[3 * i + 2], z[i]);
}

}  // namespace

// Cell edge: r_cut / div (div = 4 unless the cell tuner chose another), but at most 128 cells
// per axis.  Any edge is correct (counts and flags do not depend on it, only the order in which
// the short range sums its pairs does); a quarter keeps the candidate set close to the sphere
// the scoring kernel needs while the row count stays small.
static CellGrid make_grid(double b, double r_cut, int div) {
  CellGrid g{};
  double e = r_cut / (double)(div > 0 ? div : 4);
  const double e_min = 2.0 * b / 128.0;
  if (!(e > e_min)) e = e_min;
  g.origin = -b;
  g.edge = e;
  g.inv_edge = 1.0 / e;
  g.dim = (int)ceil(2.0 * b * g.inv_edge);
  if (g.dim < 1) g.dim = 1;
  if (g.dim > 128) g.dim = 128;
  g.ncells = g.dim * g.dim * g.dim;
  return g;
}

rsd_status build_cells(Context* ctx, Tensor* t, const double* d_charges, const double* d_positions) {
  const int64_t N = t->N;
  t->cells = make_grid(t->b, t->sp.r_cut, t->cell_div);
  const CellGrid g = t->cells;
  t->cell_bytes = sizeof(int) * (size_t)(g.ncells + 1);
  RSD_TRY(ctx->dev_alloc((void**)&t->cell_start, t->cell_bytes));
  if (!t->atoms) RSD_TRY(ctx->dev_alloc((void**)&t->atoms, sizeof(double4) * (size_t)(N > 0 ? N : 1)));
  // scratch: cell_of[N], count[ncells], cursor[ncells], order[N]
  size_t scratch = sizeof(int) * (size_t)(2 * (N > 0 ? N : 1) + 2 * (int64_t)g.ncells);
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(scratch, &ws));
  int* cell_of = (int*)ws;
  int* count = cell_of + (N > 0 ? N : 1);
  int* cursor = count + g.ncells;
  int* order = cursor + g.ncells;
  hipStream_t s = ctx->stream;
  RSD_HIP(hipMemsetAsync(count, 0, sizeof(int) * (size_t)g.ncells * 2, s));
  const int TB = 256;
  const unsigned nb = (unsigned)((N + TB - 1) / TB);
  if (N > 0) {
    RSD_TIMED_LAUNCH(ctx, "cells", (k_cell_count<<<nb, TB, 0, s>>>(d_positions, N, g, cell_of, count)));
  }
  RSD_TIMED_LAUNCH(ctx, "cells", (k_scan_single<<<1, 1024, 0, s>>>(count, g.ncells, t->cell_start)));
  if (N > 0) {
    RSD_TIMED_LAUNCH(ctx, "cells", (k_cell_scatter<<<nb, TB, 0, s>>>(cell_of, N, t->cell_start, cursor, order)));
    RSD_TIMED_LAUNCH(ctx, "cells", (k_cell_sort<<<(g.ncells + TB - 1) / TB, TB, 0, s>>>(g.ncells, t->cell_start, order)));
    RSD_TIMED_LAUNCH(ctx, "cells", (k_cell_gather<<<nb, TB, 0, s>>>(order, N, d_positions, d_charges, t->atoms)));
  }
  RSD_HIP(hipStreamSynchronize(s));
  return RSD_OK;
}
// The tensor's cell list again with edge r_cut / div, from the atoms it keeps on the host.
rsd_status rebuild_cells(Context* ctx, Tensor* t, int div) {
  RSD_CHECK(div >= 2 && div <= 12, RSD_E_INVALID, "cell divisor %d outside [2, 12]", div);
  const int64_t N = t->N;
  const size_t nz = sizeof(double) * (size_t)(N > 0 ? N : 1);
  double* d_z = nullptr;
  double* d_pos = nullptr;
  RSD_TRY(ctx->dev_alloc((void**)&d_z, nz));
  rsd_status st = ctx->dev_alloc((void**)&d_pos, 3 * nz);
  if (st == RSD_OK && N > 0) {
    hipError_t e = hipMemcpyAsync(d_z, t->host_charges.data(), sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_pos, t->host_positions.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
      set_error("cell list upload: %s", hipGetErrorString(e));
      st = RSD_E_HIP;
    }
  }
  if (st == RSD_OK) {
    (void)hipStreamSynchronize(ctx->stream);   // no queued work still reads the old cell list
    ctx->dev_free(t->cell_start, t->cell_bytes);
    t->cell_start = nullptr;
    t->cell_div = div;
    st = build_cells(ctx, t, d_z, d_pos);
  }
  if (d_pos) ctx->dev_free(d_pos, 3 * nz);
  ctx->dev_free(d_z, nz);
  return st;
}

}  // namespace rsd
