// C ABI of librsdock: contexts, resident tensors, scoring entry point, file I/O, timing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include <rocblas/rocblas.h>

#include "internal.h"

namespace rsd {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------- context memory
rsd_status Context::dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (budget != 0 && in_use + bytes > budget) block_trim();
  RSD_CHECK(budget == 0 || in_use + bytes <= budget, RSD_E_OOM,
            "HBM budget exceeded: %zu in use + %zu requested > %zu", in_use, bytes, budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess && (!block_cache.empty() || !scratch_cache.empty())) {
    (void)hipGetLastError();
    block_trim();
    e = hipMalloc(p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return RSD_E_OOM;
  }
  in_use += bytes;
  return RSD_OK;
}

void Context::dev_free(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  if (bytes == 0) bytes = 8;
  in_use = in_use >= bytes ? in_use - bytes : 0;
}

rsd_status Context::block_alloc(void** p, size_t* bytes) {
  const size_t want = *bytes == 0 ? 8 : *bytes;
  int best = -1;
  for (int i = 0; i < (int)block_cache.size(); ++i) {
    const size_t have = block_cache[i].second;
    if (have >= want && have <= 2 * want + (64u << 20) && (best < 0 || have < block_cache[best].second)) best = i;
  }
  if (best >= 0) {
    *p = block_cache[best].first;
    *bytes = block_cache[best].second;
    block_cache.erase(block_cache.begin() + best);
    return RSD_OK;
  }
  *bytes = want;
  return dev_alloc(p, want);
}

void Context::block_release(void* p, size_t bytes) {
  if (!p) return;
  block_cache.emplace_back(p, bytes);
  if (block_cache.size() > 4) {   // keep the four largest
    int small = 0;
    for (int i = 1; i < (int)block_cache.size(); ++i)
      if (block_cache[i].second < block_cache[small].second) small = i;
    dev_free(block_cache[small].first, block_cache[small].second);
    block_cache.erase(block_cache.begin() + small);
  }
}

void Context::block_trim() {
  if (block_cache.empty() && scratch_cache.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (auto& b : block_cache) dev_free(b.first, b.second);
  block_cache.clear();
  for (auto& b : scratch_cache) dev_free(b.first, b.second);
  scratch_cache.clear();
}

rsd_status Context::scratch_get(void** p, size_t bytes) {
  const size_t want = bytes == 0 ? 8 : bytes;
  int best = -1;
  for (int i = 0; i < (int)scratch_cache.size(); ++i) {
    const size_t have = scratch_cache[i].second;
    if (have >= want && have <= want + want / 4 + (1u << 20) && (best < 0 || have < scratch_cache[best].second))
      best = i;
  }
  if (best >= 0) {
    *p = scratch_cache[best].first;
    scratch_live.push_back(scratch_cache[best]);
    scratch_cache.erase(scratch_cache.begin() + best);
    return RSD_OK;
  }
  RSD_TRY(dev_alloc(p, want));
  scratch_live.emplace_back(*p, want);
  return RSD_OK;
}

void Context::scratch_end() {
  if (scratch_live.empty()) return;
  (void)hipStreamSynchronize(stream);   // the call's streams have joined this one
  for (auto& b : scratch_live) scratch_cache.push_back(b);
  scratch_live.clear();
  // keep at most 96 blocks and 4 GiB: small builds then reuse everything, while the Gram
  // matrices of a large grid (3 n^2 doubles) are not held between calls
  size_t total = 0;
  for (auto& b : scratch_cache) total += b.second;
  while (scratch_cache.size() > 96 || total > ((size_t)4 << 30)) {
    int drop = 0;   // the smallest while over the count, else the largest
    for (int i = 1; i < (int)scratch_cache.size(); ++i) {
      const bool smaller = scratch_cache[i].second < scratch_cache[drop].second;
      if (scratch_cache.size() > 96 ? smaller : !smaller) drop = i;
    }
    total -= scratch_cache[drop].second;
    dev_free(scratch_cache[drop].first, scratch_cache[drop].second);
    scratch_cache.erase(scratch_cache.begin() + drop);
  }
}

rsd_status Context::workspace(size_t bytes, void** out) {
  if (bytes > ws_bytes) {
    if (ws) {
      RSD_HIP(hipStreamSynchronize(stream));
      dev_free(ws, ws_bytes);
      ws = nullptr;
      ws_bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    RSD_TRY(dev_alloc(&ws, want));
    ws_bytes = want;
  }
  *out = ws;
  return RSD_OK;
}

rsd_status Context::aux_streams() {
  for (int i = 0; i < 2; ++i) {
    if (!aux_stream[i]) RSD_HIP(hipStreamCreateWithFlags(&aux_stream[i], hipStreamNonBlocking));
    if (!aux_blas[i]) {
      rocblas_handle h = nullptr;
      RSD_CHECK(rocblas_create_handle(&h) == rocblas_status_success, RSD_E_HIP, "rocblas_create_handle failed");
      aux_blas[i] = h;
    }
    RSD_CHECK(rocblas_set_stream((rocblas_handle)aux_blas[i], aux_stream[i]) == rocblas_status_success, RSD_E_HIP,
              "rocblas_set_stream failed");
  }
  return RSD_OK;
}

rsd_status Context::timer_begin(const char* name, KernelTimer* t) {
  t->name = name;
  RSD_HIP(hipEventCreate(&t->start));
  RSD_HIP(hipEventCreate(&t->stop));
  RSD_HIP(hipEventRecord(t->start, stream));
  return RSD_OK;
}

rsd_status Context::timer_end(KernelTimer* t) {
  RSD_HIP(hipEventRecord(t->stop, stream));
  pending.push_back(*t);
  return RSD_OK;
}

rsd_status Context::collect_timers() {
  if (pending.empty()) return RSD_OK;
  RSD_HIP(hipStreamSynchronize(stream));
  for (auto& t : pending) {
    float ms = 0.f;
    RSD_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
    auto& acc = ktime[t.name];
    acc.first += 1;
    acc.second += (double)ms;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  pending.clear();
  return RSD_OK;
}

size_t Tensor::bytes() const {
  return F_bytes + cell_bytes + sizeof(double4) * (size_t)(N > 0 ? N : 1) + sizeof(double) * 2 * kMaxTerms +
         (U3 ? sizeof(double) * (size_t)nm[2] * u3_ld + sizeof(int) * (size_t)R : 0);
}

void sinc_table(const rsd_sinc_params& sp, double* t, double* w) {
  const double root_pi = std::sqrt(M_PI);
  for (int k = 0; k <= sp.M; ++k) {
    const double kh = (double)k * sp.h_M;
    t[k] = std::sinh(kh) / sp.L_s;
    const double a = sp.h_M * std::cosh(kh) / (root_pi * sp.L_s);
    w[k] = k == 0 ? a : 2.0 * a;
  }
}

// ---------------------------------------------------------------- helpers
rsd_status check_sinc(const rsd_sinc_params* sp) {
  RSD_CHECK(sp != nullptr, RSD_E_INVALID, "sinc params are NULL");
  RSD_CHECK(sp->M >= 0 && sp->M + 1 <= kMaxTerms, RSD_E_INVALID, "M=%d out of range [0, %d]", sp->M, kMaxTerms - 1);
  RSD_CHECK(sp->K_long >= 0 && sp->K_long <= sp->M + 1, RSD_E_INVALID, "K_long=%d out of range", sp->K_long);
  RSD_CHECK(std::isfinite(sp->h_M) && sp->h_M > 0, RSD_E_INVALID, "h_M must be finite and > 0");
  RSD_CHECK(std::isfinite(sp->L_s) && sp->L_s > 0, RSD_E_INVALID, "L_s must be finite and > 0");
  RSD_CHECK(std::isfinite(sp->r_cut) && sp->r_cut >= 0, RSD_E_INVALID, "r_cut must be finite and >= 0");
  RSD_CHECK(std::isfinite(sp->eps) && sp->eps >= 0 && sp->eps < 1, RSD_E_INVALID, "eps must be in [0, 1)");
  return RSD_OK;
}

rsd_status check_grid(int32_t n, double b) {
  RSD_CHECK(n >= 4 && n <= 32768 && n % 2 == 0, RSD_E_INVALID, "n=%d must be even and in [4, 32768]", n);
  RSD_CHECK(std::isfinite(b) && b > 0, RSD_E_INVALID, "b must be finite and > 0");
  return RSD_OK;
}

static bool is_device_ptrs(uint32_t f) { return (f & RSD_DEVICE_PTRS) != 0; }

// Copy `count` doubles from a caller array (host or device) into a host vector.
static rsd_status to_host(const double* src, size_t count, bool dev, std::vector<double>* out) {
  out->resize(count);
  if (count == 0) return RSD_OK;
  if (dev) {
    RSD_HIP(hipMemcpy(out->data(), src, sizeof(double) * count, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out->data(), src, sizeof(double) * count);
  }
  return RSD_OK;
}

rsd_status check_protein(const std::vector<double>& z, const std::vector<double>& pos, int32_t n, double b) {
  double h, X0, inv_h;
  grid_constants(n, b, &h, &X0, &inv_h);
  for (size_t i = 0; i < z.size(); ++i) {
    RSD_CHECK(std::isfinite(z[i]), RSD_E_INVALID, "protein charge %zu is not finite", i);
    for (int d = 0; d < 3; ++d) {
      const double x = pos[3 * i + d];
      RSD_CHECK(std::isfinite(x) && x >= X0 && x <= b, RSD_E_INVALID,
                "protein atom %zu coordinate %d = %g outside the grid node range [%g, %g]", i, d, x, X0, b);
    }
  }
  return RSD_OK;
}

// The short-range kernel g(x) = sum_k w_k exp(-t_k^2 x), x = d^2, as piecewise polynomials:
// intervals of width d1 = 0.5 / t_max^2 on [0, x1) and of width d2 = 0.5 / t_c^2 on [x1, r_c^2],
// where x1 = 25 A^2 and t_c^2 is the largest t_k^2 whose term can still reach e^-45 of the
// widest one beyond x1 (the others are below 1e-18 of g there).  On each interval g is
// interpolated at the 8 Chebyshev points (values in long double), and the interpolant is
// stored as monomial coefficients in s in [-1, 1].  With t^2 times the width at most 1/2 the
// interpolation error of every term is below about 3e-12 of its size; the table is checked
// against the exact sum at 16 points per interval and discarded (the kernels then evaluate
// the exponentials) if any relative error exceeds 1e-11, or if it would exceed 8 MB.
bool build_short_poly(const ShortTable& st, double rc2, std::vector<double>* coef, int* n1, double* x1,
                      double* d1, double* d2) {
  coef->clear();
  if (st.S <= 0 || !(rc2 > 0.0)) return false;
  double amax = 0.0, amin = st.t2[0];
  for (int k = 0; k < st.S; ++k) {
    amax = std::max(amax, st.t2[k]);
    amin = std::min(amin, st.t2[k]);
  }
  if (!(amax > 0.0)) return false;
  const double X1 = std::min(25.0, rc2);
  double ac = amin;
  for (int k = 0; k < st.S; ++k)
    if ((st.t2[k] - amin) * X1 <= 45.0) ac = std::max(ac, st.t2[k]);
  *x1 = X1;
  *d1 = 0.5 / amax;
  *d2 = 0.5 / std::max(ac, 1e-300);
  *n1 = (int)std::ceil(X1 / *d1);
  const double n2d = rc2 > X1 ? std::ceil((rc2 - X1) / *d2) + 1.0 : 0.0;
  const double total = (double)*n1 + n2d;
  if (total * kPolyCoef * sizeof(double) > 8.0 * 1024 * 1024) return false;
  const int n = (int)total;
  coef->resize((size_t)n * kPolyCoef);
  auto g = [&](double x) {   // terms in double, summed in long double
    long double s = 0.0L;
    for (int k = 0; k < st.S; ++k) s += (long double)(st.w[k] * std::exp(-st.t2[k] * x));
    return s;
  };
  // Chebyshev polynomials T_0..T_7 in the power basis
  long double T[kPolyCoef][kPolyCoef] = {};
  T[0][0] = 1.0L;
  T[1][1] = 1.0L;
  for (int m = 2; m < kPolyCoef; ++m)
    for (int j = 0; j < kPolyCoef; ++j) T[m][j] = (j > 0 ? 2.0L * T[m - 1][j - 1] : 0.0L) - T[m - 2][j];
  const long double pi = 3.141592653589793238462643383279502884L;
  long double node[kPolyCoef], cosm[kPolyCoef][kPolyCoef];
  for (int j = 0; j < kPolyCoef; ++j) {
    node[j] = std::cos(pi * (j + 0.5L) / kPolyCoef);
    for (int m = 0; m < kPolyCoef; ++m) cosm[m][j] = std::cos(pi * m * (j + 0.5L) / kPolyCoef);
  }
  double worst = 0.0;
  for (int i = 0; i < n; ++i) {
    const double a = i < *n1 ? i * *d1 : X1 + (i - *n1) * *d2;
    const double w = i < *n1 ? *d1 : *d2;
    long double f[kPolyCoef], c[kPolyCoef];
    for (int j = 0; j < kPolyCoef; ++j) f[j] = g((double)((long double)a + (long double)w * (node[j] + 1.0L) * 0.5L));
    for (int m = 0; m < kPolyCoef; ++m) {
      long double sm = 0.0L;
      for (int j = 0; j < kPolyCoef; ++j) sm += f[j] * cosm[m][j];
      c[m] = sm * 2.0L / kPolyCoef;
    }
    c[0] *= 0.5L;
    long double p[kPolyCoef] = {};
    for (int m = 0; m < kPolyCoef; ++m)
      for (int j = 0; j < kPolyCoef; ++j) p[j] += c[m] * T[m][j];
    for (int j = 0; j < kPolyCoef; ++j) (*coef)[(size_t)i * kPolyCoef + j] = (double)p[j];
    for (int q = 0; q < 16; ++q) {   // check at points spread over the interval
      const double s = -1.0 + 2.0 * (q + 0.5) / 16.0;
      double v = (*coef)[(size_t)i * kPolyCoef + kPolyCoef - 1];
      for (int j = kPolyCoef - 2; j >= 0; --j) v = std::fma(v, s, (*coef)[(size_t)i * kPolyCoef + j]);
      const long double ex = g(a + w * (s + 1.0) * 0.5);
      if (ex > 0.0L) worst = std::max(worst, (double)std::fabs(((long double)v - ex) / ex));
    }
  }
  if (!(worst <= 1e-11)) {
    coef->clear();
    return false;
  }
  return true;
}

// Create the tensor shell: grid constants, short-range table, protein copies, cell list.
static rsd_status tensor_common(Context* ctx, Tensor* t, int32_t n, double b, const rsd_sinc_params* sp,
                                std::vector<double>&& z, std::vector<double>&& pos, double** d_z,
                                double** d_pos) {
  t->ctx = ctx;
  t->n = n;
  t->b = b;
  grid_constants(n, b, &t->h, &t->X0, &t->inv_h);
  for (int d = 0; d < 3; ++d) {
    t->X0m[d] = t->X0;
    t->nm[d] = n;
  }
  t->sp = *sp;
  t->N = (int64_t)z.size();
  t->host_charges = std::move(z);
  t->host_positions = std::move(pos);
  double tk[kMaxTerms], wk[kMaxTerms];
  sinc_table(*sp, tk, wk);
  t->shrt.S = sp->M + 1 - sp->K_long;
  double tab[2 * kMaxTerms] = {0};
  for (int k = 0; k < t->shrt.S; ++k) {
    t->shrt.t2[k] = tk[sp->K_long + k] * tk[sp->K_long + k];
    t->shrt.w[k] = wk[sp->K_long + k];
    tab[k] = t->shrt.t2[k];
    tab[kMaxTerms + k] = t->shrt.w[k];
  }
  RSD_TRY(ctx->dev_alloc((void**)&t->short_tab, sizeof(tab)));
  RSD_HIP(hipMemcpy(t->short_tab, tab, sizeof(tab), hipMemcpyHostToDevice));
  if (ctx->opt_short_poly) {
    // one table per quadrature and cutoff, kept by the context and shared by its tensors
    const auto key = std::make_tuple(sp->M, sp->K_long, sp->h_M, sp->L_s, sp->r_cut);
    auto it = ctx->poly_cache.find(key);
    if (it == ctx->poly_cache.end()) {
      Context::Poly pc{};
      std::vector<double> coef;
      double d1 = 0.0, d2 = 0.0;
      if (build_short_poly(t->shrt, sp->r_cut * sp->r_cut, &coef, &pc.n1, &pc.x1, &d1, &d2)) {
        pc.inv_d1 = 1.0 / d1;
        pc.inv_d2 = 1.0 / d2;
        pc.bytes = sizeof(double) * coef.size();
        RSD_TRY(ctx->dev_alloc((void**)&pc.p, pc.bytes));
        RSD_HIP(hipMemcpy(pc.p, coef.data(), pc.bytes, hipMemcpyHostToDevice));
      }
      it = ctx->poly_cache.emplace(key, pc).first;
    }
    const Context::Poly& pc = it->second;
    t->short_poly = pc.p;
    t->poly_n1 = pc.n1;
    t->poly_x1 = pc.x1;
    t->poly_inv_d1 = pc.inv_d1;
    t->poly_inv_d2 = pc.inv_d2;
  }
  // device copies of the protein (freed by the caller of tensor_common)
  const size_t N = (size_t)t->N;
  RSD_TRY(ctx->dev_alloc((void**)d_z, sizeof(double) * (N ? N : 1)));
  RSD_TRY(ctx->dev_alloc((void**)d_pos, sizeof(double) * 3 * (N ? N : 1)));
  if (N) {
    RSD_HIP(hipMemcpy(*d_z, t->host_charges.data(), sizeof(double) * N, hipMemcpyHostToDevice));
    RSD_HIP(hipMemcpy(*d_pos, t->host_positions.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice));
  }
  RSD_TRY(build_cells(ctx, t, *d_z, *d_pos));
  return RSD_OK;
}

static void context_destroy(Context* ctx) {
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& t : ctx->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  ctx->pending.clear();
  ctx->scratch_end();
  ctx->block_trim();
  for (auto& kv : ctx->poly_cache)
    if (kv.second.p) ctx->dev_free(kv.second.p, kv.second.bytes);
  ctx->poly_cache.clear();
  ctx->dev_free(ctx->ws, ctx->ws_bytes);
  ctx->ws = nullptr;
  if (ctx->blas) rocblas_destroy_handle((rocblas_handle)ctx->blas);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  for (int i = 0; i < 2; ++i) {
    if (ctx->aux_stream[i]) (void)hipStreamSynchronize(ctx->aux_stream[i]);
    if (ctx->aux_blas[i]) rocblas_destroy_handle((rocblas_handle)ctx->aux_blas[i]);
    if (ctx->aux_stream[i]) (void)hipStreamDestroy(ctx->aux_stream[i]);
  }
  delete static_cast<rsd_context*>(ctx);
}

static void tensor_release(Tensor* t) {
  if (!t) return;
  Context* c = t->ctx;
  if (c) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);   // scoring work queued on the stream may still read the tensor
    c->dev_free(t->F, t->F_bytes);
    c->dev_free(t->atoms, sizeof(double4) * (size_t)(t->N > 0 ? t->N : 1));
    c->dev_free(t->cell_start, t->cell_bytes);
    c->dev_free(t->short_tab, sizeof(double) * 2 * kMaxTerms);
    if (t->U3) c->dev_free(t->U3, sizeof(double) * (size_t)t->nm[2] * t->u3_ld);
    if (t->slice) c->dev_free(t->slice, sizeof(int) * (size_t)t->R);
    c->live_tensors -= 1;
  }
  delete static_cast<rsd_tensor*>(t);
  if (c && c->closing && c->live_tensors == 0) context_destroy(c);
}

// Row-major n x R (device) -> column-chunked layout (device), zero padded.
__global__ void k_relayout(const double* __restrict__ src, int64_t R, int n, int nchunk, double* __restrict__ dst) {
  const int64_t total = (int64_t)nchunk * n * kChunk;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % kChunk);
    const int64_t rest = e / kChunk;
    const int i = (int)(rest % n);
    const int c = (int)(rest / n);
    const int64_t col = (int64_t)c * kChunk + j;
    dst[e] = col < R ? src[(int64_t)i * R + col] : 0.0;
  }
}

__global__ void k_unlayout(const double* __restrict__ src, int64_t R, int n, double* __restrict__ dst) {
  const int64_t total = (int64_t)n * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R, col = e % R;
    dst[e] = src[((col / kChunk) * n + i) * kChunk + (col % kChunk)];
  }
}

rsd_status alloc_factors(Context* ctx, Tensor* t, int64_t R) {
  t->R = R;
  t->nchunk = (int)((R + kChunk - 1) / kChunk);
  t->F_bytes = sizeof(double) * 3 * (size_t)t->nchunk * (size_t)t->n * kChunk;
  return ctx->dev_alloc((void**)&t->F, t->F_bytes);
}

rsd_status import_factors(Context* ctx, Tensor* t, const double* const F[3], int64_t R, bool dev) {
  RSD_TRY(alloc_factors(ctx, t, R));
  if (t->nchunk == 0) return RSD_OK;
  const size_t one = sizeof(double) * (size_t)t->n * (size_t)R;
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(one, &ws));
  const int64_t mode = (int64_t)t->nchunk * t->n * kChunk;
  for (int d = 0; d < 3; ++d) {
    RSD_HIP(hipMemcpyAsync(ws, F[d], one, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    k_relayout<<<1024, 256, 0, ctx->stream>>>((const double*)ws, R, t->n, t->nchunk, t->F + d * mode);
    RSD_HIP(hipGetLastError());
    RSD_HIP(hipStreamSynchronize(ctx->stream));
  }
  return RSD_OK;
}

}  // namespace rsd

using namespace rsd;

// ================================================================ C ABI
extern "C" {

rsd_status rsd_version(int32_t* major, int32_t* minor) {
  if (major) *major = 1;
  if (minor) *minor = 0;
  return RSD_OK;
}

const char* rsd_last_error(void) { return g_err.c_str(); }

rsd_status rsd_context_create(int32_t device, void* hip_stream, size_t hbm_budget_bytes, rsd_context** out) {
  clear_error();
  RSD_CHECK(out != nullptr, RSD_E_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  RSD_HIP(hipGetDeviceCount(&count));
  RSD_CHECK(device >= 0 && device < count, RSD_E_INVALID, "device %d not present (%d devices)", device, count);
  RSD_HIP(hipSetDevice(device));
  rsd_context* c = new (std::nothrow) rsd_context();
  RSD_CHECK(c != nullptr, RSD_E_OOM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->budget = hbm_budget_bytes;
  const rsd_status st = noalloc_scratch_init(device);   // rsd_score_poses_noalloc's static scratch
  if (st != RSD_OK) {
    delete c;
    return st;
  }
  *out = c;
  return RSD_OK;
}

rsd_status rsd_context_set_stream(rsd_context* ctx, void* hip_stream) {
  clear_error();
  RSD_CHECK(ctx != nullptr, RSD_E_INVALID, "ctx is NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  RSD_HIP(hipStreamSynchronize(ctx->stream));
  RSD_TRY(ctx->collect_timers());
  ctx->stream = (hipStream_t)hip_stream;
  return RSD_OK;
}

rsd_status rsd_context_memory(const rsd_context* ctx, size_t* bytes_in_use, size_t* budget) {
  clear_error();
  RSD_CHECK(ctx != nullptr, RSD_E_INVALID, "ctx is NULL");
  if (bytes_in_use) *bytes_in_use = ctx->in_use;
  if (budget) *budget = ctx->budget;
  return RSD_OK;
}

void rsd_context_free(rsd_context* ctx) {
  if (!ctx || ctx->closing) return;
  if (ctx->live_tensors > 0) {   // released when the last of its tensors is freed
    ctx->closing = true;
    return;
  }
  context_destroy(ctx);
}

static rsd_status make_tensor(rsd_context* ctx, const double* const F[3], int64_t R, bool build, int32_t n,
                              double b, const rsd_sinc_params* sp, const double* charges,
                              const double* positions, int64_t N, uint32_t mem_flags, rsd_tensor** out) {
  clear_error();
  RSD_CHECK(out != nullptr, RSD_E_INVALID, "out is NULL");
  *out = nullptr;
  RSD_CHECK(ctx != nullptr && !ctx->closing, RSD_E_INVALID, "ctx is NULL or freed");
  RSD_TRY(check_sinc(sp));
  RSD_TRY(check_grid(n, b));
  RSD_CHECK(N >= (build ? 1 : 0) && N <= (int64_t)1 << 30, RSD_E_INVALID, "N=%lld out of range", (long long)N);
  RSD_CHECK(N == 0 || (charges && positions), RSD_E_INVALID, "charges/positions are NULL");
  const bool dev = is_device_ptrs(mem_flags);
  RSD_HIP(hipSetDevice(ctx->device));
  std::vector<double> z, pos;
  RSD_TRY(to_host(charges, (size_t)N, dev, &z));
  RSD_TRY(to_host(positions, 3 * (size_t)N, dev, &pos));
  RSD_TRY(check_protein(z, pos, n, b));
  rsd_tensor* t = new (std::nothrow) rsd_tensor();
  RSD_CHECK(t != nullptr, RSD_E_OOM, "host allocation failed");
  t->ctx = ctx;
  ctx->live_tensors += 1;
  double* d_z = nullptr;
  double* d_pos = nullptr;
  rsd_status st = tensor_common(ctx, t, n, b, sp, std::move(z), std::move(pos), &d_z, &d_pos);
  if (st == RSD_OK) {
    if (build) {
      t->galerkin = (ctx->opt_factors & 1) != 0;
      t->snapped = (ctx->opt_factors & 2) != 0;
      if (t->snapped) {
        // eq. 2.5: every charge moves to its nearest grid node, j = floor((x - X_0)/h + 1/2)
        // clipped to [0, n-1], at X_j = -b + (j + 1) h; the long-range factors are those of the
        // moved charges (a reference Gaussian centred on the node, windowed onto the grid), while
        // the short range and the vdW test keep the true positions
        std::vector<double> snap(t->host_positions.size());
        for (size_t i = 0; i < snap.size(); ++i) {
          double j = std::floor((t->host_positions[i] - t->X0) * t->inv_h + 0.5);
          j = std::min(std::max(j, 0.0), (double)(n - 1));
          snap[i] = -b + (j + 1.0) * t->h;
        }
        double* d_snap = nullptr;
        st = ctx->dev_alloc((void**)&d_snap, sizeof(double) * snap.size());
        if (st == RSD_OK) {
          hipError_t e = hipMemcpy(d_snap, snap.data(), sizeof(double) * snap.size(), hipMemcpyHostToDevice);
          if (e != hipSuccess) {
            set_error("hipMemcpy: %s", hipGetErrorString(e));
            st = RSD_E_HIP;
          }
          if (st == RSD_OK) st = build_factors(ctx, t, d_z, d_snap);
          (void)hipStreamSynchronize(ctx->stream);
          ctx->dev_free(d_snap, sizeof(double) * snap.size());
        }
      } else {
        st = build_factors(ctx, t, d_z, d_pos);
      }
    } else {
      st = import_factors(ctx, t, F, R, dev);
    }
  }
  if (st == RSD_OK) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
      st = RSD_E_HIP;
    }
  }
  ctx->dev_free(d_z, sizeof(double) * (size_t)(N ? N : 1));
  ctx->dev_free(d_pos, sizeof(double) * 3 * (size_t)(N ? N : 1));
  if (st != RSD_OK) {
    std::string keep = g_err;
    tensor_release(t);
    g_err = keep;
    return st;
  }
  *out = t;
  return RSD_OK;
}

rsd_status rsd_tensor_restrict(rsd_context* ctx, const rsd_tensor* src, const double lo[3], const double hi[3],
                               double eps, rsd_tensor** out) {
  clear_error();
  RSD_CHECK(out != nullptr, RSD_E_INVALID, "out is NULL");
  *out = nullptr;
  RSD_CHECK(ctx != nullptr && !ctx->closing, RSD_E_INVALID, "ctx is NULL or freed");
  RSD_CHECK(src != nullptr && lo != nullptr && hi != nullptr, RSD_E_INVALID, "NULL argument");
  RSD_CHECK(src->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(std::isfinite(eps) && eps > 0 && eps < 1, RSD_E_INVALID, "eps must be in (0, 1)");
  for (int d = 0; d < 3; ++d) {
    RSD_CHECK(std::isfinite(lo[d]) && std::isfinite(hi[d]) && lo[d] < hi[d], RSD_E_INVALID,
              "box axis %d: need finite lo < hi", d);
    RSD_CHECK(hi[d] >= src->X0m[d] && lo[d] <= src->X0m[d] + (src->nm[d] - 1) * src->h, RSD_E_INVALID,
              "box axis %d misses the grid", d);
  }
  RSD_HIP(hipSetDevice(ctx->device));
  rsd_sinc_params sp = src->sp;
  sp.eps = eps;
  rsd_tensor* t = new (std::nothrow) rsd_tensor();
  RSD_CHECK(t != nullptr, RSD_E_OOM, "host allocation failed");
  t->ctx = ctx;
  ctx->live_tensors += 1;
  double* d_z = nullptr;
  double* d_pos = nullptr;
  std::vector<double> z = src->host_charges, pos = src->host_positions;
  const int64_t N = (int64_t)z.size();
  rsd_status st = tensor_common(ctx, t, src->n, src->b, &sp, std::move(z), std::move(pos), &d_z, &d_pos);
  int i_lo[3] = {0, 0, 0};
  if (st == RSD_OK) {
    // the mesh is the source's (a restricted source's n is its largest row count, not the grid's)
    t->h = src->h;
    t->inv_h = src->inv_h;
    t->X0 = src->X0;
    // rows of the source grid that evaluation inside [lo, hi] reaches (the source may itself be
    // restricted: its mode d starts at row offset (X0m[d] - X0) / h of the full grid)
    int nmax = 0;
    for (int d = 0; d < 3; ++d) {
      int a = (int)std::floor((lo[d] - src->X0m[d]) * src->inv_h);
      int c = (int)std::floor((hi[d] - src->X0m[d]) * src->inv_h) + 1;
      a = std::min(std::max(a, 0), src->nm[d] - 2);
      c = std::min(std::max(c, a + 1), src->nm[d] - 1);
      i_lo[d] = a;
      t->nm[d] = c - a + 1;
      t->X0m[d] = src->X0m[d] + (double)a * src->h;
      nmax = std::max(nmax, t->nm[d]);
    }
    if (!src->restricted)   // rows of the full grid: origins as the grid nodes -b + (i + 1) h
      for (int d = 0; d < 3; ++d) t->X0m[d] = -src->b + (double)(i_lo[d] + 1) * src->h;
    t->n = nmax;
    t->restricted = true;
    const Tensor* one = src;
    st = reduce_factors(ctx, &one, 1, t, i_lo);
  }
  if (st == RSD_OK) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
      st = RSD_E_HIP;
    }
  }
  ctx->dev_free(d_z, sizeof(double) * (size_t)(N ? N : 1));
  ctx->dev_free(d_pos, sizeof(double) * 3 * (size_t)(N ? N : 1));
  if (st != RSD_OK) {
    std::string keep = g_err;
    tensor_release(t);
    g_err = keep;
    return st;
  }
  *out = t;
  return RSD_OK;
}

rsd_status rsd_tensor_combine(rsd_context* ctx, const rsd_tensor* const* tensors, int32_t count, double eps,
                              rsd_tensor** out) {
  clear_error();
  RSD_CHECK(out != nullptr, RSD_E_INVALID, "out is NULL");
  *out = nullptr;
  RSD_CHECK(ctx != nullptr && !ctx->closing, RSD_E_INVALID, "ctx is NULL or freed");
  RSD_CHECK(tensors != nullptr, RSD_E_INVALID, "tensors is NULL");
  RSD_CHECK(count >= 1 && count <= 4096, RSD_E_INVALID, "count %d outside [1, 4096]", (int)count);
  RSD_CHECK(std::isfinite(eps) && eps > 0 && eps < 1, RSD_E_INVALID, "eps must be in (0, 1)");
  const rsd_tensor* s0 = tensors[0];
  RSD_CHECK(s0 != nullptr, RSD_E_INVALID, "tensor 0 is NULL");
  std::vector<const Tensor*> src((size_t)count);
  size_t atoms = 0;
  for (int k = 0; k < count; ++k) {
    const rsd_tensor* sk = tensors[k];
    RSD_CHECK(sk != nullptr, RSD_E_INVALID, "tensor %d is NULL", k);
    RSD_CHECK(sk->ctx->device == ctx->device, RSD_E_INVALID, "tensor %d lives on another device", k);
    RSD_CHECK(sk->n == s0->n && sk->b == s0->b && sk->h == s0->h && sk->restricted == s0->restricted,
              RSD_E_UNSUPPORTED, "tensor %d is on another grid", k);
    for (int d = 0; d < 3; ++d)
      RSD_CHECK(sk->X0m[d] == s0->X0m[d] && sk->nm[d] == s0->nm[d], RSD_E_UNSUPPORTED,
                "tensor %d covers other rows of mode %d", k, d);
    RSD_CHECK(sk->sp.M == s0->sp.M && sk->sp.K_long == s0->sp.K_long && sk->sp.h_M == s0->sp.h_M &&
                  sk->sp.L_s == s0->sp.L_s && sk->sp.r_cut == s0->sp.r_cut,
              RSD_E_UNSUPPORTED, "tensor %d has other sinc parameters", k);
    src[k] = sk;
    atoms += sk->host_charges.size();
  }
  RSD_HIP(hipSetDevice(ctx->device));
  rsd_sinc_params sp = s0->sp;
  sp.eps = eps;
  std::vector<double> z, pos;
  z.reserve(atoms);
  pos.reserve(3 * atoms);
  for (const Tensor* sk : src) {
    z.insert(z.end(), sk->host_charges.begin(), sk->host_charges.end());
    pos.insert(pos.end(), sk->host_positions.begin(), sk->host_positions.end());
  }
  rsd_tensor* t = new (std::nothrow) rsd_tensor();
  RSD_CHECK(t != nullptr, RSD_E_OOM, "host allocation failed");
  t->ctx = ctx;
  ctx->live_tensors += 1;
  double* d_z = nullptr;
  double* d_pos = nullptr;
  const int64_t N = (int64_t)z.size();
  rsd_status st = tensor_common(ctx, t, s0->n, s0->b, &sp, std::move(z), std::move(pos), &d_z, &d_pos);
  if (st == RSD_OK) {
    t->h = s0->h;
    t->inv_h = s0->inv_h;
    t->X0 = s0->X0;
    for (int d = 0; d < 3; ++d) {
      t->X0m[d] = s0->X0m[d];
      t->nm[d] = s0->nm[d];
    }
    t->restricted = s0->restricted;
    const int i_lo[3] = {0, 0, 0};
    st = reduce_factors(ctx, src.data(), count, t, i_lo);
  }
  if (st == RSD_OK) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
      st = RSD_E_HIP;
    }
  }
  ctx->dev_free(d_z, sizeof(double) * (size_t)(N ? N : 1));
  ctx->dev_free(d_pos, sizeof(double) * 3 * (size_t)(N ? N : 1));
  if (st != RSD_OK) {
    std::string keep = g_err;
    tensor_release(t);
    g_err = keep;
    return st;
  }
  *out = t;
  return RSD_OK;
}

rsd_status rsd_self_energy(rsd_context* ctx, const rsd_tensor* t, double* E_long, double* E_short) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr && E_long != nullptr && E_short != nullptr, RSD_E_INVALID,
            "NULL argument");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(!t->restricted, RSD_E_UNSUPPORTED, "a restricted tensor does not cover the molecule's atoms");
  *E_long = 0.0;
  *E_short = 0.0;
  if (t->N == 0) return RSD_OK;
  RSD_HIP(hipSetDevice(ctx->device));
  return launch_self_energy(ctx, t, E_long, E_short);
}

rsd_status rsd_tensor_centre(const rsd_tensor* t, double centre[3]) {
  clear_error();
  RSD_CHECK(t != nullptr && centre != nullptr, RSD_E_INVALID, "NULL argument");
  RSD_CHECK(t->N > 0, RSD_E_INVALID, "the tensor has no atoms");
  double c[3] = {0.0, 0.0, 0.0};
  for (int64_t m = 0; m < t->N; ++m)
    for (int d = 0; d < 3; ++d) c[d] = c[d] + t->host_positions[3 * m + d];
  for (int d = 0; d < 3; ++d) centre[d] = c[d] / (double)t->N;
  return RSD_OK;
}

rsd_status rsd_contact_poses(rsd_context* ctx, const rsd_tensor* t, const double* lig_positions, int64_t L,
                             const double* dirs, int64_t U, const double* quats, int64_t Q, const double centre[3],
                             double sigma, double gap, double* rho, double* pose_quats, double* pose_trans) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr && centre != nullptr, RSD_E_INVALID, "NULL argument");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(L >= 1 && L <= kMaxLigand, RSD_E_UNSUPPORTED, "L=%lld outside [1, %d]", (long long)L, kMaxLigand);
  RSD_CHECK(U >= 0 && Q >= 0 && (U == 0 || Q <= ((int64_t)1 << 33) / U), RSD_E_INVALID, "U=%lld, Q=%lld out of range",
            (long long)U, (long long)Q);
  RSD_CHECK(std::isfinite(sigma) && sigma > 0, RSD_E_INVALID, "sigma must be finite and > 0");
  RSD_CHECK(std::isfinite(gap) && gap >= 0, RSD_E_INVALID, "gap must be finite and >= 0");
  for (int d = 0; d < 3; ++d) RSD_CHECK(std::isfinite(centre[d]), RSD_E_INVALID, "centre is not finite");
  if (U == 0 || Q == 0) return RSD_OK;
  RSD_CHECK(lig_positions && dirs && quats && rho && pose_quats && pose_trans, RSD_E_INVALID, "NULL array");
  RSD_HIP(hipSetDevice(ctx->device));
  return launch_contact(ctx, t, lig_positions, (int)L, dirs, U, quats, Q, centre, sigma, gap, rho, pose_quats,
                        pose_trans);
}

rsd_status rsd_orbit_minima(rsd_context* ctx, const double* energies, const uint8_t* flags, int64_t U, int64_t Q,
                            const int32_t* nbr_offsets, const int32_t* nbr_index, int32_t* best_rotation,
                            double* best_energy, uint8_t* is_minimum) {
  clear_error();
  RSD_CHECK(ctx != nullptr && !ctx->closing, RSD_E_INVALID, "ctx is NULL or freed");
  RSD_CHECK(U >= 0 && Q >= 1 && Q <= 0x7fffffff && (U == 0 || Q <= ((int64_t)1 << 33) / U), RSD_E_INVALID,
            "U=%lld, Q=%lld out of range", (long long)U, (long long)Q);
  if (U == 0) return RSD_OK;
  RSD_CHECK(energies && flags && nbr_offsets && nbr_index && best_rotation && best_energy && is_minimum,
            RSD_E_INVALID, "NULL array");
  RSD_HIP(hipSetDevice(ctx->device));
  // the neighbour lists steer device reads: check them on the host first
  std::vector<int32_t> off((size_t)U + 1);
  RSD_HIP(hipMemcpyAsync(off.data(), nbr_offsets, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost, ctx->stream));
  RSD_HIP(hipStreamSynchronize(ctx->stream));
  RSD_CHECK(off[0] == 0, RSD_E_INVALID, "nbr_offsets[0] must be 0");
  for (int64_t u = 0; u < U; ++u)
    RSD_CHECK(off[u + 1] >= off[u], RSD_E_INVALID, "nbr_offsets decrease at %lld", (long long)u);
  if (off[U] > 0) {
    std::vector<int32_t> idx((size_t)off[U]);
    RSD_HIP(hipMemcpyAsync(idx.data(), nbr_index, sizeof(int32_t) * idx.size(), hipMemcpyDeviceToHost, ctx->stream));
    RSD_HIP(hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k < idx.size(); ++k)
      RSD_CHECK(idx[k] >= 0 && idx[k] < U, RSD_E_INVALID, "nbr_index[%zu] = %d outside [0, %lld)", k, (int)idx[k],
                (long long)U);
  }
  return launch_orbit_minima(ctx, energies, flags, U, Q, nbr_offsets, nbr_index, best_rotation, best_energy,
                             is_minimum);
}

rsd_status rsd_tensor_grid(const rsd_tensor* t, double X0[3], int32_t rows[3], double* h) {
  clear_error();
  RSD_CHECK(t != nullptr, RSD_E_INVALID, "tensor is NULL");
  for (int d = 0; d < 3; ++d) {
    if (X0) X0[d] = t->X0m[d];
    if (rows) rows[d] = t->nm[d];
  }
  if (h) *h = t->h;
  return RSD_OK;
}

rsd_status rsd_build_rs_tensor(rsd_context* ctx, const double* charges, const double* positions, int64_t N,
                               int32_t n, double b, const rsd_sinc_params* sp, uint32_t mem_flags,
                               rsd_tensor** out) {
  return make_tensor(ctx, nullptr, 0, true, n, b, sp, charges, positions, N, mem_flags, out);
}

rsd_status rsd_tensor_import(rsd_context* ctx, const double* F1, const double* F2, const double* F3, int64_t R,
                             int32_t n, double b, const rsd_sinc_params* sp, const double* charges,
                             const double* positions, int64_t N, uint32_t mem_flags, rsd_tensor** out) {
  clear_error();
  RSD_CHECK(R >= 0 && R <= (int64_t)1 << 24, RSD_E_INVALID, "R=%lld out of range", (long long)R);
  RSD_CHECK(R == 0 || (F1 && F2 && F3), RSD_E_INVALID, "factor pointers are NULL");
  if (R > 0 && !is_device_ptrs(mem_flags)) {
    for (const double* F : {F1, F2, F3})
      for (int64_t e = 0; e < (int64_t)n * R; ++e)
        RSD_CHECK(std::isfinite(F[e]), RSD_E_INVALID, "factor entry %lld is not finite", (long long)e);
  }
  const double* F[3] = {F1, F2, F3};
  return make_tensor(ctx, F, R, false, n, b, sp, charges, positions, N, mem_flags, out);
}

rsd_status rsd_tensor_query(const rsd_tensor* t, int32_t* n, int64_t* R, int32_t ranks[3], size_t* bytes) {
  clear_error();
  RSD_CHECK(t != nullptr, RSD_E_INVALID, "tensor is NULL");
  if (n) *n = t->n;
  if (R) *R = t->R;
  if (ranks) {
    for (int d = 0; d < 3; ++d) ranks[d] = t->ranks[d];
  }
  if (bytes) *bytes = t->bytes();
  return RSD_OK;
}

rsd_status rsd_tensor_layout(const rsd_tensor* t, int32_t* nchunk, int32_t* shared_mode3) {
  clear_error();
  RSD_CHECK(t != nullptr, RSD_E_INVALID, "tensor is NULL");
  if (nchunk) *nchunk = t->nchunk;
  if (shared_mode3) *shared_mode3 = t->U3 ? t->u3_chunks : 0;
  return RSD_OK;
}

rsd_status rsd_probe_gather(rsd_context* ctx, int32_t n, int32_t iters, double* ms, double* bytes) {
  clear_error();
  RSD_CHECK(ctx != nullptr && ms != nullptr && bytes != nullptr, RSD_E_INVALID, "NULL argument");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_HIP(hipSetDevice(ctx->device));
  return probe_gather(ctx, n, iters, ms, bytes);
}

rsd_status rsd_tensor_export(const rsd_tensor* t, double* F1, double* F2, double* F3) {
  clear_error();
  RSD_CHECK(t != nullptr, RSD_E_INVALID, "tensor is NULL");
  RSD_CHECK(t->R == 0 || (F1 && F2 && F3), RSD_E_INVALID, "output pointers are NULL");
  if (t->R == 0) return RSD_OK;
  Context* ctx = t->ctx;
  RSD_HIP(hipSetDevice(ctx->device));
  const size_t one = sizeof(double) * (size_t)t->n * (size_t)t->R;
  void* ws = nullptr;
  RSD_TRY(ctx->workspace(one, &ws));
  double* out[3] = {F1, F2, F3};
  const int64_t mode = (int64_t)t->nchunk * t->n * kChunk;
  for (int d = 0; d < 3; ++d) {
    k_unlayout<<<1024, 256, 0, ctx->stream>>>(t->F + d * mode, t->R, t->n, (double*)ws);
    RSD_HIP(hipGetLastError());
    RSD_HIP(hipMemcpyAsync(out[d], ws, one, hipMemcpyDeviceToHost, ctx->stream));
    RSD_HIP(hipStreamSynchronize(ctx->stream));
  }
  return RSD_OK;
}

void rsd_tensor_free(rsd_tensor* t) { tensor_release(t); }

rsd_status rsd_score_poses_noalloc(rsd_context* ctx, const rsd_tensor* t, const double* lig_charges,
                                   const double* lig_positions, int64_t L, const double* quats, const double* trans,
                                   int64_t P, double vdw_min, uint32_t mem_flags, double* energies,
                                   double* energies_long, uint8_t* flags, int32_t* counts, double* grads) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr, RSD_E_INVALID, "ctx or tensor is NULL");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(is_device_ptrs(mem_flags), RSD_E_INVALID, "the allocation-free call takes device pointers only");
  RSD_CHECK(L >= 1 && L <= kMaxLigand, RSD_E_UNSUPPORTED, "L=%lld outside [1, %d]", (long long)L, kMaxLigand);
  RSD_CHECK(P >= 0 && P <= (int64_t)INT32_MAX, RSD_E_INVALID, "P=%lld out of range", (long long)P);
  RSD_CHECK(std::isfinite(vdw_min) && vdw_min >= 0, RSD_E_INVALID, "vdw_min must be finite and >= 0");
  RSD_CHECK(lig_charges && lig_positions, RSD_E_INVALID, "ligand pointers are NULL");
  if (P == 0) return RSD_OK;
  RSD_CHECK(quats && trans && energies && flags && counts, RSD_E_INVALID, "pose/output pointers are NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  ScoreIO io{};
  io.lig_charges = lig_charges;
  io.lig_positions = lig_positions;
  io.L = (int)L;
  io.quats = quats;
  io.trans = trans;
  io.P = P;
  io.vdw_min = vdw_min;
  io.E = energies;
  io.El = energies_long;
  io.flags = flags;
  io.counts = counts;
  io.grads = grads;
  return score_noalloc(ctx, t, io);
}

rsd_status rsd_score_poses(rsd_context* ctx, const rsd_tensor* t, const double* lig_charges,
                           const double* lig_positions, int64_t L, const double* quats, const double* trans,
                           int64_t P, double vdw_min, uint32_t mem_flags, double* energies,
                           double* energies_long, uint8_t* flags, int32_t* counts, double* grads) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr, RSD_E_INVALID, "ctx or tensor is NULL");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(L >= 1 && L <= kMaxLigand, RSD_E_UNSUPPORTED, "L=%lld outside [1, %d]", (long long)L, kMaxLigand);
  RSD_CHECK(P >= 0 && P <= (int64_t)INT32_MAX, RSD_E_INVALID, "P=%lld out of range", (long long)P);
  RSD_CHECK(std::isfinite(vdw_min) && vdw_min >= 0, RSD_E_INVALID, "vdw_min must be finite and >= 0");
  RSD_CHECK(lig_charges && lig_positions, RSD_E_INVALID, "ligand pointers are NULL");
  if (P == 0) return RSD_OK;
  RSD_CHECK(quats && trans && energies && flags && counts, RSD_E_INVALID, "pose/output pointers are NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  const bool dev = is_device_ptrs(mem_flags);
  ScoreIO io{};
  io.L = (int)L;
  io.P = P;
  io.vdw_min = vdw_min;
  if (dev) {
    io.lig_charges = lig_charges;
    io.lig_positions = lig_positions;
    io.quats = quats;
    io.trans = trans;
    io.E = energies;
    io.El = energies_long;
    io.flags = flags;
    io.counts = counts;
    io.grads = grads;
    return launch_score(ctx, t, io);
  }
  // host pointers: validate, stage, run, copy back, synchronise
  for (int64_t l = 0; l < L; ++l) {
    RSD_CHECK(std::isfinite(lig_charges[l]) && std::isfinite(lig_positions[3 * l]) &&
                  std::isfinite(lig_positions[3 * l + 1]) && std::isfinite(lig_positions[3 * l + 2]),
              RSD_E_INVALID, "ligand atom %lld is not finite", (long long)l);
  }
  for (int64_t p = 0; p < P; ++p) {
    const double* q = quats + 4 * p;
    const double* tt = trans + 3 * p;
    const double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    const bool ok = std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]) && std::isfinite(q[3]) &&
                    std::isfinite(tt[0]) && std::isfinite(tt[1]) && std::isfinite(tt[2]) &&
                    std::fabs(qq - 1.0) <= 1e-12;
    RSD_CHECK(ok, RSD_E_INVALID, "pose %lld: non-finite input or |q|^2 - 1 beyond 1e-12", (long long)p);
  }
  // staging buffer: inputs then outputs (separate from the context workspace used by the kernels)
  const size_t nin = (size_t)L * 4 + (size_t)P * 7;
  const size_t nout = (size_t)P * (2 + (grads ? 6 : 0));
  const size_t bytes = sizeof(double) * (nin + nout) + (size_t)P * (sizeof(int32_t) + 1) + 64;
  char* stage = nullptr;
  size_t stage_bytes = bytes;
  RSD_TRY(ctx->block_alloc((void**)&stage, &stage_bytes));
  double* d = (double*)stage;
  io.lig_charges = d;
  io.lig_positions = d + L;
  io.quats = d + 4 * L;
  io.trans = d + 4 * L + 4 * P;
  io.E = d + nin;
  io.El = io.E + P;
  io.grads = grads ? io.El + P : nullptr;
  io.counts = (int32_t*)(d + nin + nout);
  io.flags = (uint8_t*)(io.counts + P);
  hipStream_t s = ctx->stream;
  rsd_status st = RSD_OK;
  auto cp = [&](void* dst, const void* src, size_t n, hipMemcpyKind k) {
    if (st != RSD_OK || n == 0) return;
    hipError_t e = hipMemcpyAsync(dst, src, n, k, s);
    if (e != hipSuccess) {
      set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
      st = RSD_E_HIP;
    }
  };
  cp((void*)io.lig_charges, lig_charges, sizeof(double) * L, hipMemcpyHostToDevice);
  cp((void*)io.lig_positions, lig_positions, sizeof(double) * 3 * L, hipMemcpyHostToDevice);
  cp((void*)io.quats, quats, sizeof(double) * 4 * P, hipMemcpyHostToDevice);
  cp((void*)io.trans, trans, sizeof(double) * 3 * P, hipMemcpyHostToDevice);
  if (st == RSD_OK) st = launch_score(ctx, t, io);
  cp(energies, io.E, sizeof(double) * P, hipMemcpyDeviceToHost);
  if (energies_long) cp(energies_long, io.El, sizeof(double) * P, hipMemcpyDeviceToHost);
  cp(flags, io.flags, (size_t)P, hipMemcpyDeviceToHost);
  cp(counts, io.counts, sizeof(int32_t) * P, hipMemcpyDeviceToHost);
  if (grads) cp(grads, io.grads, sizeof(double) * 6 * P, hipMemcpyDeviceToHost);
  hipError_t e = hipStreamSynchronize(s);
  if (st == RSD_OK && e != hipSuccess) {
    set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
    st = RSD_E_HIP;
  }
  ctx->block_release(stage, stage_bytes);   // reused in stream order by later calls
  return st;
}

rsd_status rsd_pose_order(rsd_context* ctx, const rsd_tensor* t, const double* quats, const double* trans, int64_t P,
                          int32_t* perm, double* quats_out, double* trans_out, int32_t* sorted) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr && !ctx->closing, RSD_E_INVALID, "ctx or tensor is NULL or freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(P >= 0 && P <= ((int64_t)1 << 31) - 1, RSD_E_INVALID, "P=%lld out of range", (long long)P);
  RSD_CHECK(P == 0 || (trans && perm), RSD_E_INVALID, "trans or perm is NULL");
  RSD_CHECK(quats || !quats_out, RSD_E_INVALID, "quats_out needs quats");
  RSD_HIP(hipSetDevice(ctx->device));
  int flag = 0;
  const rsd_status st = pose_order(ctx, t, quats, trans, P, perm, quats_out, trans_out, &flag);
  if (sorted) *sorted = flag;
  return st;
}

// ---------------------------------------------------------------- launch-shape tuner
rsd_status rsd_autotune(rsd_context* ctx, const rsd_tensor* t, const double* lig_charges,
                        const double* lig_positions, int64_t L, const double* quats, const double* trans,
                        int64_t P, double vdw_min, int32_t grads, rsd_tune_report* report) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr, RSD_E_INVALID, "ctx or tensor is NULL");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(L >= 1 && L <= kMaxLigand, RSD_E_UNSUPPORTED, "L=%lld outside [1, %d]", (long long)L, kMaxLigand);
  RSD_CHECK(P >= 1 && P <= (int64_t)INT32_MAX, RSD_E_INVALID, "P=%lld out of range", (long long)P);
  RSD_CHECK(std::isfinite(vdw_min) && vdw_min >= 0, RSD_E_INVALID, "vdw_min must be finite and >= 0");
  RSD_CHECK(lig_charges && lig_positions && quats && trans, RSD_E_INVALID, "input pointers are NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  // scratch outputs: E | E_long unused | gradients | counts | flags
  size_t bytes = (size_t)P * (sizeof(double) * (1 + (grads ? 6 : 0)) + sizeof(int32_t) + 1) + 256;
  char* out = nullptr;
  RSD_TRY(ctx->block_alloc((void**)&out, &bytes));
  ScoreIO io{};
  io.lig_charges = lig_charges;
  io.lig_positions = lig_positions;
  io.L = (int)L;
  io.quats = quats;
  io.trans = trans;
  io.P = P;
  io.vdw_min = vdw_min;
  io.E = (double*)out;
  io.El = nullptr;
  io.grads = grads ? io.E + P : nullptr;
  io.counts = (int32_t*)(io.E + P * (grads ? 7 : 1));
  io.flags = (uint8_t*)(io.counts + P);
  const rsd_status st = rsd::autotune(ctx, t, io, report);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->block_release(out, bytes);
  return st;
}

rsd_status rsd_autotune_cells(rsd_context* ctx, rsd_tensor* t, const double* lig_charges,
                              const double* lig_positions, int64_t L, const double* quats, const double* trans,
                              int64_t P, double vdw_min, int32_t grads, int32_t* best_div, double* ms) {
  clear_error();
  RSD_CHECK(ctx != nullptr && t != nullptr, RSD_E_INVALID, "ctx or tensor is NULL");
  RSD_CHECK(!ctx->closing, RSD_E_INVALID, "context has been freed");
  RSD_CHECK(t->ctx->device == ctx->device, RSD_E_INVALID, "tensor lives on another device");
  RSD_CHECK(L >= 1 && L <= kMaxLigand, RSD_E_UNSUPPORTED, "L=%lld outside [1, %d]", (long long)L, kMaxLigand);
  RSD_CHECK(P >= 1 && P <= (int64_t)INT32_MAX, RSD_E_INVALID, "P=%lld out of range", (long long)P);
  RSD_CHECK(std::isfinite(vdw_min) && vdw_min >= 0, RSD_E_INVALID, "vdw_min must be finite and >= 0");
  RSD_CHECK(lig_charges && lig_positions && quats && trans, RSD_E_INVALID, "input pointers are NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  size_t bytes = (size_t)P * (sizeof(double) * (1 + (grads ? 6 : 0)) + sizeof(int32_t) + 1) + 256;
  char* out = nullptr;
  RSD_TRY(ctx->block_alloc((void**)&out, &bytes));
  ScoreIO io{};
  io.lig_charges = lig_charges;
  io.lig_positions = lig_positions;
  io.L = (int)L;
  io.quats = quats;
  io.trans = trans;
  io.P = P;
  io.vdw_min = vdw_min;
  io.E = (double*)out;
  io.El = nullptr;
  io.grads = grads ? io.E + P : nullptr;
  io.counts = (int32_t*)(io.E + P * (grads ? 7 : 1));
  io.flags = (uint8_t*)(io.counts + P);
  const rsd_status st = rsd::autotune_cells(ctx, t, io, best_div, ms);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->block_release(out, bytes);
  return st;
}

// ---------------------------------------------------------------- file I/O
static const char kMagic[8] = {'R', 'S', 'D', 'T', 'E', 'N', 'S', '1'};

static uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct FileHeader {
  char magic[8];
  uint32_t version;
  int32_t n;
  double b;
  int64_t R;
  int32_t ranks[3];
  int32_t pad;
  rsd_sinc_params sp;
  int64_t N;
};

rsd_status rsd_tensor_save(const rsd_tensor* t, const char* path) {
  clear_error();
  RSD_CHECK(t != nullptr && path != nullptr, RSD_E_INVALID, "tensor or path is NULL");
  RSD_CHECK(!t->restricted, RSD_E_UNSUPPORTED, "a tensor restricted to a sub-box cannot be saved");
  const size_t nR = (size_t)t->n * (size_t)t->R;
  std::vector<double> F(3 * nR);
  if (t->R > 0) RSD_TRY(rsd_tensor_export(t, F.data(), F.data() + nR, F.data() + 2 * nR));
  FileHeader hd{};
  std::memcpy(hd.magic, kMagic, 8);
  hd.version = 1;
  hd.n = t->n;
  hd.b = t->b;
  hd.R = t->R;
  for (int d = 0; d < 3; ++d) hd.ranks[d] = t->ranks[d];
  hd.sp = t->sp;
  hd.N = t->N;
  FILE* f = std::fopen(path, "wb");
  RSD_CHECK(f != nullptr, RSD_E_IO, "cannot open %s for writing", path);
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &hd, sizeof(hd));
  h = fnv1a(h, F.data(), sizeof(double) * F.size());
  h = fnv1a(h, t->host_charges.data(), sizeof(double) * t->host_charges.size());
  h = fnv1a(h, t->host_positions.data(), sizeof(double) * t->host_positions.size());
  bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1;
  ok = ok && (F.empty() || std::fwrite(F.data(), sizeof(double), F.size(), f) == F.size());
  ok = ok && (t->N == 0 || std::fwrite(t->host_charges.data(), sizeof(double), t->host_charges.size(), f) ==
                               t->host_charges.size());
  ok = ok && (t->N == 0 || std::fwrite(t->host_positions.data(), sizeof(double), t->host_positions.size(), f) ==
                               t->host_positions.size());
  ok = ok && std::fwrite(&h, sizeof(h), 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  RSD_CHECK(ok, RSD_E_IO, "write to %s failed", path);
  return RSD_OK;
}

rsd_status rsd_tensor_load(rsd_context* ctx, const char* path, rsd_tensor** out) {
  clear_error();
  RSD_CHECK(ctx != nullptr && path != nullptr && out != nullptr, RSD_E_INVALID, "NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  RSD_CHECK(f != nullptr, RSD_E_IO, "cannot open %s", path);
  FileHeader hd{};
  bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, kMagic, 8) == 0 && hd.version == 1 &&
            hd.R >= 0 && hd.R <= ((int64_t)1 << 24) && hd.N >= 0 && hd.N <= ((int64_t)1 << 30) && hd.n >= 4 &&
            hd.n <= 32768;
  if (!ok) {
    std::fclose(f);
    set_error("%s is not a tensor file of this version", path);
    return RSD_E_IO;
  }
  const size_t nR = (size_t)hd.n * (size_t)hd.R;
  std::vector<double> F(3 * nR), z((size_t)hd.N), pos(3 * (size_t)hd.N);
  uint64_t stored = 0;
  ok = (F.empty() || std::fread(F.data(), sizeof(double), F.size(), f) == F.size()) &&
       (z.empty() || std::fread(z.data(), sizeof(double), z.size(), f) == z.size()) &&
       (pos.empty() || std::fread(pos.data(), sizeof(double), pos.size(), f) == pos.size()) &&
       std::fread(&stored, sizeof(stored), 1, f) == 1;
  std::fclose(f);
  RSD_CHECK(ok, RSD_E_IO, "%s is truncated", path);
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &hd, sizeof(hd));
  h = fnv1a(h, F.data(), sizeof(double) * F.size());
  h = fnv1a(h, z.data(), sizeof(double) * z.size());
  h = fnv1a(h, pos.data(), sizeof(double) * pos.size());
  RSD_CHECK(h == stored, RSD_E_IO, "%s: checksum mismatch", path);
  RSD_TRY(rsd_tensor_import(ctx, F.data(), F.data() + nR, F.data() + 2 * nR, hd.R, hd.n, hd.b, &hd.sp, z.data(),
                            pos.data(), hd.N, 0u, out));
  for (int d = 0; d < 3; ++d) (*out)->ranks[d] = hd.ranks[d];
  return RSD_OK;
}

// ---------------------------------------------------------------- batches
struct rsd_batch {
  rsd::Batch* b;
  rsd_context* ctx;
};

rsd_status rsd_batch_create(rsd_context* ctx, const rsd_request* requests, int32_t n_requests, rsd_batch** out) {
  clear_error();
  RSD_CHECK(out != nullptr, RSD_E_INVALID, "out is NULL");
  *out = nullptr;
  RSD_CHECK(ctx != nullptr && !ctx->closing, RSD_E_INVALID, "ctx is NULL or freed");
  RSD_HIP(hipSetDevice(ctx->device));
  rsd::Batch* b = nullptr;
  RSD_TRY(rsd::batch_create(ctx, requests, n_requests, &b));
  rsd_batch* h = new (std::nothrow) rsd_batch{b, ctx};
  if (!h) {
    rsd::batch_free(b);
    set_error("host allocation failed");
    return RSD_E_OOM;
  }
  ctx->live_tensors += 1;   // the batch keeps its context alive like a tensor does
  *out = h;
  return RSD_OK;
}

rsd_status rsd_batch_run(rsd_batch* batch) {
  clear_error();
  RSD_CHECK(batch != nullptr, RSD_E_INVALID, "batch is NULL");
  RSD_HIP(hipSetDevice(batch->ctx->device));
  return rsd::batch_run(batch->b);
}

void rsd_batch_free(rsd_batch* batch) {
  if (!batch) return;
  rsd_context* ctx = batch->ctx;
  (void)hipSetDevice(ctx->device);
  rsd::batch_free(batch->b);
  delete batch;
  ctx->live_tensors -= 1;
  if (ctx->closing && ctx->live_tensors == 0) context_destroy(ctx);
}

// ---------------------------------------------------------------- tuning
rsd_status rsd_context_set_option(rsd_context* ctx, const char* name, int64_t value) {
  clear_error();
  RSD_CHECK(ctx != nullptr && name != nullptr, RSD_E_INVALID, "NULL argument");
  if (std::strcmp(name, "score_mode") == 0) {
    RSD_CHECK(value >= 0 && value <= 2, RSD_E_INVALID, "score_mode must be 0, 1 or 2");
    ctx->opt_score_mode = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "poses_per_wave") == 0) {
    RSD_CHECK(value >= 0 && value <= 4, RSD_E_INVALID, "poses_per_wave must be in [0, 4]");
    ctx->opt_poses_per_wave = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "eig_solver") == 0) {
    RSD_CHECK(value >= 0 && value <= 2, RSD_E_INVALID, "eig_solver must be 0, 1 or 2");
    ctx->opt_eig = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "t2c_solver") == 0) {
    RSD_CHECK(value >= 0 && value <= 3, RSD_E_INVALID, "t2c_solver must be 0, 1, 2 or 3");
    ctx->opt_t2c = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "short_waves") == 0) {
    RSD_CHECK(value == 0 || value == 1 || value == 2 || value == 4, RSD_E_INVALID, "short_waves must be 0, 1, 2 or 4");
    ctx->opt_short_waves = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "use_tuning") == 0) {
    RSD_CHECK(value == 0 || value == 1, RSD_E_INVALID, "use_tuning must be 0 or 1");
    ctx->opt_use_tuning = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "shared_mode3") == 0) {
    RSD_CHECK(value == 0 || value == 1, RSD_E_INVALID, "shared_mode3 must be 0 or 1");
    ctx->opt_shared_mode3 = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "short_poly") == 0) {
    RSD_CHECK(value == 0 || value == 1, RSD_E_INVALID, "short_poly must be 0 or 1");
    ctx->opt_short_poly = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "pose_order") == 0) {
    RSD_CHECK(value >= 0 && value <= 2, RSD_E_INVALID, "pose_order must be 0, 1 or 2");
    ctx->opt_pose_order = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "chunks_per_item") == 0) {
    RSD_CHECK(value >= 0 && value <= 4, RSD_E_INVALID, "chunks_per_item must be 0 .. 4");
    ctx->opt_cpi = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "qr_solver") == 0) {
    RSD_CHECK(value == 0 || value == 1, RSD_E_INVALID, "qr_solver must be 0 or 1");
    ctx->opt_qr = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "batch_mode") == 0) {
    RSD_CHECK(value >= 0 && value <= 2, RSD_E_INVALID, "batch_mode must be 0, 1 or 2");
    ctx->opt_batch_mode = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "overlap") == 0) {
    RSD_CHECK(value == 0 || value == 1, RSD_E_INVALID, "overlap must be 0 or 1");
    ctx->opt_overlap = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "factors") == 0) {
    RSD_CHECK(value >= 0 && value <= 3, RSD_E_INVALID, "factors must be 0, 1, 2 or 3");
    ctx->opt_factors = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "svd_solver") == 0) {
    RSD_CHECK(value >= 0 && value <= 4, RSD_E_INVALID, "svd_solver must be 0, 1, 2, 3 or 4");
    ctx->opt_svd = (int)value;
    return RSD_OK;
  }
  if (std::strcmp(name, "gram_solver") == 0) {
    RSD_CHECK(value >= 0 && value <= 2, RSD_E_INVALID, "gram_solver must be 0, 1 or 2");
    ctx->opt_gram = (int)value;
    return RSD_OK;
  }
  set_error("unknown option '%s'", name);
  return RSD_E_INVALID;
}

// ---------------------------------------------------------------- timing
rsd_status rsd_context_set_timing(rsd_context* ctx, int32_t enable) {
  clear_error();
  RSD_CHECK(ctx != nullptr, RSD_E_INVALID, "ctx is NULL");
  RSD_HIP(hipSetDevice(ctx->device));
  RSD_TRY(ctx->collect_timers());
  ctx->timing = enable != 0;
  ctx->ktime.clear();
  return RSD_OK;
}

rsd_status rsd_kernel_time(rsd_context* ctx, const char* kernel, int64_t* launches, double* total_ms) {
  clear_error();
  RSD_CHECK(ctx != nullptr && kernel != nullptr, RSD_E_INVALID, "NULL argument");
  RSD_HIP(hipSetDevice(ctx->device));
  RSD_TRY(ctx->collect_timers());
  auto it = ctx->ktime.find(kernel);
  if (launches) *launches = it == ctx->ktime.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == ctx->ktime.end() ? 0.0 : it->second.second;
  return RSD_OK;
}

}  // extern "C"
