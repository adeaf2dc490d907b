// Host-side checks of librsdock built with AddressSanitizer and UndefinedBehaviorSanitizer on
// its host code (device code is built as usual).  Runs without a GPU: every C-ABI entry point
// with missing or invalid arguments, the host argument checks, the quadrature table and the
// short-range polynomial table of the two reference quadratures.  Exit status 0 when every
// check holds; the sanitizers abort the run on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

static int failures = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

int main() {
  int32_t major = 0, minor = 0;
  EXPECT(rsd_version(&major, &minor) == RSD_OK && major >= 1);
  // null handles and outputs: argument errors before any device call, with a message
  EXPECT(rsd_context_create(0, nullptr, 0, nullptr) == RSD_E_INVALID);
  EXPECT(std::strlen(rsd_last_error()) > 0);
  double one = 1.0, pos[3] = {0, 0, 0}, q[4] = {1, 0, 0, 0}, E = 0;
  uint8_t fl = 0;
  int32_t cnt = 0;
  EXPECT(rsd_score_poses(nullptr, nullptr, &one, pos, 1, q, pos, 1, 2.5, 0, &E, nullptr, &fl, &cnt, nullptr) ==
         RSD_E_INVALID);
  EXPECT(rsd_score_poses_noalloc(nullptr, nullptr, &one, pos, 1, q, pos, 1, 2.5, RSD_DEVICE_PTRS, &E, nullptr, &fl,
                                 &cnt, nullptr) == RSD_E_INVALID);
  rsd_sinc_params sp{24, 12, 0.2622, 83.14, 43.8, 1e-8};
  rsd_tensor* t = nullptr;
  EXPECT(rsd_build_rs_tensor(nullptr, &one, pos, 1, 512, 24.0, &sp, 0, &t) == RSD_E_INVALID && t == nullptr);
  int32_t n = 0, ranks[3];
  int64_t R = 0;
  size_t bytes = 0;
  EXPECT(rsd_tensor_query(nullptr, &n, &R, ranks, &bytes) == RSD_E_INVALID);
  EXPECT(rsd_tensor_layout(nullptr, &n, &n) == RSD_E_INVALID);
  EXPECT(rsd_tensor_export(nullptr, nullptr, nullptr, nullptr) == RSD_E_INVALID);
  double ms = 0, b = 0;
  EXPECT(rsd_probe_gather(nullptr, 2048, 16, &ms, &b) == RSD_E_INVALID);
  EXPECT(rsd_context_set_option(nullptr, "score_mode", 0) == RSD_E_INVALID);
  rsd_tensor_free(nullptr);
  rsd_context_free(nullptr);
  // without a GPU the context cannot be made; with one it can (then free it)
  rsd_context* ctx = nullptr;
  const rsd_status st = rsd_context_create(0, nullptr, 0, &ctx);
  EXPECT(st == RSD_OK || st == RSD_E_HIP || st == RSD_E_INVALID);
  if (st == RSD_OK) rsd_context_free(ctx);

  // host argument checks
  EXPECT(rsd::check_sinc(&sp) == RSD_OK);
  rsd_sinc_params bad = sp;
  bad.M = 64;
  EXPECT(rsd::check_sinc(&bad) == RSD_E_INVALID);
  bad = sp;
  bad.h_M = std::nan("");
  EXPECT(rsd::check_sinc(&bad) == RSD_E_INVALID);
  EXPECT(rsd::check_sinc(nullptr) == RSD_E_INVALID);
  EXPECT(rsd::check_grid(512, 24.0) == RSD_OK);
  EXPECT(rsd::check_grid(511, 24.0) != RSD_OK);
  EXPECT(rsd::check_grid(512, -1.0) != RSD_OK);
  std::vector<double> z = {0.3, -0.3}, x = {0, 0, 0, 1, 1, 1};
  EXPECT(rsd::check_protein(z, x, 512, 24.0) == RSD_OK);
  x[4] = 1e9;
  EXPECT(rsd::check_protein(z, x, 512, 24.0) != RSD_OK);
  x[4] = std::nan("");
  EXPECT(rsd::check_protein(z, x, 512, 24.0) != RSD_OK);

  // quadrature and short-range tables of the 200-atom and 5,000-atom workloads' quadratures
  const rsd_sinc_params qs[2] = {{24, 12, 0.2622, 83.138438763306, 43.836, 1e-8},
                                 {32, 22, 0.2239, 180.13328398716, 15.963, 1e-8}};
  for (const auto& p : qs) {
    double tk[rsd::kMaxTerms], wk[rsd::kMaxTerms];
    rsd::sinc_table(p, tk, wk);
    double g1 = 0.0;   // the Gaussian sum at r = 1 A approximates 1/r
    for (int k = 0; k <= p.M; ++k) g1 += wk[k] * std::exp(-tk[k] * tk[k]);
    EXPECT(std::fabs(g1 - 1.0) < 1e-6);
    rsd::ShortTable sh{};
    sh.S = p.M + 1 - p.K_long;
    for (int k = 0; k < sh.S; ++k) {
      sh.t2[k] = tk[p.K_long + k] * tk[p.K_long + k];
      sh.w[k] = wk[p.K_long + k];
    }
    std::vector<double> coef;
    int n1 = 0;
    double x1 = 0, d1 = 0, d2 = 0;
    const bool ok = rsd::build_short_poly(sh, p.r_cut * p.r_cut, &coef, &n1, &x1, &d1, &d2);
    EXPECT(ok && !coef.empty() && n1 > 0 && d1 > 0 && d2 > 0);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
