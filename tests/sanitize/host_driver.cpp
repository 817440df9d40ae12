// Host-side checks of libps under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by tests/test_sanitize.py with the sanitizers on the host code only;
// no GPU is touched).  Exercises the host-only entry points and the argument
// validation of the device entry points, which must reject each call before
// any HIP call.  Exit status 0 when every expectation holds.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "ps.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
  do {                                                                      \
    if (!(cond)) {                                                          \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

int main() {
  // coefficients
  std::vector<double> c(171), p(61), q(61), cc(86);
  EXPECT(ps_coef_taylor_exp(170, c.data()) == PS_OK);
  EXPECT(c[0] == 1.0 && c[1] == 1.0 && c[2] == 0.5);
  EXPECT(ps_coef_taylor_exp(171, c.data()) == PS_ERR_ARG);
  EXPECT(ps_coef_pade_exp(60, p.data(), q.data()) == PS_OK);
  EXPECT(ps_coef_pade_exp(61, p.data(), q.data()) == PS_ERR_ARG);
  EXPECT(ps_coef_taylor_cos(85, cc.data()) == PS_OK);
  // planner over random-ish norms, every dtype, r up to the limit
  for (int r = 0; r < PS_MAX_BLOCKS; r += 7)
    for (int dt = 0; dt <= 2; ++dt) {
      std::vector<double> nb(r + 1), u(r + 1);
      std::vector<int> tier(r + 1);
      for (int i = 0; i <= r; ++i) nb[i] = 1.0 / (1.0 + i * i * i);
      int nu = -1;
      ps_opts o;
      memset(&o, 0, sizeof o);
      o.mode = PS_MODE_MIXED;
      EXPECT(ps_plan((ps_dtype)dt, r, nb.data(), 0.5, &o, tier.data(), u.data(), &nu) == PS_OK);
      EXPECT(nu >= 1 && nu <= r + 1);
      double cr = -1, ml = -1;
      EXPECT(ps_model_cost((ps_dtype)dt, 4, r, tier.data(), &cr, &ml) == PS_OK);
      EXPECT(cr >= 0.0 && cr < 1.0 && ml >= 0.0 && ml <= 1.0);
      nb[0] = 0.0;
      EXPECT(ps_plan((ps_dtype)dt, r, nb.data(), 0.0, &o, tier.data(), u.data(), &nu) == PS_OK);
    }
  EXPECT(ps_plan(PS_F64, PS_MAX_BLOCKS, nullptr, 1.0, nullptr, nullptr, nullptr, nullptr) == PS_ERR_ARG);
  double th = 0;
  for (int m = 0; m <= 170; m += 17) EXPECT(ps_theta_taylor(PS_F64, m, &th) == PS_OK && th > 0);
  // workspace sizes
  size_t b = 0;
  EXPECT(ps_workspace_size(PS_F64, 1024, 30, 6, 6, &b) == PS_OK && b > 0);
  EXPECT(ps_workspace_size(PS_F32, 1, 0, 0, 0, &b) == PS_OK);
  EXPECT(ps_workspace_size(PS_F64, 0, 30, 6, 6, &b) == PS_ERR_ARG);
  EXPECT(ps_workspace_size_auto(PS_F64, 100, 30, 6, &b) == PS_OK);
  EXPECT(ps_workspace_size_select(PS_F64, 100, 170, &b) == PS_OK);
  EXPECT(ps_workspace_size_vars(PS_F32, 100, 40, 2, &b) == PS_OK);
  EXPECT(ps_workspace_size_dd(100, 30, 6, 2, &b) == PS_OK);
  int degs[3] = {13, 13, 12};
  EXPECT(ps_workspace_size_multi(PS_F64, 200, 3, degs, 0, 1, &b) == PS_OK);
  EXPECT(ps_workspace_size_strided(PS_F64, 7, 64, 18, 5, 2, &b) == PS_OK);
  int32_t ns[5] = {1, 8, 64, 65, 256}, ss[5] = {0, 4, 5, 0, 4};
  EXPECT(ps_workspace_size_batched(PS_F32, 5, ns, 18, ss, &b) == PS_OK);
  EXPECT(ps_workspace_size_backward(PS_F32, 3, 128, 18, 5, 3, 1, &b) == PS_OK);
  EXPECT(ps_workspace_size_solve(PS_F64, 2048, &b) == PS_OK);
  EXPECT(ps_workspace_size_pade(PS_F64, 300, 13, 0, 2, &b) == PS_OK);
  // device entry points: rejected on the host (fake device addresses, never touched)
  void* A = (void*)0x10000000;
  void* E = (void*)0x20000000;
  void* W = (void*)0x40000000;
  EXPECT(ps_expm(PS_F64, 0, A, 1, nullptr, 6, 0, 0, E, 1, nullptr, nullptr, W, 1 << 30, nullptr) == PS_ERR_ARG);
  EXPECT(ps_expm(PS_F64, 4, A, 4, nullptr, 6, 0, 0, A, 4, nullptr, nullptr, W, 1 << 30, nullptr) == PS_ERR_ALIAS);
  EXPECT(ps_expm(PS_F64, 4, A, 4, nullptr, 6, 0, 0, E, 4, nullptr, nullptr, W, 16, nullptr) == PS_ERR_WORKSPACE);
  EXPECT(ps_expm_noalloc(PS_F64, 4096, A, 4096, nullptr, 30, 6, 2, E, 4096, nullptr, nullptr, nullptr) ==
         PS_ERR_WORKSPACE);
  EXPECT(ps_expm_noalloc(PS_F64, 4, A, 3, nullptr, 6, 0, 501, E, 4, nullptr, nullptr, nullptr) == PS_ERR_ARG);
  ps_opts bad;
  memset(&bad, 0, sizeof bad);
  bad.mode = 7;
  EXPECT(ps_eval(PS_F64, 4, A, 4, c.data(), 6, 0, E, 4, &bad, nullptr, W, 1 << 30, nullptr) == PS_ERR_ARG);
  const double* cps[2] = {p.data(), q.data()};
  void* outs[2] = {E, E};
  int64_t lds[2] = {4, 4};
  int dg[2] = {13, 13};
  EXPECT(ps_eval_multi(PS_F64, 4, A, 4, 2, cps, dg, 4, 0, outs, lds, nullptr, nullptr, W, 1 << 30, nullptr) ==
         PS_ERR_ALIAS);
  const void* As[2] = {A, E};
  void* Es[2] = {E, A};
  int64_t la[2] = {8, 8};
  int32_t n2[2] = {8, 300};
  EXPECT(ps_expm_batched(PS_F32, 2, n2, As, la, nullptr, 18, nullptr, nullptr, Es, la, nullptr, nullptr, W,
                         1 << 30, nullptr) == PS_ERR_ARG);
  EXPECT(ps_solve(PS_F64, 9000, A, 9000, 1, E, 9000, nullptr, nullptr, W, 1 << 30, nullptr) ==
         PS_ERR_UNSUPPORTED);
  EXPECT(ps_expm_pade(PS_F64, 4, A, 4, 61, 0, 0, E, 4, nullptr, nullptr, W, 1 << 30, nullptr) == PS_ERR_ARG);
  EXPECT(ps_expm_backward(PS_F32, 1, 8, A, 8, 64, A, 8, 64, nullptr, 6, 0, 0, A, 8, 64, 0, nullptr, W, 1 << 30,
                          nullptr) == PS_ERR_ALIAS);
  EXPECT(ps_expm_dd(8, (const double*)A, 4, nullptr, 6, 0, 0, (double*)E, 8, nullptr, nullptr, W, 1 << 30,
                    nullptr) == PS_ERR_ARG);
  EXPECT(ps_expm_auto(PS_F64, 4, A, 4, 171, 0, 0, E, 4, nullptr, nullptr, nullptr, W, 1 << 30, nullptr) ==
         PS_ERR_ARG);
  EXPECT(ps_expm_select(PS_F64, 4, A, 4, 0, E, 4, nullptr, nullptr, nullptr, W, 1 << 30, nullptr) == PS_ERR_ARG);
  EXPECT(strlen(ps_last_error()) > 0);
  for (int st = -6; st <= 0; ++st) EXPECT(ps_strerror(st) != nullptr);
  if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
  else printf("host driver: all expectations hold\n");
  return failures ? 1 : 0;
}
