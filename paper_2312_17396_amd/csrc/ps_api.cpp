// Host side of libps: argument validation, workspace layout and the launch
// sequence of the PS hot path.  See include/ps.h for the contract.
//
// Launch sequence for one evaluation (Algorithm 1 / Algorithm 3 with fixed s,
// X = beta * A, beta = 2^-sigma for the scaling-and-squaring driver):
//   1. power table  X_2 = beta^2 (A A), X_{j+1} = beta (X_j A)    s-1 GEMMs
//   2. k_assemble   B_0..B_r, ||B_i||_1, ||Y||_1, low-precision copies of Y
//   3. k_plan       tiers of the Horner products (on the device)
//   4. Horner       cast of the first block into its step's format, then
//                   P_{i-1} = B_{i-1} + P_i Y for i = first..1
//   5. squarings    R <- R R, sigma times (eq. (scal-idea))
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ps_internal.h"
#include "ps_planner.h"

using namespace psk;

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ps_status fail(ps_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define PS_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(PS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)


size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int default_s(int m) {
  if (m <= 1) return 1;
  int s = (int)ceil(sqrt((double)m));
  while ((s - 1) * (s - 1) >= m) --s;
  while (s * s < m) ++s;
  return s;
}

// exact-rational coefficients rounded once: the dd value of the rational
// (relative error ~1e-32) rounded to double is the correctly rounded double
// unless the rational lies within 1e-32 of a rounding boundary.
struct DD { double hi, lo; };
DD dd_two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
DD dd_div_int(DD x, double k) {  // x / k for a small positive integer k
  double q1 = x.hi / k;
  double p = q1 * k;
  double e = fma(q1, k, -p);
  double r = ((x.hi - p) - e) + x.lo;
  double q2 = r / k;
  DD s = dd_two_sum(q1, q2);
  return s;
}

bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

size_t mat_span_bytes(int64_t n, int64_t ld, int esize) {
  return (size_t)((n - 1) * ld + n) * esize;
}

struct Opts {
  int mode = PS_MODE_FIXED;
  unsigned mask = 0xF;
  double delta = 10.0;
  const int* override_tiers = nullptr;
  int profile = 0;
  int rule = PS_RULE_BLOCKS;
  int check_finite = 0;
};

Opts read_opts(const ps_opts* o, int working) {
  Opts r;
  if (o) {
    r.mode = o->mode;
    r.mask = o->tier_mask ? o->tier_mask : 0xF;
    r.delta = o->delta > 0 ? o->delta : 10.0;
    r.override_tiers = o->tier_override;
    r.profile = o->profile;
    r.rule = o->rule;
    r.check_finite = o->check_finite;
  }
  r.mask |= 1u << working;
  for (int t = 0; t < working; ++t) r.mask &= ~(1u << t);
  return r;
}

}  // namespace

namespace psk {

Layout make_layout(ps_dtype dt, int64_t n, int m, int s, int sigma, int square_arg, int npow_min, int colsum_rows) {
  Layout L;
  memset(&L, 0, sizeof L);
  L.n = n;
  L.m = m;
  L.s = s;
  L.r = m / s;
  L.sigma = sigma;
  L.working = dt == PS_F64 ? 0 : 1;
  L.esize = dt == PS_F64 ? 8 : 4;
  L.square_arg = square_arg;
  L.trivial_last = (L.r >= 1 && m == s * L.r) ? 1 : 0;
  L.nB = L.trivial_last ? L.r : L.r + 1;
  L.first_step = L.trivial_last ? L.r - 1 : L.r;
  L.Mp = round_up(n, kTile);
  L.Kp = round_up(n, kKPad);
  L.slot = al256((size_t)n * n * L.esize);
  size_t packed8 = (size_t)L.Mp * L.Kp + (size_t)L.Mp * (L.Kp / 32);
  size_t packed16 = (size_t)L.Mp * L.Kp * 2;
  L.pslot = al256(std::max({L.slot, packed8, packed16}));
  size_t off = 0;
  L.npow = std::max((s >= 2 ? s - 1 : 0) + (square_arg ? 1 : 0), npow_min);
  L.off_pow = off;   off += L.npow * L.slot;
  L.off_B = off;     off += (size_t)L.nB * L.slot;
  L.off_P0 = off;    off += L.pslot;
  L.off_P1 = off;    off += L.pslot;
  L.off_R = off;     off += (sigma > 0 ? L.slot : 0);
  L.off_yf32 = off;  off += (L.working == 0 ? al256((size_t)n * n * 4) : 0);
  L.off_ybf16 = off; off += al256((size_t)L.Mp * L.Kp * 2);
  L.off_yfp8 = off;  off += al256((size_t)L.Mp * L.Kp);
  L.off_yfp8s = off; off += al256((size_t)L.Mp * (L.Kp / 32));
  L.colsum_rows = colsum_rows;
  L.off_colsum = off; off += al256((size_t)(L.nB + 2) * ((n + colsum_rows - 1) / colsum_rows) * n * 8);
  L.off_plan = off;  off += al256(sizeof(Plan));
  L.bytes = al256(off);
  return L;
}

}  // namespace psk

namespace {

// Validation shared by the single / strided entry points.
ps_status check_common(ps_dtype dt, int64_t n, int m, int* s, int sigma) {
  if (dt != PS_F64 && dt != PS_F32) return fail(PS_ERR_ARG, "dtype must be PS_F64 or PS_F32");
  if (n < 1 || n > (1LL << 20)) return fail(PS_ERR_ARG, "n = %lld out of range [1, 2^20]", (long long)n);
  if (m < 0 || m > kMaxDegree) return fail(PS_ERR_ARG, "degree m = %d out of range [0, %d]", m, kMaxDegree);
  if (*s == 0) *s = default_s(m);
  if (*s < 1 || *s > std::max(m, 1)) return fail(PS_ERR_ARG, "block size s = %d out of range [1, max(m,1)]", *s);
  if (m / *s + 1 > PS_MAX_BLOCKS) return fail(PS_ERR_ARG, "r + 1 = %d exceeds %d blocks", m / *s + 1, PS_MAX_BLOCKS);
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range [0, %d]", sigma, kMaxSigma);
  return PS_OK;
}

ps_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
  if (ws_bytes < need) return fail(PS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (need && !ws) return fail(PS_ERR_WORKSPACE, "workspace pointer is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(PS_ERR_WORKSPACE, "workspace pointer not 256-byte aligned");
  return PS_OK;
}

ps_status check_opts(const Opts& o) {
  if (o.mode != PS_MODE_FIXED && o.mode != PS_MODE_MIXED) return fail(PS_ERR_ARG, "opts.mode must be 0 or 1");
  if (o.rule != PS_RULE_BLOCKS && o.rule != PS_RULE_APRIORI) return fail(PS_ERR_ARG, "opts.rule must be 0 or 1");
  return PS_OK;
}

// One PS evaluation (+ squarings) for a uniform batch, all matrices sharing L.
struct Job {
  const Layout* L;
  int batch;
  MatArg X1;             // base matrix of the power table (A, or Z = A^2 in the workspace)
  double beta;           // X_1 = beta * X1
  const double* coef;
  MatArg out;            // final result
  char* ws;
  size_t ws_stride;
  Opts opts;
  bool write_y;          // produce the low-precision copies of Y (first polynomial only)
  bool build_powers;     // run the power table (first polynomial only)
  bool skip_square;      // squarings handled by the caller
  int pow_shift = 0;     // power slots hold 2^(-j pow_shift) X_j (prebuilt, exact rescaling)
  bool y32 = false;      // Y = X_s lives in the slot of its FP32 copy (y32_allowed)
};

// Y = X_s formed by an FP32 product under an FP64 working precision.  By
// eq. (cond-Y) Y needs the accuracy u_nu of the first lower-precision Horner
// step; the FP32 product's error (~5.4 u32 measured) meets it when that step
// is BF16 or FP8, or FP32 with u_nu >= kY32Margin u32.  The plan is only
// known on the device, so each polynomial's cast launch forms Y in FP64 too
// (and rounds it into the FP32 copy) whenever its plan keeps a product in
// FP64 or has an FP32 product below that margin (the report counts it).  Only for n > 512: below that an n^3 product is bound
// by latency, so FP32 saves nothing and a second product in FP64 would add
// its latency.  Decided by the caller for all jobs sharing the powers.
bool y32_allowed(const Layout& L, const Opts& o) {
  return L.working == 0 && L.n > 512 && L.s >= 2 && (o.mode == PS_MODE_MIXED || o.override_tiers) &&
         ((o.mask >> 1) & 1u);
}

MatArg ws_mat(char* ws, size_t off, int64_t n, size_t stride_bytes, int esize) {
  MatArg a;
  a.p = ws + off;
  a.ld = n;
  a.stride = (int64_t)(stride_bytes / esize);
  return a;
}

// eq. (Cr) as the saving and Table 2's M_low from a plan's tiers (host)
void model_cost(int working, int s, int r, const int* tier, double* saving, double* m_low) {
  const double D = -std::log10(tier_unit_roundoff(working));
  const double half = std::sqrt(tier_unit_roundoff(working));
  // 1 - ((s-1) D + sum d_i) / ((s+r-1) D) written as sum (D - d_i) / ((s+r-1) D),
  // which is exactly 0 when every product runs in the working precision
  double gap = 0.0;
  int low = 0;
  for (int i = 1; i <= r; ++i) {
    const double ut = tier_unit_roundoff(tier[i]);
    gap += D + std::log10(ut);
    low += ut >= half ? 1 : 0;
  }
  const int prods = s - 1 + r;
  *saving = prods > 0 ? gap / (prods * D) : 0.0;
  *m_low = prods > 0 ? (double)low / prods : 0.0;
}

// opts.check_finite: one counting pass over `batch` matrices, then a
// read-back in chunks of a stack buffer (no allocation); wg: device scratch of
// norm1_groups(n) doubles per matrix, wg_stride bytes apart
ps_status nonfinite_or_ok(int W, int64_t n, int batch, MatArg M, char* wg, size_t wg_stride, hipStream_t st,
                          const char* what) {
  PS_HIP(launch_count_nonfinite(W, n, batch, M, wg, wg_stride, st));
  const int64_t G = norm1_groups(n);
  double h[256];
  for (int b = 0; b < batch; ++b)
    for (int64_t g0 = 0; g0 < G; g0 += 256) {
      const int64_t cnt = std::min<int64_t>(256, G - g0);
      PS_HIP(hipMemcpyAsync(h, (const double*)(wg + (size_t)b * wg_stride) + g0, cnt * sizeof(double),
                            hipMemcpyDeviceToHost, st));
      PS_HIP(hipStreamSynchronize(st));
      for (int64_t k = 0; k < cnt; ++k)
        if (h[k] != 0.0) return fail(PS_ERR_NONFINITE, "%s %d holds NaN or infinite entries", what, b);
    }
  return PS_OK;
}

struct Timer {
  bool on = false;
  hipEvent_t ev[8];
  int k = 0;
  hipStream_t st;
  ps_status init(bool enable, hipStream_t s) {
    on = enable;
    st = s;
    if (!on) return PS_OK;
    for (auto& e : ev) PS_HIP(hipEventCreate(&e));
    return PS_OK;
  }
  ps_status mark() {
    if (on) PS_HIP(hipEventRecord(ev[k++], st));
    return PS_OK;
  }
  float between(int a, int b) {
    float ms = 0.f;
    if (on && b < k) (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms;
  }
  ~Timer() {
    if (on) for (auto& e : ev) (void)hipEventDestroy(e);
  }
};

ps_status run_job(const Job& J, hipStream_t st, float* phase_ms /*4 or null*/) {
  const Layout& L = *J.L;
  const int W = L.working;
  const int64_t n = L.n;
  const size_t wss = J.ws_stride;
  Timer tm;
  if (ps_status e = tm.init(phase_ms != nullptr, st)) return e;
  if (ps_status e = tm.mark()) return e;
  // 1. power table
  auto power = [&](int j) {
    return j == 1 ? J.X1 : ws_mat(J.ws, L.off_pow + (size_t)(j - 2 + (L.square_arg ? 1 : 0)) * L.slot, n, wss, L.esize);
  };
  auto power_alpha = [&](int j) { return (pow_a(j) == 1 ? J.beta : 1.0) * (pow_b(j) == 1 ? J.beta : 1.0); };
  const bool yl = J.y32;
  if (J.build_powers && L.s >= 2) {
    // X_j = X_a X_b (a = ceil(j/2), b = floor(j/2)), one grouped launch per
    // level (j in (2^(l-1), 2^l]); X_1 = beta X1 enters through alpha
    for (int top = 2; top / 2 < L.s; top *= 2) {
      const int lo = top / 2 + 1, hi = std::min(top, L.s);   // level: j in (top/2, top]
      for (int j0 = lo; j0 <= hi; j0 += kMaxGroup) {
        GemmGroup g;
        memset(&g, 0, sizeof g);
        for (int j = j0; j <= std::min(hi, j0 + kMaxGroup - 1); ++j) {
          const int a = pow_a(j), b = pow_b(j), k = g.count++;
          g.A[k] = power(a);
          g.B[k] = power(b);
          g.C[k] = power(j);
          g.alpha[k] = power_alpha(j);
          if (yl && j == L.s) {   // Y in FP32, into the slot of its FP32 copy
            g.f32[k] = 1;
            g.C[k] = ws_mat(J.ws, L.off_yf32, n, wss, 4);
          }
        }
        PS_HIP(launch_gemm_group(W, n, J.batch, g, st));
      }
    }
  }
  if (ps_status e = tm.mark()) return e;
  // 2. assemble blocks, norms, Y copies
  Coefs cf;
  memset(&cf, 0, sizeof cf);
  for (int k = 0; k <= L.m; ++k) cf.c[k] = J.coef[k];
  if (W == 1)  // FP32 working precision: the coefficients enter FP32 arithmetic
    for (int k = 0; k <= L.m; ++k) cf.c[k] = (double)(float)cf.c[k];
  AssembleArgs aa;
  aa.n = n;
  aa.nv = n;
  aa.m = L.m;
  aa.s = L.s;
  aa.r = L.r;
  aa.nB = L.nB;
  aa.trivial_last = L.trivial_last;
  aa.X1 = J.X1;
  aa.x1_scale = J.beta;
  aa.pow_shift = J.pow_shift;
  aa.ws = J.ws;
  aa.ws_stride = wss;
  aa.L = L;
  aa.tier_mask = (J.opts.mode == PS_MODE_MIXED || J.opts.override_tiers) && J.write_y ? J.opts.mask : 0u;
  aa.y_f32 = yl ? 1 : 0;
  PS_HIP(launch_assemble(W, aa, cf, J.batch, st));
  if (ps_status e = tm.mark()) return e;
  // 3. plan
  PlanArgs pa;
  memset(&pa, 0, sizeof pa);
  pa.r = L.r;
  pa.mode = J.opts.mode;
  pa.working = W;
  pa.nB = L.nB;
  pa.trivial_last = L.trivial_last;
  pa.mask = J.opts.mask;
  pa.delta = J.opts.delta;
  pa.abs_cm = fabs(cf.c[L.m]);
  pa.rule = J.opts.rule;
  pa.use_override = J.opts.override_tiers != nullptr;
  if (pa.use_override)
    for (int i = 0; i <= L.r; ++i) pa.override_tier[i] = J.opts.override_tiers[i];
  pa.ws = J.ws;
  pa.ws_stride = wss;
  pa.L = L;
  PS_HIP(launch_plan(pa, J.batch, st));
  // 4. Horner
  const bool square = L.sigma > 0 && !J.skip_square;
  MatArg hout = square ? ws_mat(J.ws, L.off_R, n, wss, L.esize) : J.out;
  HornerArgs ha;
  memset(&ha, 0, sizeof ha);
  ha.n = n;
  ha.ws = J.ws;
  ha.ws_stride = wss;
  ha.L = L;
  ha.out = hout;
  if (L.s == 1) {
    ha.ysrc = J.X1;
    ha.yscale = J.beta;
  } else {
    ha.ysrc = ws_mat(J.ws, L.off_pow + (size_t)(L.s - 2 + (L.square_arg ? 1 : 0)) * L.slot, n, wss, L.esize);
    ha.yscale = ldexp(1.0, L.s * J.pow_shift);
  }
  const int i0 = L.first_step;
  // cast of the first block into the operand format of step i0 (or the result)
  ha.cast_only = 1;
  ha.step = i0;
  ha.final_out = (i0 == 0);
  ha.off_bsrc = L.off_B + (size_t)i0 * L.slot;
  ha.off_pout = L.off_P0;
  if (yl) {
    ha.y_cond = 1;
    ha.ya = power(pow_a(L.s));
    ha.yb = power(pow_b(L.s));
    ha.yc = power(L.s);
    ha.y_alpha = power_alpha(L.s);
    ha.y_cm = cf.c[L.m];   // as the assembly's fold
  }
  PS_HIP(launch_horner(W, ha, J.batch, st));
  ha.y_cond = 0;
  ha.cast_only = 0;
  for (int i = i0; i >= 1; --i) {
    const int k = i0 - i;
    ha.step = i;
    ha.final_out = (i == 1);
    ha.off_pin = (k & 1) ? L.off_P1 : L.off_P0;
    ha.off_pout = (k & 1) ? L.off_P0 : L.off_P1;
    ha.off_bsrc = L.off_B + (size_t)(i - 1) * L.slot;
    PS_HIP(launch_horner(W, ha, J.batch, st));
  }
  if (ps_status e = tm.mark()) return e;
  // 5. squarings: R <- R R (working precision), last product into the output
  if (square) {
    MatArg bufs[2] = {ws_mat(J.ws, L.off_R, n, wss, L.esize), ws_mat(J.ws, L.off_P0, n, wss, L.esize)};
    for (int t = 1; t <= L.sigma; ++t) {
      MatArg src = bufs[(t - 1) & 1];
      MatArg dst = (t == L.sigma) ? J.out : bufs[t & 1];
      PS_HIP(launch_gemm(W, n, J.batch, src, 0, src, 0, dst, 1.0, 0, st));
    }
  }
  if (ps_status e = tm.mark()) return e;
  if (phase_ms) {
    PS_HIP(hipStreamSynchronize(st));
    phase_ms[0] = tm.between(0, 1);
    phase_ms[1] = tm.between(1, 2);
    phase_ms[2] = tm.between(2, 3);
    phase_ms[3] = tm.between(3, 4);
  }
  return PS_OK;
}

ps_status fill_report(const Layout& L, const Job& J, int b, ps_report* rep, hipStream_t st, const float* ms) {
  Plan P;
  PS_HIP(hipMemcpyAsync(&P, J.ws + (size_t)b * J.ws_stride + L.off_plan, sizeof P, hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  memset(rep, 0, sizeof *rep);
  rep->s = L.s;
  rep->r = L.r;
  rep->nu = P.nu;
  rep->first_step = L.first_step;
  for (int i = 0; i <= L.r; ++i) {
    rep->tier[i] = P.tier[i];
    rep->u[i] = P.u[i];
    rep->normB[i] = P.normB[i];
  }
  rep->normY = P.normY;
  rep->normX = P.normX;
  model_cost(L.working, L.s, L.r, P.tier, &rep->cost_saving, &rep->m_low);
  rep->gemms[L.working] += L.npow + L.sigma;
  for (int i = L.first_step; i >= 1; --i) rep->gemms[P.tier[i]] += 1;
  if (J.y32) {   // Y by an FP32 product, again in FP64 if a Horner product is
    bool fp64_step = false;
    for (int i = 1; i <= L.r; ++i)
      fp64_step = fp64_step || P.tier[i] == L.working || (P.tier[i] == 1 && P.u[i] < kY32Margin * 0x1p-24);
    rep->gemms[1] += 1;
    if (!fp64_step) rep->gemms[L.working] -= 1;
  }
  if (ms) {
    rep->ms_power = ms[0];
    rep->ms_assemble = ms[1];
    rep->ms_horner = ms[2];
    rep->ms_square = ms[3];
  }
  return PS_OK;
}

}  // namespace

ps_status ps_set_error(ps_status st, const char* msg) {
  g_last_error = msg ? msg : "";
  return st;
}

// ===========================================================================
// exported entry points
// ===========================================================================
// ---------------------------------------------------------------------------
// automatic scaling (section 3.2, eq. (alpha_m-X)): sigma from the alpha_m
// bound on the Taylor truncation error
// ---------------------------------------------------------------------------
namespace {

// Taylor remainder sum_{k > m} t^k / k! (t >= 0), long double
long double taylor_tail(long double t, int m) {
  long double term = 1.0L;
  for (int k = 1; k <= m + 1; ++k) term *= t / k;
  long double sum = term;
  for (int k = m + 2; k < m + 2000; ++k) {
    term *= t / k;
    sum += term;
    if (term <= sum * 1e-21L) break;
  }
  return sum;
}

// largest theta with taylor_tail(theta, m) <= u (bisection; the tail is increasing)
double theta_taylor(int m, double u) {
  long double lo = 0.0L, hi = 1.0L;
  while (taylor_tail(hi, m) <= u && hi < 1e4L) hi *= 2;
  for (int it = 0; it < 200; ++it) {
    const long double mid = 0.5L * (lo + hi);
    if (taylor_tail(mid, m) <= u) lo = mid;
    else hi = mid;
  }
  return (double)lo;
}

// d* = max{d >= 1 : d (d - 1) <= m + 1}
int alpha_dstar(int m) {
  int d = 1;
  while ((d + 1) * d <= m + 1) ++d;
  return d;
}

// max over the workgroup pieces written by launch_norm1 (host side, after a sync)
ps_status read_norm1(const double* dev, int64_t n, hipStream_t st, double* out) {
  std::vector<double> h((size_t)norm1_groups(n));
  PS_HIP(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  double m = 0.0;
  for (double v : h)
    if (v > m || v != v) m = v;
  *out = m;
  return PS_OK;
}

int ceil_log2_ratio(double a, double b) {   // smallest k >= 0 with a <= 2^k b
  if (!(a > b)) return 0;
  int k = (int)std::ceil(std::log2(a / b));
  while (k > 0 && std::ldexp(b, k - 1) >= a) --k;
  while (std::ldexp(b, k) < a) ++k;
  return k;
}

// The acceptance test of eq. (alpha_m-X) for X = 2^-sigma A: the Taylor tail
// at t = 2^-sigma alpha_m(A) is at most u xi(X), with xi(X) = ||B_0(X)||_1,
// B_0 = sum_{j<s} X^j / j! (the leading PS block, section 3.1's stand-in for
// e^X), as the estimate of ||e^X||_1.  t > 800 is rejected without the series
// (the tail then exceeds e^t / 2, beyond u times any double).
constexpr double kTailCap = 800.0;

// Least sigma >= 0 accepted by that test.  power(1) is A itself and power(j)
// (j = 2..s-1) is X0^j with X0 = 2^-sigma0 A, so X = 2^-sigma A and
// X^j = 2^(j (sigma0 - sigma)) X0^j.  Scalings below a
// host lower bound (the tail above u times the triangle-inequality bound
// sum_j |c_j| (2^-sigma ||A||_1)^j of xi, with a margin for rounding) cannot
// pass; from there, windows of kXiWin scalings are decided with one launch of
// k_xi_norms and one read-back each.  Fails with PS_ERR_ARG when no sigma up to
// kMaxSigma passes.
template <typename PowerFn>
ps_status least_accepted_sigma(int W, int64_t n, int m, int s, double u, double alphaA, double normA, int sigma0,
                               PowerFn power, double* wg, hipStream_t st, int* out) {
  std::vector<double> c(s);
  {
    DD x = {1.0, 0.0};
    c[0] = 1.0;
    for (int j = 1; j < s; ++j) {
      x = dd_div_int(x, (double)j);
      c[j] = x.hi + x.lo;
    }
  }
  int lo = 0;
  while (lo <= kMaxSigma && !(std::ldexp(alphaA, -lo) <= kTailCap)) ++lo;
  for (; lo <= kMaxSigma; ++lo) {
    const long double t = std::ldexp(alphaA, -lo), x = std::ldexp(normA, -lo);
    long double up = 0.0L, xp = 1.0L;
    for (int j = 0; j < s; ++j, xp *= x) up += (long double)c[j] * xp;
    if (!(taylor_tail(t, m) > (long double)u * up * 1.001L)) break;
  }
  const int64_t G = norm1_groups(n);
  std::vector<double> h((size_t)kXiWin * G);
  for (int base = lo; base <= kMaxSigma; base += kXiWin) {
    XiArgs xa;
    memset(&xa, 0, sizeof xa);
    xa.J = s - 1;
    xa.K = std::min(kXiWin, kMaxSigma - base + 1);
    for (int j = 1; j < s; ++j) xa.M[j - 1] = power(j);
    for (int k = 0; k < xa.K; ++k) {
      const int sg = base + k;
      xa.w[k][0] = c[0];
      if (s > 1) xa.w[k][1] = std::ldexp(c[1], -sg);
      for (int j = 2; j < s; ++j) xa.w[k][j] = std::ldexp(c[j], j * (sigma0 - sg));
    }
    xa.wg = wg;
    PS_HIP(launch_xi_norms(W, n, xa, st));
    PS_HIP(hipMemcpyAsync(h.data(), wg, (size_t)xa.K * G * sizeof(double), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < xa.K; ++k) {
      const int sg = base + k;
      const double t = std::ldexp(alphaA, -sg);
      if (!(t <= kTailCap)) continue;
      double xi = 0.0;
      for (int64_t g = 0; g < G; ++g)
        if (h[(size_t)k * G + g] > xi || h[(size_t)k * G + g] != h[(size_t)k * G + g]) xi = h[(size_t)k * G + g];
      if (!std::isfinite(xi)) continue;
      if (taylor_tail(t, m) <= (long double)u * (long double)xi) {
        *out = sg;
        return PS_OK;
      }
    }
  }
  return fail(PS_ERR_ARG, "no scaling up to %d squarings meets the alpha_m bound (m = %d)", kMaxSigma, m);
}

}  // namespace

// Variable block size (Algorithm 2 with fix_params = false): the power slots
// X^2..X^m come first in every layout with npow = m - 1, so the powers built
// while s grows stay where the layout of the final s expects them.  After the
// largest of those layouts: the running B_0 and the norm scratch.
struct VarsLayout {
  size_t off_b0, off_wg, bytes;
};
static VarsLayout vars_layout(ps_dtype dtype, int64_t n, int m, int s0, int sigma) {
  const int np = std::max(m - 1, 0);
  size_t mx = 0;
  for (int s = s0; s <= std::max(m, s0); ++s) mx = std::max(mx, make_layout(dtype, n, m, s, sigma, 0, np).bytes);
  VarsLayout V;
  V.off_b0 = mx;
  V.off_wg = V.off_b0 + make_layout(dtype, n, m, s0, sigma, 0, np).slot;
  V.bytes = al256(V.off_wg + 2 * (size_t)norm1_groups(n) * sizeof(double));
  return V;
}

// host maxima of the two workgroup arrays written by launch_comb_norm
static ps_status read_norm_pair(const double* dev, int64_t n, hipStream_t st, double* nb, double* ny) {
  const size_t g = (size_t)norm1_groups(n);
  std::vector<double> h(2 * g);
  PS_HIP(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  double v[2] = {0.0, 0.0};
  for (int q = 0; q < 2; ++q)
    for (size_t k = 0; k < g; ++k)
      if (h[q * g + k] > v[q] || h[q * g + k] != h[q * g + k]) v[q] = h[q * g + k];
  *nb = v[0];
  *ny = v[1];
  return PS_OK;
}

// Joint choice of the degree and the scaling.  Candidates are the degrees
// m = q^2 and m = q(q+1) up to m_max, for which PS with s = ceil(sqrt(m))
// costs s - 1 powers and floor(m/s) - [s | m] Horner products.  One power
// table X0^2 .. X0^j serves the alpha_m bound of the candidates and the
// evaluation; the workspace holds it up to D = the largest of s and d* + 1
// over the candidates.
struct SelectPlan {
  std::vector<int> cand;   // candidate degrees, increasing
  int D = 1;               // highest power formed
  size_t off_wg = 0, bytes = 0;
};
static int ps_cost(int m) {
  const int s = default_s(m), r = m / s;
  return (s - 1) + (r - ((r >= 1 && m == s * r) ? 1 : 0));
}
static SelectPlan select_plan(ps_dtype dtype, int64_t n, int m_max) {
  SelectPlan P;
  for (int q = 1; q * q <= m_max; ++q) {
    P.cand.push_back(q * q);
    if (q * (q + 1) <= m_max) P.cand.push_back(q * (q + 1));
  }
  for (int m : P.cand) P.D = std::max(P.D, std::max(default_s(m), alpha_dstar(m) + 1));
  size_t mx = 0;
  for (int m : P.cand) mx = std::max(mx, make_layout(dtype, n, m, default_s(m), 1, 0, P.D - 1).bytes);
  P.off_wg = mx;
  P.bytes = al256(mx + (size_t)(P.D + kXiWin) * norm1_groups(n) * sizeof(double));
  return P;
}

static Layout auto_layout(ps_dtype dtype, int64_t n, int m, int s) {
  const int D = std::max(s, alpha_dstar(m) + 1);
  return make_layout(dtype, n, m, s, 1, 0, D - 1);
}

extern "C" {

int ps_version(void) { return 10000; }

const char* ps_strerror(int status) {
  switch (status) {
    case PS_OK: return "success";
    case PS_ERR_ARG: return "invalid argument";
    case PS_ERR_ALIAS: return "output overlaps an input";
    case PS_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case PS_ERR_NONFINITE: return "non-finite values in an input or a result";
    case PS_ERR_UNSUPPORTED: return "unsupported request";
    case PS_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

ps_status ps_coef_taylor_exp(int m, double* coef) {
  if (m < 0 || m > 170 || !coef) return fail(PS_ERR_ARG, "ps_coef_taylor_exp: m in [0,170], coef != NULL");
  DD x = {1.0, 0.0};
  coef[0] = 1.0;
  for (int k = 1; k <= m; ++k) {
    x = dd_div_int(x, (double)k);
    coef[k] = x.hi + x.lo;
  }
  return PS_OK;
}

ps_status ps_coef_taylor_cos(int m, double* coef) {
  if (m < 0 || m > 85 || !coef) return fail(PS_ERR_ARG, "ps_coef_taylor_cos: m in [0,85], coef != NULL");
  DD x = {1.0, 0.0};
  coef[0] = 1.0;
  for (int k = 1; k <= m; ++k) {
    x = dd_div_int(x, (double)(2 * k - 1));
    x = dd_div_int(x, (double)(2 * k));
    double v = x.hi + x.lo;
    coef[k] = (k & 1) ? -v : v;
  }
  return PS_OK;
}

ps_status ps_coef_pade_exp(int deg, double* p, double* q) {
  if (deg < 0 || deg > 60 || !p || !q) return fail(PS_ERR_ARG, "ps_coef_pade_exp: deg in [0,60], p,q != NULL");
  // p_j = (2d-j)! d! / ((2d)! j! (d-j)!), via p_j = p_{j-1} (d-j+1) / (j (2d-j+1))
  DD x = {1.0, 0.0};
  p[0] = q[0] = 1.0;
  for (int j = 1; j <= deg; ++j) {
    // multiply by the integer (d-j+1) exactly in dd, then divide by j and (2d-j+1)
    double f = (double)(deg - j + 1);
    double hi = x.hi * f;
    double e = fma(x.hi, f, -hi);
    DD y = dd_two_sum(hi, e + x.lo * f);
    y = dd_div_int(y, (double)j);
    y = dd_div_int(y, (double)(2 * deg - j + 1));
    x = y;
    p[j] = x.hi + x.lo;
    q[j] = (j & 1) ? -p[j] : p[j];
  }
  return PS_OK;
}

ps_status ps_plan(ps_dtype dtype, int r, const double* normB, double normY, const ps_opts* opts, int* tier,
                  double* u, int* nu) {
  if (dtype != PS_F64 && dtype != PS_F32 && dtype != PS_DD)
    return fail(PS_ERR_ARG, "dtype must be PS_F64, PS_F32 or PS_DD");
  if (r < 0 || r + 1 > PS_MAX_BLOCKS) return fail(PS_ERR_ARG, "r = %d out of range", r);
  if (!normB || !tier || !u || !nu) return fail(PS_ERR_ARG, "NULL output or norm array");
  const int W = dtype == PS_F64 ? 0 : dtype == PS_F32 ? 1 : kTierDD;
  Opts o = read_opts(opts, W == kTierDD ? 0 : W);
  if (W == kTierDD) o.mask = (opts && opts->tier_mask ? opts->tier_mask : 0xFu) & 0xFu;   // every IEEE tier is lower
  if (o.mode == PS_MODE_FIXED) {
    for (int i = 0; i <= r; ++i) { tier[i] = W; u[i] = tier_unit_roundoff(W); }
    *nu = r + 1;
    return PS_OK;
  }
  plan_tiers(r, normB, normY, W, o.mask, o.delta, tier, u, nu);
  return PS_OK;
}

ps_status ps_model_cost(ps_dtype dtype, int s, int r, const int* tier, double* cost_saving, double* m_low) {
  if (dtype != PS_F64 && dtype != PS_F32 && dtype != PS_DD)
    return fail(PS_ERR_ARG, "dtype must be PS_F64, PS_F32 or PS_DD");
  if (s < 1 || r < 0 || r + 1 > PS_MAX_BLOCKS) return fail(PS_ERR_ARG, "s = %d, r = %d out of range", s, r);
  if (!tier || !cost_saving || !m_low) return fail(PS_ERR_ARG, "NULL argument");
  for (int i = 1; i <= r; ++i)
    if (tier[i] < 0 || tier[i] > kTierDD) return fail(PS_ERR_ARG, "tier[%d] = %d not a tier", i, tier[i]);
  model_cost(dtype == PS_F64 ? 0 : dtype == PS_F32 ? 1 : kTierDD, s, r, tier, cost_saving, m_low);
  return PS_OK;
}

ps_status ps_workspace_size(ps_dtype dtype, int64_t n, int m, int s, int sigma, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  if (ps_status e = check_common(dtype, n, m, &s, sigma)) return e;
  *bytes = make_layout(dtype, n, m, s, sigma, 0).bytes;
  return PS_OK;
}

ps_status ps_workspace_size_strided(ps_dtype dtype, int batch, int64_t n, int m, int s, int sigma, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  if (batch < 1 || batch > 65535) return fail(PS_ERR_ARG, "batch = %d out of range [1, 65535]", batch);
  if (ps_status e = check_common(dtype, n, m, &s, sigma)) return e;
  *bytes = make_layout(dtype, n, m, s, sigma, 0).bytes * (size_t)batch;
  return PS_OK;
}

static ps_status expm_impl(ps_dtype dtype, int batch, int64_t n, const void* A, int64_t lda, int64_t strideA,
                           const double* coef, int m, int s, int sigma, double beta, void* E, int64_t lde,
                           int64_t strideE, const ps_opts* opts, ps_report* reports, void* ws, size_t ws_bytes,
                           void* stream) {
  if (ps_status e = check_common(dtype, n, m, &s, sigma)) return e;
  if (batch < 1 || batch > 65535) return fail(PS_ERR_ARG, "batch = %d out of range [1, 65535]", batch);
  if (!A || !E) return fail(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || lde < n) return fail(PS_ERR_ARG, "leading dimension smaller than n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  if (batch > 1) {
    if (strideA < (int64_t)((n - 1) * lda + n) || strideE < (int64_t)((n - 1) * lde + n))
      return fail(PS_ERR_ARG, "batch stride smaller than one matrix");
  }
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) {
    const int r = m / s;
    for (int i = 1; i <= r; ++i)
      if (o.override_tiers[i] < (dtype == PS_F64 ? 0 : 1) || o.override_tiers[i] > 3)
        return fail(PS_ERR_ARG, "tier_override[%d] = %d not a usable tier", i, o.override_tiers[i]);
  }
  const size_t spanA = (size_t)(batch - 1) * strideA * esize + mat_span_bytes(n, lda, esize);
  const size_t spanE = (size_t)(batch - 1) * strideE * esize + mat_span_bytes(n, lde, esize);
  if (overlap(A, spanA, E, spanE)) return fail(PS_ERR_ALIAS, "output overlaps the input matrix");
  Layout L = make_layout(dtype, n, m, s, sigma, 0);
  if (ps_status e = check_ws(ws, ws_bytes, L.bytes * (size_t)batch)) return e;
  if (overlap(ws, L.bytes * (size_t)batch, E, spanE) || overlap(ws, L.bytes * (size_t)batch, A, spanA))
    return fail(PS_ERR_ALIAS, "workspace overlaps a matrix argument");
  double c[kMaxDegree + 1];
  if (coef) {
    for (int k = 0; k <= m; ++k) c[k] = coef[k];
  } else {
    if (m > 170) return fail(PS_ERR_ARG, "built-in Taylor coefficients need m <= 170");
    ps_coef_taylor_exp(m, c);
  }
  Job J;
  J.L = &L;
  J.batch = batch;
  J.X1 = MatArg{A, lda, strideA};
  J.beta = beta;
  J.coef = c;
  J.out = MatArg{E, lde, strideE};
  J.ws = (char*)ws;
  J.ws_stride = L.bytes;
  J.opts = o;
  J.write_y = true;
  J.build_powers = true;
  J.skip_square = false;
  J.y32 = y32_allowed(L, o);
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  char* wg = (char*)ws + L.off_colsum;   // scratch of each matrix until its blocks are assembled
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, batch, J.X1, wg, L.bytes, st, "input matrix")) return e;
  float ms[4] = {0, 0, 0, 0};
  if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
  if (reports)
    for (int b = 0; b < batch; ++b)
      if (ps_status e = fill_report(L, J, b, &reports[b], st, o.profile ? ms : nullptr)) return e;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, batch, J.out, wg, L.bytes, st, "result")) return e;
  return PS_OK;
}

ps_status ps_theta_taylor(ps_dtype dtype, int m, double* theta) {
  if (dtype != PS_F64 && dtype != PS_F32) return fail(PS_ERR_ARG, "dtype must be PS_F64 or PS_F32");
  if (m < 0 || m > 170 || !theta) return fail(PS_ERR_ARG, "ps_theta_taylor: m in [0,170], theta != NULL");
  *theta = theta_taylor(m, dtype == PS_F64 ? 0x1p-53 : 0x1p-24);
  return PS_OK;
}

ps_status ps_workspace_size_auto(ps_dtype dtype, int64_t n, int m, int s, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  if (ps_status e = check_common(dtype, n, m, &s, 1)) return e;
  *bytes = auto_layout(dtype, n, m, s).bytes;
  return PS_OK;
}

ps_status ps_expm_auto(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m, int s, int norm_guard, void* E,
                       int64_t lde, const ps_opts* opts, ps_report* report, int* sigma_out, void* ws,
                       size_t ws_bytes, void* stream) {
  if (ps_status e = check_common(dtype, n, m, &s, 1)) return e;
  if (m > 170) return fail(PS_ERR_ARG, "the automatic scaling uses the Taylor coefficients: m <= 170");
  if (!A || !E) return fail(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || lde < n) return fail(PS_ERR_ARG, "leading dimension smaller than n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanA = mat_span_bytes(n, lda, esize), spanE = mat_span_bytes(n, lde, esize);
  if (overlap(A, spanA, E, spanE)) return fail(PS_ERR_ALIAS, "output overlaps the input matrix");
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) return fail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_expm_auto");
  Layout L = auto_layout(dtype, n, m, s);
  if (ps_status e = check_ws(ws, ws_bytes, L.bytes)) return e;
  if (overlap(ws, L.bytes, E, spanE) || overlap(ws, L.bytes, A, spanA))
    return fail(PS_ERR_ALIAS, "workspace overlaps a matrix argument");
  // the column-sum region (at least 3n doubles, 256-byte rounded) holds the
  // kXiWin * ceil(n/8) workgroup maxima of the acceptance windows
  if (L.off_plan - L.off_colsum < (size_t)kXiWin * norm1_groups(n) * sizeof(double))
    return fail(PS_ERR_UNSUPPORTED, "ps_expm_auto: scratch region too small");
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  const double theta = theta_taylor(m, W == 0 ? 0x1p-53 : 0x1p-24);
  const int dstar = alpha_dstar(m), D = std::max(s, dstar + 1);
  double* wg = (double*)((char*)ws + L.off_colsum);   // scratch until the blocks are assembled
  const MatArg X1{A, lda, 0};
  auto power = [&](int j) { return j == 1 ? X1 : ws_mat((char*)ws, L.off_pow + (size_t)(j - 2) * L.slot, n, 0, esize); };
  // 1. ||A||_1 and the first scaling sigma0 (||X0||_1 <= theta for X0 = 2^-sigma0 A)
  double nA = 0.0;
  PS_HIP(launch_norm1(W, n, X1, wg, st));
  if (ps_status e = read_norm1(wg, n, st, &nA)) return e;
  if (!std::isfinite(nA))
    return fail(o.check_finite ? PS_ERR_NONFINITE : PS_ERR_ARG, "input matrix has non-finite entries");
  const int sigma0 = ceil_log2_ratio(nA, theta);
  if (sigma0 > kMaxSigma) return fail(PS_ERR_ARG, "||A||_1 = %g needs more than %d squarings", nA, kMaxSigma);
  const double beta0 = ldexp(1.0, -sigma0);
  // 2. X0^2 .. X0^D by the level schedule of the power table
  for (int top = 2; top / 2 < D; top *= 2) {
    const int lo = top / 2 + 1, hi = std::min(top, D);
    for (int j0 = lo; j0 <= hi; j0 += kMaxGroup) {
      GemmGroup g;
      memset(&g, 0, sizeof g);
      for (int j = j0; j <= std::min(hi, j0 + kMaxGroup - 1); ++j) {
        const int a = pow_a(j), b = pow_b(j), k = g.count++;
        g.A[k] = power(a);
        g.B[k] = power(b);
        g.C[k] = power(j);
        g.alpha[k] = (a == 1 ? beta0 : 1.0) * (b == 1 ? beta0 : 1.0);
      }
      PS_HIP(launch_gemm_group(W, n, 1, g, st));
    }
  }
  // 3. alpha_m(X0) = max(||X0^d*||^(1/d*), ||X0^(d*+1)||^(1/(d*+1))), sigma for A
  double nd[2];
  for (int q = 0; q < 2; ++q) {
    const int d = dstar + q;
    if (d == 1) {
      nd[q] = beta0 * nA;
      continue;
    }
    PS_HIP(launch_norm1(W, n, power(d), wg, st));
    if (ps_status e = read_norm1(wg, n, st, &nd[q])) return e;
  }
  const double alpha0 = std::max(std::pow(nd[0], 1.0 / dstar), std::pow(nd[1], 1.0 / (dstar + 1)));
  // alpha_m(A) = 2^sigma0 alpha_m(X0); sigma the least scaling that passes
  // the acceptance test with xi(X) = ||B_0(X)||_1
  int sigma = 0;
  if (ps_status e = least_accepted_sigma(W, n, m, s, W == 0 ? 0x1p-53 : 0x1p-24, ldexp(alpha0, sigma0), nA, sigma0,
                                         power, wg, st, &sigma))
    return e;
  if (norm_guard) sigma = std::max(sigma, ceil_log2_ratio(M_E * nA, (double)s));   // ||X||_1 <= s / e
  if (sigma > kMaxSigma) return fail(PS_ERR_ARG, "the norm guard needs more than %d squarings", kMaxSigma);
  // 4. evaluation on X = 2^-sigma A with the prebuilt powers: X^j = 2^(j (sigma0 - sigma)) X0^j
  std::vector<double> c(m + 1);
  ps_coef_taylor_exp(m, c.data());
  L.sigma = sigma;
  Job J;
  J.L = &L;
  J.batch = 1;
  J.X1 = X1;
  J.beta = ldexp(1.0, -sigma);
  J.coef = c.data();
  J.out = MatArg{E, lde, 0};
  J.ws = (char*)ws;
  J.ws_stride = L.bytes;
  J.opts = o;
  J.write_y = true;
  J.build_powers = false;
  J.skip_square = false;
  J.pow_shift = sigma0 - sigma;
  float ms[4] = {0, 0, 0, 0};
  if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
  if (sigma_out) *sigma_out = sigma;
  if (report)
    if (ps_status e = fill_report(L, J, 0, report, st, o.profile ? ms : nullptr)) return e;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, J.out, (char*)wg, 0, st, "result")) return e;
  return PS_OK;
}

ps_status ps_workspace_size_select(ps_dtype dtype, int64_t n, int m_max, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  int s = 0;
  if (ps_status e = check_common(dtype, n, m_max, &s, 1)) return e;
  if (m_max < 1 || m_max > 170) return fail(PS_ERR_ARG, "m_max = %d out of range [1, 170]", m_max);
  *bytes = select_plan(dtype, n, m_max).bytes;
  return PS_OK;
}

ps_status ps_expm_select(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m_max, void* E, int64_t lde,
                         const ps_opts* opts, ps_report* report, int* chosen, void* ws, size_t ws_bytes,
                         void* stream) {
  int s_chk = 0;
  if (ps_status e = check_common(dtype, n, m_max, &s_chk, 1)) return e;
  if (m_max < 1 || m_max > 170) return fail(PS_ERR_ARG, "m_max = %d out of range [1, 170]", m_max);
  if (!A || !E) return fail(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || lde < n) return fail(PS_ERR_ARG, "leading dimension smaller than n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanA = mat_span_bytes(n, lda, esize), spanE = mat_span_bytes(n, lde, esize);
  if (overlap(A, spanA, E, spanE)) return fail(PS_ERR_ALIAS, "output overlaps the input matrix");
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) return fail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_expm_select");
  const SelectPlan SP = select_plan(dtype, n, m_max);
  if (ps_status e = check_ws(ws, ws_bytes, SP.bytes)) return e;
  if (overlap(ws, SP.bytes, E, spanE) || overlap(ws, SP.bytes, A, spanA))
    return fail(PS_ERR_ALIAS, "workspace overlaps a matrix argument");
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  const double u = W == 0 ? 0x1p-53 : 0x1p-24;
  char* wsc = (char*)ws;
  double* wg = (double*)(wsc + SP.off_wg);
  const int64_t G = norm1_groups(n);
  const MatArg X1{A, lda, 0};
  // the power slots sit at the start of every candidate's layout
  const Layout L0 = make_layout(dtype, n, SP.cand.back(), default_s(SP.cand.back()), 1, 0, SP.D - 1);
  auto power = [&](int j) { return j == 1 ? X1 : ws_mat(wsc, L0.off_pow + (size_t)(j - 2) * L0.slot, n, 0, esize); };
  // 1. ||A||_1; sigma0 from the largest candidate's theta (the smallest scaling)
  const double theta_last = theta_taylor(SP.cand.back(), u);
  double nA = 0.0;
  PS_HIP(launch_norm1(W, n, X1, wg, st));
  if (ps_status e = read_norm1(wg, n, st, &nA)) return e;
  if (!std::isfinite(nA))
    return fail(o.check_finite ? PS_ERR_NONFINITE : PS_ERR_ARG, "input matrix has non-finite entries");
  const int sigma0 = ceil_log2_ratio(nA, theta_last);
  if (sigma0 > kMaxSigma) return fail(PS_ERR_ARG, "||A||_1 = %g needs more than %d squarings", nA, kMaxSigma);
  const double beta0 = ldexp(1.0, -sigma0);
  // 2. candidates in increasing m; PS cost grows strictly along them, so the
  //    search stops at the first candidate whose products alone reach the
  //    best total.  Powers X0^j are formed as far as the examined candidates
  //    need them (X_j = X_ceil(j/2) X_floor(j/2), grouped), with one norm
  //    read-back per extension.
  std::vector<double> nrm(SP.D + 2, 0.0);
  nrm[1] = beta0 * nA;
  int built = 1;
  auto build_to = [&](int need) -> ps_status {
    if (need <= built) return PS_OK;
    const int first = built + 1;
    while (built < need) {
      const int lo = built + 1, hi = std::min(std::min(need, 2 * built), built + kMaxGroup);
      GemmGroup g;
      memset(&g, 0, sizeof g);
      for (int j = lo; j <= hi; ++j) {
        const int a = pow_a(j), b = pow_b(j), k = g.count++;
        g.A[k] = power(a);
        g.B[k] = power(b);
        g.C[k] = power(j);
        g.alpha[k] = (a == 1 ? beta0 : 1.0) * (b == 1 ? beta0 : 1.0);
      }
      PS_HIP(launch_gemm_group(W, n, 1, g, st));
      for (int j = lo; j <= hi; ++j) PS_HIP(launch_norm1(W, n, power(j), wg + (size_t)(j - 1) * G, st));
      built = hi;
    }
    std::vector<double> h((size_t)(need - first + 1) * G);
    PS_HIP(hipMemcpyAsync(h.data(), wg + (size_t)(first - 1) * G, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    PS_HIP(hipStreamSynchronize(st));
    for (int d = first; d <= need; ++d)
      for (int64_t k = 0; k < G; ++k) {
        const double v = h[(size_t)(d - first) * G + k];
        if (v > nrm[d] || v != v) nrm[d] = v;
      }
    return PS_OK;
  };
  // 3. per candidate: alpha_m(A) = 2^sigma0 alpha_m(X0), the least sigma that
  //    passes the acceptance test (with that candidate's s), and the products
  //    it costs
  int best = -1, best_cost = 0, best_sigma = 0;
  for (size_t k = 0; k < SP.cand.size(); ++k) {
    const int m = SP.cand[k], d = alpha_dstar(m);
    if (best >= 0 && ps_cost(m) >= best_cost) break;
    if (ps_status e = build_to(std::max(default_s(m), d + 1))) return e;
    const double a0 = std::max(std::pow(nrm[d], 1.0 / d), std::pow(nrm[d + 1], 1.0 / (d + 1)));
    int sg = 0;
    const ps_status e = least_accepted_sigma(W, n, m, default_s(m), u, ldexp(a0, sigma0), nA, sigma0, power,
                                             wg + (size_t)SP.D * G, st, &sg);
    if (e == PS_ERR_HIP) return e;
    if (e != PS_OK) continue;   // no scaling within kMaxSigma for this degree
    const int cost = ps_cost(m) + sg;
    if (best < 0 || cost < best_cost) {
      best = (int)k;
      best_cost = cost;
      best_sigma = sg;
    }
  }
  if (best < 0) return fail(PS_ERR_ARG, "no candidate degree meets the bound within %d squarings", kMaxSigma);
  const int m = SP.cand[best], s = default_s(m), sigma = best_sigma;
  // 4. evaluation with the chosen (m, s, sigma) on the power table
  std::vector<double> c(m + 1);
  ps_coef_taylor_exp(m, c.data());
  Layout L = make_layout(dtype, n, m, s, sigma, 0, SP.D - 1);
  Job J;
  J.L = &L;
  J.batch = 1;
  J.X1 = X1;
  J.beta = ldexp(1.0, -sigma);
  J.coef = c.data();
  J.out = MatArg{E, lde, 0};
  J.ws = wsc;
  J.ws_stride = L.bytes;
  J.opts = o;
  J.write_y = true;
  J.build_powers = false;
  J.skip_square = false;
  J.pow_shift = sigma0 - sigma;   // X^j = 2^(j (sigma0 - sigma)) X0^j, exact (either sign)
  float ms[4] = {0, 0, 0, 0};
  if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
  if (chosen) {
    chosen[0] = m;
    chosen[1] = s;
    chosen[2] = sigma;
  }
  if (report)
    if (ps_status e = fill_report(L, J, 0, report, st, o.profile ? ms : nullptr)) return e;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, J.out, (char*)wg, 0, st, "result")) return e;
  return PS_OK;
}

ps_status ps_workspace_size_vars(ps_dtype dtype, int64_t n, int m, int sigma, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  int s0 = 0;
  if (ps_status e = check_common(dtype, n, m, &s0, sigma)) return e;
  *bytes = vars_layout(dtype, n, m, s0, sigma).bytes;
  return PS_OK;
}

ps_status ps_expm_vars(ps_dtype dtype, int64_t n, const void* A, int64_t lda, const double* coef, int m, int sigma,
                       void* E, int64_t lde, const ps_opts* opts, ps_report* report, int* s_out, void* ws,
                       size_t ws_bytes, void* stream) {
  int s0 = 0;
  if (ps_status e = check_common(dtype, n, m, &s0, sigma)) return e;
  if (!A || !E) return fail(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || lde < n) return fail(PS_ERR_ARG, "leading dimension smaller than n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanA = mat_span_bytes(n, lda, esize), spanE = mat_span_bytes(n, lde, esize);
  if (overlap(A, spanA, E, spanE)) return fail(PS_ERR_ALIAS, "output overlaps the input matrix");
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) return fail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_expm_vars");
  const VarsLayout V = vars_layout(dtype, n, m, s0, sigma);
  if (ps_status e = check_ws(ws, ws_bytes, V.bytes)) return e;
  if (overlap(ws, V.bytes, E, spanE) || overlap(ws, V.bytes, A, spanA))
    return fail(PS_ERR_ALIAS, "workspace overlaps a matrix argument");
  std::vector<double> c(m + 1);
  if (coef) {
    for (int k = 0; k <= m; ++k) c[k] = coef[k];
  } else {
    if (m > 170) return fail(PS_ERR_ARG, "built-in Taylor coefficients need m <= 170");
    ps_coef_taylor_exp(m, c.data());
  }
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  const int np = std::max(m - 1, 0);
  const double beta = ldexp(1.0, -sigma);
  char* wsc = (char*)ws;
  double* wg = (double*)(wsc + V.off_wg);
  const MatArg X1{A, lda, 0};
  Layout L = make_layout(dtype, n, m, s0, sigma, 0, np);
  auto power = [&](int j) { return j == 1 ? X1 : ws_mat(wsc, L.off_pow + (size_t)(j - 2) * L.slot, n, 0, esize); };
  // 1. ||X||_1 for X = 2^-sigma A (exact power-of-two scaling of the column sums)
  double nA = 0.0;
  PS_HIP(launch_norm1(W, n, X1, wg, st));
  if (ps_status e = read_norm1(wg, n, st, &nA)) return e;
  if (!std::isfinite(nA))
    return fail(o.check_finite ? PS_ERR_NONFINITE : PS_ERR_ARG, "input matrix has non-finite entries");
  const double nX = ldexp(nA, -sigma);
  int s = s0;
  bool built = false;
  // 2. the variable-s branch runs only for ||X||_1 <= s/e (section 3.3); it
  //    grows s while ||Y|| > ||B_0|| ||X||^s, adding c_s Y to B_0 each time
  if (nX <= s0 / M_E && s0 < m) {
    for (int top = 2; top / 2 < s0; top *= 2) {
      const int lo = top / 2 + 1, hi = std::min(top, s0);
      GemmGroup g;
      memset(&g, 0, sizeof g);
      for (int j = lo; j <= hi; ++j) {
        const int a = pow_a(j), b = pow_b(j), k = g.count++;
        g.A[k] = power(a);
        g.B[k] = power(b);
        g.C[k] = power(j);
        g.alpha[k] = (a == 1 ? beta : 1.0) * (b == 1 ? beta : 1.0);
      }
      PS_HIP(launch_gemm_group(W, n, 1, g, st));
    }
    built = true;
    const MatArg B0 = ws_mat(wsc, V.off_b0, n, 0, esize);
    CombArgs ca;
    memset(&ca, 0, sizeof ca);
    for (int j = 1; j < s0; ++j) {
      ca.M[ca.count] = power(j);
      ca.c[ca.count++] = j == 1 ? c[1] * beta : c[j];
    }
    ca.c_id = c[0];
    ca.accumulate = 0;
    ca.B = B0;
    ca.Y = power(s0);
    ca.wgB = wg;
    ca.wgY = wg + norm1_groups(n);
    PS_HIP(launch_comb_norm(W, n, ca, st));
    double nB0 = 0.0, nY = 0.0;
    if (ps_status e = read_norm_pair(wg, n, st, &nB0, &nY)) return e;
    while (nY > nB0 * std::pow(nX, s) && s < m) {
      GemmGroup g;   // X_{s+1} = X X_s
      memset(&g, 0, sizeof g);
      g.A[0] = X1;
      g.B[0] = power(s);
      g.C[0] = power(s + 1);
      g.alpha[0] = beta;
      g.count = 1;
      PS_HIP(launch_gemm_group(W, n, 1, g, st));
      memset(&ca, 0, sizeof ca);
      ca.M[0] = power(s);   // B_0 += c_s X^s
      ca.c[0] = c[s];
      ca.count = 1;
      ca.accumulate = 1;
      ca.B = B0;
      ca.Y = power(s + 1);
      ca.wgB = wg;
      ca.wgY = wg + norm1_groups(n);
      PS_HIP(launch_comb_norm(W, n, ca, st));
      if (ps_status e = read_norm_pair(wg, n, st, &nB0, &nY)) return e;
      ++s;
    }
  }
  // 3. blocks, plan, Horner and squarings with the chosen s
  L = make_layout(dtype, n, m, s, sigma, 0, np);
  Job J;
  J.L = &L;
  J.batch = 1;
  J.X1 = X1;
  J.beta = beta;
  J.coef = c.data();
  J.out = MatArg{E, lde, 0};
  J.ws = wsc;
  J.ws_stride = L.bytes;
  J.opts = o;
  J.write_y = true;
  J.build_powers = !built;
  J.skip_square = false;
  float ms[4] = {0, 0, 0, 0};
  if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
  if (s_out) *s_out = s;
  if (report)
    if (ps_status e = fill_report(L, J, 0, report, st, o.profile ? ms : nullptr)) return e;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, J.out, (char*)wg, 0, st, "result")) return e;
  return PS_OK;
}

ps_status ps_eval(ps_dtype dtype, int64_t n, const void* A, int64_t lda, const double* coef, int m, int s, void* P,
                  int64_t ldp, const ps_opts* opts, ps_report* report, void* ws, size_t ws_bytes, void* stream) {
  if (!coef) return fail(PS_ERR_ARG, "coef == NULL");
  return expm_impl(dtype, 1, n, A, lda, 0, coef, m, s, 0, 1.0, P, ldp, 0, opts, report, ws, ws_bytes, stream);
}

ps_status ps_expm(ps_dtype dtype, int64_t n, const void* A, int64_t lda, const double* coef, int m, int s, int sigma,
                  void* E, int64_t lde, const ps_opts* opts, ps_report* report, void* ws, size_t ws_bytes,
                  void* stream) {
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range [0, %d]", sigma, kMaxSigma);
  return expm_impl(dtype, 1, n, A, lda, 0, coef, m, s, sigma, ldexp(1.0, -sigma), E, lde, 0, opts, report, ws,
                   ws_bytes, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// ps_expm_noalloc: ps_expm with its workspace in a static device array, for
// callers that cannot allocate device memory.  Each device holds its own copy
// of `scratch` (from the library's load until the process ends); host code
// reaches it only through the address hipGetSymbolAddress returns for the
// device that is current, taken once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = PS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
// device address of the current device's scratch array (looked up once per device)
ps_status scratch_address(hipStream_t st, void** out) {
  int dev = -1;
  PS_HIP(hipGetDevice(&dev));
  if (st) {
    int sdev = -1;
    PS_HIP(hipStreamGetDevice(st, &sdev));
    if (sdev != dev) return fail(PS_ERR_ARG, "stream belongs to device %d, current device is %d", sdev, dev);
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(PS_ERR_UNSUPPORTED, "device index %d above %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255) != 0) return fail(PS_ERR_HIP, "scratch array address %p not usable", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PS_OK;
}
}  // namespace

extern "C" {

ps_status ps_expm_noalloc(ps_dtype dtype, int64_t n, const void* A, int64_t lda, const double* coef, int m, int s,
                          int sigma, void* E, int64_t lde, const ps_opts* opts, ps_report* report, void* stream) {
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range [0, %d]", sigma, kMaxSigma);
  if (ps_status e = check_common(dtype, n, m, &s, sigma)) return e;
  if (opts && opts->profile) return fail(PS_ERR_UNSUPPORTED, "ps_expm_noalloc: opts.profile creates events");
  const size_t need = make_layout(dtype, n, m, s, sigma, 0).bytes;
  if (need > kScratchBytes)
    return fail(PS_ERR_WORKSPACE, "ps_expm_noalloc: n = %lld, m = %d, s = %d needs %zu bytes of scratch, above the "
                "static %zu", (long long)n, m, s, need, kScratchBytes);
  void* ws = nullptr;
  if (ps_status e = scratch_address((hipStream_t)stream, &ws)) return e;
  return expm_impl(dtype, 1, n, A, lda, 0, coef, m, s, sigma, ldexp(1.0, -sigma), E, lde, 0, opts, report, ws,
                   kScratchBytes, stream);
}

ps_status ps_expm_strided_batched(ps_dtype dtype, int batch, int64_t n, const void* A, int64_t lda, int64_t strideA,
                                  const double* coef, int m, int s, int sigma, void* E, int64_t lde, int64_t strideE,
                                  const ps_opts* opts, ps_report* reports, void* ws, size_t ws_bytes, void* stream) {
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range [0, %d]", sigma, kMaxSigma);
  return expm_impl(dtype, batch, n, A, lda, strideA, coef, m, s, sigma, ldexp(1.0, -sigma), E, lde, strideE, opts,
                   reports, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// several polynomials sharing one power table
// ---------------------------------------------------------------------------
static ps_status multi_layouts(ps_dtype dtype, int64_t n, int k, const int* degrees, int* s, int square_arg,
                               std::vector<Layout>& Ls, size_t* total) {
  if (k < 1 || k > 16) return fail(PS_ERR_ARG, "k = %d polynomials out of range [1, 16]", k);
  if (!degrees) return fail(PS_ERR_ARG, "degrees == NULL");
  int mmax = 0;
  for (int t = 0; t < k; ++t) {
    if (degrees[t] < 0 || degrees[t] > kMaxDegree) return fail(PS_ERR_ARG, "degree %d out of range", degrees[t]);
    mmax = std::max(mmax, degrees[t]);
  }
  int sv = *s;
  if (ps_status e = check_common(dtype, n, mmax, &sv, 0)) return e;
  for (int t = 0; t < k; ++t)
    if (degrees[t] / sv + 1 > PS_MAX_BLOCKS) return fail(PS_ERR_ARG, "too many blocks for degree %d", degrees[t]);
  *s = sv;
  // shared part: the power table (and Z = A^2) and the Y copies live in the
  // layout of polynomial 0; every other polynomial gets a private section
  // holding its blocks, iterates, column sums and plan.
  Ls.clear();
  Layout base = make_layout(dtype, n, degrees[0], sv, 0, square_arg);
  // make sure polynomial 0's section fits the largest block count
  size_t off = base.bytes;
  Ls.push_back(base);
  for (int t = 1; t < k; ++t) {
    Layout Lt = make_layout(dtype, n, degrees[t], sv, 0, square_arg);
    Layout priv = Lt;
    // private offsets: B, P0, P1, colsum, plan relocated after `off`
    size_t o = off;
    priv.off_B = o;      o += (size_t)Lt.nB * Lt.slot;
    priv.off_P0 = o;     o += Lt.pslot;
    priv.off_P1 = o;     o += Lt.pslot;
    priv.off_colsum = o; o += al256((size_t)(Lt.nB + 2) * ((n + kRowChunk - 1) / kRowChunk) * n * 8);
    priv.off_plan = o;   o += al256(sizeof(Plan));
    // shared offsets from polynomial 0
    priv.off_pow = base.off_pow;
    priv.npow = base.npow;
    priv.off_yf32 = base.off_yf32;
    priv.off_ybf16 = base.off_ybf16;
    priv.off_yfp8 = base.off_yfp8;
    priv.off_yfp8s = base.off_yfp8s;
    priv.off_R = base.off_R;
    off = al256(o);
    Ls.push_back(priv);
  }
  *total = off;
  for (auto& L : Ls) L.bytes = off;
  return PS_OK;
}

ps_status ps_workspace_size_multi(ps_dtype dtype, int64_t n, int k, const int* degrees, int s, int square_arg,
                                  size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  std::vector<Layout> Ls;
  return multi_layouts(dtype, n, k, degrees, &s, square_arg ? 1 : 0, Ls, bytes);
}

ps_status ps_eval_multi(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int k, const double* const* coefs,
                        const int* degrees, int s, int square_arg, void* const* P, const int64_t* ldp,
                        const ps_opts* opts, ps_report* reports, void* ws, size_t ws_bytes, void* stream) {
  std::vector<Layout> Ls;
  size_t total = 0;
  square_arg = square_arg ? 1 : 0;
  if (ps_status e = multi_layouts(dtype, n, k, degrees, &s, square_arg, Ls, &total)) return e;
  if (!A || !coefs || !P || !ldp) return fail(PS_ERR_ARG, "NULL argument");
  if (lda < n) return fail(PS_ERR_ARG, "lda < n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanA = mat_span_bytes(n, lda, esize);
  for (int t = 0; t < k; ++t) {
    if (!coefs[t] || !P[t]) return fail(PS_ERR_ARG, "NULL coefficient or output pointer for polynomial %d", t);
    if (ldp[t] < n) return fail(PS_ERR_ARG, "ldp[%d] < n", t);
    const size_t spanP = mat_span_bytes(n, ldp[t], esize);
    if (overlap(A, spanA, P[t], spanP)) return fail(PS_ERR_ALIAS, "output %d overlaps the input", t);
    if (overlap(ws, total, P[t], spanP)) return fail(PS_ERR_ALIAS, "output %d overlaps the workspace", t);
    for (int u2 = 0; u2 < t; ++u2)
      if (overlap(P[u2], mat_span_bytes(n, ldp[u2], esize), P[t], spanP))
        return fail(PS_ERR_ALIAS, "outputs %d and %d overlap", u2, t);
  }
  if (ps_status e = check_ws(ws, ws_bytes, total)) return e;
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) return fail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_eval_multi");
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  MatArg X1{A, lda, 0};
  char* wgc = (char*)ws + Ls[0].off_colsum;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, X1, wgc, 0, st, "input matrix")) return e;
  if (square_arg) {
    MatArg Z = ws_mat((char*)ws, Ls[0].off_pow, n, total, esize);
    PS_HIP(launch_gemm(W, n, 1, X1, 0, X1, 0, Z, 1.0, 0, st));
    X1 = Z;
  }
  for (int t = 0; t < k; ++t) {
    Job J;
    J.L = &Ls[t];
    J.batch = 1;
    J.X1 = X1;
    J.beta = 1.0;
    J.coef = coefs[t];
    J.out = MatArg{P[t], ldp[t], 0};
    J.ws = (char*)ws;
    J.ws_stride = total;
    J.opts = o;
    J.write_y = (t == 0);
    J.build_powers = (t == 0);
    J.skip_square = true;   // Y stays in FP64: each chain's plan could call for it
    float ms[4] = {0, 0, 0, 0};
    if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
    if (reports)
      if (ps_status e = fill_report(Ls[t], J, 0, &reports[t], st, o.profile ? ms : nullptr)) return e;
  }
  if (o.check_finite)
    for (int t = 0; t < k; ++t)
      if (ps_status e = nonfinite_or_ok(W, n, 1, MatArg{P[t], ldp[t], 0}, wgc, 0, st, "result of polynomial"))
        return e;
  return PS_OK;
}

// ---------------------------------------------------------------------------
// linear solve and the Pade form of exp
// ---------------------------------------------------------------------------
ps_status ps_workspace_size_solve(ps_dtype dtype, int64_t n, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  if (dtype != PS_F64 && dtype != PS_F32) return fail(PS_ERR_UNSUPPORTED, "ps_solve: FP64 or FP32 only");
  if (n < 1) return fail(PS_ERR_ARG, "n = %lld < 1", (long long)n);
  if (n > kMaxSolveOrder) return fail(PS_ERR_UNSUPPORTED, "ps_solve: n = %lld above %lld", (long long)n,
                                      (long long)kMaxSolveOrder);
  *bytes = lu_solve_ws_bytes(n);
  return PS_OK;
}

ps_status ps_solve(ps_dtype dtype, int64_t n, void* Q, int64_t ldq, int64_t nrhs, void* P, int64_t ldp,
                   int32_t* ipiv, int* info, void* ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (ps_status e = ps_workspace_size_solve(dtype, n, &need)) return e;
  if (!Q) return fail(PS_ERR_ARG, "Q == NULL");
  if (ldq < n) return fail(PS_ERR_ARG, "ldq < n");
  if (nrhs < 0 || nrhs > (int64_t)1 << 30) return fail(PS_ERR_ARG, "nrhs = %lld out of range", (long long)nrhs);
  if (nrhs > 0 && !P) return fail(PS_ERR_ARG, "P == NULL");
  if (nrhs > 0 && ldp < n) return fail(PS_ERR_ARG, "ldp < n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanQ = mat_span_bytes(n, ldq, esize);
  const size_t spanP = nrhs > 0 ? (size_t)((nrhs - 1) * ldp + n) * esize : 0;
  if (nrhs > 0 && overlap(Q, spanQ, P, spanP)) return fail(PS_ERR_ALIAS, "P overlaps Q");
  if (ps_status e = check_ws(ws, ws_bytes, need)) return e;
  if (overlap(ws, need, Q, spanQ) || (nrhs > 0 && overlap(ws, need, P, spanP)))
    return fail(PS_ERR_ALIAS, "the workspace overlaps Q or P");
  if (ipiv && (overlap(ipiv, (size_t)n * 4, Q, spanQ) || (nrhs > 0 && overlap(ipiv, (size_t)n * 4, P, spanP)) ||
               overlap(ipiv, (size_t)n * 4, ws, need)))
    return fail(PS_ERR_ALIAS, "ipiv overlaps Q, P or the workspace");
  hipStream_t st = (hipStream_t)stream;
  PS_HIP(launch_lu_solve(dtype == PS_F64 ? 0 : 1, n, Q, ldq, nrhs, P, ldp, ipiv, (char*)ws, st));
  if (info) {
    PS_HIP(hipMemcpyAsync(info, ws, sizeof(int), hipMemcpyDeviceToHost, st));
    PS_HIP(hipStreamSynchronize(st));
  }
  return PS_OK;
}

static ps_status pade_layout(ps_dtype dtype, int64_t n, int m, int* s, std::vector<Layout>& Ls, size_t* total,
                             size_t* off_q, size_t* off_w, size_t* off_solve) {
  if (dtype != PS_F64 && dtype != PS_F32) return fail(PS_ERR_UNSUPPORTED, "ps_expm_pade: FP64 or FP32 only");
  if (m < 1 || m > 60) return fail(PS_ERR_ARG, "Pade degree m = %d out of range [1, 60]", m);
  if (n > kMaxSolveOrder) return fail(PS_ERR_UNSUPPORTED, "ps_expm_pade: n = %lld above %lld", (long long)n,
                                      (long long)kMaxSolveOrder);
  const int degrees[2] = {m, m};
  size_t base = 0;
  if (ps_status e = multi_layouts(dtype, n, 2, degrees, s, 0, Ls, &base)) return e;
  const size_t slot = Ls[0].slot;
  *off_q = base;
  *off_w = base + slot;
  *off_solve = base + 2 * slot;
  *total = *off_solve + al256(lu_solve_ws_bytes(n));
  return PS_OK;
}

ps_status ps_workspace_size_pade(ps_dtype dtype, int64_t n, int m, int s, int sigma, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "bytes == NULL");
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range", sigma);
  std::vector<Layout> Ls;
  size_t oq, ow, os;
  return pade_layout(dtype, n, m, &s, Ls, bytes, &oq, &ow, &os);
}

ps_status ps_expm_pade(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m, int s, int sigma, void* E,
                       int64_t lde, const ps_opts* opts, ps_report* reports, void* ws, size_t ws_bytes,
                       void* stream) {
  if (sigma < 0 || sigma > kMaxSigma) return fail(PS_ERR_ARG, "sigma = %d out of range", sigma);
  std::vector<Layout> Ls;
  size_t total = 0, off_q = 0, off_w = 0, off_solve = 0;
  if (ps_status e = pade_layout(dtype, n, m, &s, Ls, &total, &off_q, &off_w, &off_solve)) return e;
  if (!A || !E) return fail(PS_ERR_ARG, "NULL argument");
  if (lda < n || lde < n) return fail(PS_ERR_ARG, "lda or lde < n");
  const int esize = dtype == PS_F64 ? 8 : 4;
  const size_t spanA = mat_span_bytes(n, lda, esize), spanE = mat_span_bytes(n, lde, esize);
  if (overlap(A, spanA, E, spanE)) return fail(PS_ERR_ALIAS, "E overlaps A");
  if (ps_status e = check_ws(ws, ws_bytes, total)) return e;
  if (overlap(ws, total, E, spanE) || overlap(ws, total, A, spanA))
    return fail(PS_ERR_ALIAS, "the workspace overlaps A or E");
  Opts o = read_opts(opts, dtype == PS_F64 ? 0 : 1);
  if (ps_status e = check_opts(o)) return e;
  if (o.override_tiers) return fail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_expm_pade");
  double pc[61], qc[61];
  if (ps_status e = ps_coef_pade_exp(m, pc, qc)) return e;
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  char* w = (char*)ws;
  // the squarings alternate between E and a workspace slot and end in E, so
  // r_m lands in E when sigma is even and in the slot when it is odd
  MatArg Eo{E, lde, 0};
  MatArg Wk = ws_mat(w, off_w, n, total, esize);
  MatArg Qk = ws_mat(w, off_q, n, total, esize);
  MatArg R0 = (sigma % 2 == 0) ? Eo : Wk;
  char* wgc = w + Ls[0].off_colsum;
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, MatArg{A, lda, 0}, wgc, 0, st, "input matrix")) return e;
  for (int t = 0; t < 2; ++t) {
    Job J;
    J.L = &Ls[t];
    J.batch = 1;
    J.X1 = MatArg{A, lda, 0};
    J.beta = ldexp(1.0, -sigma);
    J.coef = t == 0 ? pc : qc;
    J.out = t == 0 ? R0 : Qk;
    J.ws = w;
    J.ws_stride = total;
    J.opts = o;
    J.write_y = (t == 0);
    J.build_powers = (t == 0);
    J.skip_square = true;
    float ms[4] = {0, 0, 0, 0};
    if (ps_status e = run_job(J, st, o.profile ? ms : nullptr)) return e;
    if (reports)
      if (ps_status e = fill_report(Ls[t], J, 0, &reports[t], st, o.profile ? ms : nullptr)) return e;
  }
  // r_m = q_m^{-1} p_m (section 4.1)
  PS_HIP(launch_lu_solve(W, n, (void*)Qk.p, n, n, (void*)R0.p, R0.ld, nullptr, w + off_solve, st));
  MatArg cur = R0;
  for (int i = 0; i < sigma; ++i) {
    MatArg dst = (cur.p == E) ? Wk : Eo;
    PS_HIP(launch_gemm(W, n, 1, cur, 0, cur, 0, dst, 1.0, 0, st));
    cur = dst;
  }
  if (o.check_finite)
    if (ps_status e = nonfinite_or_ok(W, n, 1, Eo, wgc, 0, st, "result")) return e;
  return PS_OK;
}

}  // extern "C"
