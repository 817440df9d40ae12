// Reverse-mode adjoint of PS evaluation inside scaling and squaring:
// gradA = d<G, r(A)>/dA for r(A) = p(2^-sigma A)^(2^sigma), which equals the
// Frechet derivative L_r(A^T, G).
//
// The call first runs the forward evaluation in the working precision
// (Algorithm 1 with the same s), keeping what the reverse pass needs, then
// walks the forward graph backwards:
//   squarings      R_{t+1} = R_t R_t      ->  Rbar_t = Rbar_{t+1} R_t^T + R_t^T Rbar_{t+1}
//   Horner step i  P_{i-1} = B_{i-1} + P_i Y
//                  ->  Bbar_{i-1} = Pbar_{i-1},  Pbar_i = Pbar_{i-1} Y^T,  Ybar += P_i^T Pbar_{i-1}
//   block assembly B_i = sum_j c_{si+j} X_j  ->  Xbar_j += c_{si+j} Bbar_i  (the folded step
//                  r when s divides m contributes c_m Pbar to Ybar the same way)
//   power chain    X_{j+1} = X_j X        ->  Xbar_j += Xbar_{j+1} X^T,  Xbar += X_j^T Xbar_{j+1}
//   scaling        X = 2^-sigma A         ->  Abar = 2^-sigma Xbar
// Every product is an n x n GEMM of k_gemm (transposed operands, accumulate
// epilogue); 2 (s - 1) + 2 (Horner products) + 2 sigma GEMMs in all, twice the
// forward count.  recompute = 0 stores the Horner iterates P_1..P_{first-1};
// recompute = 1 keeps two buffers and re-runs the Horner recurrence from the
// top whenever an iterate is needed.
// In mixed mode the forward pass also runs the planning kernel on its block
// norms (the same plan as the mixed forward evaluation), and the two products
// of reverse Horner step i, Pbar_i = Pbar_{i-1} Y^T and Ybar += P_i^T Pbar_{i-1},
// run in the tier of forward step i (k_tpack + k_tgemm read it on the
// device).  The stored iterates, the power chain, the block scatter and the
// squarings stay in the working precision.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ps_internal.h"

using namespace psk;

namespace {

size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }

struct BLayout {
  Layout F;
  size_t off_Pst;   // stored iterates P_1..P_{i0-1} (store) or two running buffers (recompute)
  int nPst;
  size_t off_R;     // R_0..R_{sigma-1}
  size_t off_G[2];  // adjoint ping-pong
  size_t off_Xbar;  // Xbar_1..Xbar_s
  size_t off_GX;
  size_t off_Q[2];  // operand copies of a tiered reverse product
  size_t bytes;
};

BLayout make_blayout(ps_dtype dt, int64_t n, int m, int s, int sigma, int recompute) {
  BLayout B;
  B.F = make_layout(dt, n, m, s, sigma, 0);
  const size_t slot = B.F.slot;
  size_t off = B.F.bytes;
  const int i0 = B.F.first_step;
  B.nPst = recompute ? 2 : std::max(i0 - 1, 0);
  B.off_Pst = off;  off += (size_t)B.nPst * slot;
  B.off_R = off;    off += (size_t)sigma * slot;
  B.off_G[0] = off; off += slot;
  B.off_G[1] = off; off += slot;
  B.off_Xbar = off; off += (size_t)s * slot;
  B.off_GX = off;   off += slot;
  for (int q = 0; q < 2; ++q) { B.off_Q[q] = off; off += B.F.pslot; }
  B.bytes = al256b(off);
  return B;
}

int default_s_b(int m) {
  if (m <= 1) return 1;
  int s = (int)ceil(sqrt((double)m));
  while ((s - 1) * (s - 1) >= m) --s;
  while (s * s < m) ++s;
  return s;
}

thread_local char err_buf[512];   // message of the failing HIP call (per thread, like ps_last_error)

ps_status bad(ps_status st, const char* msg) { return ps_set_error(st, msg); }

ps_status validate(ps_dtype dt, int batch, int64_t n, int m, int* s, int sigma) {
  if (dt != PS_F64 && dt != PS_F32) return bad(PS_ERR_ARG, "dtype must be PS_F64 or PS_F32");
  if (batch < 1 || batch > 65535) return bad(PS_ERR_ARG, "batch out of range [1, 65535]");
  if (n < 1 || n > (1LL << 20)) return bad(PS_ERR_ARG, "n out of range");
  if (m < 0 || m > kMaxDegree) return bad(PS_ERR_ARG, "degree m out of range");
  if (*s == 0) *s = default_s_b(m);
  if (*s < 1 || *s > std::max(m, 1)) return bad(PS_ERR_ARG, "block size s out of range [1, max(m,1)]");
  if (m / *s + 1 > PS_MAX_BLOCKS) return bad(PS_ERR_ARG, "too many blocks");
  if (sigma < 0 || sigma > 500) return bad(PS_ERR_ARG, "sigma out of range [0, 500]");
  return PS_OK;
}

#define BK_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      snprintf(err_buf, sizeof err_buf, "%s: %s", #call, hipGetErrorString(e_));       \
      return bad(PS_ERR_HIP, err_buf);                                                 \
    }                                                                                  \
  } while (0)

}  // namespace

extern "C" {

ps_status ps_workspace_size_backward(ps_dtype dtype, int batch, int64_t n, int m, int s, int sigma, int recompute,
                                     size_t* bytes) {
  if (!bytes) return bad(PS_ERR_ARG, "bytes == NULL");
  if (ps_status e = validate(dtype, batch, n, m, &s, sigma)) return e;
  *bytes = make_blayout(dtype, n, m, s, sigma, recompute ? 1 : 0).bytes * (size_t)batch;
  return PS_OK;
}

ps_status ps_expm_backward(ps_dtype dtype, int batch, int64_t n, const void* A, int64_t lda, int64_t strideA,
                           const void* G, int64_t ldg, int64_t strideG, const double* coef, int m, int s, int sigma,
                           void* gradA, int64_t ldga, int64_t strideGA, int recompute, const ps_opts* opts, void* ws,
                           size_t ws_bytes, void* stream) {
  if (ps_status e = validate(dtype, batch, n, m, &s, sigma)) return e;
  if (!A || !G || !gradA) return bad(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || ldg < n || ldga < n) return bad(PS_ERR_ARG, "leading dimension smaller than n");
  const int64_t span = (n - 1) * std::max({lda, ldg, ldga}) + n;
  if (batch > 1 && (strideA < (n - 1) * lda + n || strideG < (n - 1) * ldg + n || strideGA < (n - 1) * ldga + n))
    return bad(PS_ERR_ARG, "batch stride smaller than one matrix");
  if (opts && opts->mode != PS_MODE_FIXED && opts->mode != PS_MODE_MIXED) return bad(PS_ERR_ARG, "opts.mode");
  if (opts && opts->rule != PS_RULE_BLOCKS && opts->rule != PS_RULE_APRIORI) return bad(PS_ERR_ARG, "opts.rule");
  if (opts && opts->check_finite) return bad(PS_ERR_UNSUPPORTED, "check_finite is not supported by ps_expm_backward");
  const int W = dtype == PS_F64 ? 0 : 1;
  const bool mixed = opts && opts->mode == PS_MODE_MIXED;
  const int es = W == 0 ? 8 : 4;
  auto span_of = [&](const void* p, int64_t ld, int64_t stride) {
    return std::make_pair((const char*)p, (size_t)(((int64_t)(batch - 1) * stride + (n - 1) * ld + n) * es));
  };
  (void)span;
  auto ov = [](std::pair<const char*, size_t> a, std::pair<const char*, size_t> b) {
    return a.first < b.first + b.second && b.first < a.first + a.second;
  };
  auto sA = span_of(A, lda, strideA), sG = span_of(G, ldg, strideG), sO = span_of(gradA, ldga, strideGA);
  if (ov(sO, sA) || ov(sO, sG)) return bad(PS_ERR_ALIAS, "gradA overlaps A or G");
  BLayout B = make_blayout(dtype, n, m, s, sigma, recompute ? 1 : 0);
  const size_t total = B.bytes * (size_t)batch;
  if (ws_bytes < total) return bad(PS_ERR_WORKSPACE, "workspace too small for ps_expm_backward");
  if (!ws || ((uintptr_t)ws & 255)) return bad(PS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (ov(std::make_pair((const char*)ws, total), sO)) return bad(PS_ERR_ALIAS, "workspace overlaps gradA");

  std::vector<double> c(m + 1);
  if (coef) {
    for (int k = 0; k <= m; ++k) c[k] = coef[k];
  } else {
    if (m > 170) return bad(PS_ERR_ARG, "built-in Taylor coefficients need m <= 170");
    ps_coef_taylor_exp(m, c.data());
  }
  if (W == 1)
    for (int k = 0; k <= m; ++k) c[k] = (double)(float)c[k];

  hipStream_t st = (hipStream_t)stream;
  const Layout& L = B.F;
  const size_t wss = B.bytes;
  char* base = (char*)ws;
  auto slot = [&](size_t off) { return MatArg{base + off, n, (int64_t)(wss / es)}; };
  const MatArg Am{A, lda, strideA};
  const double beta = ldexp(1.0, -sigma);
  const int i0 = L.first_step;
  const int r = L.r;

  // X_j as (matrix, alpha): X_1 = beta * A, X_j (j >= 2) from the power slots
  auto Xj = [&](int j) { return slot(L.off_pow + (size_t)(j - 2) * L.slot); };
  // Y = X_s as (matrix, alpha)
  const MatArg Ym = (s == 1) ? Am : Xj(s);
  const double yalpha = (s == 1) ? beta : 1.0;
  auto Bslot = [&](int i) { return slot(L.off_B + (size_t)i * L.slot); };

  // ---------------- forward (working precision) ----------------
  for (int j = 2; j <= s; ++j) {
    const MatArg prev = (j == 2) ? Am : Xj(j - 1);
    BK_HIP(launch_gemm(W, n, batch, prev, 0, Am, 0, Xj(j), (j == 2) ? beta * beta : beta, 0, st));
  }
  {
    Coefs cf;
    memset(&cf, 0, sizeof cf);
    for (int k = 0; k <= m; ++k) cf.c[k] = c[k];
    AssembleArgs aa;
    aa.n = n;
    aa.nv = n;
    aa.m = m;
    aa.s = s;
    aa.r = r;
    aa.nB = L.nB;
    aa.trivial_last = L.trivial_last;
    aa.X1 = Am;
    aa.x1_scale = beta;
    aa.pow_shift = 0;
    aa.ws = base;
    aa.ws_stride = wss;
    aa.L = L;
    aa.tier_mask = 0;
    aa.y_f32 = 0;
    BK_HIP(launch_assemble(W, aa, cf, batch, st));
  }
  if (mixed) {
    // the forward plan from the block norms (tiers of the reverse Horner products)
    PlanArgs pa;
    memset(&pa, 0, sizeof pa);
    pa.r = r;
    pa.mode = PS_MODE_MIXED;
    pa.working = W;
    pa.nB = L.nB;
    pa.trivial_last = L.trivial_last;
    pa.rule = opts->rule;
    unsigned mask = opts->tier_mask ? opts->tier_mask : 0xFu;
    mask |= 1u << W;
    for (int t = 0; t < W; ++t) mask &= ~(1u << t);
    pa.mask = mask;
    pa.delta = opts->delta > 0 ? opts->delta : 10.0;
    pa.abs_cm = fabs(c[m]);
    pa.use_override = opts->tier_override != nullptr;
    if (pa.use_override)
      for (int i = 0; i <= r; ++i) pa.override_tier[i] = opts->tier_override[i];
    pa.ws = base;
    pa.ws_stride = wss;
    pa.L = L;
    BK_HIP(launch_plan(pa, batch, st));
  }
  // Horner iterate P_i (i >= 1): B_{i0} for i = i0, stored slot otherwise
  auto Pst = [&](int i) { return slot(B.off_Pst + (size_t)(i - 1) * L.slot); };
  // one Horner step into dst: dst = B_{i-1} + alpha_y * (P_i Y)
  auto horner_step = [&](MatArg Pi, int i, MatArg dst) -> ps_status {
    BK_HIP(launch_scale_copy(W, n, batch, Bslot(i - 1), dst, 1.0, st));
    BK_HIP(launch_gemm(W, n, batch, Pi, 0, Ym, 0, dst, yalpha, 1, st));
    return PS_OK;
  };
  // P_i for the reverse pass (recompute mode: from the top into running buffers)
  auto iterate = [&](int i, MatArg* out) -> ps_status {
    if (i == i0) { *out = Bslot(i0); return PS_OK; }
    if (!recompute) { *out = Pst(i); return PS_OK; }
    MatArg bufs[2] = {Pst(1), Pst(2)};
    MatArg cur = Bslot(i0);
    int k = 0;
    for (int q = i0; q > i; --q) {
      if (ps_status e = horner_step(cur, q, bufs[k & 1])) return e;
      cur = bufs[k & 1];
      ++k;
    }
    *out = cur;
    return PS_OK;
  };
  MatArg R0 = slot(B.off_R);
  if (!recompute) {
    MatArg cur = Bslot(i0);
    for (int i = i0; i >= 2; --i) {
      if (ps_status e = horner_step(cur, i, Pst(i - 1))) return e;
      cur = Pst(i - 1);
    }
    if (sigma > 0) {
      if (i0 >= 1) { if (ps_status e = horner_step(cur, 1, R0)) return e; }
      else BK_HIP(launch_scale_copy(W, n, batch, Bslot(0), R0, 1.0, st));
    }
  } else if (sigma > 0) {
    if (i0 >= 1) {
      MatArg p1;
      if (ps_status e = iterate(1, &p1)) return e;
      if (ps_status e = horner_step(p1, 1, R0)) return e;
    } else {
      BK_HIP(launch_scale_copy(W, n, batch, Bslot(0), R0, 1.0, st));
    }
  }
  for (int t = 1; t < sigma; ++t) {
    MatArg Rp = slot(B.off_R + (size_t)(t - 1) * L.slot), Rt = slot(B.off_R + (size_t)t * L.slot);
    BK_HIP(launch_gemm(W, n, batch, Rp, 0, Rp, 0, Rt, 1.0, 0, st));
  }

  // ---------------- reverse ----------------
  MatArg Gb[2] = {slot(B.off_G[0]), slot(B.off_G[1])};
  int cur = 0;
  BK_HIP(launch_scale_copy(W, n, batch, MatArg{G, ldg, strideG}, Gb[0], 1.0, st));
  for (int t = sigma - 1; t >= 0; --t) {
    MatArg Rt = slot(B.off_R + (size_t)t * L.slot);
    BK_HIP(launch_gemm(W, n, batch, Gb[cur], 0, Rt, 1, Gb[cur ^ 1], 1.0, 0, st));
    BK_HIP(launch_gemm(W, n, batch, Rt, 1, Gb[cur], 0, Gb[cur ^ 1], 1.0, 1, st));
    cur ^= 1;
  }
  // Pbar_0 = Gb[cur]; zero Xbar_1..Xbar_s and GX
  for (int j = 1; j <= s; ++j)
    BK_HIP(launch_fill_identity(W, n, batch, slot(B.off_Xbar + (size_t)(j - 1) * L.slot), 0.0, st));
  BK_HIP(launch_fill_identity(W, n, batch, slot(B.off_GX), 0.0, st));
  auto Xbar = [&](int j) { return slot(B.off_Xbar + (size_t)(j - 1) * L.slot); };
  auto scatter_block = [&](int i, MatArg src) -> ps_status {
    // Xbar_j += c_{si+j} Bbar_i, j = 1..s-1 (and j = s for the folded step)
    ScatterArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.n = n;
    sa.nd = s;
    sa.src = src;
    sa.dst = base + B.off_Xbar;
    sa.dst_step = L.slot;
    sa.ws_stride = wss;
    bool any = false;
    for (int j = 1; j <= s; ++j) {
      const int k = s * i + j;
      const bool ok = (j < s || (L.trivial_last && i == i0)) && k <= m;
      sa.coef[j - 1] = ok ? c[k] : 0.0;
      any = any || (ok && c[k] != 0.0);
    }
    if (any) BK_HIP(launch_scatter(W, sa, batch, st));
    return PS_OK;
  };
  // C = alpha op(A) op(B) (+ C) in the tier of forward Horner step i
  auto tiered = [&](int i, MatArg A_, int tA, MatArg B_, int tB, MatArg C_, double alpha, int acc) -> ps_status {
    TPackArgs pk;
    memset(&pk, 0, sizeof pk);
    pk.n = n;
    pk.step = i;
    pk.ws = base;
    pk.ws_stride = wss;
    pk.L = L;
    pk.role = 0;
    pk.src = A_;
    pk.trans = tA;
    pk.off_dst = B.off_Q[0];
    BK_HIP(launch_tpack(W, pk, batch, st));
    pk.role = 1;
    pk.src = B_;
    pk.trans = tB;
    pk.off_dst = B.off_Q[1];
    BK_HIP(launch_tpack(W, pk, batch, st));
    TGemmArgs tg;
    memset(&tg, 0, sizeof tg);
    tg.n = n;
    tg.step = i;
    tg.A = A_;
    tg.B = B_;
    tg.C = C_;
    tg.transA = tA;
    tg.transB = tB;
    tg.alpha = alpha;
    tg.accumulate = acc;
    tg.off_pa = B.off_Q[0];
    tg.off_pb = B.off_Q[1];
    tg.ws = base;
    tg.ws_stride = wss;
    tg.L = L;
    BK_HIP(launch_tgemm(W, tg, batch, st));
    return PS_OK;
  };
  for (int i = 1; i <= i0; ++i) {
    // Gb[cur] = Pbar_{i-1} = Bbar_{i-1}
    if (ps_status e = scatter_block(i - 1, Gb[cur])) return e;
    MatArg Pi;
    if (ps_status e = iterate(i, &Pi)) return e;
    // Ybar += P_i^T Pbar_{i-1} (times yalpha when Y = beta A: the chain rule
    // through Y = beta A is applied at the end with Xbar_1)
    // Pbar_i = Pbar_{i-1} Y^T
    if (mixed) {
      if (ps_status e = tiered(i, Pi, 1, Gb[cur], 0, Xbar(s), 1.0, 1)) return e;
      if (ps_status e = tiered(i, Gb[cur], 0, Ym, 1, Gb[cur ^ 1], yalpha, 0)) return e;
    } else {
      BK_HIP(launch_gemm(W, n, batch, Pi, 1, Gb[cur], 0, Xbar(s), 1.0, 1, st));
      BK_HIP(launch_gemm(W, n, batch, Gb[cur], 0, Ym, 1, Gb[cur ^ 1], yalpha, 0, st));
    }
    cur ^= 1;
  }
  if (ps_status e = scatter_block(i0, Gb[cur])) return e;
  // power chain X_{j+1} = X_j X, X = beta A
  for (int j = s - 1; j >= 1; --j) {
    BK_HIP(launch_gemm(W, n, batch, Xbar(j + 1), 0, Am, 1, Xbar(j), beta, 1, st));
    const MatArg Xjm = (j == 1) ? Am : Xj(j);
    BK_HIP(launch_gemm(W, n, batch, Xjm, 1, Xbar(j + 1), 0, slot(B.off_GX), (j == 1) ? beta : 1.0, 1, st));
  }
  // dL/dA = beta (GX + Xbar_1)
  BK_HIP(launch_axpby(W, n, batch, slot(B.off_GX), Xbar(1), MatArg{gradA, ldga, strideGA}, beta, st));
  return PS_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// uneven batch of adjoints: matrix b has order n[b], block size s[b] and
// scaling sigma[b].  Consecutive matrices with the same order, block size,
// scaling and leading dimensions whose pointers advance by one constant
// stride each (for A, G and gradA) form a run, evaluated as one strided
// batch; every matrix owns the workspace slice of its single-matrix size.
// ---------------------------------------------------------------------------
namespace {
ps_status backward_batch_sizes(ps_dtype dtype, int batch, const int32_t* n, int m, const int32_t* s,
                               const int32_t* sigma, int recompute, std::vector<size_t>* each, size_t* total) {
  if (batch < 1 || batch > (1 << 22)) return bad(PS_ERR_ARG, "batch out of range");
  if (!n) return bad(PS_ERR_ARG, "n == NULL");
  size_t t = 0;
  for (int b = 0; b < batch; ++b) {
    size_t one = 0;
    if (ps_status e = ps_workspace_size_backward(dtype, 1, n[b], m, s ? s[b] : 0, sigma ? sigma[b] : 0, recompute,
                                                 &one))
      return e;
    if (each) each->push_back(al256b(one));
    t += al256b(one);
  }
  *total = t;
  return PS_OK;
}
}  // namespace

extern "C" {

ps_status ps_workspace_size_backward_batched(ps_dtype dtype, int batch, const int32_t* n, int m, const int32_t* s,
                                             const int32_t* sigma, int recompute, size_t* bytes) {
  if (!bytes) return bad(PS_ERR_ARG, "bytes == NULL");
  return backward_batch_sizes(dtype, batch, n, m, s, sigma, recompute, nullptr, bytes);
}

ps_status ps_expm_backward_batched(ps_dtype dtype, int batch, const int32_t* n, const void* const* A,
                                   const int64_t* lda, const void* const* G, const int64_t* ldg, const double* coef,
                                   int m, const int32_t* s, const int32_t* sigma, void* const* gradA,
                                   const int64_t* ldga, int recompute, const ps_opts* opts, void* ws, size_t ws_bytes,
                                   void* stream) {
  std::vector<size_t> each;
  size_t total = 0;
  if (ps_status e = backward_batch_sizes(dtype, batch, n, m, s, sigma, recompute, &each, &total)) return e;
  if (!A || !lda || !G || !ldg || !gradA || !ldga) return bad(PS_ERR_ARG, "NULL array argument");
  if (ws_bytes < total) return bad(PS_ERR_WORKSPACE, "workspace too small for ps_expm_backward_batched");
  if (!ws || ((uintptr_t)ws & 255)) return bad(PS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (opts && opts->check_finite) return bad(PS_ERR_UNSUPPORTED, "check_finite is not supported by ps_expm_backward");
  const int es = dtype == PS_F64 ? 8 : 4;
  auto ov = [](const void* a, size_t as, const void* b, size_t bs) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bs && y < x + as;
  };
  // every matrix checked before any device work
  for (int b = 0; b < batch; ++b) {
    const int64_t nb = n[b];
    if (!A[b] || !G[b] || !gradA[b]) return bad(PS_ERR_ARG, "NULL matrix pointer");
    if (lda[b] < nb || ldg[b] < nb || ldga[b] < nb) return bad(PS_ERR_ARG, "leading dimension smaller than n");
    const size_t so = (size_t)((nb - 1) * ldga[b] + nb) * es;
    if (ov(gradA[b], so, A[b], (size_t)((nb - 1) * lda[b] + nb) * es) ||
        ov(gradA[b], so, G[b], (size_t)((nb - 1) * ldg[b] + nb) * es))
      return bad(PS_ERR_ALIAS, "gradA overlaps A or G");
    if (ov(gradA[b], so, ws, total)) return bad(PS_ERR_ALIAS, "workspace overlaps gradA");
  }
  if (opts && opts->mode != PS_MODE_FIXED && opts->mode != PS_MODE_MIXED) return bad(PS_ERR_ARG, "opts.mode");
  if (opts && opts->rule != PS_RULE_BLOCKS && opts->rule != PS_RULE_APRIORI) return bad(PS_ERR_ARG, "opts.rule");
  char* wsc = (char*)ws;
  size_t off = 0;
  for (int b0 = 0; b0 < batch;) {
    // extend the run b0 .. b1-1 while shapes match and the strides stay constant
    auto same = [&](int x, int y) {
      return n[x] == n[y] && (s ? s[x] : 0) == (s ? s[y] : 0) && (sigma ? sigma[x] : 0) == (sigma ? sigma[y] : 0) &&
             lda[x] == lda[y] && ldg[x] == ldg[y] && ldga[x] == ldga[y];
    };
    const int64_t nb = n[b0];
    int b1 = b0 + 1;
    int64_t sA = 0, sG = 0, sO = 0;
    if (b1 < batch && same(b0, b1)) {
      sA = ((const char*)A[b1] - (const char*)A[b0]) / es;
      sG = ((const char*)G[b1] - (const char*)G[b0]) / es;
      sO = ((const char*)gradA[b1] - (const char*)gradA[b0]) / es;
      const bool ok = sA >= (nb - 1) * lda[b0] + nb && sG >= (nb - 1) * ldg[b0] + nb &&
                      sO >= (nb - 1) * ldga[b0] + nb &&
                      (const char*)A[b0] + sA * es == (const char*)A[b1] &&
                      (const char*)G[b0] + sG * es == (const char*)G[b1] &&
                      (const char*)gradA[b0] + sO * es == (const char*)gradA[b1];
      if (ok) {
        b1 = b0 + 2;
        while (b1 < batch && same(b0, b1) && (const char*)A[b1] == (const char*)A[b1 - 1] + sA * es &&
               (const char*)G[b1] == (const char*)G[b1 - 1] + sG * es &&
               (const char*)gradA[b1] == (const char*)gradA[b1 - 1] + sO * es)
          ++b1;
      }
    }
    const int cnt = b1 - b0;
    const size_t bytes = each[b0] * (size_t)cnt;   // equal shapes: equal per-matrix sizes
    if (ps_status e = ps_expm_backward(dtype, cnt, nb, A[b0], lda[b0], sA, G[b0], ldg[b0], sG, coef, m,
                                       s ? s[b0] : 0, sigma ? sigma[b0] : 0, gradA[b0], ldga[b0], sO, recompute,
                                       opts, wsc + off, bytes, stream))
      return e;
    off += bytes;
    b0 = b1;
  }
  return PS_OK;
}

}  // extern "C"
