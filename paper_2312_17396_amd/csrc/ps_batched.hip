// Many matrices of uneven order in one persistent launch.
//
// Each workgroup repeatedly takes the next matrix from a device work counter
// (matrices ordered by decreasing modelled cost, so the large ones start
// first) and runs the whole evaluation for it with its own 256 threads:
// X = 2^-sigma A, the power table, the block assembly with norms, the
// precision plan (section 2, eq. (choose-ui); section 4.1.1 tiers), the
// Horner chain in the planned tiers and the squarings (eq. (scal-idea)).
// Phases are separated by workgroup barriers only; no grid-wide
// synchronisation exists, every workgroup leaves the loop once the counter
// passes the batch size.
//
// The block size is chosen per matrix among floor(sqrt m) and ceil(sqrt m)
// (the two equally cheap choices of the paper's section 1) by the modelled
// cost sum over products of 1 / rate(tier) under an a-priori plan from
// ||X||_1 (||B_i|| ~ sum_j |c_{si+j}| ||X||^j, ||Y|| ~ ||X||^s); ties keep
// ceil(sqrt m), the paper's default.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "ps_device.h"

namespace psk {

struct BatchItem {
  const void* A;
  int64_t lda;
  void* E;
  int64_t lde;
  int64_t ws_off;       // byte offset of the matrix's workspace region
  int sigma;
  int s_fixed;          // 0: choose between L[0] (floor sqrt m) and L[1] (ceil sqrt m)
  Layout L[2];
};

struct BatchArgs {
  const BatchItem* items;
  const int* order;
  int* counter;
  int batch;
  int mode;
  unsigned mask;
  double delta;
  char* ws;
  int* chosen;          // per matrix: chosen block size (for reports)
  Coefs cf;
};

template <typename W>
constexpr int persist_smem() { return 2 * STAGE * (int)sizeof(W); }

// modelled relative cost of one n^3 product per tier (inverse MFMA rates)
__device__ inline double tier_cost(int t) { return t == 0 ? 2.0 : t == 1 ? 1.0 : t == 2 ? 1.0 / 16 : 1.0 / 32; }

__device__ inline double apriori_cost(const Layout& L, const Coefs& cf, double x, int working, unsigned mask,
                                      double delta) {
  double nb[PS_MAX_BLOCKS];
  const int s = L.s, r = L.r, m = L.m;
  for (int i = 0; i <= r; ++i) {
    double v = 0.0, p = 1.0;
    const int jmax = (i < r) ? s - 1 : m - s * r;
    for (int j = 0; j <= jmax; ++j) {
      v += fabs(cf.c[s * i + j]) * p;
      p *= x;
    }
    nb[i] = v;
  }
  double ny = 1.0;
  for (int j = 0; j < s; ++j) ny *= x;
  int tier[PS_MAX_BLOCKS];
  double u[PS_MAX_BLOCKS];
  int nu;
  plan_tiers(r, nb, ny, working, mask, delta, tier, u, &nu);
  double c = (L.s - 1) * tier_cost(working);
  for (int i = L.first_step; i >= 1; --i) c += tier_cost(tier[i]);
  return c;
}

template <typename W>
__device__ void run_matrix(const BatchArgs& a, const BatchItem& it, int idx, char* smem, double* red, double* norms) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const W* A = (const W*)it.A;
  const int64_t lda = it.lda;
  const int64_t n = it.L[0].n;
  const int sigma = it.sigma;
  const double beta = ldexp(1.0, -sigma);
  // ---- block size
  int pick = 1;
  if (!it.s_fixed && it.L[0].s != it.L[1].s) {
    // ||X||_1 = beta * max column abs sum of A
    double mx = 0.0;
    for (int64_t c = w; c < n; c += NW) {
      double v = 0.0;
      for (int64_t rw = lane; rw < n; rw += 64) v += fabs((double)A[rw + c * lda]);
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (v > mx || v != v) mx = v;
    }
    if (lane == 0) red[w] = mx;
    __syncthreads();
    if (t == 0) {
      double x = red[0];
      for (int k = 1; k < NW; ++k) if (red[k] > x || red[k] != red[k]) x = red[k];
      x *= beta;
      const double c0 = apriori_cost(it.L[0], a.cf, x, WT, a.mask, a.delta);
      const double c1 = apriori_cost(it.L[1], a.cf, x, WT, a.mask, a.delta);
      red[NW] = (c0 < c1) ? 0.0 : 1.0;
    }
    __syncthreads();
    pick = red[NW] != 0.0 ? 1 : 0;
    __syncthreads();
  }
  const Layout& L = it.L[pick];
  if (t == 0 && a.chosen) a.chosen[idx] = L.s;
  char* ws = a.ws + it.ws_off;
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  const int ntiles = ntm * ntn;
  const int64_t se = (int64_t)(L.slot / sizeof(W));
  W* pw = (W*)(ws + L.off_pow);
  // ---- 1. power table: X_2 = beta^2 (A A), X_{j+1} = beta (X_j A)
  for (int j = 2; j <= L.s; ++j) {
    const W* src = (j == 2) ? A : pw + (int64_t)(j - 3) * se;
    const int64_t lds = (j == 2) ? lda : n;
    const double alpha = (j == 2) ? beta * beta : beta;
    for (int tile = 0; tile < ntiles; ++tile)
      gemm_tile<W, false, false>(src, lds, A, lda, pw + (int64_t)(j - 2) * se, n, n, (int64_t)(tile % ntm) * kTileM,
                                 (int64_t)(tile / ntm) * kTileN, alpha, 0, smem);
  }
  // ---- 2. blocks, norms, low-precision copies of Y
  AssembleArgs aa;
  aa.n = n;
  aa.m = L.m;
  aa.s = L.s;
  aa.r = L.r;
  aa.nB = L.nB;
  aa.trivial_last = L.trivial_last;
  aa.X1 = MatArg{A, lda, 0};
  aa.x1_scale = beta;
  aa.ws = ws;
  aa.ws_stride = 0;
  aa.L = L;
  aa.tier_mask = a.mode == PS_MODE_MIXED ? a.mask : 0u;
  const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
  for (int64_t c = w; c < n; c += NW)
    for (int64_t ch = 0; ch < nch; ++ch) assemble_column<W>(aa, a.cf, ws, A, c, ch);
  __syncthreads();
  // ---- 3. plan
  PlanArgs pa;
  pa.r = L.r;
  pa.mode = a.mode;
  pa.working = WT;
  pa.nB = L.nB;
  pa.trivial_last = L.trivial_last;
  pa.mask = a.mask;
  pa.delta = a.delta;
  pa.abs_cm = fabs(a.cf.c[L.m]);
  pa.use_override = 0;
  pa.ws = ws;
  pa.ws_stride = 0;
  pa.L = L;
  plan_matrix(pa, L, ws, red, norms);
  const Plan* P = (const Plan*)(ws + L.off_plan);
  // ---- 4. Horner chain
  const bool square = sigma > 0;
  W* R = (W*)(ws + L.off_R);
  HornerTile<W> h;
  h.n = n;
  h.Mp = L.Mp;
  h.Kp = L.Kp;
  if (L.s == 1) {
    h.ysrc = A;
    h.ldy = lda;
    h.yscale = beta;
  } else {
    h.ysrc = pw + (int64_t)(L.s - 2) * se;
    h.ldy = n;
    h.yscale = 1.0;
  }
  h.yf32 = (const float*)(ws + L.off_yf32);
  h.ybf16 = (const uint16_t*)(ws + L.off_ybf16);
  h.yfp8 = (const uint8_t*)(ws + L.off_yfp8);
  h.yfp8s = (const uint8_t*)(ws + L.off_yfp8s);
  W* fin = square ? R : (W*)it.E;
  const int64_t ldfin = square ? n : it.lde;
  const int i0 = L.first_step;
  for (int k = -1; k < i0; ++k) {
    // k = -1: cast of B_{i0}; k >= 0: step i = i0 - k
    const int i = i0 - k;
    const bool cast = (k < 0);
    const bool final_out = cast ? (i0 == 0) : (i == 1);
    h.t_in = cast ? -1 : P->tier[i];
    h.t_out = final_out ? WT : P->tier[cast ? i0 : i - 1];
    // the cast writes P0; step k >= 0 reads P0 (k even) or P1 (k odd) and writes the other
    h.pin = ws + ((k & 1) ? L.off_P1 : L.off_P0);
    h.pout = ws + ((k & 1) ? L.off_P0 : L.off_P1);
    if (cast) h.pout = ws + L.off_P0;
    h.bsrc = (const W*)(ws + L.off_B) + (int64_t)(cast ? i0 : i - 1) * se;
    h.outw = final_out ? fin : (W*)h.pout;
    h.ldo = final_out ? ldfin : n;
    for (int tile = 0; tile < ntiles; ++tile)
      horner_tile<W>(h, (int64_t)(tile % ntm) * kTileM, (int64_t)(tile / ntm) * kTileN, smem);
  }
  // ---- 5. squarings
  if (square) {
    W* bufs[2] = {R, (W*)(ws + L.off_P0)};
    for (int q = 1; q <= sigma; ++q) {
      const W* src = bufs[(q - 1) & 1];
      W* dst = (q == sigma) ? (W*)it.E : bufs[q & 1];
      const int64_t ldd = (q == sigma) ? it.lde : n;
      for (int tile = 0; tile < ntiles; ++tile)
        gemm_tile<W, false, false>(src, n, src, n, dst, ldd, n, (int64_t)(tile % ntm) * kTileM,
                                   (int64_t)(tile / ntm) * kTileN, 1.0, 0, smem);
    }
  }
}

template <typename W>
__global__ __launch_bounds__(NT) void k_ps_persistent(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[persist_smem<W>()];
  __shared__ double red[NT];
  __shared__ double norms[PS_MAX_BLOCKS + 1];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(a.counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= a.batch) break;   // uniform across the workgroup
    const int b = a.order[idx];
    run_matrix<W>(a, a.items[b], b, smem, red, norms);
  }
}

__global__ void k_zero_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

}  // namespace psk

// ===========================================================================
// host side
// ===========================================================================
using namespace psk;

namespace {

thread_local std::string g_batch_err;

ps_status bfail(ps_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_batch_err = buf;
  return st;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan2 {
  std::vector<BatchItem> items;
  std::vector<int> order;
  size_t off_items, off_order, off_counter, off_chosen, off_mats, total;
};

int s_floor(int m) {
  int s = (int)floor(sqrt((double)m));
  while ((s + 1) * (s + 1) <= m) ++s;
  while (s * s > m) --s;
  return std::max(s, 1);
}
int s_ceil(int m) {
  if (m <= 1) return 1;
  int s = s_floor(m);
  return s * s == m ? s : s + 1;
}

ps_status build_plan(ps_dtype dt, int batch, const int32_t* n, int m, const int32_t* s, const int32_t* sigma,
                     const void* const* A, const int64_t* lda, void* const* E, const int64_t* lde, Plan2& P,
                     bool need_ptrs) {
  if (dt != PS_F64 && dt != PS_F32) return bfail(PS_ERR_ARG, "dtype must be PS_F64 or PS_F32");
  if (batch < 1 || batch > (1 << 24)) return bfail(PS_ERR_ARG, "batch = %d out of range", batch);
  if (!n) return bfail(PS_ERR_ARG, "n == NULL");
  if (m < 0 || m > kMaxDegree) return bfail(PS_ERR_ARG, "degree m = %d out of range", m);
  const int esize = dt == PS_F64 ? 8 : 4;
  P.items.resize(batch);
  std::vector<double> cost(batch);
  size_t off = 0;
  for (int b = 0; b < batch; ++b) {
    const int64_t nb = n[b];
    if (nb < 1 || nb > 256) return bfail(PS_ERR_ARG, "n[%d] = %lld out of range [1, 256]", b, (long long)nb);
    int sb = s ? s[b] : 0;
    if (sb < 0 || sb > std::max(m, 1)) return bfail(PS_ERR_ARG, "s[%d] = %d out of range", b, sb);
    const int sg = sigma ? sigma[b] : 0;
    if (sg < 0 || sg > 500) return bfail(PS_ERR_ARG, "sigma[%d] = %d out of range", b, sg);
    BatchItem& it = P.items[b];
    memset(&it, 0, sizeof it);
    const int s0 = sb ? sb : s_floor(m), s1 = sb ? sb : s_ceil(m);
    if (m / s0 + 1 > PS_MAX_BLOCKS || m / s1 + 1 > PS_MAX_BLOCKS) return bfail(PS_ERR_ARG, "too many blocks");
    it.L[0] = make_layout(dt, nb, m, s0, 1, 0);
    it.L[1] = make_layout(dt, nb, m, s1, 1, 0);
    it.s_fixed = sb != 0;
    it.sigma = sg;
    it.ws_off = (int64_t)off;
    off += al256(std::max(it.L[0].bytes, it.L[1].bytes));
    if (need_ptrs) {
      if (!A || !E || !lda || !lde || !A[b] || !E[b]) return bfail(PS_ERR_ARG, "NULL pointer for matrix %d", b);
      if (lda[b] < nb || lde[b] < nb) return bfail(PS_ERR_ARG, "leading dimension < n for matrix %d", b);
      const size_t span = (size_t)((nb - 1) * std::max(lda[b], lde[b]) + nb) * esize;
      const char* pa = (const char*)A[b];
      const char* pe = (const char*)E[b];
      if (pa < pe + span && pe < pa + span) return bfail(PS_ERR_ALIAS, "output %d overlaps its input", b);
      it.A = A[b];
      it.lda = lda[b];
      it.E = E[b];
      it.lde = lde[b];
    }
    const int gem = (std::max(s0, s1) - 1) + (m / s0) + sg;
    cost[b] = (double)nb * nb * nb * gem;
  }
  P.order.resize(batch);
  std::iota(P.order.begin(), P.order.end(), 0);
  std::stable_sort(P.order.begin(), P.order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  P.off_mats = 0;
  P.off_items = al256(off);
  P.off_order = al256(P.off_items + sizeof(BatchItem) * (size_t)batch);
  P.off_chosen = al256(P.off_order + sizeof(int) * (size_t)batch);
  P.off_counter = al256(P.off_chosen + sizeof(int) * (size_t)batch);
  P.total = al256(P.off_counter + 256);
  return PS_OK;
}

ps_status fill_args(ps_dtype dt, const double* coef, int m, const ps_opts* opts, BatchArgs& ba) {
  memset(&ba, 0, sizeof ba);
  const int W = dt == PS_F64 ? 0 : 1;
  ba.mode = opts ? opts->mode : PS_MODE_FIXED;
  if (ba.mode != PS_MODE_FIXED && ba.mode != PS_MODE_MIXED) return bfail(PS_ERR_ARG, "opts.mode must be 0 or 1");
  if (opts && opts->tier_override) return bfail(PS_ERR_UNSUPPORTED, "tier_override is not supported for batches");
  unsigned mask = (opts && opts->tier_mask) ? opts->tier_mask : 0xFu;
  mask |= 1u << W;
  for (int t = 0; t < W; ++t) mask &= ~(1u << t);
  ba.mask = mask;
  ba.delta = (opts && opts->delta > 0) ? opts->delta : 10.0;
  if (coef) {
    for (int k = 0; k <= m; ++k) ba.cf.c[k] = coef[k];
  } else {
    if (m > 170) return bfail(PS_ERR_ARG, "built-in Taylor coefficients need m <= 170");
    ps_coef_taylor_exp(m, ba.cf.c);
  }
  if (W == 1)
    for (int k = 0; k <= m; ++k) ba.cf.c[k] = (double)(float)ba.cf.c[k];
  return PS_OK;
}

ps_status upload_and_args(const Plan2& P, char* ws, hipStream_t st, BatchArgs& ba) {
  hipError_t e = hipMemcpyAsync(ws + P.off_items, P.items.data(), sizeof(BatchItem) * P.items.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + P.off_order, P.order.data(), sizeof(int) * P.order.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host vectors are released on return
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "descriptor upload: %s", hipGetErrorString(e));
  ba.items = (const BatchItem*)(ws + P.off_items);
  ba.order = (const int*)(ws + P.off_order);
  ba.counter = (int*)(ws + P.off_counter);
  ba.chosen = (int*)(ws + P.off_chosen);
  ba.batch = (int)P.items.size();
  ba.ws = ws;
  return PS_OK;
}

ps_status launch_batch(int W, const BatchArgs& ba, hipStream_t st) {
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipError_t e;
  if (W == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ps_persistent<double>, NT, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_ps_persistent<float>, NT, 0);
  if (e != hipSuccess || per < 1) per = 1;
  const int grid = std::max(1, std::min(ba.batch, cus * per));
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, ba.counter);
  if (W == 0) hipLaunchKernelGGL(k_ps_persistent<double>, dim3(grid), dim3(NT), 0, st, ba);
  else hipLaunchKernelGGL(k_ps_persistent<float>, dim3(grid), dim3(NT), 0, st, ba);
  e = hipGetLastError();
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "persistent launch: %s", hipGetErrorString(e));
  return PS_OK;
}

}  // namespace

struct ps_batched_exec {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {



ps_status ps_workspace_size_batched(ps_dtype dtype, int batch, const int32_t* n, int m, const int32_t* s,
                                    size_t* bytes) {
  if (!bytes) return ps_set_error(bfail(PS_ERR_ARG, "bytes == NULL"), g_batch_err.c_str());
  Plan2 P;
  ps_status st = build_plan(dtype, batch, n, m, s, nullptr, nullptr, nullptr, nullptr, nullptr, P, false);
  if (st) return ps_set_error(st, g_batch_err.c_str());
  *bytes = P.total;
  return PS_OK;
}

static ps_status batched_common(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                                const double* coef, int m, const int32_t* s, const int32_t* sigma, void* const* E,
                                const int64_t* lde, const ps_opts* opts, void* ws, size_t ws_bytes, void* stream,
                                Plan2& P, BatchArgs& ba) {
  ps_status st = build_plan(dtype, batch, n, m, s, sigma, A, lda, E, lde, P, true);
  if (st) return st;
  if (ws_bytes < P.total) return bfail(PS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, P.total);
  if (!ws || ((uintptr_t)ws & 255)) return bfail(PS_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  for (int b = 0; b < batch; ++b) {
    const int64_t nb = n[b];
    const size_t span = (size_t)((nb - 1) * lde[b] + nb) * (dtype == PS_F64 ? 8 : 4);
    const char* pe = (const char*)E[b];
    const char* pw = (const char*)ws;
    if (pe < pw + P.total && pw < pe + span) return bfail(PS_ERR_ALIAS, "output %d overlaps the workspace", b);
  }
  if ((st = fill_args(dtype, coef, m, opts, ba))) return st;
  return upload_and_args(P, (char*)ws, (hipStream_t)stream, ba);
}

ps_status ps_expm_batched(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s, const int32_t* sigma, void* const* E,
                          const int64_t* lde, const ps_opts* opts, int32_t* tiers_out, void* ws, size_t ws_bytes,
                          void* stream) {
  Plan2 P;
  BatchArgs ba;
  hipStream_t st = (hipStream_t)stream;
  ps_status r = batched_common(dtype, batch, n, A, lda, coef, m, s, sigma, E, lde, opts, ws, ws_bytes, stream, P, ba);
  if (r) return ps_set_error(r, g_batch_err.c_str());
  if ((r = launch_batch(dtype == PS_F64 ? 0 : 1, ba, st))) return ps_set_error(r, g_batch_err.c_str());
  if (tiers_out) {
    std::vector<int> chosen(batch);
    hipError_t e = hipMemcpyAsync(chosen.data(), ba.chosen, sizeof(int) * batch, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int b = 0; b < batch && e == hipSuccess; ++b) {
      const BatchItem& it = P.items[b];
      const Layout& L = (chosen[b] == it.L[0].s) ? it.L[0] : it.L[1];
      Plan pl;
      e = hipMemcpy(&pl, (char*)ws + it.ws_off + L.off_plan, sizeof pl, hipMemcpyDeviceToHost);
      for (int i = 0; i < PS_MAX_BLOCKS; ++i) tiers_out[(size_t)b * PS_MAX_BLOCKS + i] = (i <= L.r) ? pl.tier[i] : -1;
      tiers_out[(size_t)b * PS_MAX_BLOCKS + PS_MAX_BLOCKS - 1] = L.s;   // last slot: chosen block size
    }
    if (e != hipSuccess) return ps_set_error(PS_ERR_HIP, hipGetErrorString(e));
  }
  return PS_OK;
}

ps_status ps_batched_prepare(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                             const double* coef, int m, const int32_t* s, const int32_t* sigma, void* const* E,
                             const int64_t* lde, const ps_opts* opts, void* ws, size_t ws_bytes, void* stream,
                             ps_batched_handle* out) {
  if (!out) return ps_set_error(PS_ERR_ARG, "out == NULL");
  *out = nullptr;
  Plan2 P;
  BatchArgs ba;
  ps_status r = batched_common(dtype, batch, n, A, lda, coef, m, s, sigma, E, lde, opts, ws, ws_bytes, stream, P, ba);
  if (r) return ps_set_error(r, g_batch_err.c_str());
  // capture on a private stream (the legacy null stream cannot be captured)
  hipStream_t cap;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return ps_set_error(PS_ERR_HIP, hipGetErrorString(e));
  ps_batched_exec* h = new ps_batched_exec();
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    r = launch_batch(dtype == PS_F64 ? 0 : 1, ba, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &h->graph);
    if (r == PS_OK && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess && r == PS_OK) e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess || r != PS_OK) {
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
    return ps_set_error(r ? r : PS_ERR_HIP, r ? g_batch_err.c_str() : hipGetErrorString(e));
  }
  *out = h;
  return PS_OK;
}

ps_status ps_batched_launch(ps_batched_handle h, void* stream) {
  if (!h || !h->exec) return ps_set_error(PS_ERR_ARG, "invalid handle");
  hipError_t e = hipGraphLaunch(h->exec, (hipStream_t)stream);
  if (e != hipSuccess) return ps_set_error(PS_ERR_HIP, hipGetErrorString(e));
  return PS_OK;
}

ps_status ps_batched_destroy(ps_batched_handle h) {
  if (!h) return ps_set_error(PS_ERR_ARG, "invalid handle");
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  delete h;
  return PS_OK;
}

}  // extern "C"
