// Many matrices of uneven order, evaluated together.
//
// The evaluation of every matrix goes through the same phases: choice of the
// block size, X = 2^-sigma A and the power table, the block assembly with
// norms, the precision plan (section 2, eq. (choose-ui); section 4.1.1
// tiers), the Horner chain in the planned tiers and the squarings
// (eq. (scal-idea)).  Each phase step is one launch over the whole batch: a
// task table built on the host at set-up lists (matrix, output tile) pairs,
// largest matrices first, and workgroup g takes task g.  The workgroups of a
// launch go to the eight XCDs in turn, so the table keeps all tiles of a
// matrix on one XCD (every eighth entry) and its operand panels in one L2.
// Matrices that have no work in a step (a smaller block size, fewer
// squarings) leave at once.
// Every matrix is first copied into a zero-padded square of order
// np = ceil(n / 64) 64 inside its workspace region, and all later phases work
// on order np: every tile and K slab is then whole, so the GEMM and Horner
// tiles take the unconditional vector-load path.  The padding stays exactly
// zero through every phase (the identity terms of the blocks are placed on
// the first n diagonal entries only), adding zeros does not change the
// sums, and only rows and columns < n reach the output: the results are the
// same as those of the unpadded single-matrix path.
// A batch is thus a fixed sequence of about s + r + sigma + 5 launches, which
// ps_batched_prepare captures into one hipGraph; the plan and the block-size
// choice are made on the device, so nothing returns to the host in between.
//
// Size classes and branches: a matrix's class is its padded order / 64.  A
// schedule assigns each class to a branch; every branch is a launch sequence
// of its own over its matrices' tasks, and the branches run concurrently
// (forked from the caller's stream by events and joined at the end), so the
// latency-bound phases of one class overlap the products of another.  The
// schedule changes only which launch processes a tile, never a tile's
// arithmetic, so every schedule gives the same bits.  ps_batched_tune times
// the candidate schedules (the groupings of the classes, in order of order,
// into up to four branches) on the caller's batch and keeps the fastest in a
// process-wide cache keyed by device architecture, dtype, degree and the
// batch's classes; ps_expm_batched and ps_batched_prepare use a cached
// schedule when one matches (otherwise one branch), and ps_autotune_save /
// ps_autotune_load keep the cache in a JSON file.  A schedule can also hand
// the class of orders up to 64 (one tile per matrix) to k_bwhole, which runs
// every phase of a matrix in one workgroup: one launch for the class, the
// same tile routines in the same order, the same bits.
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
#include <map>
#include <mutex>
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
  int64_t off_x1;       // byte offset (in the region) of the zero-padded copy of A
  int64_t nv;           // order n of the matrix; the layouts are for the padded order
  int sigma;
  int s_fixed;          // 0: choose between L[0] (floor sqrt m) and L[1] (ceil sqrt m)
  Layout L[2];
};

// per-matrix descriptor resolved on the device once the block size is chosen
struct BatchRes {
  char* ws;             // the matrix's workspace region
  const void* X1;       // zero-padded copy of A, order L.n, leading dimension L.n
  void* E;
  int64_t lde;
  int64_t nv;           // order of the matrix (<= L.n)
  int sigma;
  Layout L;             // the chosen layout (padded order)
};

struct BatchArgs {
  const BatchItem* items;
  BatchRes* res;
  const int* tile_tasks;  // (matrix << 8) | tile in XCD lanes, largest matrices first, -1: none (this branch's)
  const int* mat_tasks;   // matrices of this branch (per-matrix kernels)
  int* pick;              // per matrix: 0 -> L[0], 1 -> L[1]
  int* chosen;            // per matrix: chosen block size (for reports)
  int batch;
  int mode;
  int rule;
  unsigned mask;
  double delta;
  char* ws;
  Coefs cf;
};

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

__device__ inline int tiles_m(int64_t n) { return (int)((n + kTileM - 1) / kTileM); }


// ---- block size: ||X||_1 = 2^-sigma ||A||_1, then the cheaper of the two layouts
// (whole workgroup; red: NW + 1 doubles of LDS).  Returns the pick (0: L[0],
// 1: L[1]) to every thread; thread 0 also records it and the matrix's
// resolved descriptor.
template <typename W>
__device__ __forceinline__ int bchoose_body(const BatchArgs& a, int b, double* red) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  const BatchItem& it = a.items[b];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  int pick = 1;
  if (!it.s_fixed && it.L[0].s != it.L[1].s) {
    const W* A = (const W*)it.A;
    const int64_t n = it.nv, lda = it.lda;
    // column sums, four columns of four row blocks per step: the sixteen
    // loads of a step are unconditional (clamped indices) and in flight together
    double mx = 0.0;
    for (int64_t c0 = 4 * w; c0 < n; c0 += 4 * NW) {
      double v[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int64_t c = c0 + cc;
        v[cc] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {   // n <= 256 = 4 x 64 rows
          const int64_t rw = lane + 64 * q;
          const bool in = rw < n && c < n;
          const double x = fabs((double)A[(in ? rw : 0) + (in ? c : 0) * lda]);
          v[cc] += in ? x : 0.0;
        }
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        double u = v[cc];
        for (int off = 32; off >= 1; off >>= 1) u += __shfl_xor(u, off, 64);
        if (c0 + cc < n && (u > mx || u != u)) mx = u;
      }
    }
    if (lane == 0) red[w] = mx;
    __syncthreads();
    if (t == 0) {
      double x = red[0];
      for (int k = 1; k < NW; ++k) if (red[k] > x || red[k] != red[k]) x = red[k];
      x *= ldexp(1.0, -it.sigma);
      const double c0 = apriori_cost(it.L[0], a.cf, x, WT, a.mask, a.delta);
      const double c1 = apriori_cost(it.L[1], a.cf, x, WT, a.mask, a.delta);
      red[NW] = (c0 < c1) ? 0.0 : 1.0;
    }
    __syncthreads();
    pick = red[NW] != 0.0 ? 1 : 0;
  }
  if (t == 0) {
    a.pick[b] = pick;
    if (a.chosen) a.chosen[b] = it.L[pick].s;
    BatchRes& r = a.res[b];
    r.ws = a.ws + it.ws_off;
    r.X1 = a.ws + it.ws_off + it.off_x1;
    r.E = it.E;
    r.lde = it.lde;
    r.nv = it.nv;
    r.sigma = it.sigma;
    r.L = it.L[pick];
  }
  return pick;
}

template <typename W>
__global__ __launch_bounds__(NT) void k_bchoose(BatchArgs a) {
  __shared__ double red[NW + 1];
  (void)bchoose_body<W>(a, a.mat_tasks[blockIdx.x], red);
}

// ---- zero-padded copy of A: one 64 x kTileN tile of the padded square per workgroup
template <typename W>
__device__ __forceinline__ void bpad_tile(const BatchArgs& a, int b, int tile) {
  const BatchItem& it = a.items[b];
  const int64_t np = it.L[0].n, n = it.nv;
  const int ntm = tiles_m(np);
  const int64_t m0 = (int64_t)(tile % ntm) * kTileM, n0 = (int64_t)(tile / ntm) * kTileN;
  const W* A = (const W*)it.A;
  W* X = (W*)(a.ws + it.ws_off + it.off_x1);
  const int t = threadIdx.x, row = t & 63;
  W v[TILE_Q];
#pragma unroll
  for (int q = 0; q < TILE_Q; ++q) {
    const int64_t gr = m0 + row, gc = n0 + (t >> 6) + NW * q;
    const bool in = gr < n && gc < n;
    const W x = A[(in ? gr : 0) + (in ? gc : 0) * it.lda];
    v[q] = in ? x : W(0);
  }
#pragma unroll
  for (int q = 0; q < TILE_Q; ++q) X[m0 + row + (n0 + (t >> 6) + NW * q) * np] = v[q];
}

template <typename W>
__global__ __launch_bounds__(NT) void k_bpad(BatchArgs a) {
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  bpad_tile<W>(a, task >> 8, task & 255);
}

// Sums over the 64 lanes of a wave of eight values per lane: three exchange
// steps that each keep half of the values (lane bits 5, 4, 3 pick the half),
// then a butterfly over lane bits 2..0.  On return lane L holds the total of
// v[L >> 3].  10 shuffles instead of 48 for eight separate butterflies.
__device__ __forceinline__ double wave_sum8(const double v[8]) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double a4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double send = b5 ? v[k] : v[4 + k];
    a4[k] = (b5 ? v[4 + k] : v[k]) + __shfl_xor(send, 32, 64);   // column 4 b5 + k
  }
  double a2[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = b4 ? a4[k] : a4[2 + k];
    a2[k] = (b4 ? a4[2 + k] : a4[k]) + __shfl_xor(send, 16, 64);   // column 4 b5 + 2 b4 + k
  }
  const double send = b3 ? a2[0] : a2[1];
  double c = (b3 ? a2[1] : a2[0]) + __shfl_xor(send, 8, 64);       // column 4 b5 + 2 b4 + b3
  c += __shfl_xor(c, 4, 64);
  c += __shfl_xor(c, 2, 64);
  c += __shfl_xor(c, 1, 64);
  return c;
}

// ---- block assembly of one 64 x 64 tile of the padded order, in the epilogue
// of the launch that forms Y = X_s (or, for s = 1, on its own): Y into its
// power slot, B_0..B_r (the same terms in the same order as the column pass
// of the single-matrix path: c_{si} I, then c_{si+j} X_j for increasing j, the
// trivial last step folded into B_{r-1}), the low-precision copies of Y, and
// the 64-row partial column abs sums of B_i, Y and X_1 that the plan reads
// (the layout's colsum_rows = 64 = the tile height).  Each wave holds 64
// rows of one column per element q, as in the column pass, so the E8M0
// blocks of 32 rows are half-waves.  ycs: the product tile in LDS (Y =
// alpha ycs), or nullptr when s = 1 (Y = X_1, read from memory).
constexpr int kAsmGather = 5;   // FP32: the powers X_1..X_{s-1} of a tile gathered at once for s <= this

// X_1..X_{s-1} of the thread's elements of a tile (zero outside the order nv
// and for j >= s), all loads in flight together
template <typename W>
__device__ __forceinline__ void gather_powers(const BatchRes& it, int64_t m0, int64_t n0,
                                              W x[kAsmGather - 1][TILE_Q]) {
  const Layout& L = it.L;
  const int64_t n = L.n, nv = it.nv, se = (int64_t)(L.slot / sizeof(W));
  const W* pw = (const W*)(it.ws + L.off_pow);
  const W* X1 = (const W*)it.X1;
  const double x1s = ldexp(1.0, -it.sigma);
  const int t = threadIdx.x;
  const int64_t gr = m0 + (t & 63);
#pragma unroll
  for (int jj = 0; jj < kAsmGather - 1; ++jj)
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const int64_t gc = n0 + (t >> 6) + NW * q;
      const bool in = jj + 1 < L.s && gr < nv && gc < nv;
      const int64_t rr = in ? gr : 0, cc = in ? gc : 0;
      const W v = (jj == 0) ? (W)(x1s * (double)X1[rr + cc * n]) : pw[(int64_t)(jj - 1) * se + rr + cc * n];
      x[jj][q] = in ? v : W(0);
    }
}

// HAVE_X: x already holds gather_powers' values (FP32, s <= kAsmGather)
template <typename W, bool HAVE_X>
__device__ __forceinline__ void assemble_tile(const BatchArgs& a, const BatchRes& it, const W* ycs, double alpha,
                                              int64_t m0, int64_t n0, W (&x)[kAsmGather - 1][TILE_Q]) {
  const Layout& L = it.L;
  const int64_t n = L.n, nv = it.nv;
  const int s = L.s, r = L.r, m = L.m, nB = L.nB;
  const int64_t se = (int64_t)(L.slot / sizeof(W));
  char* ws = it.ws;
  W* pw = (W*)(ws + L.off_pow);
  W* Bm = (W*)(ws + L.off_B);
  double* colsum = (double*)(ws + L.off_colsum);
  const int64_t nch = (n + L.colsum_rows - 1) / L.colsum_rows, chunk = m0 / L.colsum_rows;
  const double x1s = ldexp(1.0, -it.sigma);
  const W* X1 = (const W*)it.X1;
  const unsigned mask = a.mode == PS_MODE_MIXED ? a.mask : 0u;
  const bool want32 = std::is_same<W, double>::value && ((mask >> 1) & 1u);
  const bool want16 = (mask >> 2) & 1u, want8 = (mask >> 3) & 1u;
  const int64_t Kp = L.Kp, Ks = Kp / 32;
  float* yf32 = (float*)(ws + L.off_yf32);
  uint16_t* ybf = (uint16_t*)(ws + L.off_ybf16);
  uint8_t* y8 = (uint8_t*)(ws + L.off_yfp8);
  uint8_t* y8s = (uint8_t*)(ws + L.off_yfp8s);
  const int t = threadIdx.x, lane = t & 63;
  const int64_t gr = m0 + lane;
  if (m0 == 0 && n0 == 0 && t < 64) {   // |c_k| for the a-priori planning rule
    Plan* P = (Plan*)(ws + L.off_plan);
    for (int k = lane; k <= m; k += 64) P->abs_coef[k] = fabs(a.cf.c[k]);
  }
  // the thread's TILE_Q elements: row gr, columns n0 + (t >> 6) + NW q
  auto col_q = [&](int q) { return n0 + (t >> 6) + NW * q; };
  auto inner_q = [&](int q) { return gr < nv && col_q(q) < nv; };
  // X_j (j < s) of these elements, zero outside the matrix's order
  auto load_x = [&](int j, W xv[TILE_Q]) {
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const bool in = inner_q(q);
      const int64_t gc = in ? col_q(q) : 0, rr = in ? gr : 0;
      const W v = (j == 1) ? (W)(x1s * (double)X1[rr + gc * n]) : pw[(int64_t)(j - 2) * se + rr + gc * n];
      xv[q] = in ? v : W(0);
    }
  };
  // column abs sums over this tile's 64 rows (lane = row): lane 8c holds the
  // sum of column c of the wave's eight
  auto put_sums = [&](int qty, double v[TILE_Q]) {
    const double tot = wave_sum8(v);
    if ((lane & 7) == 0) colsum[((int64_t)qty * nch + chunk) * n + col_q(lane >> 3)] = tot;
  };
  // Y, its copies and column sums
  W y[TILE_Q];
  if (ycs) {
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const W v = (W)(alpha * (double)ycs[((t >> 6) + NW * q) * CSTR + lane]);
      y[q] = inner_q(q) ? v : W(0);
      pw[(int64_t)(s - 2) * se + gr + col_q(q) * n] = y[q];
    }
  } else {
    load_x(1, y);
  }
  {
    double sv[TILE_Q];
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const int64_t gc = col_q(q);
      sv[q] = fabs((double)y[q]);
      if (want32) yf32[gr + gc * n] = (float)y[q];
      if (want16) ybf[gc * Kp + gr] = bf16_bits_rne((float)y[q]);
      if (want8) {
        float av = fabsf((float)y[q]);
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) av = fmaxf(av, __shfl_xor(av, off, 64));
        const int sbyte = e8m0_for(av);
        float qv = ldexpf((float)y[q], -(sbyte - 127));
        qv = fminf(fmaxf(qv, -448.0f), 448.0f);
        const int wv = __builtin_amdgcn_cvt_pk_fp8_f32(qv, 0.0f, 0, false);
        y8[gc * Kp + gr] = (uint8_t)(wv & 0xff);
        if ((gr & 31) == 0) y8s[gc * Ks + gr / 32] = (uint8_t)sbyte;
      }
    }
    if (s == 1) {   // X_1 is Y
      double sx[TILE_Q];
#pragma unroll
      for (int q = 0; q < TILE_Q; ++q) sx[q] = sv[q];
      put_sums(nB + 1, sx);
    }
    put_sums(nB, sv);
  }
  // block i: c_{si} I, then c_{si+j} X_j for increasing j; stored with the
  // trivial last step folded in, its column sums from the unfolded values
  auto finish_block = [&](int i, const W bv[TILE_Q]) {
    double v[TILE_Q];
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      v[q] = fabs((double)bv[q]);
      W outv = bv[q];
      if (L.trivial_last && i == r - 1) outv += (W)a.cf.c[m] * y[q];   // step r: c_m I * Y
      if (inner_q(q)) Bm[(int64_t)i * se + gr + col_q(q) * n] = outv;
    }
    put_sums(i, v);
  };
  auto init_block = [&](int i, W bv[TILE_Q]) {
    const W c0 = (i < nB && s * i <= m) ? (W)a.cf.c[s * i] : W(0);
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) bv[q] = (gr == col_q(q) && gr < nv) ? c0 : W(0);
  };
  // FP32: every power X_1..X_{s-1} of the elements loaded at once (s <= PG),
  // before the GEMM main loop when the caller passes them in xpre
  constexpr int PG = std::is_same<W, float>::value ? kAsmGather : 1;
  if (PG > 1 && s <= PG) {
    if (!HAVE_X) gather_powers<W>(it, m0, n0, x);
    if (s > 1) {
      double sx[TILE_Q];
#pragma unroll
      for (int q = 0; q < TILE_Q; ++q) sx[q] = fabs((double)x[0][q]);
      put_sums(nB + 1, sx);
    }
    for (int i = 0; i < nB; ++i) {
      W bv[TILE_Q];
      init_block(i, bv);
#pragma unroll
      for (int jj = 0; jj < PG - 1; ++jj) {
        const int k = s * i + jj + 1;
        if (jj + 1 < s && k <= m) {
          const W ck = (W)a.cf.c[k];
#pragma unroll
          for (int q = 0; q < TILE_Q; ++q) bv[q] += ck * x[jj][q];
        }
      }
      finish_block(i, bv);
    }
    return;
  }
  // otherwise blocks in chunks of BC, the powers read once per chunk
  constexpr int BC = sizeof(W) == 8 ? 1 : 2;
  for (int i0 = 0; i0 < nB; i0 += BC) {
    W bv[BC][TILE_Q];
#pragma unroll
    for (int ii = 0; ii < BC; ++ii) init_block(i0 + ii, bv[ii]);
    for (int j = 1; j < s; ++j) {
      W xj[TILE_Q];
      load_x(j, xj);
      if (j == 1 && i0 == 0) {
        double sx[TILE_Q];
#pragma unroll
        for (int q = 0; q < TILE_Q; ++q) sx[q] = fabs((double)xj[q]);
        put_sums(nB + 1, sx);
      }
#pragma unroll
      for (int ii = 0; ii < BC; ++ii) {
        const int k = s * (i0 + ii) + j;
        if (i0 + ii < nB && k <= m) {
          const W ck = (W)a.cf.c[k];
#pragma unroll
          for (int q = 0; q < TILE_Q; ++q) bv[ii][q] += ck * xj[q];
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < BC; ++ii)
      if (i0 + ii < nB) finish_block(i0 + ii, bv[ii]);
  }
}

// ---- power table step j: X_j = X_a X_b (a = ceil(j/2), b = floor(j/2), X_1 = beta A).
// ASM = false: the tiles of matrices with j < s; ASM = true: those with j = s
// (Y), whose block assembly follows in the same workgroup.  Two kernels, so
// that the plain products keep the register count (and occupancy) of a GEMM.
template <typename W, bool ASM>
__device__ __forceinline__ void bpower_tile(const BatchArgs& a, const BatchRes& it, int tile, int j, char* smem) {
  const Layout& L = it.L;
  if (ASM ? (j != L.s) : (j >= L.s)) return;   // uniform: the whole workgroup leaves
  const int64_t n = L.n;
  const int ntm = tiles_m(n);
  const W* X1 = (const W*)it.X1;
  const double beta = ldexp(1.0, -it.sigma);
  const int64_t se = (int64_t)(L.slot / sizeof(W));
  W* pw = (W*)(it.ws + L.off_pow);
  // X_j = X_a X_b, a = ceil(j/2), b = floor(j/2): the same products as the
  // single-matrix path
  const int pa = (j + 1) / 2, pb = j / 2;
  const W* xa = (pa == 1) ? X1 : pw + (int64_t)(pa - 2) * se;
  const W* xb = (pb == 1) ? X1 : pw + (int64_t)(pb - 2) * se;
  const double alpha = (pa == 1 ? beta : 1.0) * (pb == 1 ? beta : 1.0);
  const int64_t m0 = (int64_t)(tile % ntm) * kTileM, n0 = (int64_t)(tile / ntm) * kTileN;
  if (!ASM) {
    gemm_tile<W, false, false>(xa, n, xb, n, pw + (int64_t)(j - 2) * se, n, n, n, m0, n0, alpha, 0, smem);
    return;
  }
  typename MF<W>::V acc[2];
  mainloop_lds<W, false, false>(xa, n, xb, n, n, m0, n0, smem, acc);
  W* Cs = (W*)smem;
  frag_to_cs<W, W>(acc, Cs, 1.0);
  __syncthreads();
  // the assembly's power loads are issued after the main loop: loaded before
  // it, they held enough registers to halve the GEMM's occupancy (slower)
  W x[kAsmGather - 1][TILE_Q];
  assemble_tile<W, false>(a, it, Cs, alpha, m0, n0, x);
}

template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bpower(BatchArgs a, int j) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  bpower_tile<W, false>(a, a.res[task >> 8], task & 255, j, smem);
}

template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bpower_asm(BatchArgs a, int j) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  bpower_tile<W, true>(a, a.res[task >> 8], task & 255, j, smem);
}

// ---- block assembly of the matrices with s = 1 (no power products: Y = X_1)
template <typename W>
__device__ __forceinline__ void bassemble1_tile(const BatchArgs& a, const BatchRes& it, int tile) {
  const int ntm = tiles_m(it.L.n);
  W x[kAsmGather - 1][TILE_Q];
  assemble_tile<W, false>(a, it, (const W*)nullptr, 1.0, (int64_t)(tile % ntm) * kTileM,
                          (int64_t)(tile / ntm) * kTileN, x);
}

template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bassemble1(BatchArgs a) {
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  const BatchRes& it = a.res[task >> 8];
  if (it.L.s != 1) return;   // uniform
  bassemble1_tile<W>(a, it, task & 255);
}

// ---- precision plan: one workgroup per matrix
// red: 8 NW doubles, norms: PS_MAX_BLOCKS + 2 doubles of LDS; ends with a barrier
template <typename W>
__device__ __forceinline__ void bplan_body(const BatchArgs& a, const BatchRes& it, double* red, double* norms) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  const Layout& L = it.L;
  PlanArgs pa;
  pa.r = L.r;
  pa.mode = a.mode;
  pa.working = WT;
  pa.nB = L.nB;
  pa.trivial_last = L.trivial_last;
  pa.mask = a.mask;
  pa.delta = a.delta;
  pa.abs_cm = fabs(a.cf.c[L.m]);
  pa.rule = a.rule;
  pa.use_override = 0;
  pa.ws = it.ws;
  pa.ws_stride = 0;
  pa.L = L;
  plan_matrix<NT>(pa, L, pa.ws, red, norms);
}

template <typename W>
__global__ __launch_bounds__(NT) void k_bplan(BatchArgs a) {
  __shared__ double red[8 * NW];
  __shared__ double norms[PS_MAX_BLOCKS + 2];
  bplan_body<W>(a, a.res[a.mat_tasks[blockIdx.x]], red, norms);
}

// ---- Horner step k: k = -1 casts B_{i0} into the format of step i0; k >= 0
// is step i = i0 - k.  The cast writes P0; step k reads P0 (k even) or P1
// (k odd) and writes the other buffer.
// tier_in, tier_out: the plan's tiers of step i and of the next step
// (ignored where the cast or the final output fixes them)
template <typename W>
__device__ __forceinline__ void bhorner_tile(const BatchArgs& a, const BatchRes& it, int tile, int k, int tier_in,
                                             int tier_out, char* smem) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  const Layout& L = it.L;
  const int i0 = L.first_step;
  const int64_t n = L.n;
  const int ntm = tiles_m(n);
  char* ws = it.ws;
  const int64_t se = (int64_t)(L.slot / sizeof(W));
  const W* pw = (const W*)(ws + L.off_pow);
  const bool square = it.sigma > 0;
  HornerTile<W> h;
  h.n = n;
  h.Mp = L.Mp;
  h.Kp = L.Kp;
  if (L.s == 1) {
    h.ysrc = (const W*)it.X1;
    h.ldy = n;
    h.yscale = ldexp(1.0, -it.sigma);
  } else {
    h.ysrc = pw + (int64_t)(L.s - 2) * se;
    h.ldy = n;
    h.yscale = 1.0;
  }
  h.yf32 = (const float*)(ws + L.off_yf32);
  h.ybf16 = (const uint16_t*)(ws + L.off_ybf16);
  h.yfp8 = (const uint8_t*)(ws + L.off_yfp8);
  h.yfp8s = (const uint8_t*)(ws + L.off_yfp8s);
  const int i = i0 - k;
  const bool cast = (k < 0);
  h.fy64 = nullptr;
  h.fy32 = nullptr;
  h.fyc = 0.0;
  const bool final_out = cast ? (i0 == 0) : (i == 1);
  h.t_in = cast ? -1 : tier_in;
  h.t_out = final_out ? WT : tier_out;
  h.pin = ws + ((k & 1) ? L.off_P1 : L.off_P0);
  h.pout = cast ? ws + L.off_P0 : ws + ((k & 1) ? L.off_P0 : L.off_P1);
  h.bsrc = (const W*)(ws + L.off_B) + (int64_t)(cast ? i0 : i - 1) * se;
  h.outw = final_out ? (square ? (W*)(ws + L.off_R) : (W*)it.E) : (W*)h.pout;
  h.ldo = final_out ? (square ? n : it.lde) : n;
  h.nv = (final_out && !square) ? it.nv : n;
  h.nvb = it.nv;
  horner_tile<W, false>(h, (int64_t)(tile % ntm) * kTileM, (int64_t)(tile / ntm) * kTileN, smem);
}

template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bhorner(BatchArgs a, int k) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  const BatchRes& it = a.res[task >> 8];
  const int i0 = it.L.first_step;
  if (k >= i0) return;   // uniform
  const Plan* P = (const Plan*)(it.ws + it.L.off_plan);
  const int i = i0 - k;
  bhorner_tile<W>(a, it, task & 255, k, k < 0 ? -1 : P->tier[i], P->tier[k < 0 ? i0 : i - 1], smem);
}

// ---- squaring q (1..sigma): R_q = R_{q-1}^2, R_0 in L.off_R, ping-pong with P0
template <typename W>
__device__ __forceinline__ void bsquare_tile(const BatchRes& it, int tile, int q, char* smem) {
  const Layout& L = it.L;
  const int64_t n = L.n;
  const int ntm = tiles_m(n);
  char* ws = it.ws;
  W* const r0 = (W*)(ws + L.off_R);
  W* const r1 = (W*)(ws + L.off_P0);
  const W* src = (q & 1) ? r0 : r1;
  W* dst = (q == it.sigma) ? (W*)it.E : ((q & 1) ? r1 : r0);
  const int64_t ldd = (q == it.sigma) ? it.lde : n;
  gemm_tile<W, false, false>(src, n, src, n, dst, ldd, n, (q == it.sigma) ? it.nv : n, (int64_t)(tile % ntm) * kTileM,
                             (int64_t)(tile / ntm) * kTileN, 1.0, 0, smem);
}

template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bsquare(BatchArgs a, int q) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  const int task = a.tile_tasks[blockIdx.x];
  if (task < 0) return;   // a hole of the XCD-lane layout
  const BatchRes& it = a.res[task >> 8];
  if (q > it.sigma) return;   // uniform
  bsquare_tile<W>(it, task & 255, q, smem);
}

// a tier of the plan this workgroup has just written: a vector load (never
// the scalar cache, which the workgroup's own stores do not update)
__device__ inline int plan_tier(const Plan* P, int i) {
  return __hip_atomic_load(&P->tier[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---- the whole evaluation of a matrix of padded order 64 (a single tile) in
// one workgroup: the phases above, in their order, on the same tile, each one
// finished (its stores complete, then a barrier) before the next reads what it
// wrote.  The arithmetic is that of the per-phase launches, so are the bits;
// a size class of such matrices takes one launch instead of s + r + sigma + 5.
template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bwhole(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  __shared__ double red[8 * NW];
  __shared__ double norms[PS_MAX_BLOCKS + 2];
  // the matrix's resolved descriptor in LDS: read where each phase needs it,
  // not held in registers across the phases
  __shared__ BatchRes s_it;
  const int b = a.mat_tasks[blockIdx.x];
  const int pick = bchoose_body<W>(a, b, red);
  if (threadIdx.x == 0) {
    const BatchItem& item = a.items[b];
    s_it.ws = a.ws + item.ws_off;
    s_it.X1 = a.ws + item.ws_off + item.off_x1;
    s_it.E = item.E;
    s_it.lde = item.lde;
    s_it.nv = item.nv;
    s_it.sigma = item.sigma;
    s_it.L = item.L[pick];
  }
  bpad_tile<W>(a, b, 0);
  __syncthreads();
  const BatchRes& it = s_it;
  const int s = it.L.s;
  for (int j = 2; j < s; ++j) bpower_tile<W, false>(a, it, 0, j, smem);
  if (s >= 2) bpower_tile<W, true>(a, it, 0, s, smem);
  else bassemble1_tile<W>(a, it, 0);
  __syncthreads();
  bplan_body<W>(a, it, red, norms);
  const Plan* P = (const Plan*)(it.ws + it.L.off_plan);
  const int i0 = it.L.first_step;
  for (int k = -1; k < i0; ++k) {
    const int i = i0 - k;
    bhorner_tile<W>(a, it, 0, k, k < 0 ? -1 : plan_tier(P, i), plan_tier(P, k < 0 ? i0 : i - 1), smem);
  }
  for (int q = 1; q <= it.sigma; ++q) bsquare_tile<W>(it, 0, q, smem);
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

constexpr int kMaxClass = 4;     // padded orders 64, 128, 192, 256
constexpr int kMaxBranch = 4;
constexpr int kMaxCand = 16;     // schedules the tuner can time: 8 groupings, 4 with k_bwhole
constexpr int kXcd = 8;          // XCDs, to which a launch's workgroups go in turn

// one branch of a batch: its matrices, their tiles and the bounds of its
// launch loops
struct Branch {
  std::vector<int> mats, tiles;   // matrices (and their tiles) that take the per-phase launches
  std::vector<int> whole;         // matrices evaluated by k_bwhole, one workgroup each
  int smax = 1, kmax = 0, sigmax = 0;
  std::vector<char> s_possible;   // s_possible[s]: some matrix of the branch may take block size s
  size_t off_mats = 0, off_tiles = 0, off_whole = 0;
  bool empty() const { return mats.empty() && whole.empty(); }
};

struct Plan2 {
  std::vector<BatchItem> items;
  std::vector<Branch> br;
  int cls_count[kMaxClass + 1] = {0, 0, 0, 0, 0};   // matrices per class (index = padded order / 64)
  size_t off_items, off_res, off_pick, off_chosen, total;
};

// schedule: group[c - 1] = branch of class c (c = 1..kMaxClass); whole64 = 1:
// the matrices of class 1 (padded order 64, one tile) are evaluated by
// k_bwhole, one workgroup per matrix, instead of the per-phase launches
struct Schedule {
  int group[kMaxClass] = {0, 0, 0, 0};
  int whole64 = 0;
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
                     bool need_ptrs, const Schedule& sch) {
  if (dt != PS_F64 && dt != PS_F32) return bfail(PS_ERR_ARG, "dtype must be PS_F64 or PS_F32");
  if (batch < 1 || batch > (1 << 22)) return bfail(PS_ERR_ARG, "batch = %d out of range", batch);
  if (!n) return bfail(PS_ERR_ARG, "n == NULL");
  if (m < 0 || m > kMaxDegree) return bfail(PS_ERR_ARG, "degree m = %d out of range", m);
  const int esize = dt == PS_F64 ? 8 : 4;
  P.items.resize(batch);
  int nbr = 1;
  for (int c = 0; c < kMaxClass; ++c) nbr = std::max(nbr, sch.group[c] + 1);
  P.br.assign(nbr, Branch());
  for (Branch& B : P.br) B.s_possible.assign(2, 0);
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
    const int64_t np = (nb + kTileM - 1) / kTileM * kTileM;   // padded order
    it.L[0] = make_layout(dt, np, m, s0, 1, 0, 0, kTileM);   // partial column sums per 64-row tile
    it.L[1] = make_layout(dt, np, m, s1, 1, 0, 0, kTileM);
    it.s_fixed = sb != 0;
    it.sigma = sg;
    it.nv = nb;
    it.ws_off = (int64_t)off;
    it.off_x1 = (int64_t)al256(std::max(it.L[0].bytes, it.L[1].bytes));
    off += it.off_x1 + al256((size_t)(np * np) * esize);
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
    const int cls = (int)(np / kTileM);
    P.cls_count[cls] += 1;
    Branch& B = P.br[sch.group[cls - 1]];
    if (cls == 1 && sch.whole64) {   // one workgroup does every phase: no launch bounds to widen
      B.whole.push_back(b);
      continue;
    }
    B.mats.push_back(b);
    B.smax = std::max(B.smax, std::max(s0, s1));
    if ((int)B.s_possible.size() <= std::max(s0, s1)) B.s_possible.resize(std::max(s0, s1) + 1, 0);
    B.s_possible[s0] = B.s_possible[s1] = 1;
    B.kmax = std::max(B.kmax, std::max(it.L[0].first_step, it.L[1].first_step));
    B.sigmax = std::max(B.sigmax, sg);
  }
  // per branch: matrices and their tiles, largest matrices first so the long
  // tiles start early
  P.off_items = al256(off);
  P.off_res = al256(P.off_items + sizeof(BatchItem) * (size_t)batch);
  const size_t tasks0 = al256(P.off_res + sizeof(BatchRes) * (size_t)batch);
  size_t o = tasks0;
  for (Branch& B : P.br) {
    std::stable_sort(B.mats.begin(), B.mats.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::stable_sort(B.whole.begin(), B.whole.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    // XCD lanes: workgroup g runs on XCD g mod kXcd, so the tiles of one
    // matrix go to one lane (task positions l, l + kXcd, l + 2 kXcd, ...)
    // and share that XCD's L2 for their operand panels; each matrix joins
    // the lane with the fewest tiles so far, and the shorter lanes end in
    // holes (task -1)
    std::vector<std::vector<int>> lane(kXcd);
    std::vector<size_t> load(kXcd, 0);
    for (int b : B.mats) {
      const int64_t nb = n[b];
      const int nt = (int)(((nb + kTileM - 1) / kTileM) * ((nb + kTileN - 1) / kTileN));   // tiles of the padded square
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (int t = 0; t < nt; ++t) lane[l].push_back((b << 8) | t);
      load[l] += (size_t)nt;
    }
    const size_t len = *std::max_element(load.begin(), load.end());
    B.tiles.assign(len * kXcd, -1);
    for (int l = 0; l < kXcd; ++l)
      for (size_t k = 0; k < lane[l].size(); ++k) B.tiles[k * kXcd + l] = lane[l][k];
    B.off_mats = o;
    o = al256(o + sizeof(int) * B.mats.size());
    B.off_tiles = o;
    o = al256(o + sizeof(int) * B.tiles.size());
    B.off_whole = o;
    o = al256(o + sizeof(int) * B.whole.size());
  }
  // the task arrays get a region sized for any schedule (every branch's three
  // arrays 256-byte rounded; a matrix is in one list of one branch and its
  // tiles are listed at most once; a branch's lanes differ in length by at
  // most one matrix's 16 tiles, so its holes number fewer than 16 kXcd), so
  // one workspace size covers all schedules
  size_t ntiles_all = 0;
  for (int b = 0; b < batch; ++b) ntiles_all += (size_t)(((n[b] + kTileM - 1) / kTileM) * ((n[b] + kTileN - 1) / kTileN));
  P.off_pick = al256(tasks0 + sizeof(int) * ((size_t)batch + ntiles_all + (size_t)(16 * kXcd * kMaxBranch)) +
                     (size_t)(3 * 256 * kMaxBranch));
  if (o > P.off_pick) return bfail(PS_ERR_UNSUPPORTED, "task arrays exceed their region");
  P.off_chosen = al256(P.off_pick + sizeof(int) * (size_t)batch);
  P.total = al256(P.off_chosen + sizeof(int) * (size_t)batch);
  return PS_OK;
}

// ---- the schedule cache (process-wide) ----
std::mutex g_cache_mu;
std::map<std::string, Schedule> g_cache;

// key of a batch: device architecture, dtype, degree and, per class, the
// order of magnitude of its matrix count (0 = absent, k = [2^(k-1), 2^k))
std::string schedule_key(ps_dtype dt, int m, const int cls_count[kMaxClass + 1]) {
  std::string arch = "unknown";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  char buf[160];
  int mag[kMaxClass];
  for (int c = 1; c <= kMaxClass; ++c) {
    int k = 0;
    while (k < 30 && (cls_count[c] >> k) > 0) ++k;
    mag[c - 1] = k;
  }
  snprintf(buf, sizeof buf, "%s|%s|m%d|%d,%d,%d,%d", arch.c_str(), dt == PS_F64 ? "f64" : "f32", m, mag[0], mag[1],
           mag[2], mag[3]);
  return buf;
}

void count_classes(int batch, const int32_t* n, int cls_count[kMaxClass + 1]) {
  for (int c = 0; c <= kMaxClass; ++c) cls_count[c] = 0;
  for (int b = 0; b < batch; ++b)
    if (n[b] >= 1 && n[b] <= 256) cls_count[(n[b] + kTileM - 1) / kTileM] += 1;
}

Schedule cached_schedule(ps_dtype dt, int m, int batch, const int32_t* n) {
  int cc[kMaxClass + 1];
  count_classes(batch, n, cc);
  const std::string key = schedule_key(dt, m, cc);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto it = g_cache.find(key);
  return it == g_cache.end() ? Schedule() : it->second;
}

ps_status fill_args(ps_dtype dt, const double* coef, int m, const ps_opts* opts, BatchArgs& ba) {
  memset(&ba, 0, sizeof ba);
  const int W = dt == PS_F64 ? 0 : 1;
  ba.mode = opts ? opts->mode : PS_MODE_FIXED;
  if (ba.mode != PS_MODE_FIXED && ba.mode != PS_MODE_MIXED) return bfail(PS_ERR_ARG, "opts.mode must be 0 or 1");
  if (opts && opts->tier_override) return bfail(PS_ERR_UNSUPPORTED, "tier_override is not supported for batches");
  if (opts && opts->check_finite) return bfail(PS_ERR_UNSUPPORTED, "check_finite is not supported for batches");
  ba.rule = opts ? opts->rule : PS_RULE_BLOCKS;
  if (ba.rule != PS_RULE_BLOCKS && ba.rule != PS_RULE_APRIORI) return bfail(PS_ERR_ARG, "opts.rule must be 0 or 1");
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
  for (const Branch& B : P.br) {
    if (e == hipSuccess && !B.mats.empty())
      e = hipMemcpyAsync(ws + B.off_mats, B.mats.data(), sizeof(int) * B.mats.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !B.tiles.empty())
      e = hipMemcpyAsync(ws + B.off_tiles, B.tiles.data(), sizeof(int) * B.tiles.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !B.whole.empty())
      e = hipMemcpyAsync(ws + B.off_whole, B.whole.data(), sizeof(int) * B.whole.size(), hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host vectors are released on return
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "descriptor upload: %s", hipGetErrorString(e));
  ba.items = (const BatchItem*)(ws + P.off_items);
  ba.res = (BatchRes*)(ws + P.off_res);
  ba.tile_tasks = nullptr;   // set per branch
  ba.mat_tasks = nullptr;
  ba.pick = (int*)(ws + P.off_pick);
  ba.chosen = (int*)(ws + P.off_chosen);
  ba.batch = (int)P.items.size();
  ba.ws = ws;
  return PS_OK;
}

// the fixed launch sequence of one branch (stream-ordered)
ps_status launch_branch(int W, BatchArgs ba, const Branch& B, hipStream_t st) {
  const dim3 blk(NT);
#define PS_BLAUNCH(KER, GRID, ...)                                                          \
  do {                                                                                       \
    if (W == 0) hipLaunchKernelGGL(KER<double>, dim3(GRID), blk, 0, st, ba, ##__VA_ARGS__); \
    else hipLaunchKernelGGL(KER<float>, dim3(GRID), blk, 0, st, ba, ##__VA_ARGS__);         \
  } while (0)
  if (!B.whole.empty()) {
    ba.mat_tasks = (const int*)(ba.ws + B.off_whole);
    PS_BLAUNCH(k_bwhole, (unsigned)B.whole.size());
  }
  if (B.mats.empty()) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PS_OK : bfail(PS_ERR_HIP, "batch launch: %s", hipGetErrorString(e));
  }
  ba.tile_tasks = (const int*)(ba.ws + B.off_tiles);
  ba.mat_tasks = (const int*)(ba.ws + B.off_mats);
  const unsigned nmat = (unsigned)B.mats.size(), ntile = (unsigned)B.tiles.size();
  PS_BLAUNCH(k_bchoose, nmat);
  PS_BLAUNCH(k_bpad, ntile);
  // powers: for each j, the products of the matrices with j < s, then those
  // with j = s (Y) together with their block assembly (only for the block
  // sizes some matrix can take)
  for (int j = 2; j <= B.smax; ++j) {
    if (j < B.smax) PS_BLAUNCH(k_bpower, ntile, j);
    if (B.s_possible[j]) PS_BLAUNCH(k_bpower_asm, ntile, j);
  }
  if (B.s_possible[1]) PS_BLAUNCH(k_bassemble1, ntile);
  PS_BLAUNCH(k_bplan, nmat);
  for (int k = -1; k < B.kmax; ++k) PS_BLAUNCH(k_bhorner, ntile, k);
  for (int q = 1; q <= B.sigmax; ++q) PS_BLAUNCH(k_bsquare, ntile, q);
#undef PS_BLAUNCH
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "batch launch: %s", hipGetErrorString(e));
  return PS_OK;
}

// Side streams of the branches: a pool per device, created on first use and
// kept for the life of the process (a stream destroyed with work in flight
// may drop it).  g_branch_mu is held while a multi-branch batch is queued or
// captured, so no other call puts work on a side stream meanwhile.
std::mutex g_branch_mu;
constexpr int kMaxDev = 64;
hipStream_t g_side[kMaxDev][kMaxBranch];

ps_status side_streams(hipStream_t* out, int count) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDev) return bfail(PS_ERR_UNSUPPORTED, "device index %d", dev);
  for (int k = 0; k < count; ++k) {
    if (!g_side[dev][k]) {
      e = hipStreamCreateWithFlags(&g_side[dev][k], hipStreamNonBlocking);
      if (e != hipSuccess) return bfail(PS_ERR_HIP, "side stream: %s", hipGetErrorString(e));
    }
    out[k] = g_side[dev][k];
  }
  return PS_OK;
}

int used_branches(const Plan2& P) {
  int used = 0;
  for (const Branch& B : P.br) used += B.empty() ? 0 : 1;
  return used;
}

// every branch of a batch: the first on `st`, the others on side streams
// forked from it by an event and joined back by one event each (under
// capture the fork and the joins become graph edges).  The caller holds
// g_branch_mu when more than one branch is used.
ps_status launch_batch(int W, const BatchArgs& ba, const Plan2& P, hipStream_t st) {
  if (used_branches(P) <= 1) {
    for (const Branch& B : P.br)
      if (ps_status r = launch_branch(W, ba, B, st)) return r;
    return PS_OK;
  }
  hipStream_t side[kMaxBranch] = {};
  if (ps_status r = side_streams(side, kMaxBranch - 1)) return r;
  hipEvent_t fork = nullptr, join[kMaxBranch] = {};
  ps_status r = PS_OK;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, st);
  int k = 0;
  for (size_t i = 0; i < P.br.size() && e == hipSuccess && r == PS_OK; ++i) {
    const Branch& B = P.br[i];
    if (B.empty()) continue;
    if (k == 0) {
      r = launch_branch(W, ba, B, st);
    } else {
      hipStream_t sk = side[k - 1];
      e = hipStreamWaitEvent(sk, fork, 0);
      if (e == hipSuccess) r = launch_branch(W, ba, B, sk);
      if (e == hipSuccess && r == PS_OK) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
      if (e == hipSuccess && r == PS_OK) e = hipEventRecord(join[k], sk);
      if (e == hipSuccess && r == PS_OK) e = hipStreamWaitEvent(st, join[k], 0);
    }
    ++k;
  }
  for (int i = 0; i < kMaxBranch; ++i)
    if (join[i]) (void)hipEventDestroy(join[i]);
  if (fork) (void)hipEventDestroy(fork);
  if (r != PS_OK) return r;
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "branch fork/join: %s", hipGetErrorString(e));
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
  ps_status st = build_plan(dtype, batch, n, m, s, nullptr, nullptr, nullptr, nullptr, nullptr, P, false, Schedule());
  if (st) return ps_set_error(st, g_batch_err.c_str());
  *bytes = P.total;
  return PS_OK;
}

static ps_status batched_common(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                                const double* coef, int m, const int32_t* s, const int32_t* sigma, void* const* E,
                                const int64_t* lde, const ps_opts* opts, void* ws, size_t ws_bytes, void* stream,
                                Plan2& P, BatchArgs& ba, const Schedule* sch = nullptr) {
  if (batch < 1 || !n) return bfail(PS_ERR_ARG, "batch = %d or n == NULL", batch);
  ps_status st = build_plan(dtype, batch, n, m, s, sigma, A, lda, E, lde, P, true,
                            sch ? *sch : cached_schedule(dtype, m, batch, n));
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
  {
    std::unique_lock<std::mutex> lock(g_branch_mu, std::defer_lock);
    if (used_branches(P) > 1) lock.lock();
    if ((r = launch_batch(dtype == PS_F64 ? 0 : 1, ba, P, st))) return ps_set_error(r, g_batch_err.c_str());
  }
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

ps_status ps_eval_batched(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s, void* const* P, const int64_t* ldp,
                          const ps_opts* opts, int32_t* tiers_out, void* ws, size_t ws_bytes, void* stream) {
  if (!coef) return ps_set_error(bfail(PS_ERR_ARG, "coef == NULL"), g_batch_err.c_str());
  return ps_expm_batched(dtype, batch, n, A, lda, coef, m, s, nullptr, P, ldp, opts, tiers_out, ws, ws_bytes, stream);
}

}  // extern "C"

// capture one batch's launch sequence (on a private stream: the legacy null
// stream cannot be captured) and instantiate it
static ps_status capture_batch(int W, const BatchArgs& ba, const Plan2& P, ps_batched_exec** out) {
  hipStream_t cap;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return bfail(PS_ERR_HIP, "%s", hipGetErrorString(e));
  ps_batched_exec* h = new ps_batched_exec();
  ps_status r = PS_OK;
  {
    std::unique_lock<std::mutex> lock(g_branch_mu, std::defer_lock);
    if (used_branches(P) > 1) lock.lock();   // the side streams join this capture
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      r = launch_batch(W, ba, P, cap);
      hipError_t e2 = hipStreamEndCapture(cap, &h->graph);
      if (r == PS_OK && e2 != hipSuccess) e = e2;
    }
  }
  if (e == hipSuccess && r == PS_OK) e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess || r != PS_OK) {
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
    return r ? r : bfail(PS_ERR_HIP, "%s", hipGetErrorString(e));
  }
  *out = h;
  return PS_OK;
}

// the contiguous groupings of the present classes (in increasing order) into
// at most kMaxBranch branches; where class 1 has a branch of its own, also
// with that class on k_bwhole
static std::vector<Schedule> candidate_schedules(const int cls_count[kMaxClass + 1]) {
  std::vector<int> present;
  for (int c = 1; c <= kMaxClass; ++c)
    if (cls_count[c] > 0) present.push_back(c);
  std::vector<Schedule> out;
  const int K = (int)present.size();
  if (K == 0) return {Schedule()};
  for (int cut = 0; cut < (1 << (K - 1)); ++cut) {   // bit i: a new branch starts after present class i
    Schedule sch;
    int g = 0;
    for (int i = 0; i < K; ++i) {
      sch.group[present[i] - 1] = g;
      if (i < K - 1 && ((cut >> i) & 1)) ++g;
    }
    out.push_back(sch);
  }
  if (cls_count[1] > 0) {
    const size_t ng = out.size();
    for (size_t k = 0; k < ng; ++k) {
      bool alone = true;
      for (int c = 2; c <= kMaxClass; ++c) alone = alone && !(cls_count[c] > 0 && out[k].group[c - 1] == out[k].group[0]);
      if (!alone) continue;
      Schedule w = out[k];
      w.whole64 = 1;
      out.push_back(w);
    }
  }
  return out;
}

extern "C" {

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
  if ((r = capture_batch(dtype == PS_F64 ? 0 : 1, ba, P, out))) return ps_set_error(r, g_batch_err.c_str());
  return PS_OK;
}

ps_status ps_batched_tune(ps_dtype dtype, int batch, const int32_t* n, const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s, const int32_t* sigma, void* const* E,
                          const int64_t* lde, const ps_opts* opts, void* ws, size_t ws_bytes, void* stream, int reps,
                          int32_t* groups_out, float* ms_out, int* ncand_out) {
  if (reps < 1 || reps > 1000) return ps_set_error(PS_ERR_ARG, "reps out of range [1, 1000]");
  if (batch < 1 || !n) return ps_set_error(PS_ERR_ARG, "batch < 1 or n == NULL");
  int cc[kMaxClass + 1];
  count_classes(batch, n, cc);
  const std::vector<Schedule> cand = candidate_schedules(cc);
  hipStream_t st = (hipStream_t)stream;
  const int W = dtype == PS_F64 ? 0 : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) return ps_set_error(PS_ERR_HIP, hipGetErrorString(he));
  int best = -1;
  float best_ms = 0.0f;
  ps_status r = PS_OK;
  for (size_t k = 0; k < cand.size() && r == PS_OK; ++k) {
    Plan2 P;
    BatchArgs ba;
    r = batched_common(dtype, batch, n, A, lda, coef, m, s, sigma, E, lde, opts, ws, ws_bytes, stream, P, ba,
                       &cand[k]);
    ps_batched_exec* h = nullptr;
    if (r == PS_OK) r = capture_batch(W, ba, P, &h);
    if (r != PS_OK) break;
    // one warm-up replay, then the median of reps timed replays
    std::vector<float> t;
    he = hipGraphLaunch(h->exec, st);
    for (int q = 0; q < reps && he == hipSuccess; ++q) {
      he = hipEventRecord(e0, st);
      if (he == hipSuccess) he = hipGraphLaunch(h->exec, st);
      if (he == hipSuccess) he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      t.push_back(ms);
    }
    (void)hipGraphExecDestroy(h->exec);
    (void)hipGraphDestroy(h->graph);
    delete h;
    if (he != hipSuccess) {
      r = bfail(PS_ERR_HIP, "tuning replay: %s", hipGetErrorString(he));
      break;
    }
    std::sort(t.begin(), t.end());
    const float med = t[t.size() / 2];
    if (ms_out && k < kMaxCand) ms_out[k] = med;
    if (best < 0 || med < best_ms) {
      best = (int)k;
      best_ms = med;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != PS_OK) return ps_set_error(r, g_batch_err.c_str());
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache[schedule_key(dtype, m, cc)] = cand[best];
  }
  if (groups_out) {
    for (int c = 0; c < kMaxClass; ++c) groups_out[c] = cand[best].group[c];
    groups_out[kMaxClass] = cand[best].whole64;
  }
  if (ncand_out) *ncand_out = (int)cand.size();
  return PS_OK;
}

ps_status ps_autotune_lookup(ps_dtype dtype, int batch, const int32_t* n, int m, int32_t* groups_out, int* found) {
  if (!n || batch < 1 || !groups_out || !found) return ps_set_error(PS_ERR_ARG, "NULL argument or batch < 1");
  int cc[kMaxClass + 1];
  count_classes(batch, n, cc);
  const std::string key = schedule_key(dtype, m, cc);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto it = g_cache.find(key);
  *found = it != g_cache.end();
  const Schedule sch = *found ? it->second : Schedule();
  for (int c = 0; c < kMaxClass; ++c) groups_out[c] = sch.group[c];
  groups_out[kMaxClass] = sch.whole64;
  return PS_OK;
}

ps_status ps_autotune_clear(void) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_cache.clear();
  return PS_OK;
}

ps_status ps_autotune_save(const char* path) {
  if (!path) return ps_set_error(PS_ERR_ARG, "path == NULL");
  FILE* f = fopen(path, "w");
  if (!f) return ps_set_error(PS_ERR_ARG, "cannot open the cache file for writing");
  std::lock_guard<std::mutex> lock(g_cache_mu);
  fprintf(f, "{\"ps_autotune\": 1, \"entries\": [");
  bool first = true;
  for (const auto& kv : g_cache) {
    fprintf(f, "%s\n  {\"key\": \"%s\", \"groups\": [%d, %d, %d, %d], \"whole64\": %d}", first ? "" : ",",
            kv.first.c_str(), kv.second.group[0], kv.second.group[1], kv.second.group[2], kv.second.group[3],
            kv.second.whole64);
    first = false;
  }
  fprintf(f, "\n]}\n");
  fclose(f);
  return PS_OK;
}

ps_status ps_autotune_load(const char* path) {
  if (!path) return ps_set_error(PS_ERR_ARG, "path == NULL");
  FILE* f = fopen(path, "r");
  if (!f) return ps_set_error(PS_ERR_ARG, "cannot open the cache file");
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  fclose(f);
  if (text.find("\"ps_autotune\": 1") == std::string::npos) return ps_set_error(PS_ERR_ARG, "not a cache file");
  std::map<std::string, Schedule> add;
  size_t pos = 0;
  while ((pos = text.find("\"key\": \"", pos)) != std::string::npos) {
    pos += 8;
    const size_t end = text.find('"', pos);
    const size_t gp = text.find("\"groups\": [", end == std::string::npos ? pos : end);
    if (end == std::string::npos || gp == std::string::npos) return ps_set_error(PS_ERR_ARG, "malformed cache entry");
    Schedule sch;
    if (sscanf(text.c_str() + gp + 11, "%d , %d , %d , %d", &sch.group[0], &sch.group[1], &sch.group[2],
               &sch.group[3]) != 4)
      return ps_set_error(PS_ERR_ARG, "malformed groups in the cache file");
    for (int c = 0; c < kMaxClass; ++c)
      if (sch.group[c] < 0 || sch.group[c] >= kMaxBranch) return ps_set_error(PS_ERR_ARG, "group out of range");
    // optional (files without it: per-phase launches); it belongs to this
    // entry if it comes before the next entry's key
    const size_t wp = text.find("\"whole64\": ", gp);
    const size_t next = text.find("\"key\": \"", gp);
    if (wp != std::string::npos && (next == std::string::npos || wp < next)) {
      if (sscanf(text.c_str() + wp + 11, "%d", &sch.whole64) != 1 || sch.whole64 < 0 || sch.whole64 > 1)
        return ps_set_error(PS_ERR_ARG, "malformed whole64 in the cache file");
    }
    add[text.substr(pos, end - pos)] = sch;
    pos = gp;
  }
  std::lock_guard<std::mutex> lock(g_cache_mu);
  for (const auto& kv : add) g_cache[kv.first] = kv.second;
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
