// Double-double working precision (u = 2^-106) with FP64 / FP32 / BF16 / FP8
// tiers below it: the paper's multi-precision setting (sections 1 and 4,
// Table 1), where the working precision is far above IEEE double and every
// Horner product that the plan moves to a lower tier saves most of its cost.
//
// A double-double matrix is two FP64 planes: hi at p, lo at p + ld n, both
// column-major with leading dimension ld; the value of an entry is hi + lo
// with |lo| <= ulp(hi) / 2.
//
// Kernels:
//   k_gemm_dd     C = alpha A B in double-double on the FP64 vector units
//                 (the head hi*hi of each product with its exact FMA
//                 residual, the two cross terms in the tail, lo*lo dropped;
//                 compensated summation), alpha a power of two.  Power table
//                 and squarings.
//   k_assemble_dd B_0..B_r = sum_j c_{si+j} X^j in double-double with
//                 double-double coefficients (section 2: the blocks are
//                 assembled in the working precision), column abs sums of
//                 the hi parts for the plan, FP32 / BF16 / FP8 copies of Y.
//   k_plan        shared with the IEEE path (working tier 4).
//   k_horner_dd   one Horner step P_{i-1} = B_{i-1} + P_i Y: the product in
//                 tier(i) (double-double on the vector units, or an MFMA tier
//                 on the operand formats of ps_device.h), the sum with
//                 B_{i-1} in tier(i-1).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ps_device.h"

// The error-free transformations below rely on every product and sum being
// rounded on its own: no multiply may be fused into a following add (a
// contracted a*b + c would pair an exact product with a rounded one).
#pragma clang fp contract(off)

namespace psk {

// ---------------------------------------------------------------------------
// double-double arithmetic (error-free transformations: Knuth's two-sum,
// Dekker's fast two-sum, the FMA two-product)
// ---------------------------------------------------------------------------
struct D2 {
  double hi, lo;
};
__device__ inline D2 two_sum(double a, double b) {
  const double s = a + b, v = s - a;
  return {s, (a - (s - v)) + (b - v)};
}
__device__ inline D2 fast_two_sum(double a, double b) {   // |a| >= |b| or a = 0
  const double s = a + b;
  return {s, b - (s - a)};
}
// double-double + double-double, the accurate variant (two two-sums)
__device__ inline D2 d2_add(D2 x, D2 y) {
  const D2 s = two_sum(x.hi, y.hi), t = two_sum(x.lo, y.lo);
  const D2 v = fast_two_sum(s.hi, s.lo + t.hi);
  return fast_two_sum(v.hi, t.lo + v.lo);
}
__device__ inline D2 d2_mul(D2 x, D2 y) {
  const double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, e);
  e = fma(x.lo, y.hi, e);
  return fast_two_sum(p, e);
}
// One term of a double-double dot product, in the compensated form of Ogita,
// Rump and Oishi's Dot2 ("Accurate sum and dot product", 2005): acc.hi is
// the running sum of the product heads, acc.lo collects (unnormalised) the
// two-sum errors of those additions and the product tails (FMA residual of
// hi*hi and the two cross terms).  12 FP64 operations per term; the pair is
// renormalised once at the end of the dot product (d2_finish).
__device__ inline void d2_fma_acc(D2& acc, D2 x, D2 y) {
  const double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, e);
  e = fma(x.lo, y.hi, e);
  const D2 s = two_sum(acc.hi, p);
  acc.hi = s.hi;
  acc.lo += s.lo + e;
}
__device__ inline D2 d2_finish(D2 acc) { return two_sum(acc.hi, acc.lo); }

// ---------------------------------------------------------------------------
// double-double GEMM tile: 64 x 64 outputs, 512 threads, 4 x 2 outputs per
// thread; K in slabs of 16 through LDS (hi and lo planes of both operands)
// ---------------------------------------------------------------------------
constexpr int DD_BK = 16;
constexpr int DD_LR = 64 + 4;                 // padded LDS row (doubles)
constexpr int DD_PLANE = DD_BK * DD_LR;       // one plane of one operand slab
constexpr int DD_STAGE = 4 * DD_PLANE;        // A hi, A lo, B hi, B lo
static_assert(2 * DD_STAGE * 8 <= smem_bytes<double>(), "double-double stages fit the tile LDS");
static_assert(kTileN * CSTR * 16 <= smem_bytes<double>(), "double-double epilogue tile fits the tile LDS");

struct DDMat {
  const double* p;   // hi plane; lo plane at p + plane
  int64_t ld, plane;
};

// slab loads: thread t moves 4 consecutive elements of one plane.
// A (64 rows x 16 k): plane = t >> 8, k = (t >> 4) & 15, rows 4 (t & 15) ..
// B (16 k x 64 cols): plane = t >> 8, col = (t >> 2) & 63, k = 4 (t & 3) ..
__device__ inline void dd_load_a(const DDMat& A, int64_t n, int64_t m0, int64_t k0, double alpha, int t, double r[4]) {
  const int pl = t >> 8, kk = (t >> 4) & 15, mm = (t & 15) * 4;
  const int64_t k = k0 + kk, m = m0 + mm;
  const double* q = A.p + pl * A.plane + m + k * A.ld;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = (k < n && m + i < n) ? q[i] * alpha : 0.0;
}
__device__ inline void dd_store_a(double* S, int t, const double r[4]) {
  const int pl = t >> 8, kk = (t >> 4) & 15, mm = (t & 15) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) S[pl * DD_PLANE + kk * DD_LR + mm + i] = r[i];
}
__device__ inline void dd_load_b(const DDMat& B, int64_t n, int64_t n0, int64_t k0, int t, double r[4]) {
  const int pl = t >> 8, jj = (t >> 2) & 63, kk = (t & 3) * 4;
  const int64_t j = n0 + jj, k = k0 + kk;
  const double* q = B.p + pl * B.plane + k + j * B.ld;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = (j < n && k + i < n) ? q[i] : 0.0;
}
__device__ inline void dd_store_b(double* S, int t, const double r[4]) {
  const int pl = t >> 8, jj = (t >> 2) & 63, kk = (t & 3) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) S[2 * DD_PLANE + pl * DD_PLANE + (kk + i) * DD_LR + jj] = r[i];
}

// acc[4][2] = (alpha A)(tile rows) x B(tile cols) over all of K, returned as
// normalised double-double values.  alpha is a power of two applied to A
// exactly.  Ends with a barrier.
__device__ inline void dd_mainloop(const DDMat& A, double alpha, const DDMat& B, int64_t n, int64_t m0, int64_t n0,
                                   char* smem, D2 acc[4][2]) {
  const int t = threadIdx.x;
  const int tr = t & 15, tc = t >> 4;   // rows 4 tr .. 4 tr + 3, columns 2 tc, 2 tc + 1
  double* S = (double*)smem;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = D2{0.0, 0.0};
  const int64_t nk = (n + DD_BK - 1) / DD_BK;
  double ra[4], rb[4];
  dd_load_a(A, n, m0, 0, alpha, t, ra);
  dd_load_b(B, n, n0, 0, t, rb);
  dd_store_a(S, t, ra);
  dd_store_b(S, t, rb);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    // next slab (clamped to the last one: the loads stay unconditional)
    const int64_t kn = min<int64_t>(kt + 1, nk - 1) * DD_BK;
    dd_load_a(A, n, m0, kn, alpha, t, ra);
    dd_load_b(B, n, n0, kn, t, rb);
    const double* st = S + cur * DD_STAGE;
#pragma unroll 4
    for (int k = 0; k < DD_BK; ++k) {
      D2 a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = D2{st[k * DD_LR + 4 * tr + i], st[DD_PLANE + k * DD_LR + 4 * tr + i]};
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = D2{st[2 * DD_PLANE + k * DD_LR + 2 * tc + j], st[3 * DD_PLANE + k * DD_LR + 2 * tc + j]};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) d2_fma_acc(acc[i][j], a[i], b[j]);
    }
    double* nx = S + (cur ^ 1) * DD_STAGE;
    dd_store_a(nx, t, ra);
    dd_store_b(nx, t, rb);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d2_finish(acc[i][j]);
}

__global__ __launch_bounds__(NT) void k_gemm_dd(int64_t n, DDMat A, double alpha, DDMat B, double* C, int64_t ldc,
                                                int64_t cplane) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<double>()];
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int64_t m0 = (int64_t)tm * kTileM, n0 = (int64_t)tn * kTileN;
  D2 acc[4][2];
  dd_mainloop(A, alpha, B, n, m0, n0, smem, acc);
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t gr = m0 + 4 * tr + i, gc = n0 + 2 * tc + j;
      if (gr < n && gc < n) {
        C[gr + gc * ldc] = acc[i][j].hi;
        C[cplane + gr + gc * ldc] = acc[i][j].lo;
      }
    }
}

// ---------------------------------------------------------------------------
// block assembly in double-double.  One wave per (column, 256-row chunk),
// four rows per lane, blocks four at a time.  x_j = the power slot j, x_1 =
// beta A.  Column abs sums of the hi parts go to the colsum layout of
// plan_matrix; the FP32 / BF16 / MX-FP8 copies of Y come from Y's hi part.
// ---------------------------------------------------------------------------
struct AssembleDD {
  int64_t n;
  int m, s, r, nB, trivial_last;
  DDMat X1;              // A
  double beta;           // X_1 = beta A
  char* ws;
  Layout L;              // esize 16: each slot is a hi plane and a lo plane
  const double* chi;     // coefficients, hi and lo parts (device, m + 1 each)
  const double* clo;
  unsigned tier_mask;
};

__device__ inline D2 ldd(const double* p, int64_t plane, int64_t i) { return D2{p[i], p[plane + i]}; }

__global__ __launch_bounds__(NT) void k_assemble_dd(AssembleDD a) {
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6);
  if (col >= a.n) return;   // no workgroup barrier below
  const Layout& L = a.L;
  const int64_t n = a.n, chunk = blockIdx.y;
  const int64_t plane = n * n;
  const int64_t se = (int64_t)(L.slot / 8);           // doubles per slot
  const double* pw = (const double*)(a.ws + L.off_pow);
  double* Bm = (double*)(a.ws + L.off_B);
  double* colsum = (double*)(a.ws + L.off_colsum);
  const int s = a.s, m = a.m, nB = a.nB;
  const int64_t Kp = L.Kp, Ks = Kp / 32;
  float* yf32 = (float*)(a.ws + L.off_yf32);
  uint16_t* ybf = (uint16_t*)(a.ws + L.off_ybf16);
  uint8_t* y8 = (uint8_t*)(a.ws + L.off_yfp8);
  uint8_t* y8s = (uint8_t*)(a.ws + L.off_yfp8s);
  const bool want32 = (a.tier_mask >> 1) & 1u, want16 = (a.tier_mask >> 2) & 1u, want8 = (a.tier_mask >> 3) & 1u;
  constexpr int RPL = kRowChunk / 64;
  const int64_t r_begin = chunk * kRowChunk, r_end = min<int64_t>(n, r_begin + kRowChunk);
  const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
  int64_t rw[RPL];
  bool valid[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    rw[q] = r_begin + lane + 64 * q;
    valid[q] = rw[q] < r_end;
  }
  auto load_x = [&](int j, D2 out[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int64_t rr = valid[q] ? rw[q] : r_begin;
      D2 x;
      if (j == 1) {
        const D2 v = D2{a.X1.p[rr + col * a.X1.ld], a.X1.p[a.X1.plane + rr + col * a.X1.ld]};
        x = D2{v.hi * a.beta, v.lo * a.beta};
      } else {
        x = ldd(pw + (int64_t)(j - 2) * se, plane, rr + col * n);
      }
      out[q] = valid[q] ? x : D2{0.0, 0.0};
    }
  };
  D2 y[RPL];
  load_x(s, y);
  double ysum = 0.0;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    ysum += fabs(y[q].hi);
    if (valid[q] && want32) yf32[rw[q] + col * n] = (float)y[q].hi;
    if (valid[q] && want16) ybf[col * Kp + rw[q]] = bf16_bits_rne((float)y[q].hi);
    if (want8) {
      float av = fabsf((float)y[q].hi);
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) av = fmaxf(av, __shfl_xor(av, off, 64));
      const int sbyte = e8m0_for(av);
      if (valid[q]) {
        float qv = ldexpf((float)y[q].hi, -(sbyte - 127));
        qv = fminf(fmaxf(qv, -448.0f), 448.0f);
        const int wv = __builtin_amdgcn_cvt_pk_fp8_f32(qv, 0.0f, 0, false);
        y8[col * Kp + rw[q]] = (uint8_t)(wv & 0xff);
        if ((rw[q] & 31) == 0) y8s[col * Ks + rw[q] / 32] = (uint8_t)sbyte;
      }
    }
  }
  if (col == 0 && chunk == 0) {   // |c_k| (hi parts) beside the plan
    Plan* P = (Plan*)(a.ws + L.off_plan);
    for (int k = lane; k <= m; k += 64) P->abs_coef[k] = fabs(a.chi[k]);
  }
  double xsum = 0.0;   // column abs sum of X_1 (hi parts), first pass over the blocks
  for (int i0 = 0; i0 < nB; i0 += 4) {
    D2 bv[RPL][4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = i0 + ii;
      const D2 c0 = (i < nB && s * i <= m) ? D2{a.chi[s * i], a.clo[s * i]} : D2{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < RPL; ++q) bv[q][ii] = (rw[q] == col) ? c0 : D2{0.0, 0.0};
    }
    for (int j = 1; j < s; ++j) {
      D2 xj[RPL];
      load_x(j, xj);
      if (j == 1 && i0 == 0)
#pragma unroll
        for (int q = 0; q < RPL; ++q) xsum += fabs(xj[q].hi);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int k = s * (i0 + ii) + j;
        if (i0 + ii < nB && k <= m) {
          const D2 ck = D2{a.chi[k], a.clo[k]};
#pragma unroll
          for (int q = 0; q < RPL; ++q) bv[q][ii] = d2_add(bv[q][ii], d2_mul(ck, xj[q]));
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = i0 + ii;
      if (i >= nB) continue;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        if (!valid[q]) continue;
        D2 outv = bv[q][ii];
        if (a.trivial_last && i == a.r - 1) outv = d2_add(outv, d2_mul(D2{a.chi[m], a.clo[m]}, y[q]));
        v += fabs(outv.hi);
        double* dst = Bm + (int64_t)i * se;
        dst[rw[q] + col * n] = outv.hi;
        dst[plane + rw[q] + col * n] = outv.lo;
      }
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) colsum[((int64_t)i * nch + chunk) * n + col] = v;
    }
  }
  double v = ysum;
  double vx = s == 1 ? ysum : xsum;   // s = 1: X_1 is Y
  for (int off = 32; off >= 1; off >>= 1) {
    v += __shfl_xor(v, off, 64);
    vx += __shfl_xor(vx, off, 64);
  }
  if (lane == 0) {
    colsum[((int64_t)nB * nch + chunk) * n + col] = v;
    colsum[((int64_t)(nB + 1) * nch + chunk) * n + col] = vx;
  }
}

// ---------------------------------------------------------------------------
// Horner step in the double-double setting.  Buffer formats by tier:
// 4 = double-double (two planes, ld n), 0 = FP64 column-major, 1 = FP32
// column-major, 2 / 3 = the packed K-contiguous layouts of ps_device.h.
// ---------------------------------------------------------------------------
struct HornerDD {
  int64_t n;
  int step, cast_only, final_out;
  Layout L;
  char* ws;
  size_t off_pin, off_pout, off_bsrc;
  DDMat Y;               // Y = yscale * (this matrix) in double-double
  double yscale;
  double* out;           // final result (double-double planes)
  int64_t ldo, oplane;
};

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_horner_dd(HornerDD a) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<double>()];
  const Layout& L = a.L;
  const int64_t n = a.n, plane = n * n;
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int64_t m0 = (int64_t)tm * kTileM, n0 = (int64_t)tn * kTileN;
  const Plan* P = (const Plan*)(a.ws + L.off_plan);
  const int t_in = a.cast_only ? -1 : P->tier[a.step];
  const int t_out = a.final_out ? kTierDD : P->tier[a.cast_only ? a.step : a.step - 1];
  const char* pin = a.ws + a.off_pin;
  char* pout = a.ws + a.off_pout;
  const int64_t Kp = L.Kp;
  const int t = threadIdx.x;
  // product P_i Y of the tile into Cs (hi plane) and Cl (lo plane), column-major
  double* Cs = (double*)smem;
  double* Cl = Cs + kTileN * CSTR;
  if (t_in == kTierDD) {
    D2 acc[4][2];
    dd_mainloop(DDMat{(const double*)pin, n, plane}, 1.0, a.Y, n, m0, n0, smem, acc);
    const int tr = t & 15, tc = t >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = 4 * tr + i, col = 2 * tc + j;
        Cs[col * CSTR + row] = acc[i][j].hi * a.yscale;
        Cl[col * CSTR + row] = acc[i][j].lo * a.yscale;
      }
  } else if (t_in == 0) {
    typename MF<double>::V acc[2];
    mainloop_lds<double, false, false>((const double*)pin, n, a.Y.p, a.Y.ld, n, m0, n0, smem, acc);
    frag_to_cs<double, double>(acc, Cs, a.yscale);
  } else if (t_in == 1) {
    typename MF<float>::V acc[2];
    mainloop_lds<float, false, false>((const float*)pin, n, (const float*)(a.ws + L.off_yf32), n, n, m0, n0, smem,
                                      acc);
    frag_to_cs<float, double>(acc, Cs, 1.0);
  } else if (t_in == 2) {
    f4v acc[2];
    mainloop_lowp<false>((const uint8_t*)pin, nullptr, (const uint8_t*)(a.ws + L.off_ybf16), nullptr, Kp, n, m0, n0,
                         smem, acc);
    frag_f32_to_cs_any(acc, Cs, (float*)Cs, true);
  } else if (t_in == 3) {
    f4v acc[2];
    const uint8_t* p8 = (const uint8_t*)pin;
    mainloop_lowp<true>(p8, p8 + L.Mp * Kp, (const uint8_t*)(a.ws + L.off_yfp8), (const uint8_t*)(a.ws + L.off_yfp8s),
                        Kp, n, m0, n0, smem, acc);
    frag_f32_to_cs_any(acc, Cs, (float*)Cs, true);
  }
  __syncthreads();
  // pass 1 (column-major): P_{i-1} = B_{i-1} + product in the precision of t_out
  const double* bsrc = (const double*)(a.ws + a.off_bsrc);
  const int row = t & 63;
  const int64_t gr = m0 + row;
  for (int q = 0; q < TILE_Q; ++q) {
    const int col = (t >> 6) + NW * q;
    const int64_t gc = n0 + col;
    const bool in = gr < n && gc < n;
    const int64_t e = (in ? gr : 0) + (in ? gc : 0) * n;
    const D2 b = in ? D2{bsrc[e], bsrc[plane + e]} : D2{0.0, 0.0};
    const D2 v = (t_in < 0) ? D2{0.0, 0.0} : D2{Cs[col * CSTR + row], t_in == kTierDD ? Cl[col * CSTR + row] : 0.0};
    if (t_out == kTierDD) {
      const D2 rs = d2_add(b, v);
      if (a.final_out) {
        if (in) {
          a.out[gr + gc * a.ldo] = rs.hi;
          a.out[a.oplane + gr + gc * a.ldo] = rs.lo;
        }
      } else if (in) {
        ((double*)pout)[e] = rs.hi;
        ((double*)pout)[plane + e] = rs.lo;
      }
    } else if (t_out == 0) {
      if (in) ((double*)pout)[e] = (b.hi + b.lo) + v.hi;
    } else if (t_out == 1) {
      if (in) ((float*)pout)[e] = (float)(b.hi + b.lo) + (float)v.hi;
    } else {
      Cs[col * CSTR + row] = in ? (double)((float)(b.hi + b.lo) + (float)v.hi) : 0.0;
    }
  }
  __syncthreads();
  if (t_out == 2 || t_out == 3) pack_tile_lowp<double>(Cs, t_out, pout, L.Mp, Kp, m0, n0);
}

}  // namespace psk

// ===========================================================================
// host side
// ===========================================================================
using namespace psk;

namespace {

thread_local std::string g_dd_err;

ps_status dfail(ps_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_dd_err = buf;
  return ps_set_error(st, g_dd_err.c_str());
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// double-double layout: every matrix slot holds two FP64 planes
Layout dd_layout(int64_t n, int m, int s, int sigma) {
  Layout L = make_layout(PS_F64, n, m, s, sigma, 0);   // packed Y copies, colsum, plan as for FP64
  Layout D = L;
  D.working = kTierDD;
  D.esize = 16;
  D.slot = al256((size_t)n * n * 16);
  D.pslot = al256(std::max(D.slot, L.pslot));
  size_t off = 0;
  D.off_pow = off;   off += (size_t)D.npow * D.slot;
  D.off_B = off;     off += (size_t)D.nB * D.slot;
  D.off_P0 = off;    off += D.pslot;
  D.off_P1 = off;    off += D.pslot;
  D.off_R = off;     off += (sigma > 0 ? D.slot : 0);
  D.off_yf32 = off;  off += al256((size_t)n * n * 4);
  D.off_ybf16 = off; off += al256((size_t)D.Mp * D.Kp * 2);
  D.off_yfp8 = off;  off += al256((size_t)D.Mp * D.Kp);
  D.off_yfp8s = off; off += al256((size_t)D.Mp * (D.Kp / 32));
  D.off_colsum = off; off += al256((size_t)(D.nB + 2) * ((n + kRowChunk - 1) / kRowChunk) * n * 8);
  D.off_plan = off;  off += al256(sizeof(Plan));
  D.off_coef = off;  off += al256((size_t)2 * (m + 1) * 8);
  D.bytes = al256(off);
  return D;
}

// 1/k! in double-double (long division by k of a double-double, then renormalisation)
void taylor_dd(int m, double* hi, double* lo) {
  double h = 1.0, l = 0.0;
  hi[0] = 1.0;
  lo[0] = 0.0;
  for (int k = 1; k <= m; ++k) {
    const double q1 = h / k;
    const double p = q1 * k, pe = std::fma(q1, (double)k, -p);   // q1 k exactly = p + pe
    const double r = ((h - p) - pe) + l;                          // remainder
    const double q2 = r / k;
    const double s = q1 + q2;
    h = s;
    l = q2 - (s - q1);
    hi[k] = h;
    lo[k] = l;
  }
}

bool spans_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" {

ps_status ps_workspace_size_dd(int64_t n, int m, int s, int sigma, size_t* bytes) {
  if (!bytes) return dfail(PS_ERR_ARG, "bytes == NULL");
  if (n < 1 || n > (1LL << 16)) return dfail(PS_ERR_ARG, "n = %lld out of range [1, 65536]", (long long)n);
  if (m < 0 || m > kMaxDegree) return dfail(PS_ERR_ARG, "degree m = %d out of range", m);
  if (s == 0) s = m <= 1 ? 1 : (int)std::ceil(std::sqrt((double)m) - 1e-12);
  if (s < 1 || s > std::max(m, 1)) return dfail(PS_ERR_ARG, "block size s = %d out of range", s);
  if (sigma < 0 || sigma > kMaxSigma) return dfail(PS_ERR_ARG, "sigma = %d out of range", sigma);
  *bytes = dd_layout(n, m, s, sigma).bytes;
  return PS_OK;
}

ps_status ps_expm_dd(int64_t n, const double* A, int64_t lda, const double* coef, int m, int s, int sigma, double* E,
                     int64_t lde, const ps_opts* opts, ps_report* report, void* ws, size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (ps_status e = ps_workspace_size_dd(n, m, s, sigma, &need)) return e;
  if (s == 0) s = m <= 1 ? 1 : (int)std::ceil(std::sqrt((double)m) - 1e-12);
  if (!A || !E) return dfail(PS_ERR_ARG, "NULL matrix pointer");
  if (lda < n || lde < n) return dfail(PS_ERR_ARG, "leading dimension smaller than n");
  if (!coef && m > 170) return dfail(PS_ERR_ARG, "built-in Taylor coefficients need m <= 170");
  if (m / s + 1 > PS_MAX_BLOCKS) return dfail(PS_ERR_ARG, "too many blocks (m / s >= %d)", PS_MAX_BLOCKS);
  const size_t spanA = (size_t)(2 * lda * n) * 8, spanE = (size_t)(2 * lde * n) * 8;
  if (spans_overlap(A, spanA, E, spanE)) return dfail(PS_ERR_ALIAS, "output overlaps the input matrix");
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need)
    return dfail(PS_ERR_WORKSPACE, "workspace NULL, misaligned or smaller than %zu bytes", need);
  if (spans_overlap(ws, need, E, spanE) || spans_overlap(ws, need, A, spanA))
    return dfail(PS_ERR_ALIAS, "workspace overlaps a matrix argument");
  const int mode = opts ? opts->mode : PS_MODE_FIXED;
  if (mode != PS_MODE_FIXED && mode != PS_MODE_MIXED) return dfail(PS_ERR_ARG, "opts.mode must be 0 or 1");
  if (opts && opts->tier_override) return dfail(PS_ERR_UNSUPPORTED, "tier_override is not supported by ps_expm_dd");
  if (opts && opts->check_finite) return dfail(PS_ERR_UNSUPPORTED, "check_finite is not supported by ps_expm_dd");
  if (opts && opts->rule != PS_RULE_BLOCKS) return dfail(PS_ERR_UNSUPPORTED, "ps_expm_dd plans from the block norms only");
  const unsigned mask = ((opts && opts->tier_mask) ? opts->tier_mask : 0xFu) & 0xFu;
  const double delta = (opts && opts->delta > 0) ? opts->delta : 10.0;
  hipStream_t st = (hipStream_t)stream;
  Layout L = dd_layout(n, m, s, sigma);
  char* W = (char*)ws;
  const int64_t plane = n * n;
  auto slot = [&](size_t off) { return W + off; };
  // coefficients (double-double) into the workspace
  std::vector<double> ch(m + 1), cl(m + 1);
  if (coef) {
    for (int k = 0; k <= m; ++k) {
      ch[k] = coef[k];
      cl[k] = coef[m + 1 + k];
    }
  } else {
    taylor_dd(m, ch.data(), cl.data());
  }
  std::vector<double> cbuf(2 * (m + 1));
  std::copy(ch.begin(), ch.end(), cbuf.begin());
  std::copy(cl.begin(), cl.end(), cbuf.begin() + m + 1);
  double* dcoef = (double*)slot(L.off_coef);
  hipError_t he = hipMemcpyAsync(dcoef, cbuf.data(), cbuf.size() * 8, hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);   // the host buffer is released on return
  if (he != hipSuccess) return dfail(PS_ERR_HIP, "coefficient upload: %s", hipGetErrorString(he));
  const double beta = ldexp(1.0, -sigma);
  const DDMat X1{A, lda, lda * n};
  auto power = [&](int j) { return DDMat{(const double*)slot(L.off_pow + (size_t)(j - 2) * L.slot), n, plane}; };
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  const dim3 tiles(ntm * ntn), blk(NT);
  // 1. powers X_j = X_a X_b (a = ceil(j/2), b = floor(j/2)), X_1 = beta A
  for (int j = 2; j <= s; ++j) {
    const int pa = pow_a(j), pb = pow_b(j);
    const double alpha = (pa == 1 ? beta : 1.0) * (pb == 1 ? beta : 1.0);
    double* C = (double*)slot(L.off_pow + (size_t)(j - 2) * L.slot);
    hipLaunchKernelGGL(k_gemm_dd, tiles, blk, 0, st, n, pa == 1 ? X1 : power(pa), alpha, pb == 1 ? X1 : power(pb), C,
                       n, plane);
  }
  // 2. blocks, norms, Y copies
  AssembleDD aa;
  memset(&aa, 0, sizeof aa);
  aa.n = n;
  aa.m = m;
  aa.s = s;
  aa.r = L.r;
  aa.nB = L.nB;
  aa.trivial_last = L.trivial_last;
  aa.X1 = X1;
  aa.beta = beta;
  aa.ws = W;
  aa.L = L;
  aa.chi = dcoef;
  aa.clo = dcoef + m + 1;
  aa.tier_mask = mode == PS_MODE_MIXED ? mask : 0u;
  // Y for s = 1 is X_1 = beta A: the assembly reads it through x_1
  hipLaunchKernelGGL(k_assemble_dd, dim3((unsigned)((n + NW - 1) / NW), (unsigned)((n + kRowChunk - 1) / kRowChunk)),
                     blk, 0, st, aa);
  // 3. plan (working tier double-double)
  PlanArgs pa;
  memset(&pa, 0, sizeof pa);
  pa.r = L.r;
  pa.mode = mode;
  pa.working = kTierDD;
  pa.nB = L.nB;
  pa.trivial_last = L.trivial_last;
  pa.mask = mask;
  pa.delta = delta;
  pa.abs_cm = std::fabs(ch[m]);
  pa.ws = W;
  pa.ws_stride = 0;
  pa.L = L;
  if (hipError_t e = launch_plan(pa, 1, st)) return dfail(PS_ERR_HIP, "plan launch: %s", hipGetErrorString(e));
  // 4. Horner
  const bool square = sigma > 0;
  HornerDD h;
  memset(&h, 0, sizeof h);
  h.n = n;
  h.L = L;
  h.ws = W;
  if (s == 1) {
    h.Y = X1;
    h.yscale = beta;
  } else {
    h.Y = power(s);
    h.yscale = 1.0;
  }
  h.out = square ? (double*)slot(L.off_R) : E;
  h.ldo = square ? n : lde;
  h.oplane = square ? plane : lde * n;
  const int i0 = L.first_step;
  h.cast_only = 1;
  h.step = i0;
  h.final_out = (i0 == 0);
  h.off_bsrc = L.off_B + (size_t)i0 * L.slot;
  h.off_pout = L.off_P0;
  hipLaunchKernelGGL(k_horner_dd, tiles, blk, 0, st, h);
  h.cast_only = 0;
  for (int i = i0; i >= 1; --i) {
    const int k = i0 - i;
    h.step = i;
    h.final_out = (i == 1);
    h.off_pin = (k & 1) ? L.off_P1 : L.off_P0;
    h.off_pout = (k & 1) ? L.off_P0 : L.off_P1;
    h.off_bsrc = L.off_B + (size_t)(i - 1) * L.slot;
    hipLaunchKernelGGL(k_horner_dd, tiles, blk, 0, st, h);
  }
  // 5. squarings in double-double
  if (square) {
    double* bufs[2] = {(double*)slot(L.off_R), (double*)slot(L.off_P0)};
    for (int q = 1; q <= sigma; ++q) {
      const DDMat src{bufs[(q - 1) & 1], n, plane};
      double* dst = (q == sigma) ? E : bufs[q & 1];
      hipLaunchKernelGGL(k_gemm_dd, tiles, blk, 0, st, n, src, 1.0, src, dst, q == sigma ? lde : n,
                         q == sigma ? lde * n : plane);
    }
  }
  he = hipGetLastError();
  if (he != hipSuccess) return dfail(PS_ERR_HIP, "launch: %s", hipGetErrorString(he));
  if (report) {
    Plan pl;
    he = hipMemcpyAsync(&pl, slot(L.off_plan), sizeof pl, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return dfail(PS_ERR_HIP, "report: %s", hipGetErrorString(he));
    memset(report, 0, sizeof *report);
    report->s = L.s;
    report->r = L.r;
    report->nu = pl.nu;
    report->first_step = L.first_step;
    for (int i = 0; i <= L.r; ++i) {
      report->tier[i] = pl.tier[i];
      report->u[i] = pl.u[i];
      report->normB[i] = pl.normB[i];
    }
    report->normY = pl.normY;
    report->normX = pl.normX;
    (void)ps_model_cost(PS_DD, L.s, L.r, pl.tier, &report->cost_saving, &report->m_low);
  }
  return PS_OK;
}

}  // extern "C"
