// Linear solve Q X = P with a dense square Q (section 4.1 forms the Pade
// approximant as r_km = q_km^{-1} p_km; the PS scheme gives p_km and q_km and
// this solve gives the quotient).  LU factorisation with partial pivoting,
// right-looking and blocked by panels, on the augmented matrix [Q | P]: the
// panel's row exchanges, its triangular solve and its trailing update are
// applied to P's columns as well, so that after the last panel P holds
// L^{-1} Pi P and only the back substitution with U remains.
//
// Kernels (working type T = double or float):
//   k_lu_panel       one workgroup (256 threads up to 256 rows, 512 above;
//                    FP32: 1024 from 513 to 1024 and above 2048 rows) factors
//                    the (n - k0) x nb panel
//                    held in registers (thread t owns rows k0 + t + NT q);
//                    per column a DPP wave arg-max and one barrier pick the
//                    pivot (largest |entry|, lowest position on ties); rows
//                    never move in the registers (each keeps its current
//                    position, and goes there when the panel is stored), the
//                    pivot row is read from the winning wave's LDS copy, the
//                    multipliers are formed by division and the rank-one
//                    update stays in registers.  It also writes the panel's
//                    exchanges as one gather list (<= 2 nb rows).
//   k_lu_swap_trsm   one wave per column outside the panel (Q's and P's):
//                    the gather list applied in one load/store round, then,
//                    right of the panel, the unit-lower triangular solve with
//                    the panel's L11 (lanes = rows, lane reads for the pivots).
//   k_lu_step        one launch per panel after the first: block 0 applies
//                    the previous panel's trailing update to its own columns
//                    and factors it (as k_lu_panel), the other blocks apply
//                    that update, C -= L21 U12 with K <= 32, to the 64 x 64
//                    tiles of the other columns (FMA in the working type,
//                    C's loads issued first).
//   k_lu_backstep    one step of the back substitution: the update of the
//                    rows above a solved block row (K <= 64) on the FP64 /
//                    FP32 matrix cores in 64 x 64 tiles, and in the same
//                    launch the block row just above it updated and solved.
//   k_lu_trsm_upper  back substitution with a <= 64-row diagonal block of U,
//                    one wave per right-hand side, multiplying by the
//                    reciprocals of U's diagonal (formed once per block).
// Panel width: 24 (FP64) or 32 (FP32) columns while at most 1024 rows are
// left, then 16, 8 and 4 columns up to 2048, 4096 and 8192 rows (the
// largest order), so that a thread's rows fit its registers (FP64 panels of
// more than 2048 rows on 512 threads, eight or sixteen rows each).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ps_internal.h"

namespace psk {
namespace {

constexpr int kPanelThreads = 1024;
constexpr int kListMax = 64;   // rows touched by one panel's exchanges (2 nb)

__global__ void k_fill_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// DPP controls (gfx9 encoding): row_shr:k = 0x110 + k, row_bcast:15 =
// 0x142, row_bcast:31 = 0x143.  The 64-bit value moves as two 32-bit halves.
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ double dpp_f64(double old, double src) {
  const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, ROWM, BANKM, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, ROWM, BANKM, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The largest value over the wave (operands not NaN), returned to every lane:
// row shifts build each row's maximum in its lane 15, the two row
// broadcasts carry it to lane 63, which is then read.
__device__ __forceinline__ double wave_max_f64(double x) {
  x = fmax(x, dpp_f64<0x111, 0xf, 0xf>(x, x));
  x = fmax(x, dpp_f64<0x112, 0xf, 0xf>(x, x));
  x = fmax(x, dpp_f64<0x113, 0xf, 0xf>(x, x));
  x = fmax(x, dpp_f64<0x114, 0xf, 0xe>(x, x));
  x = fmax(x, dpp_f64<0x118, 0xf, 0xc>(x, x));
  x = fmax(x, dpp_f64<0x142, 0xa, 0xf>(x, x));
  x = fmax(x, dpp_f64<0x143, 0xc, 0xf>(x, x));
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename T, int NW, int NB>
struct PanelLds {
  double val[2][NW];   // each wave's candidate |value| (-1: none), by column parity
  int pos[2][NW];      // its position
  int who[2][NW];      // its lane * 8 + slot
  T wrow[2][NW][NB];   // its row, columns j .. NB-1
  int piv[NB];
};

// Column j of the panel (a compile-time constant, so that the register array
// keeps constant indices).  No row moves in the registers: slot q of thread t
// holds one row throughout, ps[q] is its current position (the exchanges of
// partial pivoting permute positions) and bit q of `done` marks a row already
// used as a pivot.  One barrier per column (the LDS areas alternate with the
// column's parity): every wave stages its best row, then every thread picks
// the winner from the NW candidates and reads the pivot row from LDS.
template <typename T, int R, int NB, int NT, int j>
__device__ __forceinline__ void panel_column(T (&a)[R][NB], int (&ps)[R], unsigned& done,
                                             PanelLds<T, NT / 64, NB>& S, int k0, int nbe, int t, int lane, int w,
                                             int& first_zero) {
  if constexpr (j < NB) {
    if (j < nbe) {
      constexpr int NW = NT / 64, b = j & 1;
      const int kk = k0 + j;
      // this thread's best active row: largest |a| (a NaN below every
      // number), the lowest position on ties
      double bv = -1.0;
      int bp = 0x7fffffff, bq = 0;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double x = fabs((double)a[q][j]);
        const double v = ((done >> q) & 1u) ? -1.0 : ((x == x) ? x : -0.5);
        const bool take = (v > bv) | ((v == bv) & (ps[q] < bp));
        bv = take ? v : bv;
        bp = take ? ps[q] : bp;
        bq = take ? q : bq;
      }
      // the wave's best: its largest value, then the lowest position among
      // the lanes that hold it
      const double wv = wave_max_f64(bv);
      int wl = 0, wp = 0x7fffffff;
      if (wv >= -0.5) {
        unsigned long long m = __ballot(bv == wv);
        wl = __ffsll((long long)m) - 1;
        wp = __builtin_amdgcn_readlane(bp, wl);
        m &= m - 1;
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          const int p2 = __builtin_amdgcn_readlane(bp, l);
          if (p2 < wp) { wp = p2; wl = l; }
          m &= m - 1;
        }
      }
      const int wq = __builtin_amdgcn_readlane(bq, wl);
      if (lane == wl) {
        if (wv >= -0.5) {
#pragma unroll
          for (int jj = j; jj < NB; ++jj) {
            T v = a[0][jj];
#pragma unroll
            for (int q = 1; q < R; ++q) {
              T x = a[q][jj];
              // an empty asm keeps the choice a select of values: otherwise
              // the compiler folds the selects into one load at a variable
              // index and moves the whole register array to scratch memory
              asm volatile("" : "+v"(x));
              v = (wq == q) ? x : v;
            }
            S.wrow[b][w][jj] = v;
          }
        }
        S.val[b][w] = wv;
        S.pos[b][w] = wp;
        S.who[b][w] = wl * 8 + wq;
      }
      __syncthreads();
      double cv[NW];
      int cp[NW], cw[NW];
#pragma unroll
      for (int u = 0; u < NW; ++u) { cv[u] = S.val[b][u]; cp[u] = S.pos[b][u]; cw[u] = S.who[b][u]; }
      double pv = cv[0];
      int p = cp[0], ws = 0, who = cw[0];
#pragma unroll
      for (int u = 1; u < NW; ++u) {
        const bool take = (cv[u] > pv) | ((cv[u] == pv) & (cp[u] < p));
        pv = take ? cv[u] : pv;
        p = take ? cp[u] : p;
        ws = take ? u : ws;
        who = take ? cw[u] : who;
      }
      p = __builtin_amdgcn_readfirstlane(p);
      ws = __builtin_amdgcn_readfirstlane(ws);
      who = __builtin_amdgcn_readfirstlane(who);
      const int xl = who >> 3, xq = who & 7;
      // the exchange of positions kk and p; the pivot row retires
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (ps[q] == kk) ps[q] = p;
      if (w == ws && lane == xl) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (q == xq) { ps[q] = kk; done |= 1u << q; }
      }
      const T d = S.wrow[b][ws][j];
      if (t == 0) {
        S.piv[j] = p;
        if (d == T(0) && first_zero == 0) first_zero = kk + 1;
      }
      // multipliers and the rank-one update of the active rows
      if (d != T(0)) {
        T pr[NB];
#pragma unroll
        for (int jj = j + 1; jj < NB; ++jj) pr[jj] = S.wrow[b][ws][jj];
        T l[R];
#pragma unroll
        for (int q = 0; q < R; ++q) l[q] = a[q][j] / d;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          if (!((done >> q) & 1u)) {
            a[q][j] = l[q];
#pragma unroll
            for (int jj = j + 1; jj < NB; ++jj) a[q][jj] -= l[q] * pr[jj];
          }
        }
      }
    }
    panel_column<T, R, NB, NT, j + 1>(a, ps, done, S, k0, nbe, t, lane, w, first_zero);
  }
}

// The factorisation of the panel at column k0 by one workgroup of NT threads.
// Kp > 0: the panel's columns first take the trailing update of the previous
// panel (at kp = k0 - Kp): a -= L21 U12 with the sum over k formed as the
// update tiles of k_lu_step form it (a fused multiply-add chain from k = 0,
// then one subtraction).
template <typename T, int R, int NB, int NT>
__device__ __forceinline__ void panel_factor(T* __restrict__ Q, int64_t ld, int n, int k0, int* __restrict__ piv,
                                             int* __restrict__ list, int* __restrict__ info, int Kp) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbe = min(NB, n - k0);
  __shared__ PanelLds<T, NT / 64, NB> S;
  __shared__ T Us[32][NB];   // U12 of the previous panel, restricted to this panel's columns
  T a[R][NB];
  int ps[R];
  unsigned done = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int row = k0 + t + q * NT;
    ps[q] = row;
    if (row >= n) done |= 1u << q;   // no such row: never a candidate, never stored
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
      a[q][jj] = (row < n && jj < nbe) ? Q[row + (int64_t)(k0 + jj) * ld] : T(0);
  }
  if (Kp > 0) {
    const int kp = k0 - Kp;
    constexpr int UQ = (32 * NB + NT - 1) / NT;   // U12 elements per thread (Kp <= 32)
    T ru[UQ];
#pragma unroll
    for (int q = 0; q < UQ; ++q) {
      const int idx = t + NT * q;
      const int k = idx / NB, jj = idx - k * NB;
      ru[q] = (k < Kp && jj < nbe) ? Q[(kp + k) + (int64_t)(k0 + jj) * ld] : T(0);
    }
#pragma unroll
    for (int q = 0; q < UQ; ++q) {
      const int idx = t + NT * q;
      if (idx < 32 * NB) Us[idx / NB][idx % NB] = ru[q];
    }
    __syncthreads();
    // eight k at a time: the row's eight L21 loads are issued together (a
    // zero beyond Kp, whose product with U12's zero leaves the sum as it is:
    // the sums start at +0 and never become -0)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int row = k0 + t + q * NT;
      if (row < n) {
        T acc[NB];
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) acc[jj] = T(0);
        for (int kc = 0; kc < Kp; kc += 8) {
          T lk[8];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) lk[kk] = (kc + kk < Kp) ? Q[row + (int64_t)(kp + kc + kk) * ld] : T(0);
#pragma unroll
          for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) acc[jj] = fma(lk[kk], Us[kc + kk][jj], acc[jj]);
        }
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) a[q][jj] = a[q][jj] - acc[jj];
      }
    }
  }
  const unsigned valid = ~done;
  int first_zero = 0;
  panel_column<T, R, NB, NT, 0>(a, ps, done, S, k0, nbe, t, lane, w, first_zero);
  // each row to its final position
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (((valid >> q) & 1u) && ps[q] >= k0 && ps[q] < n) {
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < nbe) Q[ps[q] + (int64_t)(k0 + jj) * ld] = a[q][jj];
    }
  }
  __syncthreads();   // S.piv (written by thread 0) is read by all of wave 0
  // the panel's exchanges as one gather: new row pos <- old row org, one
  // touched row per lane of wave 0 (rows k0 .. k0 + nbe - 1 in lanes 0 ..
  // nbe - 1, then each pivot row from below the panel's block)
  if (w == 0) {
    if (lane < nbe) piv[k0 + lane] = S.piv[lane];
    int pos = lane < nbe ? k0 + lane : -1;
    int org = pos;
    int cnt = nbe;
    for (int j = 0; j < nbe; ++j) {
      const int p = S.piv[j];
      if (p == k0 + j) continue;
      const unsigned long long hit = __ballot(pos == p);
      int idx;
      if (hit) {
        idx = __ffsll((long long)hit) - 1;
      } else {
        idx = cnt++;
        if (lane == idx) { pos = p; org = p; }
      }
      const int oj = __shfl(org, j, 64), oi = __shfl(org, idx, 64);
      if (lane == j) org = oi;
      if (lane == idx) org = oj;
    }
    if (lane < cnt) { list[1 + lane] = pos; list[1 + kListMax + lane] = org; }
    if (lane == 0) {
      list[0] = cnt;
      if (first_zero != 0 && *info == 0) *info = first_zero;
    }
  }
}

template <typename T, int R, int NB, int NT>
__global__ __launch_bounds__(NT) void k_lu_panel(T* __restrict__ Q, int64_t ld, int n, int k0,
                                                int* __restrict__ piv, int* __restrict__ list,
                                                int* __restrict__ info) {
  if (n - k0 > R * NT || n <= k0) return;   // the host never launches this
  panel_factor<T, R, NB, NT>(Q, ld, n, k0, piv, list, info, 0);
}

// lane j's x, for a wave-uniform j (a scalar read instead of a permute)
template <typename T>
__device__ __forceinline__ T lane_value(T x, int j) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong((double)x);
    const int lo = __builtin_amdgcn_readlane((int)b, j), hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
    return (T)__longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int((float)x), j));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_lu_swap_trsm(T* __restrict__ Q, int64_t ldq, T* __restrict__ P, int64_t ldp,
                                                      int n, int k0, int nbe, int nrhs, const int* __restrict__ list) {
  __shared__ T Ls[32][33];   // Ls[j][i] = L(k0 + i, k0 + j)
  __shared__ int s_pos[kListMax], s_org[kListMax];
  __shared__ int s_cnt;
  const int t = threadIdx.x, lane = t & 63;
  if (t == 0) s_cnt = list[0];
  if (t < kListMax) { s_pos[t] = list[1 + t]; s_org[t] = list[1 + kListMax + t]; }
  T rl[4];   // the panel's L11 (at most 32 x 32): loads first, then the stores
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + 256 * q;
    const int i = idx & 31, j = idx >> 5;
    rl[q] = (i < nbe && j < nbe) ? Q[(k0 + i) + (int64_t)(k0 + j) * ldq] : T(0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + 256 * q;
    Ls[idx >> 5][idx & 31] = rl[q];
  }
  __syncthreads();
  const int cnt = s_cnt;
  const int64_t nleft = k0, nright = n - k0 - nbe;
  const int64_t g = (int64_t)blockIdx.x * 4 + (t >> 6);
  if (g >= nleft + nright + nrhs) return;
  T* c;
  bool trsm = true;
  if (g < nleft) {
    c = Q + g * ldq;
    trsm = false;
  } else if (g < nleft + nright) {
    c = Q + (g - nleft + k0 + nbe) * ldq;
  } else {
    c = P + (g - nleft - nright) * ldp;
  }
  T x = T(0);
  if (lane < cnt) x = c[s_org[lane]];
  if (trsm) {
    for (int j = 0; j + 1 < nbe; ++j) {
      const T xj = lane_value(x, j);
      if (lane > j && lane < nbe) x -= Ls[j][lane] * xj;
    }
  }
  if (lane < cnt) c[s_pos[lane]] = x;
}

struct UpdSeg {
  void* M;
  int64_t ld, col0, ncols;
};


// One step of the factorisation in one launch: block 0 factors the next
// panel (at r1 = k0 + K, width nbn), first applying this step's trailing
// update to its own columns (panel_factor with Kp = K), while the other
// blocks apply the trailing update of the panel at k0 (C -= L21 U12 with
// K <= 32) to the 64 x 64 tiles of C outside the next panel's columns.  The
// two parts write disjoint columns, and both read only the columns of the
// panel at k0 (rows r1 and below) and the rows above r1, which this launch
// does not write; the exchange list that block 0 writes is read by the next
// launch only.
template <typename T, int R, int NB, int NT>
__global__ __launch_bounds__(NT) void k_lu_step(T* Q, int64_t ldq, int k0, int K, int cr1, int n, int nbn,
                                               UpdSeg s0, UpdSeg s1, int tiles0, int nrt, int ntiles,
                                               int* __restrict__ piv, int* __restrict__ list, int* __restrict__ info) {
  constexpr int CPT = 4096 / NT;   // columns of the tile per thread
  __shared__ T As[32][64];         // As[k][i]
  __shared__ T Bs[32][64];         // Bs[k][c]
  const int t = threadIdx.x;
  const int cr0 = k0 + K;
  if (blockIdx.x == 0) {
    panel_factor<T, R, NB, NT>(Q, ldq, n, cr0, piv, list, info, K);
    return;
  }
  const int idx = (int)blockIdx.x - 1;
  const int ct = idx / nrt, rt = idx % nrt;
  const UpdSeg S = ct < tiles0 ? s0 : s1;
  const int64_t c0 = (int64_t)(ct < tiles0 ? ct : ct - tiles0) * 64;
  const int64_t cskip = ct == 0 ? nbn : 0;   // the next panel's columns: block 0 updates them
  const int r0 = cr0 + rt * 64;
  T* M = (T*)S.M;
  const int i = t & 63, cg = (t >> 6) * CPT;
  const int r = r0 + i;
  T cv[CPT];
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int64_t col = c0 + cg + cc;
    cv[cc] = (r < cr1 && col < S.ncols && col >= cskip) ? M[r + (S.col0 + col) * S.ld] : T(0);
  }
  // the operands: every load issued before the first LDS store
  constexpr int AQ = 64 * 32 / NT;
  T ra[AQ], rb[AQ];
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const int idx2 = t + NT * q;
    const int k = idx2 >> 6, ii = idx2 & 63;
    const int rr = r0 + ii;
    ra[q] = (k < K && rr < cr1) ? Q[rr + (int64_t)(k0 + k) * ldq] : T(0);
    const int cc = idx2 / K, kb = idx2 - cc * K;
    const int64_t col = c0 + cc;
    rb[q] = (idx2 < 64 * K && col < S.ncols) ? M[(k0 + kb) + (S.col0 + col) * S.ld] : T(0);
  }
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const int idx2 = t + NT * q;
    if (idx2 < 64 * K) {
      As[idx2 >> 6][idx2 & 63] = ra[q];
      const int cc = idx2 / K, kb = idx2 - cc * K;
      Bs[kb][cc] = rb[q];
    }
  }
  __syncthreads();
  T acc[CPT];
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) acc[cc] = T(0);
  for (int k = 0; k < K; ++k) {
    const T av = As[k][i];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) acc[cc] = fma(av, Bs[k][cg + cc], acc[cc]);
  }
  if (r < cr1) {
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int64_t col = c0 + cg + cc;
      if (col < S.ncols && col >= cskip) M[r + (S.col0 + col) * S.ld] = cv[cc] - acc[cc];
    }
  }
}

// The back substitution's update C -= A B (C: rows [0, cr1) of P, A: the
// block column of U above the diagonal block, B: the block's solved rows of
// P, K <= 64) on the matrix cores: a 64 x 64 tile of C per 256-thread
// workgroup, each wave a 32 x 32 quadrant as 2 x 2 blocks of 16 x 16 x 4
// MFMAs (lane (g, c) = (lane / 16, lane % 16) feeds A[c][k = g] and B[k =
// g][c]; the FP64 product leaves D[4v + g][c], the FP32 one D[4g + v][c] in
// its v-th value), A and B staged whole in LDS with K padded by zeros to a
// multiple of 4, this lane's C elements loaded first.
typedef double lu_d4 __attribute__((ext_vector_type(4)));
typedef float lu_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct LuMma;
template <> struct LuMma<double> {
  typedef lu_d4 V;
  static __device__ inline V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int v, int g) { return 4 * v + g; }
};
template <> struct LuMma<float> {
  typedef lu_f4 V;
  static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int v, int g) { return 4 * g + v; }
};

// One 64 x 64 tile (rows r0.., columns c0..) of M -= A(:, ac0 .. ac0 + K)
// M(kb0 .. kb0 + K, :), rows below cr1 only.  As, Bs: 64 x 65 elements of
// LDS each: As[k][i] = A(r0 + i, ac0 + k), Bs[k][c] = M(kb0 + k, c0 + c).
template <typename T>
__device__ __forceinline__ void update_tile_mfma(const T* __restrict__ A, int64_t lda, int ac0, int K, int kb0,
                                                 int cr1, T* __restrict__ M, int64_t ldm, int64_t ncols, int r0,
                                                 int64_t c0, T (*As)[65], T (*Bs)[65]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c = lane & 15;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const int K4 = (K + 3) & ~3;
  // this lane's 16 elements of C
  T cv[2][2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr + 16 * mb + LuMma<T>::row(v, g);
        const int64_t col = c0 + wc + 16 * nb + c;
        cv[mb][nb][v] = (row < cr1 && col < ncols) ? M[row + col * ldm] : T(0);
      }
  // the operands: every load of a thread issued before the first LDS store
  // (a loop with a run-time trip count would wait for each load in turn)
  T ra[16], rb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    const int k = idx >> 6, i = idx & 63;
    const int row = r0 + i;
    ra[q] = (k < K && row < cr1) ? A[row + (int64_t)(ac0 + k) * lda] : T(0);
    const int cc = idx / K4, kb = idx - cc * K4;
    const int64_t col = c0 + cc;
    rb[q] = (idx < 64 * K4 && kb < K && col < ncols) ? M[(kb0 + kb) + col * ldm] : T(0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    if (idx < 64 * K4) {
      As[idx >> 6][idx & 63] = ra[q];
      const int cc = idx / K4, kb = idx - cc * K4;
      Bs[kb][cc] = rb[q];
    }
  }
  __syncthreads();
  typename LuMma<T>::V acc[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = typename LuMma<T>::V{0, 0, 0, 0};
  for (int k = 0; k < K4; k += 4) {
    const T a0 = As[k + g][wr + c], a1 = As[k + g][wr + 16 + c];
    const T b0 = Bs[k + g][wc + c], b1 = Bs[k + g][wc + 16 + c];
    acc[0][0] = LuMma<T>::mma(a0, b0, acc[0][0]);
    acc[0][1] = LuMma<T>::mma(a0, b1, acc[0][1]);
    acc[1][0] = LuMma<T>::mma(a1, b0, acc[1][0]);
    acc[1][1] = LuMma<T>::mma(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr + 16 * mb + LuMma<T>::row(v, g);
        const int64_t col = c0 + wc + 16 * nb + c;
        if (row < cr1 && col < ncols) M[row + col * ldm] = cv[mb][nb][v] - acc[mb][nb][v];
      }
}

template <typename T>
__global__ __launch_bounds__(256) void k_lu_trsm_upper(const T* __restrict__ Q, int64_t ldq, T* __restrict__ P,
                                                       int64_t ldp, int k0, int b, int nrhs) {
  __shared__ T Us[64][65];   // Us[j][i] = U(k0 + i, k0 + j)
  __shared__ T rd[64];       // 1 / U(k0 + j, k0 + j)
  const int t = threadIdx.x, lane = t & 63;
  // the block's loads all issued before the LDS stores
  T ru[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    const int i = idx & 63, j = idx >> 6;
    ru[q] = (i < b && j < b) ? Q[(k0 + i) + (int64_t)(k0 + j) * ldq] : T(0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    Us[idx >> 6][idx & 63] = ru[q];
  }
  if (t < b) rd[t] = T(1) / Q[(k0 + t) + (int64_t)(k0 + t) * ldq];
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 4 + (t >> 6);
  if (col >= nrhs) return;
  T* c = P + col * ldp;
  T x = lane < b ? c[k0 + lane] : T(0);
  for (int j = b - 1; j >= 0; --j) {
    const T xj = lane_value(x, j) * rd[j];
    if (lane == j) x = xj;
    if (lane < j) x -= Us[j][lane] * xj;
  }
  if (lane < b) c[k0 + lane] = x;
}

// One step of the back substitution in one launch.  X_k, rows k0 .. k0 + b - 1
// of P, is solved; the rows above take its update and the block above it,
// rows d0 = k0 - 64 .. k0 - 1, is solved too.  The first ndiag workgroups
// each take 16 right-hand sides of that block: its update by X_k, as the
// update tiles form it (the same MFMA chain over k for every element), then
// the substitution with its diagonal block of U, as k_lu_trsm_upper does it
// (one wave per four right-hand sides).  The other workgroups are the 64 x 64
// update tiles of the rows above d0.  The two parts write disjoint rows and
// read only X_k besides their own rows, so no workgroup waits for another,
// and the results are those of the update and substitution launches.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_backstep(const T* __restrict__ Q, int64_t ldq, T* __restrict__ P,
                                                     int64_t ldp, int k0, int b, int nrhs, int ndiag) {
  __shared__ T S[2][64][65];
  const int d0 = k0 - 64;
  if ((int)blockIdx.x >= ndiag) {
    const int idx = blockIdx.x - ndiag, nrt = d0 / 64;
    update_tile_mfma<T>(Q, ldq, k0, b, k0, d0, P, ldp, (int64_t)nrhs, (idx % nrt) * 64, (int64_t)(idx / nrt) * 64,
                        S[0], S[1]);
    return;
  }
  T (*Us)[65] = S[0];                      // Us[k][i] = Q(d0 + i, k0 + k), then Us[j][i] = Q(d0 + i, d0 + j)
  T (*Xs)[17] = (T (*)[17])&S[1][0][0];    // Xs[k][c] = P(k0 + k, c0 + c)
  T (*Cs)[17] = Xs + 64;                   // the block's rows after the update, Cs[i][c]
  T* rd = &Cs[64][0];                      // 1 / Q(d0 + j, d0 + j)
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, c = lane & 15;
  const int64_t c0 = (int64_t)blockIdx.x * 16;
  const int K4 = (b + 3) & ~3;
  // every load of a thread issued before the first LDS store
  T ru[16], rg[16], rx[4], cv[4];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    const int k = idx >> 6, i = idx & 63;
    ru[q] = k < b ? Q[(d0 + i) + (int64_t)(k0 + k) * ldq] : T(0);
    rg[q] = Q[(d0 + i) + (int64_t)(d0 + k) * ldq];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + 256 * q;
    const int k = idx >> 4, cc = idx & 15;
    rx[q] = (k < b && c0 + cc < nrhs) ? P[(k0 + k) + (c0 + cc) * ldp] : T(0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = d0 + 16 * w + LuMma<T>::row(v, g);
    cv[v] = c0 + c < nrhs ? P[row + (c0 + c) * ldp] : T(0);
  }
  const T rdd = t < 64 ? T(1) / Q[(d0 + t) + (int64_t)(d0 + t) * ldq] : T(0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    Us[idx >> 6][idx & 63] = ru[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = t + 256 * q;
    Xs[idx >> 4][idx & 15] = rx[q];
  }
  __syncthreads();
  // wave w: rows 16 w .. 16 w + 15 of the block
  typename LuMma<T>::V acc = typename LuMma<T>::V{0, 0, 0, 0};
  for (int k = 0; k < K4; k += 4) acc = LuMma<T>::mma(Us[k + g][16 * w + c], Xs[k + g][c], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) Cs[16 * w + LuMma<T>::row(v, g)][c] = cv[v] - acc[v];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q;
    Us[idx >> 6][idx & 63] = rg[q];
  }
  if (t < 64) rd[t] = rdd;
  __syncthreads();
  // wave w: right-hand sides 4 w .. 4 w + 3, lane = row
  T x[4];
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) x[cc] = Cs[lane][4 * w + cc];
  for (int j = 63; j >= 0; --j) {
    T xj[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) xj[cc] = lane_value(x[cc], j) * rd[j];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
      if (lane == j) x[cc] = xj[cc];
    if (lane < j) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) x[cc] -= Us[j][lane] * xj[cc];
    }
  }
#pragma unroll
  for (int cc = 0; cc < 4; ++cc)
    if (c0 + 4 * w + cc < nrhs) P[(d0 + lane) + (c0 + 4 * w + cc) * ldp] = x[cc];
}

// Launches the panel factorisation at k0 for `rem` rows left, alone
// (step == nullptr) or fused with the trailing update of the previous panel
// (k_lu_step); the panel shape (rows per thread R, width NB, threads NT) is
// chosen by dispatch_panel below.
template <typename T>
struct PanelLaunch {
  T* Q;
  int64_t ldq;
  int n, k0;
  int *piv, *list, *info;
  hipStream_t st;
  // fused step: the previous panel at kp (width K), its update segments
  bool fused;
  int kp, K, tiles0, nrt, ntiles;
  UpdSeg s0, s1;
  template <int R, int NB, int NT>
  void go() const {
    if (!fused)
      hipLaunchKernelGGL((k_lu_panel<T, R, NB, NT>), dim3(1), dim3(NT), 0, st, Q, ldq, n, k0, piv, list, info);
    else
      hipLaunchKernelGGL((k_lu_step<T, R, NB, NT>), dim3((unsigned)ntiles + 1), dim3(NT), 0, st, Q, ldq, kp, K, n,
                         n, std::min(NB, n - k0), s0, s1, tiles0, nrt, ntiles, piv, list, info);
  }
};

// Panel width: 24 (FP64) or 32 (FP32) columns while at most 1024 rows are
// left, then 16, 8 and 4 columns up to 2048, 4096 and 8192 rows.  Returns
// the width.
template <typename T>
int dispatch_panel(int rem, const PanelLaunch<T>& l) {
  // 32 doubles per thread leave no room under the 128-VGPR limit of a
  // 1024-thread workgroup (the compiler moves the array to scratch)
  constexpr int NB1 = sizeof(T) == 8 ? 24 : 32;
  if (rem <= 256) {
    l.template go<1, NB1, 256>();
    return NB1;
  }
  if (rem <= 512) {
    l.template go<1, NB1, 512>();
    return NB1;
  }
  if (rem <= kPanelThreads) {
    // FP64: fewer waves per barrier, 512 threads with two rows each (64
    // FP32 values per thread would go to scratch: 1024 threads there)
    if constexpr (sizeof(T) == 8) l.template go<2, NB1, 512>();
    else l.template go<1, NB1, kPanelThreads>();
    return NB1;
  }
  if (rem <= 2 * kPanelThreads) {
    l.template go<4, 16, 512>();
    return 16;
  }
  if (rem <= 4 * kPanelThreads) {
    // FP64: 512 threads with eight rows each (1024 threads leave 128
    // registers per lane, too few for the row positions and staging)
    if constexpr (sizeof(T) == 8) l.template go<8, 8, 512>();
    else l.template go<4, 8, kPanelThreads>();
    return 8;
  }
  if constexpr (sizeof(T) == 8) l.template go<16, 4, 512>();
  else l.template go<8, 4, kPanelThreads>();
  return 4;
}

template <typename T>
hipError_t lu_solve_t(int n, T* Q, int64_t ldq, int nrhs, T* P, int64_t ldp, int* piv, int* info, int* list,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, info, 0);
  PanelLaunch<T> l{};
  l.Q = Q;
  l.ldq = ldq;
  l.n = n;
  l.piv = piv;
  l.list = list;
  l.info = info;
  l.st = st;
  l.fused = false;
  l.k0 = 0;
  int nb = dispatch_panel<T>(n, l);
  for (int k0 = 0; k0 < n;) {
    const int rem = n - k0;
    const int nbe = nb < rem ? nb : rem;
    const int64_t cols = (int64_t)n - nbe + nrhs;   // every column outside the panel
    if (cols > 0)
      hipLaunchKernelGGL(k_lu_swap_trsm<T>, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, st, Q, ldq, P, ldp, n,
                         k0, nbe, nrhs, (const int*)list);
    const int r1 = k0 + nbe;
    if (r1 >= n) break;
    // the trailing update of this panel and the next panel's factorisation
    // in one launch
    l.fused = true;
    l.k0 = r1;
    l.kp = k0;
    l.K = nbe;
    l.s0 = UpdSeg{Q, ldq, r1, n - r1};
    l.s1 = UpdSeg{P, ldp, 0, nrhs};
    l.tiles0 = (n - r1 + 63) / 64;
    l.nrt = (n - r1 + 63) / 64;
    l.ntiles = l.nrt * (l.tiles0 + (nrhs + 63) / 64);
    nb = dispatch_panel<T>(n - r1, l);
    k0 = r1;
  }
  if (nrhs > 0) {
    // the last block row alone, then per block row its update of the rows
    // above fused with the substitution of the block row above it
    const int kl = (n - 1) / 64;
    hipLaunchKernelGGL(k_lu_trsm_upper<T>, dim3((nrhs + 3) / 4), dim3(256), 0, st, (const T*)Q, ldq, P, ldp, kl * 64,
                       n - kl * 64, nrhs);
    const int ndiag = (nrhs + 15) / 16, nct = (nrhs + 63) / 64;
    for (int kb = kl; kb >= 1; --kb) {
      const int k0 = kb * 64, b = (n - k0) < 64 ? (n - k0) : 64;
      hipLaunchKernelGGL(k_lu_backstep<T>, dim3((unsigned)(ndiag + (kb - 1) * nct)), dim3(256), 0, st, (const T*)Q,
                         ldq, P, ldp, k0, b, nrhs, ndiag);
    }
  }
  return hipGetLastError();
}

}  // namespace

size_t lu_solve_ws_bytes(int64_t n) {
  return 256 + (((size_t)(1 + 2 * kListMax) * 4 + 255) & ~(size_t)255) + (((size_t)n * 4 + 255) & ~(size_t)255);
}

hipError_t launch_lu_solve(int working, int64_t n, void* Q, int64_t ldq, int64_t nrhs, void* P, int64_t ldp,
                           int* piv_out, char* ws, hipStream_t st) {
  int* info = (int*)ws;
  int* list = (int*)(ws + 256);
  int* piv = piv_out ? piv_out : (int*)(ws + 256 + (((size_t)(1 + 2 * kListMax) * 4 + 255) & ~(size_t)255));
  if (working == 0)
    return lu_solve_t<double>((int)n, (double*)Q, ldq, (int)nrhs, (double*)P, ldp, piv, info, list, st);
  return lu_solve_t<float>((int)n, (float*)Q, ldq, (int)nrhs, (float*)P, ldp, piv, info, list, st);
}

}  // namespace psk
