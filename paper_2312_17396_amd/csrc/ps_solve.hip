// Linear solve Q X = P with a dense square Q (section 4.1 forms the Pade
// approximant as r_km = q_km^{-1} p_km; the PS scheme gives p_km and q_km and
// this solve gives the quotient).  LU factorisation with partial pivoting,
// right-looking and blocked by panels, on the augmented matrix [Q | P]: the
// panel's row exchanges, its triangular solve and its trailing update are
// applied to P's columns as well, so that after the last panel P holds
// L^{-1} Pi P and only the back substitution with U remains.
//
// Kernels (working type T = double or float):
//   k_lu_panel       one workgroup (256 threads up to 256 rows, 512 up to
//                    2048 rows, 1024 above) factors the (n - k0) x nb panel
//                    held in registers (thread t owns rows k0 + t + NT q);
//                    per column a workgroup arg-max picks the pivot (largest
//                    |entry|, lowest row on ties), the two rows are exchanged
//                    through LDS, the multipliers are formed by division and
//                    the rank-one update stays in registers.  It also writes
//                    the panel's exchanges as one gather list (<= 2 nb rows).
//   k_lu_swap_trsm   one wave per column outside the panel (Q's and P's):
//                    the gather list applied in one load/store round, then,
//                    right of the panel, the unit-lower triangular solve with
//                    the panel's L11 (lanes = rows, shuffles for the pivots).
//   k_lu_update      C -= A B with K <= 32 (panels) or 64 (back
//                    substitution, LDS sized for each) for 64 x 64 tiles of C, 256
//                    threads, FMA in the working type (HBM bound: every C
//                    element is read and written once per panel).
//   k_lu_trsm_upper  back substitution with a <= 64-row diagonal block of U,
//                    one wave per right-hand side.
// Panel width: 24 (FP64) or 32 (FP32) columns while at most 1024 rows are
// left, then 16, 8 and 4 columns up to 2048, 4096 and 8192 rows (the
// largest order), so that a thread's rows fit its registers.
#include <hip/hip_runtime.h>

#include "ps_internal.h"

namespace psk {
namespace {

constexpr int kPanelThreads = 1024;
constexpr int kListMax = 64;   // rows touched by one panel's exchanges (2 nb)

__global__ void k_fill_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <typename T, int R, int NB, int NT>
__global__ __launch_bounds__(NT) void k_lu_panel(T* __restrict__ Q, int64_t ld, int n, int k0,
                                                int* __restrict__ piv, int* __restrict__ list,
                                                int* __restrict__ info) {
  constexpr int NW = NT / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (n - k0 > R * NT || n <= k0) return;   // the host never launches this
  const int nbe = min(NB, n - k0);
  __shared__ double s_val[NW];
  __shared__ int s_row[NW];
  __shared__ T s_prow[NB], s_krow[NB];
  __shared__ int s_piv[NB];

  T a[R][NB];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int row = k0 + t + q * NT;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
      a[q][jj] = (row < n && jj < nbe) ? Q[row + (int64_t)(k0 + jj) * ld] : T(0);
  }

  int first_zero = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nbe) {
      const int kk = k0 + j;
      // pivot: largest |a(row, j)| over rows >= kk, lowest row on ties
      double bv = -1.0;
      int br = kk;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int row = k0 + t + q * NT;
        if (row >= kk && row < n) {
          const double v = fabs((double)a[q][j]);
          if (v > bv) { bv = v; br = row; }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int orow = __shfl_xor(br, off, 64);
        if (ov > bv || (ov == bv && orow < br)) { bv = ov; br = orow; }
      }
      if (lane == 0) { s_val[w] = bv; s_row[w] = br; }
      __syncthreads();
      double pv = s_val[0];
      int p = s_row[0];
      for (int u = 1; u < NW; ++u) {
        const double v = s_val[u];
        const int rr = s_row[u];
        if (v > pv || (v == pv && rr < p)) { pv = v; p = rr; }
      }
      // exchange rows kk (thread j, slot 0) and p (thread pt, slot pq) through LDS
      const int pt = (p - k0) % NT, pq = (p - k0) / NT;
      if (t == pt) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (q == pq) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) s_prow[jj] = a[q][jj];
          }
      }
      if (t == j && p != kk) {
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) s_krow[jj] = a[0][jj];
      }
      __syncthreads();
      if (t == pt && p != kk) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (q == pq) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) a[q][jj] = s_krow[jj];
          }
      }
      if (t == j) {
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) a[0][jj] = s_prow[jj];
      }
      const T d = s_prow[j];
      if (t == 0) {
        s_piv[j] = p;
        if (d == T(0) && first_zero == 0) first_zero = kk + 1;
      }
      // multipliers and the rank-one update of the panel's remaining columns
      if (d != T(0)) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int row = k0 + t + q * NT;
          if (row > kk && row < n) {
            const T l = a[q][j] / d;
            a[q][j] = l;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj)
              if (jj > j) a[q][jj] -= l * s_prow[jj];
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int row = k0 + t + q * NT;
    if (row < n) {
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < nbe) Q[row + (int64_t)(k0 + jj) * ld] = a[q][jj];
    }
  }
  __syncthreads();   // s_piv (written by thread 0) is read by all of wave 0
  // the panel's exchanges as one gather: new row pos <- old row org, one
  // touched row per lane of wave 0 (rows k0 .. k0 + nbe - 1 in lanes 0 ..
  // nbe - 1, then each pivot row from below the panel's block)
  if (w == 0) {
    if (lane < nbe) piv[k0 + lane] = s_piv[lane];
    int pos = lane < nbe ? k0 + lane : -1;
    int org = pos;
    int cnt = nbe;
    for (int j = 0; j < nbe; ++j) {
      const int p = s_piv[j];
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

template <typename T>
__global__ __launch_bounds__(256) void k_lu_swap_trsm(T* __restrict__ Q, int64_t ldq, T* __restrict__ P, int64_t ldp,
                                                      int n, int k0, int nbe, int nrhs, const int* __restrict__ list) {
  __shared__ T Ls[32][33];   // Ls[j][i] = L(k0 + i, k0 + j)
  __shared__ int s_pos[kListMax], s_org[kListMax];
  __shared__ int s_cnt;
  const int t = threadIdx.x, lane = t & 63;
  if (t == 0) s_cnt = list[0];
  if (t < kListMax) { s_pos[t] = list[1 + t]; s_org[t] = list[1 + kListMax + t]; }
  for (int idx = t; idx < nbe * nbe; idx += 256) {
    const int i = idx % nbe, j = idx / nbe;
    Ls[j][i] = Q[(k0 + i) + (int64_t)(k0 + j) * ldq];
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
      const T xj = __shfl(x, j, 64);
      if (lane > j && lane < nbe) x -= Ls[j][lane] * xj;
    }
  }
  if (lane < cnt) c[s_pos[lane]] = x;
}

struct UpdSeg {
  void* M;
  int64_t ld, col0, ncols;
};

// C(r, col) -= sum_k A(r, ac0 + k) B(kb0 + k, col) for rows r in [cr0, cr1);
// C and B are the segment's matrix, columns col0 .. col0 + ncols - 1.
template <typename T, int KMAX>
__global__ __launch_bounds__(256) void k_lu_update(const T* __restrict__ A, int64_t lda, int ac0, int K, int kb0,
                                                   int cr0, int cr1, UpdSeg s0, UpdSeg s1, int tiles0) {
  __shared__ T As[KMAX][64];   // As[k][i]
  __shared__ T Bs[KMAX][64];   // Bs[k][c]
  const int t = threadIdx.x;
  const int ct = blockIdx.y;
  const UpdSeg S = ct < tiles0 ? s0 : s1;
  const int64_t c0 = (int64_t)(ct < tiles0 ? ct : ct - tiles0) * 64;
  const int r0 = cr0 + blockIdx.x * 64;
  T* M = (T*)S.M;
  for (int idx = t; idx < 64 * K; idx += 256) {
    const int k = idx >> 6, i = idx & 63;
    const int r = r0 + i;
    As[k][i] = r < cr1 ? A[r + (int64_t)(ac0 + k) * lda] : T(0);
  }
  for (int idx = t; idx < 64 * K; idx += 256) {
    const int cc = idx / K, k = idx - cc * K;
    const int64_t col = c0 + cc;
    Bs[k][cc] = col < S.ncols ? M[(kb0 + k) + (S.col0 + col) * S.ld] : T(0);
  }
  __syncthreads();
  const int i = t & 63, cg = (t >> 6) * 16;
  T acc[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) acc[cc] = T(0);
  for (int k = 0; k < K; ++k) {
    const T av = As[k][i];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc[cc] = fma(av, Bs[k][cg + cc], acc[cc]);
  }
  const int r = r0 + i;
  if (r < cr1) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int64_t col = c0 + cg + cc;
      if (col < S.ncols) {
        T* ptr = M + r + (S.col0 + col) * S.ld;
        *ptr = *ptr - acc[cc];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_lu_trsm_upper(const T* __restrict__ Q, int64_t ldq, T* __restrict__ P,
                                                       int64_t ldp, int k0, int b, int nrhs) {
  __shared__ T Us[64][65];   // Us[j][i] = U(k0 + i, k0 + j)
  const int t = threadIdx.x, lane = t & 63;
  for (int idx = t; idx < b * b; idx += 256) {
    const int i = idx % b, j = idx / b;
    Us[j][i] = Q[(k0 + i) + (int64_t)(k0 + j) * ldq];
  }
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 4 + (t >> 6);
  if (col >= nrhs) return;
  T* c = P + col * ldp;
  T x = lane < b ? c[k0 + lane] : T(0);
  for (int j = b - 1; j >= 0; --j) {
    if (lane == j) x = x / Us[j][j];
    const T xj = __shfl(x, j, 64);
    if (lane < j) x -= Us[j][lane] * xj;
  }
  if (lane < b) c[k0 + lane] = x;
}

template <typename T>
hipError_t lu_solve_t(int n, T* Q, int64_t ldq, int nrhs, T* P, int64_t ldp, int* piv, int* info, int* list,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, info, 0);
  for (int k0 = 0; k0 < n;) {
    const int rem = n - k0;
    int nb;
    // 32 doubles per thread leave no room under the 128-VGPR limit of a
    // 1024-thread workgroup (the compiler moves the array to scratch)
    constexpr int NB1 = sizeof(T) == 8 ? 24 : 32;
    if (rem <= 256) {
      nb = NB1;
      hipLaunchKernelGGL((k_lu_panel<T, 1, NB1, 256>), dim3(1), dim3(256), 0, st, Q, ldq, n, k0, piv, list, info);
    } else if (rem <= 512) {
      nb = NB1;
      hipLaunchKernelGGL((k_lu_panel<T, 1, NB1, 512>), dim3(1), dim3(512), 0, st, Q, ldq, n, k0, piv, list, info);
    } else if (rem <= kPanelThreads) {
      // FP64: fewer waves per barrier, 512 threads with two rows each (64
      // FP32 values per thread would go to scratch: 1024 threads there)
      nb = NB1;
      if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL((k_lu_panel<T, 2, NB1, 512>), dim3(1), dim3(512), 0, st, Q, ldq, n, k0, piv, list, info);
      else
        hipLaunchKernelGGL((k_lu_panel<T, 1, NB1, kPanelThreads>), dim3(1), dim3(kPanelThreads), 0, st, Q, ldq, n,
                           k0, piv, list, info);
    } else if (rem <= 2 * kPanelThreads) {
      nb = 16;
      hipLaunchKernelGGL((k_lu_panel<T, 4, 16, 512>), dim3(1), dim3(512), 0, st, Q, ldq, n, k0, piv, list, info);
    } else if (rem <= 4 * kPanelThreads) {
      nb = 8;
      hipLaunchKernelGGL((k_lu_panel<T, 4, 8, kPanelThreads>), dim3(1), dim3(kPanelThreads), 0, st, Q, ldq, n, k0,
                         piv, list, info);
    } else {
      nb = 4;
      hipLaunchKernelGGL((k_lu_panel<T, 8, 4, kPanelThreads>), dim3(1), dim3(kPanelThreads), 0, st, Q, ldq, n, k0,
                         piv, list, info);
    }
    const int nbe = nb < rem ? nb : rem;
    const int64_t cols = (int64_t)n - nbe + nrhs;   // every column outside the panel
    if (cols > 0)
      hipLaunchKernelGGL(k_lu_swap_trsm<T>, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, st, Q, ldq, P, ldp, n,
                         k0, nbe, nrhs, (const int*)list);
    const int r1 = k0 + nbe;
    if (r1 < n) {
      UpdSeg s0{Q, ldq, r1, n - r1}, s1{P, ldp, 0, nrhs};
      const int t0 = (n - r1 + 63) / 64, t1 = (nrhs + 63) / 64;
      hipLaunchKernelGGL((k_lu_update<T, 32>), dim3((n - r1 + 63) / 64, t0 + t1), dim3(256), 0, st, (const T*)Q, ldq, k0,
                         nbe, k0, r1, n, s0, s1, t0);
    }
    k0 += nbe;
  }
  if (nrhs > 0) {
    for (int kb = (n - 1) / 64; kb >= 0; --kb) {
      const int k0 = kb * 64, b = (n - k0) < 64 ? (n - k0) : 64;
      hipLaunchKernelGGL(k_lu_trsm_upper<T>, dim3((nrhs + 3) / 4), dim3(256), 0, st, (const T*)Q, ldq, P, ldp, k0, b,
                         nrhs);
      if (k0 > 0) {
        UpdSeg s0{P, ldp, 0, nrhs}, s1{nullptr, 0, 0, 0};
        const int t0 = (nrhs + 63) / 64;
        hipLaunchKernelGGL((k_lu_update<T, 64>), dim3((k0 + 63) / 64, t0), dim3(256), 0, st, (const T*)Q, ldq, k0, b, k0,
                           0, k0, s0, s1, t0);
      }
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
