// Device building blocks of the PS kernels, shared by the grid kernels
// (ps_kernels.hip) and the batched phase kernels (ps_batched.hip).
// Every function here works on one 64 x kTileN output tile, one column, or
// one matrix with the NT threads of a workgroup.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "ps_internal.h"
#include "ps_planner.h"

namespace psk {


typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

constexpr int NT = kTileM * kTileN / 8;  // threads per workgroup: one wave per 32x16 output block
                                         // (64x64 tiles: 8 waves, two per SIMD)
constexpr int NW = NT / 64;           // waves per workgroup
#ifndef PS_KCHAINS
#define PS_KCHAINS 2
#endif
#ifndef PS_BKL
#define PS_BKL 32
#endif
constexpr int BKL = PS_BKL;           // K slab of the LDS main loop
constexpr int LROWA = kTileM + 16;    // padded LDS rows (elements): a fragment read covers k-rows
constexpr int LROWB = kTileN + 16;    //   k and k+1 in one half-wave pass; 640 B (384 B) apart, the
                                      //   two rows land on disjoint banks
constexpr int KCH = PS_KCHAINS;       // independent accumulator chains per MFMA block (k-step parity)
constexpr int CSTR = kTileM + 1;      // epilogue tile column stride (elements)
constexpr int SLABA = BKL * LROWA;    // elements of the A slab of one stage
constexpr int SLABB = BKL * LROWB;    // elements of the B slab of one stage
constexpr int STAGE = SLABA + SLABB;
// LDS of one tile workgroup with working type W: two FP64/FP32 slab stages
// (80 KiB for FP64, 40 KiB for FP32, so up to four FP32 workgroups share a
// compute unit); the low-precision stages and the epilogue tile fit in it
template <typename W>
constexpr int smem_bytes() { return 2 * STAGE * (int)sizeof(W); }
constexpr int RUNA = BKL * kTileM / NT;      // consecutive elements each thread moves per slab
constexpr int RUNB = BKL * kTileN / NT;
constexpr int TPA = kTileM / RUNA;           // threads per k-row of a normal A slab
constexpr int TPB = kTileN / RUNB;           // threads per k-row of a transposed B slab
constexpr int TILE_Q = kTileM * kTileN / NT; // tile elements per thread in the epilogue passes (8)

static_assert(kTileM == 64 && kTileN == 64, "tile shape");
static_assert(RUNA % 2 == 0 && RUNB % 2 == 0 && TPA * RUNA == kTileM && TPB * RUNB == kTileN, "slab split");

// Wave layout of an output tile: wave w owns rows [32 (w & 1), +32) and
// columns [16 (w >> 1), +16) as two 16x16 MFMA blocks interleaved in M:
// block bi holds the rows wr + 2 r + bi (r = 0..15), so the two A values a
// lane feeds to the pair of MFMAs of one k-step are adjacent in LDS and come
// in one 2-element read.
__device__ inline int wave_row0() { return ((threadIdx.x >> 6) & 1) * 32; }
__device__ inline int wave_col0() { return (threadIdx.x >> 7) * 16; }

// ---------------------------------------------------------------------------
// tile scheduling: workgroups are dispatched round-robin over the 8 XCDs; each
// XCD is given a contiguous range of tiles, walked in groups of 4 tile-rows,
// so the workgroups sharing an L2 also share A row panels and B column panels.
// ---------------------------------------------------------------------------
__device__ inline void tile_of_block(int ntm, int ntn, int& tm, int& tn) {
  const int total = ntm * ntn;
  int bid = blockIdx.x;
  int t = bid;
  if ((total & 7) == 0) t = (bid & 7) * (total >> 3) + (bid >> 3);
  const int GM = 4;
  const int per_group = GM * ntn;
  const int group = t / per_group;
  const int first = group * GM;
  const int gsize = min(ntm - first, GM);
  const int local = t - group * per_group;
  tm = first + local % gsize;
  tn = local / gsize;
}

template <typename T> struct MF;
template <> struct MF<double> {
  typedef d4v V;
  static __device__ inline V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int v, int g) { return 4 * v + g; }
};
template <> struct MF<float> {
  typedef f4v V;
  static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int v, int g) { return 4 * g + v; }
};

// ---- global -> register slab loads.  Each thread moves a run of RUNA (A)
// or RUNB (B) consecutive elements (contiguous in memory) of the 64 x BKL A
// slab and the BKL x kTileN B slab.  On the full-tile path every run is one
// or two 16-byte vector loads; otherwise runs fully inside the n x n matrix
// and 16-byte aligned still use vector loads and the rest guarded element
// loads (zero fill).  Runs along k (A transposed, B normal) are laid out
// lane -> row / column so that each LDS store instruction of a wave writes
// consecutive elements of one k-row.
//
// Run of R elements p[x0 + i + y ld], i < R, of an n x n matrix stored with
// leading dimension ld (x the contiguous index).
template <typename T, int R, bool FULL>
__device__ inline void load_run(const T* __restrict__ p, int64_t ld, int64_t n, int64_t x0, int64_t y, T r[R]) {
  typedef T v2 __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int W = 16 / sizeof(T);
  const T* q = p + x0 + y * ld;
  const int64_t lim = (y < n) ? min<int64_t>(R, n - x0) : 0;
  if (FULL || (lim >= R && (((uintptr_t)q) & 15) == 0)) {
#pragma unroll
    for (int i = 0; i < R; i += W) {
      v2 x = *(const v2*)(q + i);
#pragma unroll
      for (int j = 0; j < W; ++j) r[i + j] = x[j];
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) r[i] = (i < lim) ? q[i] : T(0);
  }
}
// A(m,k): TA = false -> A[m + k lda] (run along m), true -> A[k + m lda] (run along k)
template <typename T, bool TA, bool FULL>
__device__ inline void load_a(const T* __restrict__ A, int64_t lda, int64_t n, int64_t m0, int64_t k0, int t,
                              T r[RUNA]) {
  if (!TA) {
    const int kk = t / TPA, mm = (t % TPA) * RUNA;
    load_run<T, RUNA, FULL>(A, lda, n, m0 + mm, k0 + kk, r);
  } else {
    const int mm = t & 63, kk = (t >> 6) * RUNA;
    load_run<T, RUNA, FULL>(A, lda, n, k0 + kk, m0 + mm, r);
  }
}
template <typename T, bool TA>
__device__ inline void store_a(T* As, int t, const T r[RUNA]) {
  if (!TA) {
    const int kk = t / TPA, mm = (t % TPA) * RUNA;
#pragma unroll
    for (int i = 0; i < RUNA; ++i) As[kk * LROWA + mm + i] = r[i];
  } else {
    const int mm = t & 63, kk = (t >> 6) * RUNA;
#pragma unroll
    for (int i = 0; i < RUNA; ++i) As[(kk + i) * LROWA + mm] = r[i];
  }
}
// B(k,j): TB = false -> B[k + j ldb] (run along k), true -> B[j + k ldb] (run along j)
template <typename T, bool TB, bool FULL>
__device__ inline void load_b(const T* __restrict__ B, int64_t ldb, int64_t n, int64_t n0, int64_t k0, int t,
                              T r[RUNB]) {
  if (!TB) {
    const int jj = t % kTileN, kk = (t / kTileN) * RUNB;
    load_run<T, RUNB, FULL>(B, ldb, n, k0 + kk, n0 + jj, r);
  } else {
    const int kk = t / TPB, jj = (t % TPB) * RUNB;
    load_run<T, RUNB, FULL>(B, ldb, n, n0 + jj, k0 + kk, r);
  }
}
template <typename T, bool TB>
__device__ inline void store_b(T* Bs, int t, const T r[RUNB]) {
  if (!TB) {
    const int jj = t % kTileN, kk = (t / kTileN) * RUNB;
#pragma unroll
    for (int i = 0; i < RUNB; ++i) Bs[(kk + i) * LROWB + jj] = r[i];
  } else {
    const int kk = t / TPB, jj = (t % TPB) * RUNB;
#pragma unroll
    for (int i = 0; i < RUNB; ++i) Bs[kk * LROWB + jj + i] = r[i];
  }
}

template <typename T>
__device__ __forceinline__ void mma_slab(const T* as, const T* bs, int wr, int wc, int g, int c,
                                typename MF<T>::V acc[2 * KCH]) {
  typedef T v2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int ks = 0; ks < BKL / 4; ++ks) {
    const int k = ks * 4 + g;
    const int ch = (ks % KCH) * 2;
    const v2 a01 = *(const v2*)(as + k * LROWA + wr + 2 * c);   // rows wr + 2c (block 0), wr + 2c + 1 (block 1)
    const T b0 = bs[k * LROWB + wc + c];
    acc[ch] = MF<T>::mma(a01[0], b0, acc[ch]);
    acc[ch + 1] = MF<T>::mma(a01[1], b0, acc[ch + 1]);
  }
}

// ---- FP64 / FP32 main loop: acc[bi] += A-tile x B-tile over all of K for the
// wave's two 16x16 blocks.  Two LDS stages and two register sets: the global
// loads of slab kt+2 are issued before the MFMAs of slab kt, and slab kt+1
// (loaded one iteration earlier) is stored to the other stage after them.
// The loop multiplies K slabs [sb, se) (se > sb).
// TL: the element type of A and B in memory (T, or FP64 operands of an FP32
// product, rounded to FP32 as they are stored to LDS).
template <typename T, bool TA, bool TB, bool FULL, typename TL = T>
__device__ __forceinline__ void mainloop_lds_impl(const TL* __restrict__ A, int64_t lda, const TL* __restrict__ B, int64_t ldb,
                                    int64_t n, int64_t m0, int64_t n0, char* smem, typename MF<T>::V acc[2],
                                    int64_t sb, int64_t se) {
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, c = lane & 15;
  const int wr = wave_row0(), wc = wave_col0();
  T* const S = (T*)smem;   // stage q: A slab at S + q STAGE, B slab after it
  typename MF<T>::V chains[2 * KCH];
#pragma unroll
  for (int i = 0; i < 2 * KCH; ++i) chains[i] = typename MF<T>::V{0, 0, 0, 0};
  const int64_t nk = se - sb;
  // two register sets: the global loads of slab kt+2 are issued while slab
  // kt+1 is still in flight, so each load has two slab times to arrive.  The
  // loads and LDS stores are unconditional (past the last slab the last slab
  // is fetched again and stored into the idle stage): a branch around them
  // would make the memory-counter wait before each store cover the newer
  // loads as well, which cancels the prefetch.
  TL ra0[RUNA], rb0[RUNB], ra1[RUNA], rb1[RUNB];
  // LDS stores of a register set, rounded to T when the operands are wider
  auto put = [&](T* st, const TL* ra, const TL* rb) {
    T ca[RUNA], cb[RUNB];
#pragma unroll
    for (int i = 0; i < RUNA; ++i) ca[i] = (T)ra[i];
#pragma unroll
    for (int i = 0; i < RUNB; ++i) cb[i] = (T)rb[i];
    store_a<T, TA>(st, t, ca);
    store_b<T, TB>(st + SLABA, t, cb);
  };
  const int64_t k0 = sb * BKL, k1 = (sb + min<int64_t>(1, nk - 1)) * BKL;
  load_a<TL, TA, FULL>(A, lda, n, m0, k0, t, ra0);
  load_b<TL, TB, FULL>(B, ldb, n, n0, k0, t, rb0);
  load_a<TL, TA, FULL>(A, lda, n, m0, k1, t, ra1);
  load_b<TL, TB, FULL>(B, ldb, n, n0, k1, t, rb1);
  put(S, ra0, rb0);
  __syncthreads();
  auto step = [&](int64_t kt, TL* rna, TL* rnb, const TL* rfa, const TL* rfb) {
    // rna/rnb: free set (receives slab kt+2); rfa/rfb: slab kt+1, in flight
    const int cur = (int)(kt & 1);
    const int64_t kn = (sb + min<int64_t>(kt + 2, nk - 1)) * BKL;
    load_a<TL, TA, FULL>(A, lda, n, m0, kn, t, rna);
    load_b<TL, TB, FULL>(B, ldb, n, n0, kn, t, rnb);
    if (kt < nk) mma_slab<T>(S + cur * STAGE, S + cur * STAGE + SLABA, wr, wc, g, c, chains);
    put(S + (cur ^ 1) * STAGE, rfa, rfb);
    __syncthreads();
  };
  for (int64_t kt = 0; kt < nk; kt += 2) {
    step(kt, ra0, rb0, ra1, rb1);
    step(kt + 1, ra1, rb1, ra0, rb0);
  }
  acc[0] = chains[0];
  acc[1] = chains[1];
#pragma unroll
  for (int ch = 1; ch < KCH; ++ch) {
    acc[0] += chains[2 * ch];
    acc[1] += chains[2 * ch + 1];
  }
}

// Full-tile fast path: when every tile and K slab is whole (n a multiple of 64)
// and both operands allow aligned 16-byte loads at every run, the slab loads
// are unconditional vector loads.  Besides saving the bounds arithmetic this
// keeps the loop free of divergent branches around the loads, so the memory
// counter waits before each LDS store cover only the slab being stored and
// the next slab's loads stay in flight.
template <typename T>
__device__ inline bool full_tiles(const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n) {
  constexpr int64_t V = 16 / sizeof(T);
  return (n % 64) == 0 && (lda % V) == 0 && (ldb % V) == 0 && ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0;
}
template <typename T, bool TA, bool TB, typename TL = T>
__device__ __forceinline__ void mainloop_lds(const TL* __restrict__ A, int64_t lda, const TL* __restrict__ B, int64_t ldb,
                                    int64_t n, int64_t m0, int64_t n0, char* smem, typename MF<T>::V acc[2]) {
  const int64_t nk = (n + BKL - 1) / BKL;
  if (full_tiles(A, lda, B, ldb, n)) mainloop_lds_impl<T, TA, TB, true, TL>(A, lda, B, ldb, n, m0, n0, smem, acc, 0, nk);
  else mainloop_lds_impl<T, TA, TB, false, TL>(A, lda, B, ldb, n, m0, n0, smem, acc, 0, nk);
}



// accumulator fragments -> LDS tile Cs[col * CSTR + row] (type W)
template <typename T, typename W>
__device__ __forceinline__ void frag_to_cs(const typename MF<T>::V acc[2], W* Cs, double scale) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int wr = wave_row0(), wc = wave_col0();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = wr + 2 * MF<T>::row(v, g) + bi;
      const int col = wc + c;
      Cs[col * CSTR + row] = (W)((double)acc[bi][v] * scale);
    }
}

__device__ __forceinline__ void frag_f32_to_cs_any(const f4v acc[2], double* Csd, float* Csf, bool isd) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int wr = wave_row0(), wc = wave_col0();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = wr + 16 * bi + 4 * g + v;
      const int col = wc + c;
      if (isd) Csd[col * CSTR + row] = (double)acc[bi][v];
      else Csf[col * CSTR + row] = acc[bi][v];
    }
}

// ---------------------------------------------------------------------------
// low-precision main loops (operands packed K-contiguous, zero-masked past n)
// ---------------------------------------------------------------------------
__device__ inline uint16_t bf16_bits_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---- BF16 / FP8 main loop.  The operands are packed K-contiguous: row r of
// P_i (and column j of Y) is a run of Kp elements, FP8 rows followed by E8M0
// scales (one byte per 32 elements).  A slab is 128 bytes of K per row (FP8:
// 128 elements, BF16: 64); the workgroup stages the 64 A rows and 64 B
// columns of a slab in LDS (each thread one 16-byte chunk of each, K beyond n
// zeroed there), so every byte is fetched from memory once per workgroup and
// by wide coalesced loads; the waves then read their MFMA fragments from LDS.
// Two LDS stages and two register sets, as in the FP64/FP32 loop.
constexpr int LP_RS = 144;                      // LDS row stride (bytes): 16-byte fragment reads of
                                                //   16 consecutive rows hit distinct banks
constexpr int LP_OPER = 64 * LP_RS;             // one operand slab
constexpr int LP_STAGE = 2 * LP_OPER + 2 * 64 * 4;   // A, B, then A and B scale words
static_assert(2 * LP_STAGE <= smem_bytes<float>(), "low-precision stages fit the tile LDS");
static_assert(kTileN * CSTR * 4 <= smem_bytes<float>(), "epilogue tile fits the tile LDS");

struct LpRegs { uint4 a, b; uint32_t s; };

// zero the elements >= n of a 16-byte chunk whose first element is k (EB bytes per element)
template <int EB>
__device__ inline uint4 lp_mask(uint4 v, int64_t k, int64_t n) {
  constexpr int PW = 4 / EB;   // elements per 32-bit word
  union { uint4 q; uint32_t w[4]; } u;
  u.q = v;
#pragma unroll
  for (int wd = 0; wd < 4; ++wd) {
    const int64_t nv = n - (k + PW * wd);
    const uint32_t mk = nv >= PW ? 0xffffffffu : nv <= 0 ? 0u : (1u << (8 * EB * nv)) - 1u;
    u.w[wd] &= mk;
  }
  return u.q;
}

// the slab-i loads of thread t (raw: K past n not yet masked)
template <bool FP8>
__device__ __forceinline__ void lp_load_raw(const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
                                   const uint8_t* __restrict__ B, const uint8_t* __restrict__ Bs, int64_t rsb,
                                   int64_t Ks, int64_t m0, int64_t n0, int64_t i, int t, LpRegs& r) {
  const int row = t >> 3, ch = t & 7;
  const int64_t kbyte = 128 * i + 16 * ch;
  r.a = *(const uint4*)(A + (m0 + row) * rsb + kbyte);
  r.b = *(const uint4*)(B + (n0 + row) * rsb + kbyte);
  // one word = the 4 E8M0 scales of this slab for one row of A (t < 64) or
  // one column of B
  if (FP8 && t < 128)
    r.s = (t < 64) ? *(const uint32_t*)(As + (m0 + t) * Ks + 4 * i)
                   : *(const uint32_t*)(Bs + (n0 + t - 64) * Ks + 4 * i);
}
// zero the elements >= n of slab i; scale blocks wholly past n get the
// neutral scale 2^0
template <bool FP8>
__device__ __forceinline__ void lp_fix(int64_t n, int64_t i, int t, LpRegs& r) {
  constexpr int EB = FP8 ? 1 : 2;
  const int ch = t & 7;
  const int64_t k = (128 * i + 16 * ch) / EB;
  if (k + 16 / EB > n) {
    r.a = lp_mask<EB>(r.a, k, n);
    r.b = lp_mask<EB>(r.b, k, n);
  }
  if (FP8 && t < 128) {
#pragma unroll
    for (int bk = 0; bk < 4; ++bk)
      if ((4 * i + bk) * 32 >= n) r.s = (r.s & ~(0xffu << (8 * bk))) | (127u << (8 * bk));
  }
}
template <bool FP8>
__device__ __forceinline__ void lp_load(const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
                               const uint8_t* __restrict__ B, const uint8_t* __restrict__ Bs, int64_t rsb,
                               int64_t Ks, int64_t n, int64_t m0, int64_t n0, int64_t i, int t, LpRegs& r) {
  lp_load_raw<FP8>(A, As, B, Bs, rsb, Ks, m0, n0, i, t, r);
  lp_fix<FP8>(n, i, t, r);
}

template <bool FP8>
__device__ __forceinline__ void lp_store(char* st, int t, const LpRegs& r) {
  const int row = t >> 3, ch = t & 7;
  *(uint4*)(st + row * LP_RS + 16 * ch) = r.a;
  *(uint4*)(st + LP_OPER + row * LP_RS + 16 * ch) = r.b;
  if (FP8 && t < 128) *(uint32_t*)(st + 2 * LP_OPER + 4 * t) = r.s;
}

template <bool FP8>
__device__ __forceinline__ void lp_mma(const char* st, int wr, int wc, int g, int c, f4v acc[2]) {
  const char* a0p = st + (wr + c) * LP_RS + 16 * g;
  const char* a1p = a0p + 16 * LP_RS;
  const char* bp = st + LP_OPER + (wc + c) * LP_RS + 16 * g;
  if (FP8) {
    union U { uint4 q[2]; i8v v; } a0, a1, bb;
    a0.q[0] = *(const uint4*)a0p; a0.q[1] = *(const uint4*)(a0p + 64);
    a1.q[0] = *(const uint4*)a1p; a1.q[1] = *(const uint4*)(a1p + 64);
    bb.q[0] = *(const uint4*)bp;  bb.q[1] = *(const uint4*)(bp + 64);
    const uint8_t* sc = (const uint8_t*)(st + 2 * LP_OPER);
    const int sa0 = sc[(wr + c) * 4 + g], sa1 = sc[(wr + 16 + c) * 4 + g];
    const int sb = sc[256 + (wc + c) * 4 + g];
    acc[0] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a0.v, bb.v, acc[0], 0, 0, 0, sa0, 0, sb);
    acc[1] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a1.v, bb.v, acc[1], 0, 0, 0, sa1, 0, sb);
  } else {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      union U { uint4 q; bf8v v; } a0, a1, bb;
      a0.q = *(const uint4*)(a0p + 64 * j);
      a1.q = *(const uint4*)(a1p + 64 * j);
      bb.q = *(const uint4*)(bp + 64 * j);
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.v, bb.v, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.v, bb.v, acc[1], 0, 0, 0);
    }
  }
}

// FP8 (FP8 = true): A = P8 [Mp][Kp] bytes, As = its scales [Mp][Kp/32], B = Y8, Bs = its scales.
// BF16: A = P [Mp][Kp] bf16 bits, B = Yb [Mp][Kp]; As, Bs unused.
// The scaled f8f6f4 16x16x128 MFMA orders K inside a 128-slab as: lane group
// g = l/16 holds slab elements [16g, 16g+16) in bytes 0..15 and
// [64+16g, 64+16g+16) in bytes 16..31, and the E8M0 scale of the 32-element
// slab block b of row (column) l%16 is the one passed by lane l%16 + 16b.
// Reading each lane's halves from those two offsets makes every hardware
// scale block coincide with one 32-element block of the packed layout.
// after_issue() runs once the loads of the first two slabs are issued (as in
// mainloop_fp8_all: loads it issues retire after theirs).
template <bool FP8, typename F>
__device__ __forceinline__ void mainloop_lowp(const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
                                     const uint8_t* __restrict__ B, const uint8_t* __restrict__ Bs, int64_t Kp,
                                     int64_t n, int64_t m0, int64_t n0, char* smem, f4v acc[2], F&& after_issue) {
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, c = lane & 15;
  const int wr = wave_row0(), wc = wave_col0();
  const int64_t rsb = FP8 ? Kp : 2 * Kp;             // row stride in bytes
  const int64_t Ks = Kp / 32;
  const int64_t ns = FP8 ? (n + 127) / 128 : (n + 63) / 64;
  acc[0] = f4v{0, 0, 0, 0};
  acc[1] = f4v{0, 0, 0, 0};
  // loads and stores unconditional, as in mainloop_lds_impl
  LpRegs r0, r1;
  lp_load<FP8>(A, As, B, Bs, rsb, Ks, n, m0, n0, 0, t, r0);
  lp_load<FP8>(A, As, B, Bs, rsb, Ks, n, m0, n0, min<int64_t>(1, ns - 1), t, r1);
  after_issue();
  lp_store<FP8>(smem, t, r0);
  __syncthreads();
  auto step = [&](int64_t kt, LpRegs& rn, const LpRegs& rf) {
    const int cur = (int)(kt & 1);
    lp_load<FP8>(A, As, B, Bs, rsb, Ks, n, m0, n0, min<int64_t>(kt + 2, ns - 1), t, rn);
    if (kt < ns) lp_mma<FP8>(smem + cur * LP_STAGE, wr, wc, g, c, acc);
    lp_store<FP8>(smem + (cur ^ 1) * LP_STAGE, t, rf);
    __syncthreads();
  };
  for (int64_t kt = 0; kt < ns; kt += 2) {
    step(kt, r0, r1);
    step(kt + 1, r1, r0);
  }
}
template <bool FP8>
__device__ __forceinline__ void mainloop_lowp(const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
                                     const uint8_t* __restrict__ B, const uint8_t* __restrict__ Bs, int64_t Kp,
                                     int64_t n, int64_t m0, int64_t n0, char* smem, f4v acc[2]) {
  mainloop_lowp<FP8>(A, As, B, Bs, Kp, n, m0, n0, smem, acc, [] {});
}

// FP8 with at most LP_ALL slabs (n <= 1024): the loads of every slab are
// issued first, so the workgroup waits for memory once; the slabs then pass
// through the two LDS stages (one barrier per slab: the barrier of slab k+1
// follows every wave's reads of slab k, so slab k+2 may overwrite its stage).
// after_issue() runs once the slab loads are issued: loads it issues retire
// after the slabs' (the memory counter counts in issue order), so the first
// slab does not wait for them.
constexpr int LP_ALL = 8;
template <typename F>
__device__ __forceinline__ void mainloop_fp8_all(const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
                                                 const uint8_t* __restrict__ B, const uint8_t* __restrict__ Bs,
                                                 int64_t Kp, int64_t n, int64_t m0, int64_t n0, char* smem,
                                                 f4v acc[2], F&& after_issue) {
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, c = lane & 15;
  const int wr = wave_row0(), wc = wave_col0();
  const int64_t Ks = Kp / 32;
  const int ns = (int)((n + 127) / 128);
  acc[0] = f4v{0, 0, 0, 0};
  acc[1] = f4v{0, 0, 0, 0};
  LpRegs r[LP_ALL];
#pragma unroll
  for (int i = 0; i < LP_ALL; ++i)
    if (i < ns) lp_load_raw<true>(A, As, B, Bs, Kp, Ks, m0, n0, i, t, r[i]);
  after_issue();
#pragma unroll
  for (int i = 0; i < LP_ALL; ++i) {
    if (i < ns) {
      char* st = smem + (i & 1) * LP_STAGE;
      lp_fix<true>(n, i, t, r[i]);
      lp_store<true>(st, t, r[i]);
      __syncthreads();
      lp_mma<true>(st, wr, wc, g, c, acc);
    }
  }
  __syncthreads();   // the epilogue reuses the stages
}

// E4M3 quantisation of 32 floats with a shared power-of-two scale (E8M0).
// amax = f 2^e with f in [0.5,1): scaled values lie in (-256, 256), inside the
// E4M3 range (max 448); conversion is round-to-nearest-even.
__device__ inline int e8m0_for(float amax) {
  if (!(amax > 0.0f) || !(amax < INFINITY)) return 127;
  int e;
  frexpf(amax, &e);
  int se = e - 8;
  se = max(-127, min(127, se));
  return se + 127;
}
__device__ inline uint32_t pack4_e4m3(float a, float b, float c, float d) {
  const float L = 448.0f;
  a = fminf(fmaxf(a, -L), L); b = fminf(fmaxf(b, -L), L);
  c = fminf(fmaxf(c, -L), L); d = fminf(fmaxf(d, -L), L);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

// ---------------------------------------------------------------------------
// one output tile of C = alpha op(A) op(B) (+ C); ends with a barrier so the
// caller may reuse smem for the next tile
// ---------------------------------------------------------------------------
// n: order of the operands (extent of the product); nv <= n: the order of the
// part of C that is written (rows and columns < nv).
template <typename T, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(const T* __restrict__ Ap, int64_t lda, const T* __restrict__ Bp, int64_t ldb,
                                 T* Cp, int64_t ldc, int64_t n, int64_t nv, int64_t m0, int64_t n0, double alpha,
                                 int accumulate, char* smem) {
  typename MF<T>::V acc[2];
  mainloop_lds<T, TA, TB>(Ap, lda, Bp, ldb, n, m0, n0, smem, acc);
  T* Cs = (T*)smem;
  frag_to_cs<T, T>(acc, Cs, 1.0);
  __syncthreads();
  const int t = threadIdx.x;
  const int row = t & 63;
  const int64_t gr = m0 + row;
#pragma unroll 4
  for (int q = 0; q < TILE_Q; ++q) {
    const int col = (t >> 6) + NW * q;
    const int64_t gc = n0 + col;
    if (gr < nv && gc < nv) {
      const T v = (T)(alpha * (double)Cs[col * CSTR + row]);
      T* dst = Cp + gr + gc * ldc;
      if (accumulate) *dst = *dst + v;
      else *dst = v;
    }
  }
  __syncthreads();
}

// C (FP32, ld ldc) = alpha A B for FP64 operands, the product in FP32: the
// operands are rounded to FP32 on their way into LDS.  One 64 x 64 tile.
__device__ __forceinline__ void gemm_tile_f32_of_f64(const double* __restrict__ Ap, int64_t lda,
                                                     const double* __restrict__ Bp, int64_t ldb, float* Cp,
                                                     int64_t ldc, int64_t n, int64_t m0, int64_t n0, double alpha,
                                                     char* smem) {
  typename MF<float>::V acc[2];
  mainloop_lds<float, false, false, double>(Ap, lda, Bp, ldb, n, m0, n0, smem, acc);
  float* Cs = (float*)smem;
  frag_to_cs<float, float>(acc, Cs, 1.0);
  __syncthreads();
  const int t = threadIdx.x;
  const int row = t & 63;
  const int64_t gr = m0 + row;
#pragma unroll 4
  for (int q = 0; q < TILE_Q; ++q) {
    const int col = (t >> 6) + NW * q;
    const int64_t gc = n0 + col;
    if (gr < n && gc < n) Cp[gr + gc * ldc] = (float)(alpha * (double)Cs[col * CSTR + row]);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// one output tile of a Horner step P_{i-1} = B_{i-1} + P_i Y (t_in < 0: cast of
// B_src into the format t_out).  The product runs in tier t_in; the epilogue
// adds B_{i-1} in the precision of t_out and writes the operand format that
// the next step reads (or the working-precision result).  Ends with a barrier.
// ---------------------------------------------------------------------------
// Pack the tile Cs (column-major, CSTR) into the K-contiguous operand layout of
// tier t_out: 2 = BF16 [Mp][Kp]; 3 = E4M3 [Mp][Kp] followed by the E8M0
// scales [Mp][Kp/32] (one per 32 columns of a row).  The caller synchronizes.
template <typename C>
__device__ __forceinline__ void pack_tile_lowp(const C* Cs, int t_out, char* pout, int64_t Mp, int64_t Kp, int64_t m0,
                                               int64_t n0) {
  const int t = threadIdx.x;
  if (t_out == 2) {
    const int r = t / (kTileN / 8), seg = (t % (kTileN / 8)) * 8;   // NT = 64 rows x kTileN/8 segments
    union { uint4 q; uint16_t h[8]; } o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o.h[e] = bf16_bits_rne((float)Cs[(seg + e) * CSTR + r]);
    *(uint4*)((uint16_t*)pout + (m0 + r) * Kp + n0 + seg) = o.q;
  } else {
    // one E8M0 block = 32 columns of a row, shared by four consecutive lanes
    // (eight values each); the block maximum by two butterfly steps
    static_assert(NT == 4 * kTileM * kTileN / 32, "four lanes per E8M0 block");
    const int q = t >> 2, part = t & 3;
    const int r = q % kTileM, blk = q / kTileM;
    float vals[8];
    float amax = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      vals[e] = (float)Cs[(32 * blk + 8 * part + e) * CSTR + r];
      amax = fmaxf(amax, fabsf(vals[e]));
    }
    amax = fmaxf(amax, __shfl_xor(amax, 1, 64));
    amax = fmaxf(amax, __shfl_xor(amax, 2, 64));
    const int sbyte = e8m0_for(amax);
    const int sexp = sbyte - 127;
    uint2 o;
    o.x = pack4_e4m3(ldexpf(vals[0], -sexp), ldexpf(vals[1], -sexp), ldexpf(vals[2], -sexp), ldexpf(vals[3], -sexp));
    o.y = pack4_e4m3(ldexpf(vals[4], -sexp), ldexpf(vals[5], -sexp), ldexpf(vals[6], -sexp), ldexpf(vals[7], -sexp));
    uint8_t* p8 = (uint8_t*)pout;
    *(uint2*)(p8 + (m0 + r) * Kp + n0 + 32 * blk + 8 * part) = o;
    if (part == 0) p8[Mp * Kp + (m0 + r) * (Kp / 32) + n0 / 32 + blk] = (uint8_t)sbyte;
  }
}

template <typename W>
struct HornerTile {
  int64_t n, Mp, Kp;
  int t_in, t_out;          // t_in = -1: cast only; t_out = working tier: W column-major output
  const char* pin;          // operand P_i in the format of t_in
  const W* ysrc;            // Y in the working precision
  int64_t ldy;
  double yscale;
  const float* yf32;        // FP32 copy of Y (W = double)
  const uint16_t* ybf16;
  const uint8_t* yfp8;
  const uint8_t* yfp8s;
  const W* bsrc;            // B_{i-1} (column-major, ld n)
  char* pout;               // next operand buffer (t_out below working)
  W* outw;                  // working-precision output (t_out = working tier)
  int64_t ldo;
  int64_t nv;               // rows and columns < nv of outw are written (nv <= n)
  int64_t nvb;              // order of the matrix inside the padded n: B_{i-1} is read
                            // for rows and columns < nvb only (zero beyond)
  // fyc != 0 (a cast of the block that holds the folded last step c_m Y,
  // where the fold used Y in FP32 but the plan keeps a product in FP64):
  // B_{i-1} + fyc (fy64 - fy32) restores the fold with Y in FP64
  const W* fy64;
  const float* fy32;
  double fyc;
};

// FP8ALL: FP8 products of order n <= 1024 load all their K slabs at once
// (mainloop_fp8_all); off for the batched kernel, whose orders stay <= 256
template <typename W, bool FP8ALL>
__device__ __forceinline__ void horner_tile(const HornerTile<W>& h, int64_t m0, int64_t n0, char* smem) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;   // working tier
  const int64_t n = h.n, Kp = h.Kp;
  const int t_in = h.t_in, t_out = h.t_out;
  W* Cs = (W*)smem;
  const int t = threadIdx.x;
  const int row = t & 63;
  const int64_t gr = m0 + row;
  // this thread's elements of B_{i-1} (the block is in the working precision
  // whatever the tier): their round trip overlaps everything up to the
  // epilogue.  FP64 and FP32 products issue them before the main loop; the
  // BF16 and FP8 loops issue them right after their first slab loads, so
  // that the first slab does not wait for them (the memory counter retires
  // loads in issue order)
  W bq[TILE_Q];
  auto load_bq = [&]() {
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const int64_t gc = n0 + (t >> 6) + NW * q;
      const bool in = gr < h.nvb && gc < h.nvb;
      const W x = h.bsrc[(in ? gr : 0) + (in ? gc : 0) * n];
      bq[q] = in ? x : W(0);
    }
  };
  const bool fp8all = FP8ALL && t_in == 3 && n <= LP_ALL * 128;
  if (t_in != 2 && t_in != 3) load_bq();
  if (t_in == WT) {
    typename MF<W>::V acc[2];
    mainloop_lds<W, false, false>((const W*)h.pin, n, h.ysrc, h.ldy, n, m0, n0, smem, acc);
    frag_to_cs<W, W>(acc, Cs, h.yscale);
  } else if (t_in == 1) {   // FP32 product below an FP64 working precision
    typename MF<float>::V acc[2];
    mainloop_lds<float, false, false>((const float*)h.pin, n, h.yf32, n, n, m0, n0, smem, acc);
    frag_to_cs<float, W>(acc, Cs, 1.0);
  } else if (t_in == 2) {
    f4v acc[2];
    mainloop_lowp<false>((const uint8_t*)h.pin, nullptr, (const uint8_t*)h.ybf16, nullptr, Kp, n, m0, n0, smem, acc,
                         load_bq);
    frag_f32_to_cs_any(acc, (double*)smem, (float*)smem, WT == 0);
  } else if (t_in == 3) {
    f4v acc[2];
    const uint8_t* p8 = (const uint8_t*)h.pin;
    if (fp8all) mainloop_fp8_all(p8, p8 + h.Mp * Kp, h.yfp8, h.yfp8s, Kp, n, m0, n0, smem, acc, load_bq);
    else mainloop_lowp<true>(p8, p8 + h.Mp * Kp, h.yfp8, h.yfp8s, Kp, n, m0, n0, smem, acc, load_bq);
    frag_f32_to_cs_any(acc, (double*)smem, (float*)smem, WT == 0);
  } else {   // cast only
    if (h.fyc != 0.0) {
#pragma unroll
      for (int q = 0; q < TILE_Q; ++q) {
        const int64_t gc = n0 + (t >> 6) + NW * q;
        if (gr < h.nvb && gc < h.nvb)
          bq[q] += (W)(h.fyc * ((double)h.fy64[gr + gc * n] - (double)h.fy32[gr + gc * n]));
      }
    }
  }
  __syncthreads();

  // pass 1 (column-major, coalesced): add B_{i-1} in the precision of t_out
#pragma unroll
  for (int q = 0; q < TILE_Q; ++q) {
    const int col = (t >> 6) + NW * q;
    const int64_t gc = n0 + col;
    const bool in = gr < n && gc < n;
    const W v = (t_in < 0) ? W(0) : Cs[col * CSTR + row];
    const W bb = bq[q];
    if (t_out == WT) {
      if (gr < h.nv && gc < h.nv) h.outw[gr + gc * h.ldo] = bb + v;
    } else if (t_out == 1) {
      if (in) ((float*)h.pout)[gr + gc * n] = (float)bb + (float)v;
    } else {
      Cs[col * CSTR + row] = in ? (W)((float)bb + (float)v) : W(0);
    }
  }
  __syncthreads();
  if (t_out < 2) return;
  // pass 2 (row-major): pack into the K-contiguous low-precision layout
  pack_tile_lowp<W>(Cs, t_out, h.pout, h.Mp, Kp, m0, n0);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// one wave: rows of chunk `chunk` of column `col` of B_0..B_r (working
// precision, the paper assembles the blocks in u), the fold of the trivial
// last step (B_r = c_m I), partial column abs sums of B_i and Y, and the
// low-precision copies of Y.  No workgroup barrier inside.
// ---------------------------------------------------------------------------
// GATHER: for block sizes up to 8, load every power of the column before the
// first use (one memory round trip per wave; the grid kernel over large
// matrices).  Otherwise the powers are read one after another (the batched
// kernel, whose many short waves run faster with the smaller code).
template <typename W, bool GATHER>
__device__ __forceinline__ void assemble_column(const AssembleArgs& a, const Coefs& cf, char* ws, const W* X1, int64_t col,
                                       int64_t chunk) {
  const Layout& L = a.L;
  const int64_t n = a.n;
  const int lane = threadIdx.x & 63;
  const int64_t se = (int64_t)(L.slot / sizeof(W));
  const W* pw = (const W*)(ws + L.off_pow) + (L.square_arg ? se : 0);  // X_2 .. X_s
  W* Bm = (W*)(ws + L.off_B);
  double* colsum = (double*)(ws + L.off_colsum);
  const int s = a.s, r = a.r, m = a.m, nB = a.nB;
  const double x1s = a.x1_scale;
  const bool want32 = std::is_same<W, double>::value && ((a.tier_mask >> 1) & 1u) && !a.y_f32;
  const bool want16 = (a.tier_mask >> 2) & 1u;
  const bool want8 = (a.tier_mask >> 3) & 1u;
  const int64_t Kp = L.Kp, Ks = Kp / 32;
  float* yf32 = (float*)(ws + L.off_yf32);
  uint16_t* ybf = (uint16_t*)(ws + L.off_ybf16);
  uint8_t* y8 = (uint8_t*)(ws + L.off_yfp8);
  uint8_t* y8s = (uint8_t*)(ws + L.off_yfp8s);

  // this wave's rows: row chunk `chunk` (kRowChunk rows) of column `col`,
  // RPL rows per lane, 64 apart
  constexpr int RPL = kRowChunk / 64;
  const int64_t r_begin = chunk * kRowChunk;
  const int64_t r_end = min<int64_t>(n, r_begin + kRowChunk);
  const int64_t nch = (n + kRowChunk - 1) / kRowChunk;
  // valid: rows of this chunk (the Y copies cover the padded order n);
  // inner: rows and column inside the matrix's own order nv.  Outside it the
  // powers are zero, so nothing there is loaded, and the blocks are neither
  // formed nor stored there (their readers mask at nv).
  const bool colv = col < a.nv;
  int64_t rw[RPL];
  bool valid[RPL], inner[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    rw[q] = r_begin + lane + 64 * q;
    valid[q] = rw[q] < r_end;
    inner[q] = colv && rw[q] < r_end && rw[q] < a.nv;
  }
  // this lane's elements of column `col` of X_j, in two phases so that the
  // loads of several powers can all be in flight before the first use:
  // load_raw issues the loads (lanes past the end read row r_begin of a
  // column inside; 64-row groups that hold no row of the matrix are skipped
  // by a wave-uniform test), finish_x scales and masks the values.
  const int64_t cl = colv ? col : 0;
  const int rlim = __builtin_amdgcn_readfirstlane((int)(colv ? min<int64_t>(r_end, a.nv) : r_begin));
  const bool yf = a.y_f32 != 0;   // Y = X_s in the FP32 copy's slot
  auto load_raw = [&](int j, W out[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      out[q] = W(0);
      if (!GATHER || r_begin + 64 * q < rlim) {
        const int64_t rr = inner[q] ? rw[q] : r_begin;
        out[q] = (j == 1) ? X1[rr + cl * a.X1.ld]
                          : (yf && j == s) ? (W)yf32[rr + cl * n] : pw[(int64_t)(j - 2) * se + rr + cl * n];
      }
    }
  };
  auto finish_x = [&](int j, W v[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const W x = (j == 1) ? (W)(x1s * (double)v[q]) : (W)ldexp((double)v[q], j * a.pow_shift);
      v[q] = inner[q] ? x : W(0);
    }
  };
  auto load_x = [&](int j, W out[RPL]) {
    load_raw(j, out);
    finish_x(j, out);
  };
  // Y statistics and low-precision copies
  double ysum = 0.0;
  auto y_copies = [&](const W y[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      ysum += fabs((double)y[q]);
      if (valid[q] && want32) yf32[rw[q] + col * n] = (float)y[q];
      if (valid[q] && want16) ybf[col * Kp + rw[q]] = bf16_bits_rne((float)y[q]);
      if (want8) {
        // E8M0 block = 32 consecutive rows = one half-wave
        float av = fabsf((float)y[q]);
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) av = fmaxf(av, __shfl_xor(av, off, 64));
        const int sbyte = e8m0_for(av);
        if (valid[q]) {
          float qv = ldexpf((float)y[q], -(sbyte - 127));
          qv = fminf(fmaxf(qv, -448.0f), 448.0f);
          const int wv = __builtin_amdgcn_cvt_pk_fp8_f32(qv, 0.0f, 0, false);
          y8[col * Kp + rw[q]] = (uint8_t)(wv & 0xff);
          if ((rw[q] & 31) == 0) y8s[col * Ks + rw[q] / 32] = (uint8_t)sbyte;
        }
      }
    }
  };
  // |c_k| for the a-priori planning rule (one wave writes them)
  if (col == 0 && chunk == 0) {
    Plan* P = (Plan*)(ws + L.off_plan);
    for (int k = lane; k <= m; k += 64) P->abs_coef[k] = fabs(cf.c[k]);
  }
  // block i's values of this lane's rows, stored with the trivial last step
  // folded in; its partial column abs sum
  auto store_block = [&](int i, const W bv[RPL], const W y[RPL]) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      if (!inner[q]) continue;
      v += fabs((double)bv[q]);
      W outv = bv[q];
      if (a.trivial_last && i == r - 1) outv += (W)cf.c[m] * y[q];   // step r: c_m I * Y
      Bm[(int64_t)i * se + rw[q] + col * n] = outv;
    }
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) colsum[((int64_t)i * nch + chunk) * n + col] = v;
  };
  // identity term of block i on this lane's rows
  auto block_init = [&](int i, W bv[RPL]) {
    const W c0 = (i < nB && s * i <= m) ? (W)cf.c[s * i] : W(0);
#pragma unroll
    for (int q = 0; q < RPL; ++q) bv[q] = (rw[q] == col && col < a.nv) ? c0 : W(0);
  };
  double xsum = 0.0;   // column abs sum of X_1
  W y[RPL];
  constexpr int PG = 8;   // block sizes up to PG: every power of the column loaded at once
  if (GATHER && s <= PG) {
    W x[PG][RPL];
#pragma unroll
    for (int jj = 0; jj < PG; ++jj) {
      if (jj < s) {
        load_raw(jj + 1, x[jj]);
      } else {
#pragma unroll
        for (int q = 0; q < RPL; ++q) x[jj][q] = W(0);
      }
    }
#pragma unroll
    for (int jj = 0; jj < PG; ++jj) finish_x(jj + 1, x[jj]);   // zero stays zero for jj >= s
#pragma unroll
    for (int q = 0; q < RPL; ++q) y[q] = x[0][q];
#pragma unroll
    for (int jj = 1; jj < PG; ++jj)
      if (jj + 1 == s)
#pragma unroll
        for (int q = 0; q < RPL; ++q) y[q] = x[jj][q];
    y_copies(y);
    if (s > 1)
#pragma unroll
      for (int q = 0; q < RPL; ++q) xsum += fabs((double)x[0][q]);
    for (int i = 0; i < nB; ++i) {
      W bv[RPL];
      block_init(i, bv);
      // B_i = c_{si} I + sum_{j=1}^{s-1} c_{si+j} X_j, terms in increasing j
#pragma unroll
      for (int j = 1; j < PG; ++j) {
        const int k = s * i + j;
        if (j < s && k <= m) {
          const W ck = (W)cf.c[k];
#pragma unroll
          for (int q = 0; q < RPL; ++q) bv[q] += ck * x[j - 1][q];
        }
      }
      store_block(i, bv, y);
    }
  } else {
    load_x(s, y);
    y_copies(y);
    // blocks in chunks of BC so their running values stay in registers (few
    // enough for six waves per SIMD in the batched kernel); the powers
    // X_1..X_{s-1} are read once per chunk, terms in increasing j
    constexpr int BC = 4;
    for (int i0 = 0; i0 < nB; i0 += BC) {
      W bv[BC][RPL];
#pragma unroll
      for (int ii = 0; ii < BC; ++ii) block_init(i0 + ii, bv[ii]);
#pragma unroll 2
      for (int j = 1; j < (colv ? s : 1); ++j) {
        W xj[RPL];
        load_x(j, xj);
        if (j == 1 && i0 == 0)
#pragma unroll
          for (int q = 0; q < RPL; ++q) xsum += fabs((double)xj[q]);
#pragma unroll
        for (int ii = 0; ii < BC; ++ii) {
          const int k = s * (i0 + ii) + j;
          if (i0 + ii < nB && k <= m) {
            const W ck = (W)cf.c[k];
#pragma unroll
            for (int q = 0; q < RPL; ++q) bv[ii][q] += ck * xj[q];
          }
        }
      }
#pragma unroll
      for (int ii = 0; ii < BC; ++ii)
        if (i0 + ii < nB) store_block(i0 + ii, bv[ii], y);
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
// per-matrix plan (whole workgroup): norms = max over columns of the summed
// partial column sums, then the tier rule of ps_planner.h.  Thread 0 writes
// the Plan; ends with a barrier.  red: NT doubles, norms: PS_MAX_BLOCKS+2
// doubles, both in LDS.
// ---------------------------------------------------------------------------
// PT: threads of the workgroup (red holds 8 PT / 64 doubles).  The norms do
// not depend on PT: a maximum is the same whatever the partition.
template <int PT>
__device__ __forceinline__ void plan_matrix(const PlanArgs& a, const Layout& L, char* ws, double* red, double* norms) {
  constexpr int PW = PT / 64;
  const int64_t n = L.n;
  const double* colsum = (const double*)(ws + L.off_colsum);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t nch = (n + L.colsum_rows - 1) / L.colsum_rows;
  // each thread: running max over its columns of every block's column sum
  // (partial sums of the row chunks added in chunk order); the loads of
  // different blocks and chunks are independent, so their latencies overlap
  const int rows = a.nB + 1;   // column-sum rows: B_0 .. B_{nB-1}, Y, X
  for (int i0 = 0; i0 <= rows; i0 += 8) {
    double mx[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) mx[ii] = 0.0;
    for (int64_t c = t; c < n; c += PT) {
      double sum[8];
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) sum[ii] = 0.0;
      // all (block, chunk) loads of this column are independent, so they are
      // in flight together
#pragma unroll 4
      for (int64_t ch = 0; ch < nch; ++ch) {
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) {
          const int i = min(i0 + ii, rows);   // clamped: every load is unconditional
          const double v = colsum[((int64_t)i * nch + ch) * n + c];
          sum[ii] += (i0 + ii <= rows) ? v : 0.0;
        }
      }
#pragma unroll
      for (int ii = 0; ii < 8; ++ii)
        if (sum[ii] > mx[ii] || sum[ii] != sum[ii]) mx[ii] = sum[ii];
    }
    // wave maxima: the eight butterflies interleaved so their shuffles overlap
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        const double o = __shfl_xor(mx[ii], off, 64);
        if (o > mx[ii] || o != o) mx[ii] = o;
      }
    if (lane == 0)
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) red[ii * PW + w] = mx[ii];
    __syncthreads();
    if (t < 8 && i0 + t <= rows) {
      double v = red[t * PW];
      for (int k = 1; k < PW; ++k) {
        const double o = red[t * PW + k];
        if (o > v || o != o) v = o;
      }
      norms[i0 + t] = v;
    }
    __syncthreads();
  }
  // plan in LDS (thread 0), then copied to the workspace Plan by all threads
  __shared__ int s_tier[PS_MAX_BLOCKS];
  __shared__ double s_u[PS_MAX_BLOCKS];
  __shared__ int s_nu;
  __shared__ double s_ny, s_nx;
  __shared__ double s_nb[PS_MAX_BLOCKS];
  if (t == 0) {
    // norms[nB] holds ||Y|| and norms[nB + 1] ||X||; with s | m, nB = r and
    // slot r then receives ||B_r|| = |c_m| (B_r = c_m I), so ||Y|| is read
    // out first
    const double ny = norms[a.nB];
    const double nx = norms[a.nB + 1];
    s_ny = ny;
    s_nx = nx;
    if (a.trivial_last) norms[a.r] = a.abs_cm;
    if (a.use_override) {
      for (int i = 0; i <= a.r; ++i) {
        s_tier[i] = (i == 0) ? a.working : a.override_tier[i];
        s_u[i] = tier_unit_roundoff(s_tier[i]);
      }
      s_nu = a.r + 1;
      for (int i = 1; i <= a.r; ++i) if (s_tier[i] != a.working) { s_nu = i; break; }
    } else if (a.mode == PS_MODE_FIXED) {
      for (int i = 0; i <= a.r; ++i) { s_tier[i] = a.working; s_u[i] = tier_unit_roundoff(a.working); }
      s_nu = a.r + 1;
    } else if (a.rule == PS_RULE_APRIORI) {
      // ||B_i|| ||Y||^i bounded by sum_{k in block i} |c_k| ||X||^k, written as
      // nb_i ||X||^(s i) with nb_i = sum_j |c_{si+j}| ||X||^j; ||B_0|| exact
      const double* ac = ((const Plan*)(ws + L.off_plan))->abs_coef;
      const int sb = L.s;
      s_nb[0] = norms[0];
      for (int i = 1; i <= a.r; ++i) {
        double v = 0.0, p = 1.0;
        for (int k = sb * i; k <= min(sb * i + sb - 1, L.m); ++k) {
          v += ac[k] * p;
          p *= nx;
        }
        s_nb[i] = v;
      }
      double nys = 1.0;
      for (int j = 0; j < sb; ++j) nys *= nx;
      int nu;
      plan_tiers(a.r, s_nb, nys, a.working, a.mask, a.delta, s_tier, s_u, &nu);
      s_nu = nu;
    } else {
      int nu;
      plan_tiers(a.r, norms, ny, a.working, a.mask, a.delta, s_tier, s_u, &nu);
      s_nu = nu;
    }
  }
  __syncthreads();
  Plan* P = (Plan*)(ws + L.off_plan);
  if (t <= a.r) {
    P->tier[t] = s_tier[t];
    P->u[t] = s_u[t];
    P->normB[t] = norms[t];
  }
  if (t == 0) {
    P->normY = s_ny;
    P->normX = s_nx;
    P->nu = s_nu;
  }
  __syncthreads();
}

}  // namespace psk
