// HIP kernels of the Paterson--Stockmeyer (PS) hot path for gfx950 (MI355X).
//
// Method: X. Liu, arXiv 2312.17396.  p(X) = sum_i B_i (X^s)^i (eq. (ps)),
// Horner in Y = X^s (eq. (ps-Horner)); mixed precision per Theorem 2.1 and
// Algorithms 2/3: product i in precision u_i, the following sum in u_{i-1}.
//
// Kernels
//   k_gemm      C = alpha op(A) op(B) (+C): power table X_{j+1} = X_j X
//               (Algorithm 1), squarings R <- R^2 (eq. (scal-idea)) and the
//               adjoint products.  FP64 or FP32 MFMA 16x16x4, 64x64 output tile
//               per 512-thread workgroup (8 waves of 32x16, each two 16x16
//               MFMA blocks), K staged through two LDS stages in slabs of 32.
//   k_gemm_group several independent products of one order in one launch
//               (the levels of the power table).
//   k_horner    one Horner step P_{i-1} = B_{i-1} + P_i Y.  The product runs in
//               the step's tier (FP64 / FP32 MFMA 16x16x4, BF16 MFMA 16x16x32,
//               FP8 E4M3 MFMA 16x16x128 with E8M0 scales per 32 K-elements);
//               the epilogue adds B_{i-1} in the next step's precision and
//               writes P_{i-1} directly in the operand format that step reads.
//   k_assemble  B_0..B_r = sum_j c_{si+j} X_j in the working precision (the
//               paper assembles the blocks in u, section 2), their column
//               absolute sums (exact ||B_i||_1, ||Y||_1 for the plan) and the
//               low-precision copies of Y, one wave per column.
//   k_plan      per-matrix precision plan from those norms (ps_planner.h).
//
// MFMA accumulator layouts used below (probed on gfx950):
//   f64 16x16x4 : lane l holds D[4v + l/16][l%16], v = 0..3
//   f32 16x16x4, bf16 16x16x32, f8f6f4 16x16x128 : D[4(l/16) + v][l%16]
//   operands (f64, f32, bf16): lane l holds A[l%16][kb + e] and
//   B[kb + e][l%16] with kb = (l/16) * (K/4), e over K/4 consecutive elements;
//   f8f6f4 16x16x128 interleaves K and its scales, see mainloop_lowp.
#include "ps_device.h"

namespace psk {

// ---------------------------------------------------------------------------
// k_gemm: one 64 x kTileN tile per workgroup
// ---------------------------------------------------------------------------
template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(NT) void k_gemm(int64_t n, MatArg A, MatArg B, MatArg C, double alpha, int accumulate) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<T>()];
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int64_t b = blockIdx.z;
  gemm_tile<T, TA, TB>((const T*)A.p + b * A.stride, A.ld, (const T*)B.p + b * B.stride, B.ld,
                       (T*)C.p + b * C.stride, C.ld, n, n, (int64_t)tm * kTileM, (int64_t)tn * kTileN, alpha,
                       accumulate, smem);
}

// k_gemm_group: product blockIdx.y of a group, one 64 x kTileN tile per workgroup
template <typename T>
__global__ __launch_bounds__(NT) void k_gemm_group(int64_t n, GemmGroup g) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<T>()];
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int k = blockIdx.y;
  const int64_t b = blockIdx.z;
  const MatArg A = g.A[k], B = g.B[k], C = g.C[k];
  if (std::is_same<T, double>::value && g.f32[k]) {   // uniform per workgroup (product k)
    gemm_tile_f32_of_f64((const double*)A.p + b * A.stride, A.ld, (const double*)B.p + b * B.stride, B.ld,
                         (float*)C.p + b * C.stride, C.ld, n, (int64_t)tm * kTileM, (int64_t)tn * kTileN,
                         g.alpha[k], smem);
    return;
  }
  gemm_tile<T, false, false>((const T*)A.p + b * A.stride, A.ld, (const T*)B.p + b * B.stride, B.ld,
                             (T*)C.p + b * C.stride, C.ld, n, n, (int64_t)tm * kTileM, (int64_t)tn * kTileN,
                             g.alpha[k], 0, smem);
}

hipError_t launch_gemm_group(int working, int64_t n, int batch, const GemmGroup& g, hipStream_t st) {
  if (g.count < 1 || g.count > kMaxGroup) return hipErrorInvalidValue;
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  dim3 grid(ntm * ntn, g.count, batch), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_gemm_group<double>, grid, block, 0, st, n, g);
  else hipLaunchKernelGGL(k_gemm_group<float>, grid, block, 0, st, n, g);
  return hipGetLastError();
}

hipError_t launch_gemm(int working, int64_t n, int batch, MatArg A, int transA, MatArg B, int transB,
                       MatArg C, double alpha, int accumulate, hipStream_t st) {
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  dim3 grid(ntm * ntn, 1, batch), block(NT);
#define PS_LAUNCH_GEMM(T, ta, tb) \
  hipLaunchKernelGGL((k_gemm<T, ta, tb>), grid, block, 0, st, n, A, B, C, alpha, accumulate)
  if (working == 0) {
    if (!transA && !transB) PS_LAUNCH_GEMM(double, false, false);
    else if (transA && !transB) PS_LAUNCH_GEMM(double, true, false);
    else if (!transA && transB) PS_LAUNCH_GEMM(double, false, true);
    else PS_LAUNCH_GEMM(double, true, true);
  } else {
    if (!transA && !transB) PS_LAUNCH_GEMM(float, false, false);
    else if (transA && !transB) PS_LAUNCH_GEMM(float, true, false);
    else if (!transA && transB) PS_LAUNCH_GEMM(float, false, true);
    else PS_LAUNCH_GEMM(float, true, true);
  }
#undef PS_LAUNCH_GEMM
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_horner: one tile of one Horner step per workgroup
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_horner(HornerArgs a) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  const Layout& L = a.L;
  const int ntm = (int)((a.n + kTileM - 1) / kTileM), ntn = (int)((a.n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int64_t b = blockIdx.z;
  char* ws = a.ws + b * a.ws_stride;
  const Plan* plan = (const Plan*)(ws + L.off_plan);
  bool y64 = false;
  if (a.y_cond) {
    // Y was formed in FP32; a Horner product in the working precision (the
    // folded step r included) needs it in the working precision as well, and
    // so does an FP32 product whose u_i is below kY32Margin u32 (eq. (cond-Y):
    // Y must be accurate to u_i, and the FP32 product's error is ~5 u32).
    // Lane i - 1 of every wave tests step i (r < PS_MAX_BLOCKS): one round
    // trip to the plan instead of one per step.
    const int i = 1 + (int)(threadIdx.x & 63);
    bool need = false;
    if (i <= L.r) {
      const int ti = plan->tier[i];
      const double ui = plan->u[i];
      need = ti == WT || (ti == 1 && ui < kY32Margin * 0x1p-24);
    }
    y64 = __any(need);
    if (y64)
      gemm_tile<W, false, false>((const W*)a.ya.p + b * a.ya.stride, a.ya.ld, (const W*)a.yb.p + b * a.yb.stride,
                                 a.yb.ld, (W*)a.yc.p + b * a.yc.stride, a.yc.ld, a.n, a.n, (int64_t)tm * kTileM,
                                 (int64_t)tn * kTileN, a.y_alpha, 0, smem);
  }
  HornerTile<W> h;
  h.fy64 = (const W*)a.yc.p + b * a.yc.stride;
  h.fy32 = (const float*)(ws + L.off_yf32);
  h.fyc = (y64 && L.trivial_last) ? a.y_cm : 0.0;   // the assembly folded c_m Y with Y in FP32
  h.n = a.n;
  h.Mp = L.Mp;
  h.Kp = L.Kp;
  h.t_in = a.cast_only ? -1 : plan->tier[a.step];
  h.t_out = a.final_out ? WT : plan->tier[a.cast_only ? a.step : a.step - 1];
  h.pin = ws + a.off_pin;
  h.ysrc = (const W*)a.ysrc.p + b * a.ysrc.stride;
  h.ldy = a.ysrc.ld;
  h.yscale = a.yscale;
  h.yf32 = (const float*)(ws + L.off_yf32);
  h.ybf16 = (const uint16_t*)(ws + L.off_ybf16);
  h.yfp8 = (const uint8_t*)(ws + L.off_yfp8);
  h.yfp8s = (const uint8_t*)(ws + L.off_yfp8s);
  h.bsrc = (const W*)(ws + a.off_bsrc);
  h.pout = ws + a.off_pout;
  h.outw = a.final_out ? ((W*)a.out.p + b * a.out.stride) : (W*)(ws + a.off_pout);
  h.ldo = a.final_out ? a.out.ld : a.n;
  h.nv = a.n;
  h.nvb = a.n;
  horner_tile<W, true>(h, (int64_t)tm * kTileM, (int64_t)tn * kTileN, smem);
  if (y64) {
    // the FP32 copy of Y that the FP32 products read becomes the rounding of
    // the working-precision Y (after the fold correction above has read the
    // FP32-formed one); this workgroup wrote the tile, and horner_tile ended
    // with a barrier
    const int t = threadIdx.x, row = t & 63;
    const int64_t gr = (int64_t)tm * kTileM + row;
    const W* yc = (const W*)a.yc.p + b * a.yc.stride;
    float* y32 = (float*)(ws + L.off_yf32);
#pragma unroll 4
    for (int q = 0; q < TILE_Q; ++q) {
      const int64_t gc = (int64_t)tn * kTileN + (t >> 6) + NW * q;
      if (gr < a.n && gc < a.n) y32[gr + gc * a.n] = (float)yc[gr + gc * a.yc.ld];
    }
  }
}

hipError_t launch_horner(int working, const HornerArgs& a, int batch, hipStream_t st) {
  const int ntm = (int)((a.n + kTileM - 1) / kTileM), ntn = (int)((a.n + kTileN - 1) / kTileN);
  dim3 grid(ntm * ntn, 1, batch), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_horner<double>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(k_horner<float>, grid, block, 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_tpack / k_tgemm: the adjoint's Horner products in the tier that the
// forward plan gave the step (read from each matrix's Plan on the device)
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) void k_tpack(TPackArgs a) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  __shared__ __attribute__((aligned(16))) W Cs[kTileN * CSTR];
  const int64_t b = blockIdx.z;
  char* ws = a.ws + b * a.ws_stride;
  const int tier = ((const Plan*)(ws + a.L.off_plan))->tier[a.step];
  if (tier == WT) return;   // uniform over the grid's matrix: nothing to pack
  const int64_t n = a.n;
  const int ntm = (int)((n + kTileM - 1) / kTileM);
  const int64_t m0 = (int64_t)(blockIdx.x % ntm) * kTileM, n0 = (int64_t)(blockIdx.x / ntm) * kTileN;
  const W* src = (const W*)a.src.p + b * a.src.stride;
  const int64_t ld = a.src.ld;
  // tile of Z = op(src) (FP32 copy, or a left operand) or Z = op(src)^T (the
  // right operand of a BF16 / FP8 product, whose columns become rows);
  // tz: Z is src transposed.  The lanes run along src's contiguous index.
  const bool tz = (tier == 1 || a.role == 0) ? a.trans != 0 : a.trans == 0;
  const int t = threadIdx.x, lane = t & 63;
#pragma unroll
  for (int q = 0; q < TILE_Q; ++q) {
    const int o = (t >> 6) + NW * q;
    const int r = tz ? o : lane, c = tz ? lane : o;   // Z(r, c) of the tile
    const int64_t zr = m0 + r, zc = n0 + c;
    const bool in = zr < n && zc < n;
    const W v = src[in ? (tz ? zc + zr * ld : zr + zc * ld) : 0];
    Cs[c * CSTR + r] = in ? v : W(0);
  }
  __syncthreads();
  char* dst = ws + a.off_dst;
  if (tier == 1) {   // FP32 product under an FP64 working precision: Z column-major, ld n
    float* d = (float*)dst;
#pragma unroll
    for (int q = 0; q < TILE_Q; ++q) {
      const int col = (t >> 6) + NW * q;
      if (m0 + lane < n && n0 + col < n) d[(m0 + lane) + (n0 + col) * n] = (float)Cs[col * CSTR + lane];
    }
  } else {
    pack_tile_lowp<W>(Cs, tier, dst, a.L.Mp, a.L.Kp, m0, n0);
  }
}

template <typename W, bool TA, bool TB>
__global__ __launch_bounds__(NT) void k_tgemm(TGemmArgs a) {
  constexpr int WT = std::is_same<W, double>::value ? 0 : 1;
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<W>()];
  const int64_t b = blockIdx.z;
  char* ws = a.ws + b * a.ws_stride;
  const int tier = ((const Plan*)(ws + a.L.off_plan))->tier[a.step];
  const int64_t n = a.n;
  const int ntm = (int)((n + kTileM - 1) / kTileM), ntn = (int)((n + kTileN - 1) / kTileN);
  int tm, tn;
  tile_of_block(ntm, ntn, tm, tn);
  const int64_t m0 = (int64_t)tm * kTileM, n0 = (int64_t)tn * kTileN;
  W* C = (W*)a.C.p + b * a.C.stride;
  if (tier == WT) {
    gemm_tile<W, TA, TB>((const W*)a.A.p + b * a.A.stride, a.A.ld, (const W*)a.B.p + b * a.B.stride, a.B.ld, C,
                         a.C.ld, n, n, m0, n0, a.alpha, a.accumulate, smem);
    return;
  }
  const char* pa = ws + a.off_pa;
  const char* pb = ws + a.off_pb;
  W* Cs = (W*)smem;
  if (tier == 1) {
    typename MF<float>::V acc[2];
    mainloop_lds<float, false, false>((const float*)pa, n, (const float*)pb, n, n, m0, n0, smem, acc);
    frag_to_cs<float, W>(acc, Cs, 1.0);
  } else {
    f4v acc[2];
    const int64_t Mp = a.L.Mp, Kp = a.L.Kp;
    const uint8_t* qa = (const uint8_t*)pa;
    const uint8_t* qb = (const uint8_t*)pb;
    if (tier == 3) mainloop_lowp<true>(qa, qa + Mp * Kp, qb, qb + Mp * Kp, Kp, n, m0, n0, smem, acc);
    else mainloop_lowp<false>(qa, nullptr, qb, nullptr, Kp, n, m0, n0, smem, acc);
    frag_f32_to_cs_any(acc, (double*)smem, (float*)smem, WT == 0);
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int row = t & 63;
  const int64_t gr = m0 + row;
#pragma unroll 4
  for (int q = 0; q < TILE_Q; ++q) {
    const int col = (t >> 6) + NW * q;
    const int64_t gc = n0 + col;
    if (gr < n && gc < n) {
      const W v = (W)(a.alpha * (double)Cs[col * CSTR + row]);
      W* dst = C + gr + gc * a.C.ld;
      if (a.accumulate) *dst = *dst + v;
      else *dst = v;
    }
  }
}

hipError_t launch_tpack(int working, const TPackArgs& a, int batch, hipStream_t st) {
  const int nt = (int)((a.n + kTileM - 1) / kTileM);
  dim3 grid(nt * nt, 1, batch), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_tpack<double>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(k_tpack<float>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_tgemm(int working, const TGemmArgs& a, int batch, hipStream_t st) {
  const int ntm = (int)((a.n + kTileM - 1) / kTileM), ntn = (int)((a.n + kTileN - 1) / kTileN);
  dim3 grid(ntm * ntn, 1, batch), block(NT);
  if (!a.transA && a.transB) {
    if (working == 0) hipLaunchKernelGGL((k_tgemm<double, false, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tgemm<float, false, true>), grid, block, 0, st, a);
  } else if (a.transA && !a.transB) {
    if (working == 0) hipLaunchKernelGGL((k_tgemm<double, true, false>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tgemm<float, true, false>), grid, block, 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_assemble: one wave per (column, row chunk)
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_assemble(AssembleArgs a, Coefs cf) {
  const int w = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * NW + w;
  if (col >= a.n) return;  // no block-wide synchronisation below
  const int64_t b = blockIdx.z;
  char* ws = a.ws + b * a.ws_stride;
  const W* X1 = (const W*)a.X1.p + b * a.X1.stride;
  assemble_column<W, true>(a, cf, ws, X1, col, blockIdx.y);
}

hipError_t launch_assemble(int working, const AssembleArgs& a, const Coefs& c, int batch, hipStream_t st) {
  dim3 grid((unsigned)((a.n + NW - 1) / NW), (unsigned)((a.n + kRowChunk - 1) / kRowChunk), batch), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_assemble<double>, grid, block, 0, st, a, c);
  else hipLaunchKernelGGL(k_assemble<float>, grid, block, 0, st, a, c);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_norm1: column abs sums (one wave per column), maximum per workgroup
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) void k_norm1(int64_t n, MatArg X, double* wgmax) {
  __shared__ double red[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t col = (int64_t)blockIdx.x * NW + w;
  const W* x = (const W*)X.p;
  double v = 0.0;
  if (col < n) {
    double part[4] = {0.0, 0.0, 0.0, 0.0};   // four independent partial sums per lane
    for (int64_t r0 = 0; r0 < n; r0 += 256) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t rw = r0 + 64 * q + lane;
        part[q] += (rw < n) ? fabs((double)x[rw + col * X.ld]) : 0.0;
      }
    }
    v = (part[0] + part[1]) + (part[2] + part[3]);
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  }
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (t == 0) {
    double m = red[0];
    for (int k = 1; k < NW; ++k)
      if (red[k] > m || red[k] != red[k]) m = red[k];
    wgmax[blockIdx.x] = m;
  }
}

hipError_t launch_norm1(int working, int64_t n, MatArg X, double* wgmax, hipStream_t st) {
  const dim3 grid((unsigned)norm1_groups(n)), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_norm1<double>, grid, block, 0, st, n, X, wgmax);
  else hipLaunchKernelGGL(k_norm1<float>, grid, block, 0, st, n, X, wgmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_comb_norm: a linear combination of matrices into B (one wave per column)
// with the column abs sums of B and Y, maximum per workgroup
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) void k_comb_norm(int64_t n, CombArgs a) {
  __shared__ double red[2][NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t col = (int64_t)blockIdx.x * NW + w;
  double vb = 0.0, vy = 0.0;
  if (col < n) {
    W* b = (W*)a.B.p + col * a.B.ld;
    const W* y = (const W*)a.Y.p + col * a.Y.ld;
    for (int64_t rw = lane; rw < n; rw += 64) {
      double v = a.accumulate ? (double)b[rw] : 0.0;
      for (int k = 0; k < a.count; ++k) v += a.c[k] * (double)((const W*)a.M[k].p)[rw + col * a.M[k].ld];
      if (rw == col) v += a.c_id;
      const W out = (W)v;
      b[rw] = out;
      vb += fabs((double)out);
      vy += fabs((double)y[rw]);
    }
    for (int off = 32; off >= 1; off >>= 1) {
      vb += __shfl_xor(vb, off, 64);
      vy += __shfl_xor(vy, off, 64);
    }
  }
  if (lane == 0) {
    red[0][w] = vb;
    red[1][w] = vy;
  }
  __syncthreads();
  if (t < 2) {
    double m = red[t][0];
    for (int k = 1; k < NW; ++k)
      if (red[t][k] > m || red[t][k] != red[t][k]) m = red[t][k];
    (t == 0 ? a.wgB : a.wgY)[blockIdx.x] = m;
  }
}

hipError_t launch_comb_norm(int working, int64_t n, const CombArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)norm1_groups(n)), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_comb_norm<double>, grid, block, 0, st, n, a);
  else hipLaunchKernelGGL(k_comb_norm<float>, grid, block, 0, st, n, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_xi_norms: column abs sums of K combinations of the same J matrices (one
// wave per column, every matrix read once), maximum per workgroup and
// combination
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) void k_xi_norms(int64_t n, XiArgs a) {
  __shared__ double red[kXiWin][NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t col = (int64_t)blockIdx.x * NW + w;
  double acc[kXiWin];
#pragma unroll
  for (int k = 0; k < kXiWin; ++k) acc[k] = 0.0;
  if (col < n) {
    for (int64_t rw = lane; rw < n; rw += 64) {
      double x[kMaxComb];
#pragma unroll
      for (int j = 0; j < kMaxComb; ++j)
        x[j] = j < a.J ? (double)((const W*)a.M[j].p)[rw + col * a.M[j].ld] : 0.0;
      const double id = rw == col ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < kXiWin; ++k) {
        double v = a.w[k][0] * id;
#pragma unroll
        for (int j = 0; j < kMaxComb; ++j)
          if (j < a.J) v += a.w[k][j + 1] * x[j];
        acc[k] += fabs(v);
      }
    }
#pragma unroll
    for (int k = 0; k < kXiWin; ++k)
      for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < kXiWin; ++k) red[k][w] = acc[k];
  __syncthreads();
  if (t < a.K) {
    double m = red[t][0];
    for (int q = 1; q < NW; ++q)
      if (red[t][q] > m || red[t][q] != red[t][q]) m = red[t][q];
    a.wg[(int64_t)t * gridDim.x + blockIdx.x] = m;
  }
}

hipError_t launch_xi_norms(int working, int64_t n, const XiArgs& a, hipStream_t st) {
  if (a.J < 0 || a.J > kMaxComb || a.K < 1 || a.K > kXiWin || NT / 64 != NW) return hipErrorInvalidValue;
  const dim3 grid((unsigned)norm1_groups(n)), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_xi_norms<double>, grid, block, 0, st, n, a);
  else hipLaunchKernelGGL(k_xi_norms<float>, grid, block, 0, st, n, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_count_nonfinite: NaN and infinity entries (one wave per column), count per
// workgroup; grid.y runs over the matrices of a batch
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(NT) void k_count_nonfinite(int64_t n, MatArg X, char* wg, size_t wg_stride) {
  __shared__ double red[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t col = (int64_t)blockIdx.x * NW + w;
  const W* x = (const W*)X.p + (int64_t)blockIdx.y * X.stride;
  double cnt = 0.0;
  if (col < n) {
    for (int64_t rw = lane; rw < n; rw += 64) cnt += isfinite((double)x[rw + col * X.ld]) ? 0.0 : 1.0;
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  }
  if (lane == 0) red[w] = cnt;
  __syncthreads();
  if (t == 0) {
    double c = 0.0;
    for (int k = 0; k < NW; ++k) c += red[k];
    ((double*)(wg + (size_t)blockIdx.y * wg_stride))[blockIdx.x] = c;
  }
}

hipError_t launch_count_nonfinite(int working, int64_t n, int batch, MatArg X, char* wg, size_t wg_stride,
                                  hipStream_t st) {
  const dim3 grid((unsigned)norm1_groups(n), (unsigned)batch), block(NT);
  if (working == 0) hipLaunchKernelGGL(k_count_nonfinite<double>, grid, block, 0, st, n, X, wg, wg_stride);
  else hipLaunchKernelGGL(k_count_nonfinite<float>, grid, block, 0, st, n, X, wg, wg_stride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_plan: one workgroup per matrix
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_plan(PlanArgs a) {
  __shared__ double red[8 * NW];
  __shared__ double norms[PS_MAX_BLOCKS + 2];
  char* ws = a.ws + (int64_t)blockIdx.x * a.ws_stride;
  plan_matrix<NT>(a, a.L, ws, red, norms);
}

hipError_t launch_plan(const PlanArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_plan, dim3(batch), dim3(NT), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
template <typename W>
__global__ void k_scale_copy(int64_t n, MatArg src, MatArg dst, double alpha) {
  const int64_t b = blockIdx.z;
  const int64_t col = blockIdx.y;
  const W* s = (const W*)src.p + b * src.stride;
  W* d = (W*)dst.p + b * dst.stride;
  for (int64_t rw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; rw < n; rw += (int64_t)gridDim.x * blockDim.x)
    d[rw + col * dst.ld] = (W)(alpha * (double)s[rw + col * src.ld]);
}
hipError_t launch_scale_copy(int working, int64_t n, int batch, MatArg src, MatArg dst, double alpha, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, batch);
  if (working == 0) hipLaunchKernelGGL(k_scale_copy<double>, grid, dim3(256), 0, st, n, src, dst, alpha);
  else hipLaunchKernelGGL(k_scale_copy<float>, grid, dim3(256), 0, st, n, src, dst, alpha);
  return hipGetLastError();
}

template <typename W>
__global__ void k_fill_identity(int64_t n, MatArg dst, double alpha) {
  const int64_t b = blockIdx.z;
  const int64_t col = blockIdx.y;
  W* d = (W*)dst.p + b * dst.stride;
  for (int64_t rw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; rw < n; rw += (int64_t)gridDim.x * blockDim.x)
    d[rw + col * dst.ld] = (rw == col) ? (W)alpha : W(0);
}
hipError_t launch_fill_identity(int working, int64_t n, int batch, MatArg dst, double alpha, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, batch);
  if (working == 0) hipLaunchKernelGGL(k_fill_identity<double>, grid, dim3(256), 0, st, n, dst, alpha);
  else hipLaunchKernelGGL(k_fill_identity<float>, grid, dim3(256), 0, st, n, dst, alpha);
  return hipGetLastError();
}

template <typename W>
__global__ void k_scatter(ScatterArgs a) {
  const int64_t b = blockIdx.z, col = blockIdx.y;
  const W* s = (const W*)a.src.p + b * a.src.stride;
  for (int64_t rw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; rw < a.n; rw += (int64_t)gridDim.x * blockDim.x) {
    const W v = s[rw + col * a.src.ld];
    for (int j = 0; j < a.nd; ++j) {
      if (a.coef[j] == 0.0) continue;
      W* d = (W*)(a.dst + b * a.ws_stride + (size_t)j * a.dst_step);
      d[rw + col * a.n] += (W)a.coef[j] * v;
    }
  }
}
hipError_t launch_scatter(int working, const ScatterArgs& a, int batch, hipStream_t st) {
  dim3 grid((unsigned)((a.n + 255) / 256), (unsigned)a.n, batch);
  if (working == 0) hipLaunchKernelGGL(k_scatter<double>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_scatter<float>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename W>
__global__ void k_axpby(int64_t n, MatArg x, MatArg y, MatArg dst, double alpha) {
  const int64_t b = blockIdx.z, col = blockIdx.y;
  const W* xs = (const W*)x.p + b * x.stride;
  const W* ys = (const W*)y.p + b * y.stride;
  W* d = (W*)dst.p + b * dst.stride;
  for (int64_t rw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; rw < n; rw += (int64_t)gridDim.x * blockDim.x)
    d[rw + col * dst.ld] = (W)(alpha * ((double)xs[rw + col * x.ld] + (double)ys[rw + col * y.ld]));
}
hipError_t launch_axpby(int working, int64_t n, int batch, MatArg x, MatArg y, MatArg dst, double alpha,
                        hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, batch);
  if (working == 0) hipLaunchKernelGGL(k_axpby<double>, grid, dim3(256), 0, st, n, x, y, dst, alpha);
  else hipLaunchKernelGGL(k_axpby<float>, grid, dim3(256), 0, st, n, x, y, dst, alpha);
  return hipGetLastError();
}

}  // namespace psk
