// Internal declarations shared by the host driver (ps_api.cpp) and the HIP
// kernel files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ps.h"

namespace psk {

constexpr int kMaxSigma = 500;  // largest number of squarings
constexpr int kMaxDegree = 255;  // coefficients travel by value in kernel arguments
constexpr int kTileM = 64;       // output tile rows of every GEMM kernel
constexpr int kTileN = 64;       // output tile columns
constexpr int kTile = kTileM;    // row padding unit of the packed layouts
constexpr int kKPad = 128;       // K padding of the packed low-precision layouts
constexpr int kRowChunk = 256;   // rows per wave in the column passes
// Y = X^s formed by an FP32 product (FP64 working precision) is kept for an
// FP32 Horner product only when that product's u_i >= kY32Margin * 2^-24: the
// FP32 product's normwise error measured ~5.4 u32 on N(0,1) matrices
constexpr double kY32Margin = 16.0;

__host__ __device__ inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Per-matrix plan as written by the planning kernel (device) or the host.
struct Plan {
  int tier[PS_MAX_BLOCKS];
  double u[PS_MAX_BLOCKS];
  double normB[PS_MAX_BLOCKS];
  double normY;
  double normX;                     // ||X||_1 (X = X_1)
  int nu;
  int pad_[3];
  double abs_coef[kMaxDegree + 1];  // |c_k|, written by the block assembly for the a-priori rule
};

struct Coefs {
  double c[kMaxDegree + 1];
};

// Byte layout of the per-matrix workspace region for one PS evaluation
// (optionally followed by squarings).  All offsets are relative to the start
// of the matrix's region and 256-byte aligned.
struct Layout {
  int64_t n;
  int m, s, r, sigma;
  int working;         // 0 = FP64, 1 = FP32, 4 = double-double
  int esize;           // bytes of the working type (16: two FP64 planes)
  int trivial_last;    // s divides m: B_r = c_m I, step r folded into B_{r-1}
  int first_step;      // index of the first Horner product formed by a GEMM (0 = none)
  int square_arg;      // power table of A^2 instead of A
  int64_t Mp, Kp;      // padded sizes of the packed BF16/FP8 layouts
  size_t slot;         // bytes of one n x n working-precision matrix
  size_t pslot;        // bytes of one Horner iterate buffer (any format)
  size_t off_pow;      // X_2..X_s (s-1 slots); with square_arg slot 0 holds Z = A^2
  int npow;            // number of power slots
  size_t off_B;        // B_0..B_{nB-1}
  int nB;
  size_t off_P0, off_P1, off_R;
  size_t off_yf32, off_ybf16, off_yfp8, off_yfp8s;
  size_t off_colsum;   // (nB + 2) * nchunks * n doubles: partial column abs sums of B_i, Y and X
  int colsum_rows;     // rows per partial column sum (nchunks = ceil(n / colsum_rows))
  size_t off_plan;
  size_t off_coef;     // double-double coefficients (hi[m+1], lo[m+1]); double-double path only
  size_t bytes;        // total per matrix
};

Layout make_layout(ps_dtype dt, int64_t n, int m, int s, int sigma, int square_arg, int npow_min = 0,
                   int colsum_rows = kRowChunk);

}  // namespace psk

// Records `msg` as the thread's last error (ps_last_error) and returns st.
ps_status ps_set_error(ps_status st, const char* msg);

namespace psk {

// ---------------------------------------------------------------------------
// Kernel launchers (defined in ps_kernels.hip).  All take a batch of matrices
// addressed as base + b * stride (strides in bytes for workspace pointers, in
// elements for user pointers).
// ---------------------------------------------------------------------------
struct MatArg {
  const void* p;
  int64_t ld;
  int64_t stride;   // elements between consecutive matrices of the batch
};

// C = alpha * op(A) op(B)  (accumulate != 0: C += alpha * op(A) op(B)).
hipError_t launch_gemm(int working, int64_t n, int batch, MatArg A, int transA, MatArg B, int transB,
                       MatArg C, double alpha, int accumulate, hipStream_t st);

// Several independent products of order n in one launch (up to 8):
// C_k = alpha_k A_k B_k, no transposes; grid (tiles, count, batch).
constexpr int kMaxGroup = 8;
struct GemmGroup {
  MatArg A[kMaxGroup], B[kMaxGroup], C[kMaxGroup];
  double alpha[kMaxGroup];
  int f32[kMaxGroup];   // FP64 working precision only: product k in FP32, its C an FP32 matrix
  int count;
};
hipError_t launch_gemm_group(int working, int64_t n, int batch, const GemmGroup& g, hipStream_t st);

// Power table by binary splitting: X_j = X_a X_b with a = ceil(j/2),
// b = floor(j/2) (X_1 = beta A).  Powers with the same ceil(log2 j) depend
// only on lower ones, so each such level is one grouped launch.
inline int pow_a(int j) { return (j + 1) / 2; }
inline int pow_b(int j) { return j / 2; }

// Column pass: B_0..B_r, folded last step, column abs sums, low-precision Y copies.
struct AssembleArgs {
  int64_t n;
  int64_t nv;           // order of the matrix inside n (rows, columns >= nv are zero padding)
  int m, s, r, nB, trivial_last;
  MatArg X1;            // X_1 = x1_scale * X1
  double x1_scale;
  int pow_shift;        // X_j = 2^(j pow_shift) * (power slot j), j >= 2 (exact rescaling)
  char* ws;             // base of matrix 0's region
  size_t ws_stride;     // bytes per matrix
  Layout L;
  unsigned tier_mask;   // which low-precision copies of Y to produce
  int y_f32;            // Y was formed in FP32 into the FP32 copy's slot: read it there
};
hipError_t launch_assemble(int working, const AssembleArgs& a, const Coefs& c, int batch, hipStream_t st);

// Per-matrix planning kernel.
struct PlanArgs {
  int r, mode, working, nB, trivial_last;
  int rule;             // PS_RULE_BLOCKS or PS_RULE_APRIORI
  unsigned mask;
  double delta;
  double abs_cm;        // |c_m| (norm of B_r = c_m I when s divides m)
  int use_override;
  int override_tier[PS_MAX_BLOCKS];
  char* ws;
  size_t ws_stride;
  Layout L;
};
hipError_t launch_plan(const PlanArgs& a, int batch, hipStream_t st);

// 1-norm pieces: wgmax[g] = max over the columns of workgroup g (NW columns)
// of the column abs sums of the n x n matrix X (leading dimension ld).
hipError_t launch_norm1(int working, int64_t n, MatArg X, double* wgmax, hipStream_t st);
inline int64_t norm1_groups(int64_t n) { return (n + 7) / 8; }

// B = (accumulate ? B : 0) + c_id I + sum_k c[k] M[k], and the per-workgroup
// maxima (norm1_groups(n) of each) of the column abs sums of the new B and of Y
constexpr int kMaxComb = 16;
struct CombArgs {
  MatArg M[kMaxComb];
  double c[kMaxComb];
  int count;
  double c_id;
  int accumulate;
  MatArg B, Y;
  double* wgB;
  double* wgY;
};
hipError_t launch_comb_norm(int working, int64_t n, const CombArgs& a, hipStream_t st);

// Estimates of ||e^X||_1 for K scalings at once (eq. (alpha_m-X)): for each
// k < K the per-workgroup maxima (norm1_groups(n) of each, at wg + k * G) of
// the column abs sums of w[k][0] I + sum_{j=1..J} w[k][j] M[j-1].
constexpr int kXiWin = 16;
struct XiArgs {
  MatArg M[kMaxComb];
  int J, K;
  double w[kXiWin][kMaxComb + 1];
  double* wg;
};
hipError_t launch_xi_norms(int working, int64_t n, const XiArgs& a, hipStream_t st);

// Non-finite entries of `batch` matrices of order n: for matrix b the count
// per workgroup (norm1_groups(n) doubles) at (double*)(wg + b * wg_stride).
hipError_t launch_count_nonfinite(int working, int64_t n, int batch, MatArg X, char* wg, size_t wg_stride,
                                  hipStream_t st);

// One Horner step: P_{i-1} = B_{i-1} + P_i Y (or, with cast_only, P = B_src
// converted to the format of the consumer step).
struct HornerArgs {
  int64_t n;
  int step;              // i (product P_i Y); for cast_only: the consumer step index
  int cast_only;
  int final_out;         // output is the working-precision result (to `out`)
  MatArg out;            // final output (working precision)
  size_t off_pin, off_pout;   // Horner iterate buffers in the workspace
  size_t off_bsrc;       // B_{i-1} (or the cast source) in the workspace
  MatArg ysrc;           // Y in working precision (X_s slot, or X1 when s == 1)
  double yscale;         // applied to the working-precision product (s == 1)
  char* ws;
  size_t ws_stride;
  Layout L;
  // cast launch only, Y formed in FP32: when the plan keeps a Horner product
  // (or the folded last step) in the working precision, the launch first
  // forms Y = y_alpha Ya Yb in the working precision into Yc (the power slot
  // of X_s)
  int y_cond;
  MatArg ya, yb, yc;
  double y_alpha;
  double y_cm;           // c_m (working precision) when s divides m: the fold c_m Y is redone with that Y
};
hipError_t launch_horner(int working, const HornerArgs& a, int batch, hipStream_t st);

// Elementwise scale/copy used by the drivers: dst = alpha * src (n x n).
hipError_t launch_scale_copy(int working, int64_t n, int batch, MatArg src, MatArg dst, double alpha,
                             hipStream_t st);

// Fill an n x n matrix with alpha * I (graph-safe replacement for memset).
hipError_t launch_fill_identity(int working, int64_t n, int batch, MatArg dst, double alpha, hipStream_t st);

// Adjoint helper: for j = 0..nd-1 with coef[j] != 0: dst_j += coef[j] * src
// (dst_j = dst base + j * dst_step bytes), all n x n column-major, per matrix
// of the batch (workspace stride ws_stride, user stride in MatArg).
struct ScatterArgs {
  int64_t n;
  int nd;
  MatArg src;
  char* dst;            // first destination (ld n)
  size_t dst_step;      // bytes between destinations
  size_t ws_stride;     // bytes between matrices for dst
  double coef[PS_MAX_BLOCKS];
};
hipError_t launch_scatter(int working, const ScatterArgs& a, int batch, hipStream_t st);

// Adjoint products in the forward plan's tiers.  The tier of Horner step
// `step` is read on the device from each matrix's Plan (L.off_plan in the
// matrix's workspace region); when it is the working precision nothing is
// packed and the product runs on the working-precision operands.
// k_tpack writes op(src) in the step's operand format into the workspace
// (L.pslot bytes at off_dst): role 0 (left operand) the rows of op(src),
// role 1 (right operand) the columns of op(src), K-contiguous for BF16 and
// FP8 (FP8 with E8M0 scales per 32 K elements); op(src) column-major for an
// FP32 product under an FP64 working precision.
struct TPackArgs {
  int64_t n;
  int step;
  int role;
  MatArg src;            // working precision
  int trans;             // op(src) = src^T
  size_t off_dst;
  char* ws;
  size_t ws_stride;
  Layout L;
};
hipError_t launch_tpack(int working, const TPackArgs& a, int batch, hipStream_t st);

// C = alpha op(A) op(B) (+ C if accumulate), the product in step's tier:
// the working-precision operands A, B when the tier is the working
// precision, otherwise the packed copies at off_pa (role 0 of op(A)) and
// off_pb (role 1 of op(B)).  Supported: (transA, transB) = (0, 1) or (1, 0).
struct TGemmArgs {
  int64_t n;
  int step;
  MatArg A, B, C;
  int transA, transB;
  double alpha;
  int accumulate;
  size_t off_pa, off_pb;
  char* ws;
  size_t ws_stride;
  Layout L;
};
hipError_t launch_tgemm(int working, const TGemmArgs& a, int batch, hipStream_t st);

// dst = alpha * (x + y) elementwise (n x n, batch).
hipError_t launch_axpby(int working, int64_t n, int batch, MatArg x, MatArg y, MatArg dst, double alpha,
                        hipStream_t st);

// LU solve Q X = P (ps_solve.hip): Q (n x n) is overwritten by its factors
// (unit L below the diagonal, U on and above), P (n x nrhs) by X.  ws holds
// lu_solve_ws_bytes(n): the first int is the first zero pivot (1-based, 0 =
// none) and the pivots follow unless piv_out (device, n ints) is given.
size_t lu_solve_ws_bytes(int64_t n);
constexpr int64_t kMaxSolveOrder = 8192;
hipError_t launch_lu_solve(int working, int64_t n, void* Q, int64_t ldq, int64_t nrhs, void* P, int64_t ldp,
                           int* piv_out, char* ws, hipStream_t st);

}  // namespace psk
