/*
 * ps.h -- C ABI of libps: Paterson--Stockmeyer (PS) evaluation of matrix
 * polynomials with scalar coefficients on AMD MI355X (gfx950), with
 * per-Horner-step precision tiers (FP64 / FP32 / BF16 / FP8 matrix cores).
 *
 * Method: X. Liu, "Mixed-Precision Paterson--Stockmeyer Method for Evaluating
 * Polynomials of Matrices", arXiv 2312.17396.
 *   p(X) = sum_{k=0}^{m} c_k X^k is written as sum_{i=0}^{r} B_i (X^s)^i,
 *   r = floor(m/s), B_i = sum_j c_{si+j} X^j (eq. (ps)), and evaluated by
 *   Horner's rule in Y = X^s (eq. (ps-Horner), Algorithm 1).  In mixed mode
 *   the product of Horner step i runs in the precision u_i chosen from
 *   ||B_0||, ||B_i|| and ||Y|| (Theorem 2.1, eq. (choose-ui), Algorithms 2
 *   and 3), rounded to the hardware tiers available (section 4.1.1).
 *
 * General conventions (every entry point):
 *  - Return value: a ps_status; PS_OK (0) on success, negative on error.
 *    Nothing throws or aborts across this boundary.
 *  - Matrices are square, real, column-major with a leading dimension
 *    (element (i,j) at ptr[i + j*ld]), ld >= n.  Since p(A^T) = p(A)^T for
 *    real coefficients, row-major data may be passed unchanged and the
 *    result comes back row-major too (the same holds for the gradient).
 *  - Pointers named A, G, P, E, grad are DEVICE pointers; coefficient arrays
 *    and size/index arrays are HOST pointers, copied before the call returns.
 *  - All arguments are validated on the host before any device work; on
 *    error no kernel is launched.  PS_ERR_ALIAS is returned when an output
 *    overlaps an input.
 *  - Work is queued asynchronously on `stream` (a hipStream_t; NULL = the
 *    null stream).  The caller keeps every buffer alive until the stream
 *    has completed.  When a ps_report is requested the call synchronises
 *    the stream before returning.
 *  - The library never allocates device memory: scratch space is the
 *    caller's `ws` of at least the size returned by the matching
 *    ps_workspace_size* query (256-byte aligned pointer required).
 *  - On error, output contents are unspecified.  IEEE non-finite values in
 *    the input propagate through the arithmetic, unless opts->check_finite
 *    is set (see ps_opts).
 */
#ifndef PS_H
#define PS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PS_OK = 0,
  PS_ERR_ARG = -1,         /* invalid size, degree, block size, pointer, ld */
  PS_ERR_ALIAS = -2,       /* output overlaps an input */
  PS_ERR_WORKSPACE = -3,   /* workspace missing, too small or misaligned */
  PS_ERR_NONFINITE = -4,   /* opts->check_finite: a NaN or infinity in an input, or in a result */
  PS_ERR_UNSUPPORTED = -5, /* valid request the library does not implement */
  PS_ERR_HIP = -6          /* a HIP runtime call failed; see ps_last_error() */
} ps_status;

/* Working (target) precision; also the element type of A and of the result. */
typedef enum {
  PS_F64 = 0,
  PS_F32 = 1,
  PS_DD = 2   /* double-double (two FP64 planes); ps_plan and the *_dd entry points only */
} ps_dtype;

/* Precision tiers of the Horner products (unit roundoffs 2^-53, 2^-24,
 * 2^-8, 2^-4).  FP8 is OCP E4M3 with a power-of-two (E8M0) scale per 32
 * consecutive elements along the reduction dimension. */
typedef enum { PS_TIER_F64 = 0, PS_TIER_F32 = 1, PS_TIER_BF16 = 2, PS_TIER_FP8 = 3 } ps_tier;

#define PS_MODE_FIXED 0   /* Algorithm 1: every product in the working precision */
#define PS_MODE_MIXED 1   /* Algorithms 2/3 (fixed s): per-step tiers from the norms.
                             With an FP64 working precision, FP32 allowed and n > 512,
                             ps_eval, ps_expm and ps_expm_strided_batched form Y = X^s by an
                             FP32 product (eq. (cond-Y): Y needs the accuracy u_nu of
                             the first lower-precision step) and again in FP64 (its
                             FP32 rounding then feeds the FP32 products) when the
                             plan keeps a Horner product in FP64 or has an FP32
                             product with u_i < 16 * 2^-24. */

#define PS_RULE_BLOCKS 0  /* tiers from the assembled blocks' 1-norms (Thm 2.1, eq. (choose-ui)) */
#define PS_RULE_APRIORI 1 /* tiers from coefficient magnitudes times powers of ||X||_1 */

#define PS_MAX_BLOCKS 64  /* r + 1 <= PS_MAX_BLOCKS */

typedef struct ps_opts {
  int mode;                  /* PS_MODE_FIXED or PS_MODE_MIXED */
  unsigned tier_mask;        /* bit t allows tier t; 0 = all tiers.  The working
                                tier is always allowed; tiers of higher precision
                                than the working one are never used. */
  double delta;              /* lower precision only where u_i >= delta*u
                                (section 3.2, default 10; <= 0 = default) */
  const int* tier_override;  /* optional host array of r+1 tiers (entry 0 ignored),
                                replaces the plan (testing); NULL = plan */
  int profile;               /* nonzero: time the phases with hipEvents */
  int rule;                  /* PS_RULE_BLOCKS (0, default): u_i from the 1-norms of
                                the assembled blocks, ||B_i|| ||Y||^i (eq. (choose-ui));
                                PS_RULE_APRIORI (1): the denominator bounded a priori by
                                sum_{k in block i} |c_k| ||X||^k, the numerator the
                                block norm ||B_0|| (never overestimated) */
  int check_finite;          /* nonzero: before any evaluation kernel the inputs are scanned
                                (one pass per matrix, then a stream synchronisation) and a
                                NaN or infinity returns PS_ERR_NONFINITE with nothing
                                evaluated; after the evaluation the results are scanned the
                                same way (an overflow returns PS_ERR_NONFINITE, the result
                                left in place).  ps_eval, ps_expm, ps_expm_noalloc,
                                ps_expm_strided_batched, ps_eval_multi, ps_expm_pade,
                                ps_expm_auto, ps_expm_select and ps_expm_vars; the others
                                return PS_ERR_UNSUPPORTED when it is set. */
} ps_opts;

typedef struct ps_report {
  int s, r, nu;              /* block size, floor(m/s), first low-precision step */
  int first_step;            /* index of the first Horner product formed as a GEMM */
  int tier[PS_MAX_BLOCKS];   /* tier[i]: precision of the product P_i * Y (i = 1..r) */
  double u[PS_MAX_BLOCKS];   /* u_i from eq. (choose-ui) (u_0 = working) */
  double normB[PS_MAX_BLOCKS]; /* ||B_i||_1 of the assembled blocks */
  double normY;              /* ||X^s||_1 (of the FP32-formed Y where mixed mode forms it so) */
  int gemms[4];              /* GEMMs per tier: powers (Y's product under its tier, counted
                                twice when it is also formed in FP64) + Horner + squarings */
  float ms_power, ms_assemble, ms_horner, ms_square;  /* profile != 0 only */
  double normX;              /* ||X||_1, X = 2^-sigma A (the first power) */
  double cost_saving;        /* C_r of eq. (Cr) read as the saving (Table 1):
                                1 - ((s-1) D + sum_{i=1..r} d_i) / ((s+r-1) D), D and d_i the
                                decimal digits -log10 u of the working precision and of
                                step i's tier (see ps_model_cost) */
  double m_low;              /* M_low of Table 2: the fraction of the s-1+r products run in
                                precision u^(1/2) or lower */
} ps_report;

/* Version of the ABI (major*10000 + minor*100 + patch). */
int ps_version(void);

/* Static text for a status code. */
const char* ps_strerror(int status);

/* Thread-local detail of the most recent failure in this thread ("" if none). */
const char* ps_last_error(void);

/* Built-in coefficients, correctly rounded to double from the exact rationals:
 *   ps_coef_taylor_exp: c_k = 1/k!, k = 0..m            (section 3)
 *   ps_coef_pade_exp:   numerator p_j and denominator q_j, j = 0..deg, of the
 *                       [deg/deg] Pade approximant of exp (section 4.1);
 *                       q_j = (-1)^j p_j
 *   ps_coef_taylor_cos: c_k = (-1)^k / (2k)!, k = 0..m, a polynomial in X^2
 *                       (section 4.2)
 * Output arrays have m+1 (deg+1) entries; m <= 170. */
ps_status ps_coef_taylor_exp(int m, double* coef);
ps_status ps_coef_pade_exp(int deg, double* p, double* q);
ps_status ps_coef_taylor_cos(int m, double* coef);

/* Precision plan of the mixed scheme from block norms (host only, no GPU).
 *   normB[0..r] = ||B_i||_1, normY = ||X^s||_1, dtype = working precision.
 *   Rule: u_i = u ||B_0|| / max_{j>=i} ||B_j|| ||Y||^j  (eq. (choose-ui) with
 *   nu = 1, made monotone as the framework of section 2 requires);
 *   nu = min{i : u_i >= delta u} (Algorithms 2, 3); tier(i) for i >= nu is the
 *   lowest-precision allowed tier whose unit roundoff does not exceed u_i
 *   (section 4.1.1); steps 1..nu-1 stay in the working precision.  A zero
 *   denominator gives u_i = +inf (the product is exactly zero).
 * Outputs tier[0..r], u[0..r] (caller arrays of r+1) and *nu. */
ps_status ps_plan(ps_dtype dtype, int r, const double* normB, double normY,
                  const ps_opts* opts, int* tier, double* u, int* nu);

/* The modelled cost of a plan (section 3.3.1, host only, no GPU): with D the
 * decimal digits -log10 u of the working precision dtype and d_i those of
 * the unit roundoff of tier[i] (2^-53, 2^-24, 2^-8, 2^-4; 2^-106 for
 * PS_DD), i = 1..r,
 *   *cost_saving = 1 - ((s-1) D + sum_i d_i) / ((s+r-1) D)   (eq. (Cr), Table 1)
 *   *m_low = #{i : u_tier(i) >= u^(1/2)} / (s-1+r)          (Table 2's M_low)
 * counting the s-1 powers in the working precision and every one of the r
 * Horner products, the trivial one of s | m included, as the paper does.
 * tier: host array of r+1 entries (entry 0 ignored), values 0..3 or 4 (dd). */
ps_status ps_model_cost(ps_dtype dtype, int s, int r, const int* tier, double* cost_saving, double* m_low);

/* ---------------------------------------------------------------------------
 * Single matrix.
 * ------------------------------------------------------------------------- */

/* Workspace bytes for ps_eval / ps_expm with these sizes (sigma = 0 for
 * ps_eval).  s = 0 selects ceil(sqrt(m)). */
ps_status ps_workspace_size(ps_dtype dtype, int64_t n, int m, int s, int sigma, size_t* bytes);

/* P = p(A) = sum_{k=0}^{m} coef[k] A^k  (Algorithm 1 in PS_MODE_FIXED,
 * Algorithm 3 with fixed s in PS_MODE_MIXED).
 *   n >= 1; A: n x n (lda >= n); coef: host array of m+1 doubles, used as
 *   given (rounded to float where an FP32 step consumes it); 0 <= m;
 *   1 <= s <= max(m,1) or s = 0 (= ceil(sqrt(m))); P: n x n output (ldp >= n),
 *   must not overlap A.  opts may be NULL (fixed mode).  report may be NULL. */
ps_status ps_eval(ps_dtype dtype, int64_t n, const void* A, int64_t lda,
                  const double* coef, int m, int s,
                  void* P, int64_t ldp, const ps_opts* opts, ps_report* report,
                  void* ws, size_t ws_bytes, void* stream);

/* E = r(A) = p(2^-sigma A)^(2^sigma): scaling and squaring (eq. (scal-idea))
 * around the PS evaluation of p at X = 2^-sigma A.  coef = NULL selects the
 * Taylor coefficients 1/k! (Algorithm 2's polynomial).  0 <= sigma <= 1000.
 * The squarings run in the working precision. */
ps_status ps_expm(ps_dtype dtype, int64_t n, const void* A, int64_t lda,
                  const double* coef, int m, int s, int sigma,
                  void* E, int64_t lde, const ps_opts* opts, ps_report* report,
                  void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ps_expm
 * with its workspace taken from a static device array of
 * PS_NOALLOC_SCRATCH_BYTES (128 MiB) that the library holds on each device it
 * runs on until the process ends (FP64, m = 30, s = 6, sigma > 0 fits up to
 * n = 1024).  Same arguments, kernels and results as ps_expm, minus the
 * workspace.  The call allocates nothing: no hipMalloc, hipFree or event; the
 * array's device address is looked up once per device (hipGetSymbolAddress,
 * under a lock).  The stream must belong to the current device.  Every call
 * on one device shares that device's array and leaves its contents behind;
 * nothing in it needs to start at zero, but calls that overlap on one device
 * (concurrent streams or host threads) race on it and must be serialised by
 * the caller.  Errors: PS_ERR_WORKSPACE when the layout of (n, m, s, sigma)
 * needs more than PS_NOALLOC_SCRATCH_BYTES (checked before any device work);
 * PS_ERR_UNSUPPORTED for opts->profile (it creates events); otherwise as
 * ps_expm. */
#define PS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
ps_status ps_expm_noalloc(ps_dtype dtype, int64_t n, const void* A, int64_t lda,
                          const double* coef, int m, int s, int sigma,
                          void* E, int64_t lde, const ps_opts* opts, ps_report* report,
                          void* stream);

/* Automatic scaling for the Taylor approximant (section 3.2, eq.
 * (alpha_m-X)).  theta_m: the largest theta with
 * sum_{k>m} theta^k / k! <= u, u the unit roundoff of dtype (2^-53 or
 * 2^-24), i.e. the bound's threshold when the estimate xi(X) of ||e^X||_1
 * is 1.  ps_expm_auto and ps_expm_select use it only for the first scaling
 * sigma0 of the powers; their acceptance test scales u by xi(X).  Host only.
 * 0 <= m <= 170. */
ps_status ps_theta_taylor(ps_dtype dtype, int m, double* theta);

/* Workspace bytes for ps_expm_auto (the power table reaches
 * max(s, d* + 1), d* = max{d : d(d-1) <= m+1}, and a squaring buffer). */
ps_status ps_workspace_size_auto(ps_dtype dtype, int64_t n, int m, int s, size_t* bytes);

/* E = p_m(2^-sigma A)^(2^sigma) with sigma chosen by the alpha_m bound:
 *   sigma0 = the smallest sigma >= 0 with 2^-sigma ||A||_1 <= theta_m;
 *   X0 = 2^-sigma0 A; the powers X0^2 .. X0^max(s, d*+1) are formed once;
 *   alpha = 2^sigma0 max(||X0^d*||_1^(1/d*), ||X0^(d*+1)||_1^(1/(d*+1)));
 *   sigma = the smallest sigma >= 0 whose X = 2^-sigma A passes eq.
 *   (alpha_m-X): sum_{k>m} t^k / k! <= u xi(X) at t = 2^-sigma alpha, with
 *   xi(X) = ||B_0(X)||_1, B_0 = sum_{j<s} X^j / j! (the leading PS block),
 *   as the estimate of ||e^X||_1 (t > 800 fails without the series; sigma
 *   may exceed sigma0 when xi < 1); with norm_guard != 0 also
 *   ||2^-sigma A||_1 <= s / e, the norm under which section 3 guarantees
 *   the decay the mixed plan relies on.
 * The PS evaluation reuses the power table (X^j = 2^(j (sigma0 - sigma)) X0^j,
 * an exact rescaling).  Taylor coefficients 1/k!, m <= 170; s as in
 * ps_expm.  The chosen sigma is written to *sigma_out (may be NULL).
 * Norms are 1-norms of the column-major matrix.  The call synchronizes the
 * stream for ||A||_1, for the two alpha_m norms and once per window of 16
 * candidate scalings (one launch forms xi for all of them), so it cannot be
 * captured into a graph.  Errors: PS_ERR_ARG also for non-finite input, and
 * when no sigma <= 500 passes. */
ps_status ps_expm_auto(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m, int s,
                       int norm_guard, void* E, int64_t lde, const ps_opts* opts,
                       ps_report* report, int* sigma_out, void* ws, size_t ws_bytes,
                       void* stream);

/* Workspace bytes for ps_expm_select (the power table up to the largest
 * candidate's max(s, d* + 1), the largest candidate layout, norm scratch). */
ps_status ps_workspace_size_select(ps_dtype dtype, int64_t n, int m_max, size_t* bytes);

/* E = p_m(2^-sigma A)^(2^sigma), Taylor coefficients, with the degree m and
 * the scaling sigma chosen together by the alpha_m bound (section 3.2, eq.
 * (alpha_m-X)): the candidates are the degrees m = q^2 and m = q(q+1) up to
 * m_max (the PS-optimal degrees: s = ceil(sqrt(m)) gives s - 1 powers and
 * floor(m/s) - [s | m] Horner products); sigma0 makes ||2^-sigma0 A||_1 at
 * most the largest candidate's theta; the powers of X0 = 2^-sigma0 A give
 * alpha_m; for each candidate the least sigma that passes the acceptance
 * test of ps_expm_auto (xi from that candidate's s) is taken, and the
 * candidate with the fewest products plus squarings (the smaller m
 * on ties) is evaluated on the same powers (exact power-of-two rescaling).
 * The candidates are examined in increasing m, and the search stops at the
 * first one whose products alone reach the best total (the PS cost grows
 * strictly along the list), so powers are formed only as far as
 * max(s, d* + 1) of the examined candidates.  chosen: host array of 3 ints
 * receiving m, s, sigma (may be NULL).  1 <= m_max <= 170.  The call
 * synchronizes the stream once for ||A||_1, once per extension of the
 * powers and once per window of candidate scalings.  The cost rule is this
 * library's own (the paper takes m from its reference algorithm).  Errors:
 * as ps_expm_auto. */
ps_status ps_expm_select(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m_max,
                         void* E, int64_t lde, const ps_opts* opts, ps_report* report,
                         int* chosen, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for ps_expm_vars: the power table X^2 .. X^m (s may grow to
 * m), the largest block / iterate / plan section over s0 <= s <= m, one
 * matrix for the running B_0 and the norm scratch. */
ps_status ps_workspace_size_vars(ps_dtype dtype, int64_t n, int m, int sigma, size_t* bytes);

/* E = p(2^-sigma A)^(2^sigma) with the block size chosen by Algorithm 2's
 * variable-s branch (fix_params = false, section 3.3): with X = 2^-sigma A and
 * s0 = ceil(sqrt(m)), if ||X||_1 <= s0 / e the call forms X^2 .. X^s0,
 * B_0 = sum_{j<s0} c_j X^j and Y = X^s0, then while ||Y||_1 > ||B_0||_1
 * ||X||_1^s and s < m it adds c_s Y to B_0, raises s by one and forms
 * Y = X Y, all in the working precision; otherwise s = s0.  The blocks, the
 * plan (the same rule as ps_expm), the Horner steps and the squarings then
 * run with the chosen s, reusing the powers.  coef = NULL selects the Taylor
 * coefficients 1/k! (m <= 170).  The chosen s goes to *s_out (may be NULL).
 * Norms are 1-norms of the column-major matrix.  The call synchronizes the
 * stream once per norm read (1 + number of growth steps + 1 when the branch
 * runs), so it cannot be captured into a graph.  Errors as ps_expm;
 * PS_ERR_ARG also for non-finite input, PS_ERR_UNSUPPORTED for
 * opts->tier_override. */
ps_status ps_expm_vars(ps_dtype dtype, int64_t n, const void* A, int64_t lda,
                       const double* coef, int m, int sigma,
                       void* E, int64_t lde, const ps_opts* opts, ps_report* report,
                       int* s_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Double-double working precision (u = 2^-106) with the FP64, FP32, BF16 and
 * MX-FP8 tiers below it: the multi-precision setting the paper is written
 * for (sections 1 and 4, Table 1), with Algorithm 3's plan over five tiers
 * (tier code 4 = double-double).
 * A double-double matrix argument points to 2 ld n doubles: the hi plane
 * (column-major, leading dimension ld) followed by the lo plane; each entry
 * is hi + lo.
 * ------------------------------------------------------------------------- */

/* Workspace bytes for ps_expm_dd.  s = 0 selects ceil(sqrt(m)). */
ps_status ps_workspace_size_dd(int64_t n, int m, int s, int sigma, size_t* bytes);

/* E = p(2^-sigma A)^(2^sigma) in double-double (scaling and squaring
 * around the PS evaluation, eq. (scal-idea)).  A, E: double-double n x n
 * (lda, lde >= n), not overlapping.  coef: host array of 2 (m+1) doubles,
 * hi parts c_0..c_m then lo parts, or NULL for the Taylor coefficients 1/k!
 * rounded to double-double (m <= 170).  0 <= sigma <= 500.  opts: mode
 * fixed (every product in double-double) or mixed (tiers 0..3 below it as
 * the plan allows; tier_override unsupported).  report may be NULL.  The
 * call synchronizes the stream once (coefficient upload) and again when a
 * report is asked for. */
ps_status ps_expm_dd(int64_t n, const double* A, int64_t lda, const double* coef, int m, int s, int sigma,
                     double* E, int64_t lde, const ps_opts* opts, ps_report* report,
                     void* ws, size_t ws_bytes, void* stream);

/* Several polynomials of one matrix sharing one power table (section 4:
 * the Pade numerator and denominator; the cosine, which is a polynomial in
 * X^2).  square_arg = 0: P_t = p_t(A); square_arg = 1: P_t = p_t(A^2)
 * (one extra product forms A^2 first).
 *   k >= 1 polynomials; coefs[t]: host array of degrees[t]+1 doubles; one
 *   block size s for all (s = 0: ceil(sqrt(max degree))); P: host array of k
 *   device pointers, ldp: host array of k leading dimensions; reports: NULL
 *   or a host array of k reports. */
ps_status ps_workspace_size_multi(ps_dtype dtype, int64_t n, int k, const int* degrees, int s,
                                  int square_arg, size_t* bytes);
ps_status ps_eval_multi(ps_dtype dtype, int64_t n, const void* A, int64_t lda,
                        int k, const double* const* coefs, const int* degrees, int s,
                        int square_arg, void* const* P, const int64_t* ldp,
                        const ps_opts* opts, ps_report* reports,
                        void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Many matrices of one size n (contiguous, fixed stride): the same
 * computation as ps_expm for each matrix b = 0..batch-1 at
 * A + b*strideA, E + b*strideE (strides in elements).  Each matrix gets its
 * own precision plan.  reports: NULL or host array of `batch` reports.
 * ------------------------------------------------------------------------- */
ps_status ps_workspace_size_strided(ps_dtype dtype, int batch, int64_t n, int m, int s, int sigma,
                                    size_t* bytes);
ps_status ps_expm_strided_batched(ps_dtype dtype, int batch, int64_t n,
                                  const void* A, int64_t lda, int64_t strideA,
                                  const double* coef, int m, int s, int sigma,
                                  void* E, int64_t lde, int64_t strideE,
                                  const ps_opts* opts, ps_report* reports,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Many matrices of uneven sizes, each phase one launch for the whole batch
 * (one hipGraph replay once prepared).  Matrix b has order
 * n[b] (1 <= n[b] <= 256), lives at device pointer A[b] with leading dimension
 * lda[b], and its result goes to E[b] (lde[b]).  Per-matrix block size s[b]
 * (0 = chosen per matrix from {floor(sqrt m), ceil(sqrt m)} by the lower
 * modelled cost) and scaling sigma[b].  Host arrays of `batch` entries.
 * Every matrix's block size and plan are chosen on the device (mixed mode),
 * with no host round trip between the phases.  The call uploads its work
 * descriptors into the workspace first and synchronises the stream once for
 * that, so it cannot itself be captured; ps_batched_prepare below does the
 * upload once and captures the launch sequence, whose replays need no host
 * work.  tiers_out: NULL or host array of batch*PS_MAX_BLOCKS ints receiving
 * each matrix's tier vector (synchronises the stream again).
 * ------------------------------------------------------------------------- */
ps_status ps_workspace_size_batched(ps_dtype dtype, int batch, const int32_t* n, int m,
                                    const int32_t* s, size_t* bytes);
ps_status ps_expm_batched(ps_dtype dtype, int batch, const int32_t* n,
                          const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s, const int32_t* sigma,
                          void* const* E, const int64_t* lde,
                          const ps_opts* opts, int32_t* tiers_out,
                          void* ws, size_t ws_bytes, void* stream);

/* P_b = p(A_b) = sum_k coef[k] A_b^k for a batch of uneven orders (Algorithm
 * 1 / Algorithm 3 with fixed s per matrix, as ps_eval): ps_expm_batched with
 * every sigma = 0 and the caller's coefficients (coef required, host array of
 * m+1).  Workspace: ps_workspace_size_batched.  Same launches, plans and
 * errors as ps_expm_batched. */
ps_status ps_eval_batched(ps_dtype dtype, int batch, const int32_t* n,
                          const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s,
                          void* const* P, const int64_t* ldp,
                          const ps_opts* opts, int32_t* tiers_out,
                          void* ws, size_t ws_bytes, void* stream);

/* Graph form of ps_expm_batched for repeated evaluation of the same batch
 * layout: ps_batched_prepare validates, uploads the work descriptors into the
 * workspace (synchronously) and captures the launch sequence into a
 * hipGraph; ps_batched_launch replays it on `stream`; ps_batched_destroy
 * frees the host-side graph.  The pointers given to prepare must stay valid
 * and keep their meaning for every launch. */
typedef struct ps_batched_exec* ps_batched_handle;
ps_status ps_batched_prepare(ps_dtype dtype, int batch, const int32_t* n,
                             const void* const* A, const int64_t* lda,
                             const double* coef, int m, const int32_t* s, const int32_t* sigma,
                             void* const* E, const int64_t* lde, const ps_opts* opts,
                             void* ws, size_t ws_bytes, void* stream, ps_batched_handle* out);
ps_status ps_batched_launch(ps_batched_handle h, void* stream);
ps_status ps_batched_destroy(ps_batched_handle h);

/* ---------------------------------------------------------------------------
 * Autotuning of the uneven batch's size-class schedule (the batching
 * pattern's tuner).  A matrix's size class is its padded order / 64 (1..4 for
 * orders up to 256).  A schedule assigns each class to one of up to four
 * branches; each branch is a launch sequence of its own over its matrices'
 * tiles, and the branches run concurrently (forked from the caller's stream
 * and joined back by events; graph edges under capture).  A schedule changes
 * which launch processes a tile, never a tile's arithmetic.  The matrices
 * of class 1 (orders up to 64: one 64 x 64 tile) can instead be evaluated
 * whole by one workgroup each, every phase in one launch (whole64 = 1), on
 * the same tile routines in the same order.  Every schedule gives the same
 * bits.
 *   ps_batched_tune: times every contiguous grouping of the batch's classes
 *     (in increasing order) into at most four branches, and each grouping
 *     that gives class 1 a branch of its own once more with whole64 = 1, on
 *     this batch (one captured graph per candidate, one warm-up replay,
 *     median of `reps` replays timed with events on `stream`, which the call
 *     synchronises), keeps the fastest in the process-wide cache under a key
 *     of device architecture, dtype, degree m and the order of magnitude of
 *     each class's matrix count, and returns it: groups_out[c-1] = branch of
 *     class c, groups_out[4] = whole64 (host array of 5; may be NULL),
 *     ms_out[k] = candidate k's median (host array of 16; may be NULL),
 *     *ncand_out = candidates (may be NULL).  Arguments and workspace as
 *     ps_batched_prepare.  ps_expm_batched, ps_eval_batched and
 *     ps_batched_prepare use the cached schedule of a matching key,
 *     otherwise one branch of per-phase launches.
 *   ps_autotune_lookup: the schedule the cache holds for such a batch, in
 *     groups_out (host array of 5, as above; *found = 0: none, groups_out
 *     then the one-branch default).
 *   ps_autotune_save / ps_autotune_load: the cache as a JSON file
 *     ({"ps_autotune": 1, "entries": [{"key": ..., "groups": [g1,g2,g3,g4],
 *     "whole64": w}]}; an entry without "whole64" reads as 0); load adds the
 *     file's entries to the cache (PS_ERR_ARG for a file that is missing or
 *     not such a cache).  ps_autotune_clear empties the cache.
 * The cache is guarded by a mutex; multi-branch batches are queued (or
 * captured) under a second mutex, since their side streams are a per-device
 * pool created on first use and kept until the process ends.
 * ------------------------------------------------------------------------- */
ps_status ps_batched_tune(ps_dtype dtype, int batch, const int32_t* n,
                          const void* const* A, const int64_t* lda,
                          const double* coef, int m, const int32_t* s, const int32_t* sigma,
                          void* const* E, const int64_t* lde, const ps_opts* opts,
                          void* ws, size_t ws_bytes, void* stream, int reps,
                          int32_t* groups_out, float* ms_out, int* ncand_out);
ps_status ps_autotune_lookup(ps_dtype dtype, int batch, const int32_t* n, int m, int32_t* groups_out, int* found);
ps_status ps_autotune_save(const char* path);
ps_status ps_autotune_load(const char* path);
ps_status ps_autotune_clear(void);

/* ---------------------------------------------------------------------------
 * Adjoint.  gradA = d<G, r(A)>/dA for r(A) = p(2^-sigma A)^(2^sigma), i.e. the
 * Frechet derivative L_r(A^T, G), by reverse-mode differentiation of the
 * squarings, the Horner recurrence, the block assembly and the power table.
 * opts NULL or mode PS_MODE_FIXED: every product in the working precision.
 * mode PS_MODE_MIXED: the forward pass also makes the plan of Theorem 2.1 /
 * eq. (choose-ui) from its block norms (tier_mask, delta, rule and
 * tier_override as for ps_expm, so the same tiers as the mixed forward
 * evaluation), and both products of reverse Horner step i
 * (Pbar_i = Pbar_{i-1} Y^T, Ybar += P_i^T Pbar_{i-1}) run in forward step
 * i's tier; the stored iterates, the power chain, the block scatter and the
 * squarings stay in the working precision.  The plan is made and read on
 * the device: the call does not synchronise.
 * recompute = 1 keeps only A and recomputes the power table and Horner
 * iterates (smaller workspace); 0 stores them from the forward pass.
 * Strided-batched over `batch` matrices of order n like
 * ps_expm_strided_batched.  G: upstream gradient, same layout as E.
 * gradA must not overlap A or G.
 * ------------------------------------------------------------------------- */
ps_status ps_workspace_size_backward(ps_dtype dtype, int batch, int64_t n, int m, int s, int sigma,
                                     int recompute, size_t* bytes);
ps_status ps_expm_backward(ps_dtype dtype, int batch, int64_t n,
                           const void* A, int64_t lda, int64_t strideA,
                           const void* G, int64_t ldg, int64_t strideG,
                           const double* coef, int m, int s, int sigma,
                           void* gradA, int64_t ldga, int64_t strideGA,
                           int recompute, const ps_opts* opts,
                           void* ws, size_t ws_bytes, void* stream);

/* Adjoints of a batch of uneven orders: gradA_b = L_r(A_b^T, G_b) as
 * ps_expm_backward for each matrix b (order n[b] <= 2^20, block size s[b],
 * 0 = ceil(sqrt m); scaling sigma[b]; s and sigma may be NULL = 0 / auto).
 * Host arrays of `batch` device pointers and leading dimensions.  Matrices
 * that follow each other with the same order, block size, scaling and
 * leading dimensions, and whose A, G and gradA pointers each advance by one
 * constant stride, run as one strided batch of ps_expm_backward; every other
 * matrix as a batch of one, in order on `stream`.  Workspace: the sum over
 * the matrices of their single-matrix ps_workspace_size_backward, 256-byte
 * rounded (ps_workspace_size_backward_batched).  Every matrix's arguments
 * are checked before any device work; errors as ps_expm_backward. */
ps_status ps_workspace_size_backward_batched(ps_dtype dtype, int batch, const int32_t* n, int m,
                                             const int32_t* s, const int32_t* sigma, int recompute,
                                             size_t* bytes);
ps_status ps_expm_backward_batched(ps_dtype dtype, int batch, const int32_t* n,
                                   const void* const* A, const int64_t* lda,
                                   const void* const* G, const int64_t* ldg,
                                   const double* coef, int m, const int32_t* s, const int32_t* sigma,
                                   void* const* gradA, const int64_t* ldga,
                                   int recompute, const ps_opts* opts,
                                   void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Linear solve Q X = P (the quotient r_km = q_km^{-1} p_km of the Pade
 * approximant, section 4.1).  LU factorisation with partial pivoting: at
 * step k the row of largest |entry| in column k at or below row k (the
 * lowest such row on ties; NaN entries are never chosen) is exchanged with
 * row k over the full width.
 *   Q: device, n x n (ldq >= n), overwritten by the factors: the multipliers
 *      of the unit lower factor L below the diagonal, U on and above it.
 *   P: device, n x nrhs (ldp >= n), overwritten by X; nrhs = 0 factors only.
 *   ipiv: NULL, or a device array of n int32: ipiv[k] = the row (0-based)
 *      exchanged with row k at step k, as LAPACK's getrf (which is 1-based).
 *   info: NULL, or a HOST int that receives 0, or k + 1 when U[k,k] is the
 *      first exactly zero pivot (then X holds non-finite values); a non-NULL
 *      info synchronises the stream.
 * FP64 and FP32, 1 <= n <= 8192 (PS_ERR_UNSUPPORTED above).  Row-major
 * data solves Q^T Z = P^T instead (Z^T = P Q^{-1}, the same matrix when P
 * and Q commute, as two polynomials in one matrix do).  Q, P, ipiv and the
 * workspace must not overlap.
 * ------------------------------------------------------------------------- */
ps_status ps_workspace_size_solve(ps_dtype dtype, int64_t n, size_t* bytes);
ps_status ps_solve(ps_dtype dtype, int64_t n, void* Q, int64_t ldq, int64_t nrhs, void* P, int64_t ldp,
                   int32_t* ipiv, int* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * exp(A) in the Pade form inside scaling and squaring (section 4.1):
 * E = r_m(X)^(2^sigma), X = 2^-sigma A, r_m = q_m^{-1} p_m the diagonal
 * [m/m] Pade approximant (1 <= m <= 60; coefficients of ps_coef_pade_exp).
 * p_m and q_m share one power table (as ps_eval_multi, block size s, 0 =
 * ceil(sqrt m)), each with its own plan in mixed mode (opts as for
 * ps_eval_multi; tier_override unsupported); the solve (ps_solve's
 * factorisation) and the squarings run in the working precision.  reports:
 * NULL or a host array of 2 (p_m, q_m).  The caller picks m and sigma so that
 * q_m(X) is nonsingular (a singular q_m gives non-finite values; nothing is
 * reported).  FP64 and FP32, n <= 8192.
 * ------------------------------------------------------------------------- */
ps_status ps_workspace_size_pade(ps_dtype dtype, int64_t n, int m, int s, int sigma, size_t* bytes);
ps_status ps_expm_pade(ps_dtype dtype, int64_t n, const void* A, int64_t lda, int m, int s, int sigma,
                       void* E, int64_t lde, const ps_opts* opts, ps_report* reports,
                       void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PS_H */
