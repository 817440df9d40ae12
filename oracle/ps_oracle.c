/*
 * ps_oracle.c -- plain, slow CPU reference for matrix polynomials with scalar
 * coefficients (Paterson--Stockmeyer evaluation, Liu, "Mixed-Precision
 * Paterson--Stockmeyer Method for Evaluating Polynomials of Matrices",
 * arXiv 2312.17396).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; it shares no header, helper, constant or kernel with the
 * HIP path.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.
 *
 * Conventions: n x n matrices are column-major, element (i,j) at [i + j*n].
 * A double-double (dd) matrix is held as two arrays (hi, lo) with value
 * hi + lo.  Coefficients are given as doubles and used exactly as given.
 *
 * Arithmetic building blocks (published error-free transformations):
 *   two_sum        -- Knuth's TwoSum (exact a+b = s+e, any magnitudes)
 *   fast_two_sum   -- Dekker's Fast2Sum (exact when |a| >= |b| or a = 0)
 *   two_prod       -- FMA-based TwoProd (exact a*b = p+e barring underflow)
 *   dd_add         -- accurate double-word + double-word addition
 *                     (Joldes, Muller, Popescu 2017, "AccurateDWPlusDW")
 *   dd_mul_d       -- double-word x double ("DWTimesFP" with FMA)
 *   dd_mul         -- double-word x double-word ("DWTimesDW" with FMA)
 * Relative error of every dd operation is a small multiple of 2^-104, i.e.
 * about twice the decimal digits of IEEE double, which is the protocol of the
 * paper's experiments (the reference solution is computed in twice the
 * working digits, section 3.3).
 *
 * Build: gcc -O2 -mfma -ffp-contract=off -fopenmp -shared -fPIC.
 * -ffp-contract=off keeps the compiler from fusing a*b+c on its own, so every
 * rounding in this file is the one written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = { s, e };
    return r;
}

static inline dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    dd r = { s, e };
    return r;
}

static inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd r = { p, e };
    return r;
}

static inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    double c = s.lo + t.hi;
    dd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

static inline dd dd_mul_d(dd a, double b) {
    dd c = two_prod(a.hi, b);
    double cl = fma(a.lo, b, c.lo);
    return fast_two_sum(c.hi, cl);
}

static inline dd dd_mul(dd a, dd b) {
    dd c = two_prod(a.hi, b.hi);
    double t = a.lo * b.lo;
    t = fma(a.hi, b.lo, t);
    double cl = fma(a.lo, b.hi, t);
    cl = c.lo + cl;
    return fast_two_sum(c.hi, cl);
}

/* ---- scalar entry points (used by the tests that pin dd against exact
 * rational arithmetic) ---- */
void orc_two_sum(double a, double b, double* out) { dd r = two_sum(a, b); out[0] = r.hi; out[1] = r.lo; }
void orc_two_prod(double a, double b, double* out) { dd r = two_prod(a, b); out[0] = r.hi; out[1] = r.lo; }
void orc_dd_add(double ah, double al, double bh, double bl, double* out) {
    dd a = { ah, al }, b = { bh, bl }; dd r = dd_add(a, b); out[0] = r.hi; out[1] = r.lo;
}
void orc_dd_mul(double ah, double al, double bh, double bl, double* out) {
    dd a = { ah, al }, b = { bh, bl }; dd r = dd_mul(a, b); out[0] = r.hi; out[1] = r.lo;
}
void orc_dd_mul_d(double ah, double al, double b, double* out) {
    dd a = { ah, al }; dd r = dd_mul_d(a, b); out[0] = r.hi; out[1] = r.lo;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/* ------------------------------------------------------------------------
 * Matrix products.
 * ---------------------------------------------------------------------- */

/* C (n x k, dd) = X (n x n, double) * B (n x k, dd).  Every output entry is
 * an ordinary dot product accumulated in dd. C must not alias B. */
void orc_gemm_d_dd(int n, int k, const double* X,
                   const double* Bh, const double* Bl, double* Ch, double* Cl) {
    #pragma omp parallel
    {
        dd* acc = (dd*)malloc((size_t)n * sizeof(dd));
        #pragma omp for schedule(static)
        for (int j = 0; j < k; ++j) {
            for (int i = 0; i < n; ++i) { acc[i].hi = 0.0; acc[i].lo = 0.0; }
            for (int l = 0; l < n; ++l) {          /* acc[i] += X(i,l) * B(l,j), l ascending */
                dd b = { Bh[l + (size_t)j * n], Bl[l + (size_t)j * n] };
                const double* xc = X + (size_t)l * n;
                for (int i = 0; i < n; ++i) acc[i] = dd_add(acc[i], dd_mul_d(b, xc[i]));
            }
            for (int i = 0; i < n; ++i) { Ch[i + (size_t)j * n] = acc[i].hi; Cl[i + (size_t)j * n] = acc[i].lo; }
        }
        free(acc);
    }
}

/* C = A * B, all n x n dd.  C must not alias A or B. */
void orc_gemm_dd(int n, const double* Ah, const double* Al,
                 const double* Bh, const double* Bl, double* Ch, double* Cl) {
    #pragma omp parallel
    {
        dd* acc = (dd*)malloc((size_t)n * sizeof(dd));
        #pragma omp for schedule(static)
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) { acc[i].hi = 0.0; acc[i].lo = 0.0; }
            for (int l = 0; l < n; ++l) {          /* acc[i] += A(i,l) * B(l,j), l ascending */
                dd b = { Bh[l + (size_t)j * n], Bl[l + (size_t)j * n] };
                for (int i = 0; i < n; ++i) {
                    dd a = { Ah[i + (size_t)l * n], Al[i + (size_t)l * n] };
                    acc[i] = dd_add(acc[i], dd_mul(a, b));
                }
            }
            for (int i = 0; i < n; ++i) { Ch[i + (size_t)j * n] = acc[i].hi; Cl[i + (size_t)j * n] = acc[i].lo; }
        }
        free(acc);
    }
}

/* ------------------------------------------------------------------------
 * R1: the plain definition  p(X) V = sum_{j=0}^{m} c_j X^j V  (the polynomial
 * of the paper's eq. (ps) before any re-association).  V is an n x k dd
 * block; V = I (k = n, Vh = NULL) gives the full matrix p(X).
 * The powers are applied one at a time: T <- X T, S <- S + c_j T.
 * ---------------------------------------------------------------------- */
void orc_poly_apply_dd(int n, const double* X, const double* coef, int m, int k,
                       const double* Vh, const double* Vl, double* Sh, double* Sl) {
    size_t nk = (size_t)n * k;
    double* Th = (double*)malloc(nk * sizeof(double));
    double* Tl = (double*)malloc(nk * sizeof(double));
    double* Uh = (double*)malloc(nk * sizeof(double));
    double* Ul = (double*)malloc(nk * sizeof(double));
    for (size_t e = 0; e < nk; ++e) {
        size_t i = e % n, j = e / n;
        double vh = Vh ? Vh[e] : (i == j ? 1.0 : 0.0);
        double vl = Vh ? (Vl ? Vl[e] : 0.0) : 0.0;
        Th[e] = vh; Tl[e] = vl;
        dd t = { vh, vl };
        dd s = dd_mul_d(t, coef[0]);
        Sh[e] = s.hi; Sl[e] = s.lo;
    }
    for (int p = 1; p <= m; ++p) {
        orc_gemm_d_dd(n, k, X, Th, Tl, Uh, Ul);
        double* sw;
        sw = Th; Th = Uh; Uh = sw;
        sw = Tl; Tl = Ul; Ul = sw;
        for (size_t e = 0; e < nk; ++e) {
            dd t = { Th[e], Tl[e] };
            dd s = { Sh[e], Sl[e] };
            s = dd_add(s, dd_mul_d(t, coef[p]));
            Sh[e] = s.hi; Sl[e] = s.lo;
        }
    }
    free(Th); free(Tl); free(Uh); free(Ul);
}

/* R3: the scaling-and-squaring approximant r(A) = p(2^-sigma A)^(2^sigma)
 * (paper eq. (scal-idea)) applied to an n x k dd block V (V = NULL: identity,
 * k must then be n and the result is the full matrix).
 * Full matrix: R = p(X) by the plain definition, then sigma dd squarings.
 * Column block: W <- p(X) W repeated 2^sigma times (no squaring needed:
 * (p(X))^(2^sigma) V is 2^sigma applications of p(X)). */
void orc_expm_apply_dd(int n, const double* A, const double* coef, int m, int sigma, int k,
                       const double* Vh, const double* Vl, double* Eh, double* El) {
    size_t nn = (size_t)n * n, nk = (size_t)n * k;
    double* X = (double*)malloc(nn * sizeof(double));
    for (size_t e = 0; e < nn; ++e) X[e] = ldexp(A[e], -sigma);   /* exact scaling by 2^-sigma */
    if (Vh == NULL) {
        double* Rh = Eh; double* Rl = El;
        orc_poly_apply_dd(n, X, coef, m, n, NULL, NULL, Rh, Rl);
        if (sigma > 0) {
            double* Qh = (double*)malloc(nn * sizeof(double));
            double* Ql = (double*)malloc(nn * sizeof(double));
            for (int t = 0; t < sigma; ++t) {
                orc_gemm_dd(n, Rh, Rl, Rh, Rl, Qh, Ql);
                memcpy(Rh, Qh, nn * sizeof(double));
                memcpy(Rl, Ql, nn * sizeof(double));
            }
            free(Qh); free(Ql);
        }
    } else {
        double* Wh = (double*)malloc(nk * sizeof(double));
        double* Wl = (double*)malloc(nk * sizeof(double));
        memcpy(Wh, Vh, nk * sizeof(double));
        if (Vl) memcpy(Wl, Vl, nk * sizeof(double)); else memset(Wl, 0, nk * sizeof(double));
        long reps = 1L << sigma;
        for (long t = 0; t < reps; ++t) {
            orc_poly_apply_dd(n, X, coef, m, k, Wh, Wl, Eh, El);
            memcpy(Wh, Eh, nk * sizeof(double));
            memcpy(Wl, El, nk * sizeof(double));
        }
        free(Wh); free(Wl);
    }
    free(X);
}

/* ------------------------------------------------------------------------
 * Paterson--Stockmeyer in dd (used only to cross-check the plain definition,
 * and as the faster dd route for large n).  Follows Algorithm 1 of the paper:
 * powers X_1..X_s by repeated multiplication, P = B_r, then
 * P = B_i + X_s P for i = r-1 down to 0, where B_i = sum_j b_{si+j} X_j.
 * ---------------------------------------------------------------------- */
void orc_ps_dd(int n, const double* X, const double* coef, int m, int s,
               double* Ph, double* Pl) {
    size_t nn = (size_t)n * n;
    int r = m / s;
    /* power table, X_0 = I implicit, X_j for j = 1..s in dd */
    double* Xh = (double*)malloc(nn * (size_t)(s + 1) * sizeof(double));
    double* Xl = (double*)malloc(nn * (size_t)(s + 1) * sizeof(double));
    for (size_t e = 0; e < nn; ++e) { size_t i = e % n, j = e / n; Xh[e] = (i == j); Xl[e] = 0.0; }
    for (int j = 1; j <= s; ++j)
        orc_gemm_d_dd(n, n, X, Xh + (j - 1) * nn, Xl + (j - 1) * nn, Xh + j * nn, Xl + j * nn);
    double* Qh = (double*)malloc(nn * sizeof(double));
    double* Ql = (double*)malloc(nn * sizeof(double));
    /* P = B_r = sum_{j=0}^{m-sr} b_{sr+j} X_j */
    for (size_t e = 0; e < nn; ++e) {
        dd acc = { 0.0, 0.0 };
        for (int j = 0; j <= m - s * r; ++j) {
            dd x = { Xh[j * nn + e], Xl[j * nn + e] };
            acc = dd_add(acc, dd_mul_d(x, coef[s * r + j]));
        }
        Ph[e] = acc.hi; Pl[e] = acc.lo;
    }
    for (int i = r - 1; i >= 0; --i) {
        /* Q = X_s P */
        orc_gemm_dd(n, Xh + (size_t)s * nn, Xl + (size_t)s * nn, Ph, Pl, Qh, Ql);
        for (size_t e = 0; e < nn; ++e) {
            dd acc = { Qh[e], Ql[e] };
            for (int j = 0; j < s; ++j) {
                dd x = { Xh[j * nn + e], Xl[j * nn + e] };
                acc = dd_add(acc, dd_mul_d(x, coef[s * i + j]));
            }
            Ph[e] = acc.hi; Pl[e] = acc.lo;
        }
    }
    free(Xh); free(Xl); free(Qh); free(Ql);
}

/* ------------------------------------------------------------------------
 * Plain IEEE double routines (no dd).  These are the fixed-precision
 * algorithm as printed in the paper (Algorithm 1) and its two degenerate
 * relatives, used (i) for exactness pins on integer data, where every
 * intermediate is an integer below 2^53 and all three must agree bitwise,
 * and (ii) as the multicore CPU timing baseline.
 * ---------------------------------------------------------------------- */

/* C = A * B in double, each dot product accumulated in ascending l.  C must
 * not alias A or B. */
void orc_gemm_f64(int n, const double* A, const double* B, double* C) {
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double* c = C + (size_t)j * n;
        for (int i = 0; i < n; ++i) c[i] = 0.0;
        for (int l = 0; l < n; ++l) {              /* c[i] += A(i,l) * B(l,j), l ascending */
            double b = B[l + (size_t)j * n];
            const double* a = A + (size_t)l * n;
            for (int i = 0; i < n; ++i) c[i] += a[i] * b;
        }
    }
}

/* Algorithm 1 (fixed-precision PS) in double with the given s (s >= 1). */
void orc_ps_f64(int n, const double* X, const double* coef, int m, int s, double* P) {
    size_t nn = (size_t)n * n;
    int r = m / s;
    double* Xp = (double*)malloc(nn * (size_t)(s + 1) * sizeof(double));
    double* Q = (double*)malloc(nn * sizeof(double));
    for (size_t e = 0; e < nn; ++e) Xp[e] = ((e % n) == (e / n)) ? 1.0 : 0.0;
    for (int j = 1; j <= s; ++j) orc_gemm_f64(n, Xp + (j - 1) * nn, X, Xp + j * nn);
    for (size_t e = 0; e < nn; ++e) {
        double acc = 0.0;
        for (int j = 0; j <= m - s * r; ++j) acc += coef[s * r + j] * Xp[j * nn + e];
        P[e] = acc;
    }
    for (int i = r - 1; i >= 0; --i) {
        orc_gemm_f64(n, Xp + (size_t)s * nn, P, Q);
        for (size_t e = 0; e < nn; ++e) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += coef[s * i + j] * Xp[j * nn + e];
            P[e] = acc + Q[e];
        }
    }
    free(Xp); free(Q);
}

/* Horner's method in double: P = c_m I; P = P X + c_k I (k = m-1..0). */
void orc_horner_f64(int n, const double* X, const double* coef, int m, double* P) {
    size_t nn = (size_t)n * n;
    double* Q = (double*)malloc(nn * sizeof(double));
    for (size_t e = 0; e < nn; ++e) P[e] = ((e % n) == (e / n)) ? coef[m] : 0.0;
    for (int k = m - 1; k >= 0; --k) {
        orc_gemm_f64(n, P, X, Q);
        for (size_t e = 0; e < nn; ++e) P[e] = Q[e] + (((e % n) == (e / n)) ? coef[k] : 0.0);
    }
    free(Q);
}

/* Explicit powers in double: sum_k c_k X^k. */
void orc_naive_f64(int n, const double* X, const double* coef, int m, double* P) {
    size_t nn = (size_t)n * n;
    double* T = (double*)malloc(nn * sizeof(double));
    double* U = (double*)malloc(nn * sizeof(double));
    for (size_t e = 0; e < nn; ++e) { T[e] = ((e % n) == (e / n)) ? 1.0 : 0.0; P[e] = coef[0] * T[e]; }
    for (int k = 1; k <= m; ++k) {
        orc_gemm_f64(n, T, X, U);
        memcpy(T, U, nn * sizeof(double));
        for (size_t e = 0; e < nn; ++e) P[e] += coef[k] * T[e];
    }
    free(T); free(U);
}

/* Scaling and squaring around Algorithm 1, all in double:
 * E = PS(2^-sigma A)^(2^sigma).  The CPU timing baseline. */
void orc_expm_ps_f64(int n, const double* A, const double* coef, int m, int s, int sigma, double* E) {
    size_t nn = (size_t)n * n;
    double* X = (double*)malloc(nn * sizeof(double));
    double* Q = (double*)malloc(nn * sizeof(double));
    for (size_t e = 0; e < nn; ++e) X[e] = ldexp(A[e], -sigma);
    orc_ps_f64(n, X, coef, m, s, E);
    for (int t = 0; t < sigma; ++t) {
        orc_gemm_f64(n, E, E, Q);
        memcpy(E, Q, nn * sizeof(double));
    }
    free(X); free(Q);
}
