/* The C part of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitize.py together with oracle/ps_oracle.c).  Every
 * routine runs on small odd orders, including n = 1, degree 0 and a block size
 * equal to the degree; on integer data all routes must agree exactly.  Exit
 * status 0 when every expectation holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_two_sum(double a, double b, double* out);
void orc_two_prod(double a, double b, double* out);
void orc_dd_add(double ah, double al, double bh, double bl, double* out);
void orc_dd_mul(double ah, double al, double bh, double bl, double* out);
void orc_dd_mul_d(double ah, double al, double b, double* out);
void orc_set_threads(int t);
void orc_gemm_d_dd(int n, int k, const double* X, const double* Bh, const double* Bl, double* Ch, double* Cl);
void orc_gemm_dd(int n, const double* Ah, const double* Al, const double* Bh, const double* Bl, double* Ch,
                 double* Cl);
void orc_poly_apply_dd(int n, const double* X, const double* coef, int m, int k, const double* Vh,
                       const double* Vl, double* Sh, double* Sl);
void orc_expm_apply_dd(int n, const double* A, const double* coef, int m, int sigma, int k, const double* Vh,
                       const double* Vl, double* Eh, double* El);
void orc_ps_dd(int n, const double* X, const double* coef, int m, int s, double* Ph, double* Pl);
void orc_gemm_f64(int n, const double* A, const double* B, double* C);
void orc_ps_f64(int n, const double* X, const double* coef, int m, int s, double* P);
void orc_horner_f64(int n, const double* X, const double* coef, int m, double* P);
void orc_naive_f64(int n, const double* X, const double* coef, int m, double* P);
void orc_expm_ps_f64(int n, const double* A, const double* coef, int m, int s, int sigma, double* E);

static int failures = 0;
#define EXPECT(c) do { if (!(c)) { fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); ++failures; } } while (0)

static int same(int len, const double* a, const double* b) {
  for (int i = 0; i < len; ++i)
    if (a[i] != b[i]) return 0;
  return 1;
}

int main(void) {
  double o[2];
  orc_two_sum(1.0, 1e-30, o);
  EXPECT(o[0] == 1.0 && o[1] == 1e-30);
  orc_two_prod(3.0, 1.0 / 3.0, o);
  orc_dd_add(1.0, 1e-20, 2.0, -1e-20, o);
  EXPECT(o[0] == 3.0 && o[1] == 0.0);
  orc_dd_mul(2.0, 0.0, 0.5, 0.0, o);
  EXPECT(o[0] == 1.0 && o[1] == 0.0);
  orc_dd_mul_d(3.0, 1e-17, 2.0, o);
  for (int threads = 1; threads <= 3; threads += 2) {
    orc_set_threads(threads);
    const int sizes[4] = {1, 2, 5, 7};
    for (int si = 0; si < 4; ++si) {
      const int n = sizes[si], nn = n * n;
      double* X = malloc(nn * sizeof(double));
      double* Z = calloc(nn, sizeof(double));
      double* P1 = malloc(nn * sizeof(double));
      double* P2 = malloc(nn * sizeof(double));
      double* P3 = malloc(nn * sizeof(double));
      double* Ph = malloc(nn * sizeof(double));
      double* Pl = malloc(nn * sizeof(double));
      double* Qh = malloc(nn * sizeof(double));
      double* Ql = malloc(nn * sizeof(double));
      for (int i = 0; i < nn; ++i) X[i] = (double)((i * 7 + 3) % 5) - 2.0;   /* entries in {-2..2} */
      const double coef[9] = {1, -2, 3, 1, -1, 2, 0, 1, -1};                  /* integers */
      for (int m = 0; m <= 8; m += 4)
        for (int s = 1; s <= (m > 1 ? m : 1); ++s) {
          orc_naive_f64(n, X, coef, m, P1);
          orc_horner_f64(n, X, coef, m, P2);
          orc_ps_f64(n, X, coef, m, s, P3);
          orc_ps_dd(n, X, coef, m, s, Ph, Pl);
          orc_poly_apply_dd(n, X, coef, m, n, NULL, NULL, Qh, Ql);
          EXPECT(same(nn, P1, P2) && same(nn, P1, P3) && same(nn, P1, Ph) && same(nn, P1, Qh));
        }
      orc_gemm_f64(n, X, X, P1);
      orc_gemm_dd(n, X, Z, X, Z, Ph, Pl);
      EXPECT(same(nn, P1, Ph));
      orc_gemm_d_dd(n, n, X, X, Z, Qh, Ql);
      EXPECT(same(nn, P1, Qh));
      double c[13];
      for (int k = 0; k <= 12; ++k) c[k] = 1.0 / tgamma(k + 1.0);
      for (int i = 0; i < nn; ++i) X[i] *= 0.05;
      orc_expm_ps_f64(n, X, c, 12, 4, 2, P1);
      orc_expm_apply_dd(n, X, c, 12, 2, n, NULL, NULL, Ph, Pl);
      for (int i = 0; i < nn; ++i) EXPECT(fabs(P1[i] - Ph[i]) <= 1e-13 * (1.0 + fabs(Ph[i])));
      /* k < n columns of a dd block */
      orc_expm_apply_dd(n, X, c, 12, 1, 1, Ph, Pl, Qh, Ql);
      free(X); free(Z); free(P1); free(P2); free(P3); free(Ph); free(Pl); free(Qh); free(Ql);
    }
  }
  if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
  else printf("oracle driver: all expectations hold\n");
  return failures ? 1 : 0;
}
