/*
 * Checks of the oracle's Gaussian elimination (oracle/ge.c), meant to be
 * built together with it under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Matrices are heap-allocated at their exact size (rows of lda >= n
 * entries), so a read or write past a row or past the buffer is reported.
 *
 * Checks: the residual of A X = B on random complex systems (several sizes,
 * padded leading dimensions, several right-hand sides); pivots in range; a
 * permutation matrix solved exactly; an exactly singular column reported as
 * info = column + 1; a partial elimination (fewer steps than n).
 * Exit status 0 when every check holds.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

long oracle_ge_eliminate(long n, long nrhs, double complex *A, long lda, int *ipiv, double complex *B, long ldb,
                         long steps);
long oracle_zgesv(long n, long nrhs, double complex *A, long lda, int *ipiv, double complex *B, long ldb);

static int fails = 0;
static uint64_t state = 0x9e3779b97f4a7c15ull;

static double uniform(void) { /* xorshift64*, values in [-1, 1) */
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  return (double)((state * 0x2545f4914f6cdd1dull) >> 11) * 0x1p-52 - 1.0;
}

static void fail(const char *what, double a, double b) {
  fprintf(stderr, "FAIL %s (%g %g)\n", what, a, b);
  ++fails;
}

static void random_solve(long n, long nrhs, long pad) {
  const long lda = n + pad, ldb = nrhs + pad;
  double complex *A = malloc(sizeof(double complex) * n * lda);
  double complex *A0 = malloc(sizeof(double complex) * n * lda);
  double complex *B = malloc(sizeof(double complex) * n * ldb);
  double complex *B0 = malloc(sizeof(double complex) * n * ldb);
  int *ipiv = malloc(sizeof(int) * n);
  for (long i = 0; i < n * lda; ++i) A[i] = A0[i] = uniform() + I * uniform();
  for (long i = 0; i < n * ldb; ++i) B[i] = B0[i] = uniform() + I * uniform();
  if (oracle_zgesv(n, nrhs, A, lda, ipiv, B, ldb) != 0) fail("random system reported singular", n, nrhs);
  for (long k = 0; k < n; ++k)
    if (ipiv[k] < k || ipiv[k] >= n) fail("pivot out of range", k, ipiv[k]);
  double anorm = 0.0, xnorm = 0.0, rmax = 0.0;
  for (long i = 0; i < n; ++i) {
    double row = 0.0;
    for (long j = 0; j < n; ++j) row += cabs(A0[i * lda + j]);
    if (row > anorm) anorm = row;
    for (long c = 0; c < nrhs; ++c)
      if (cabs(B[i * ldb + c]) > xnorm) xnorm = cabs(B[i * ldb + c]);
  }
  for (long i = 0; i < n; ++i)
    for (long c = 0; c < nrhs; ++c) {
      double complex s = -B0[i * ldb + c];
      for (long j = 0; j < n; ++j) s += A0[i * lda + j] * B[j * ldb + c];
      if (cabs(s) > rmax) rmax = cabs(s);
    }
  /* normwise backward error of a stable solve on a random matrix: a small
     multiple of n times the unit roundoff */
  const double eta = rmax / (anorm * xnorm);
  if (!(eta < 64.0 * (double)n * 0x1p-53)) fail("normwise backward error", (double)n, eta);
  free(A), free(A0), free(B), free(B0), free(ipiv);
}

static void permutation_solve(long n) {
  double complex *A = calloc((size_t)(n * n), sizeof(double complex));
  double complex *B = malloc(sizeof(double complex) * n);
  int *ipiv = malloc(sizeof(int) * n);
  /* row i has its one at column (3 i + 1) mod n, n not a multiple of 3 */
  for (long i = 0; i < n; ++i) A[i * n + (3 * i + 1) % n] = 1.0;
  for (long i = 0; i < n; ++i) B[i] = (double)i + I * (double)(2 * i);
  if (oracle_zgesv(n, 1, A, n, ipiv, B, 1) != 0) fail("permutation reported singular", n, 0);
  /* x[(3 i + 1) mod n] = b[i] exactly */
  for (long i = 0; i < n; ++i) {
    double complex want = (double)i + I * (double)(2 * i);
    if (B[(3 * i + 1) % n] != want) fail("permutation solve not exact", i, creal(B[(3 * i + 1) % n]));
  }
  free(A), free(B), free(ipiv);
}

static void singular_column(long n, long col) {
  double complex *A = malloc(sizeof(double complex) * n * n);
  double complex *B = malloc(sizeof(double complex) * n);
  int *ipiv = malloc(sizeof(int) * n);
  /* unit lower-triangular plus diagonal, with column col zeroed: the first
     zero pivot column is col */
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) A[i * n + j] = (j < i) ? 0.5 : (j == i ? 2.0 : 0.0);
  for (long i = 0; i < n; ++i) A[i * n + col] = 0.0, B[i] = 1.0;
  const long info = oracle_zgesv(n, 1, A, n, ipiv, B, 1);
  if (info != col + 1) fail("singular column info", (double)col, (double)info);
  free(A), free(B), free(ipiv);
}

static void partial_elimination(long n, long steps) {
  double complex *A = malloc(sizeof(double complex) * n * n);
  double complex *B = malloc(sizeof(double complex) * n * 2);
  int *ipiv = malloc(sizeof(int) * n);
  for (long i = 0; i < n * n; ++i) A[i] = uniform() + I * uniform();
  for (long i = 0; i < 2 * n; ++i) B[i] = uniform();
  if (oracle_ge_eliminate(n, 2, A, n, ipiv, B, 2, steps) != 0) fail("partial elimination info", n, steps);
  for (long k = 0; k < steps; ++k)
    if (ipiv[k] < k || ipiv[k] >= n) fail("partial pivot out of range", k, ipiv[k]);
  free(A), free(B), free(ipiv);
}

int main(void) {
  const long sizes[] = {1, 2, 3, 17, 64, 129};
  for (int s = 0; s < 6; ++s)
    for (long nrhs = 1; nrhs <= 3; nrhs += 2)
      for (long pad = 0; pad <= 3; pad += 3) random_solve(sizes[s], nrhs, pad);
  permutation_solve(1);
  permutation_solve(20);
  permutation_solve(64);
  singular_column(1, 0);
  singular_column(10, 0);
  singular_column(10, 6);
  singular_column(10, 9);
  partial_elimination(40, 13);
  partial_elimination(40, 40);
  if (fails) {
    fprintf(stderr, "%d check(s) failed\n", fails);
    return 1;
  }
  printf("oracle elimination checks ok\n");
  return 0;
}
