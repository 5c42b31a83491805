/*
 * Oracle (test infrastructure only; never called by the product path).
 *
 * Plain Gaussian elimination with partial pivoting on the augmented system
 * [M | B], complex double, row-major, as the dense direct solve of the paper
 * (Sec. 3.1, "Dense Solver (Type 1)": M = P L U, then forward and backward
 * substitution on all n_ch right-hand sides at once).
 *
 * Pivot rule: in column k choose the row i >= k with the largest
 * |Re a_ik| + |Im a_ik|; among equal values the smallest i.  The
 * multipliers l_ik = a_ik / a_kk overwrite the eliminated entries, so on
 * return A holds L (unit diagonal implied) and U, ipiv[k] is the row swapped
 * with row k at step k, and B holds the solution X.
 *
 * No blocking, no reordering: step k touches every row below the pivot once.
 * The row loop of each step is split over OpenMP threads; the arithmetic of
 * every entry is the same whatever the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double cabs1(double complex z) { return fabs(creal(z)) + fabs(cimag(z)); }

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Elimination steps k = 0 .. steps-1 (steps <= n).  Returns 0, or k+1 for the
 * first exactly zero pivot column k (that step is then skipped). */
long oracle_ge_eliminate(long n, long nrhs, double complex *A, long lda,
                         int *ipiv, double complex *B, long ldb, long steps) {
  long info = 0;
  if (steps > n) steps = n;
  for (long k = 0; k < steps; ++k) {
    long p = k;
    double best = cabs1(A[k * lda + k]);
    for (long i = k + 1; i < n; ++i) {
      double v = cabs1(A[i * lda + k]);
      if (v > best) { best = v; p = i; }
    }
    ipiv[k] = (int)p;
    if (best == 0.0) {
      if (info == 0) info = k + 1;
      continue;
    }
    if (p != k) {
      for (long j = 0; j < n; ++j) {
        double complex t = A[k * lda + j]; A[k * lda + j] = A[p * lda + j]; A[p * lda + j] = t;
      }
      for (long j = 0; j < nrhs; ++j) {
        double complex t = B[k * ldb + j]; B[k * ldb + j] = B[p * ldb + j]; B[p * ldb + j] = t;
      }
    }
    const double complex piv = A[k * lda + k];
#pragma omp parallel for schedule(static)
    for (long i = k + 1; i < n; ++i) {
      double complex l = A[i * lda + k] / piv;
      A[i * lda + k] = l;
      if (l == 0.0) continue;
      for (long j = k + 1; j < n; ++j) A[i * lda + j] -= l * A[k * lda + j];
      for (long j = 0; j < nrhs; ++j) B[i * ldb + j] -= l * B[k * ldb + j];
    }
  }
  return info;
}

/* Backward substitution with the upper triangle U left in A. */
void oracle_back_substitute(long n, long nrhs, const double complex *A, long lda,
                            double complex *B, long ldb) {
#pragma omp parallel for schedule(static)
  for (long j = 0; j < nrhs; ++j) {
    for (long k = n - 1; k >= 0; --k) {
      double complex s = B[k * ldb + j];
      for (long m = k + 1; m < n; ++m) s -= A[k * lda + m] * B[m * ldb + j];
      B[k * ldb + j] = s / A[k * lda + k];
    }
  }
}

/* Full solve: A X = B.  Returns the elimination info (0 = nonsingular). */
long oracle_zgesv(long n, long nrhs, double complex *A, long lda, int *ipiv,
                  double complex *B, long ldb) {
  long info = oracle_ge_eliminate(n, nrhs, A, lda, ipiv, B, ldb, n);
  if (info != 0) return info;
  oracle_back_substitute(n, nrhs, A, lda, B, ldb);
  return 0;
}
