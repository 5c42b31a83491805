// Host-side checks of the HIP library, meant to be built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host pass (the device code is built
// too, but nothing here launches it): the Lagrange-Legendre mesh and its
// kinetic + Bloch matrix (Sec. 2.2), the Coulomb functions of the matching
// (Sec. 2.3), the workspace arithmetic, and every entry point's argument
// checks, which must reject bad input before touching a device.
//
// Every output buffer is heap-allocated at its exact size, so a write past
// its end is reported by AddressSanitizer.  Exit status 0 when every check
// holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "hprmat.h"

static int g_fail = 0;

static void check(bool ok, const char *what, double a = 0.0, double b = 0.0) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s (%g %g)\n", what, a, b);
    ++g_fail;
  }
}

template <typename T>
static T *exact(size_t n) {
  return static_cast<T *>(std::malloc(n * sizeof(T)));
}

static void mesh_checks() {
  const int nrs[] = {1, 2, 3, 7, 40, 60, 100, 128};
  const double as[] = {3.0, 15.0, 30.0};
  for (int nr : nrs)
    for (double a : as) {
      double *r = exact<double>(nr), *w = exact<double>(nr), *q = exact<double>(nr);
      double *tl = exact<double>((size_t)nr * nr);
      check(hp_mesh(nr, a, r, w, q, tl) == HP_OK, "hp_mesh status", nr, a);
      double sw = 0.0;
      for (int i = 0; i < nr; ++i) {
        check(r[i] > 0.0 && r[i] < a, "node inside (0, a)", r[i], a);
        if (i) check(r[i] > r[i - 1], "nodes increasing", r[i - 1], r[i]);
        check(w[i] > 0.0, "positive weight", w[i]);
        check(std::isfinite(q[i]) && q[i] != 0.0, "surface value", q[i]);
        sw += w[i];
        for (int j = 0; j < nr; ++j) {
          const double x = tl[(size_t)i * nr + j];
          check(std::isfinite(x), "finite kinetic + Bloch entry", x);
          check(x == tl[(size_t)j * nr + i], "symmetric kinetic + Bloch", i, j);
        }
      }
      // Gauss-Legendre weights on (0, a) integrate 1 exactly
      check(std::fabs(sw - a) <= 1e-13 * a, "weights sum to a", sw, a);
      // each output is optional
      check(hp_mesh(nr, a, r, nullptr, nullptr, nullptr) == HP_OK, "hp_mesh r only", nr);
      check(hp_mesh(nr, a, nullptr, nullptr, nullptr, tl) == HP_OK, "hp_mesh tl only", nr);
      std::free(r), std::free(w), std::free(q), std::free(tl);
    }
  check(hp_mesh(0, 1.0, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "hp_mesh nr = 0");
  check(hp_mesh(5, -1.0, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "hp_mesh a < 0");
  check(hp_mesh(5, NAN, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "hp_mesh a = NaN");
}

static void coulomb_checks() {
  const int ls[] = {0, 1, 6, 20};
  const double etas[] = {0.0, 2.0, 18.2, 25.8};
  const double rhos[] = {11.2, 23.7, 58.0, 116.0};
  for (int l : ls)
    for (double eta : etas)
      for (double rho : rhos) {
        double *out = exact<double>(4);
        check(hp_coulomb(l, eta, rho, out) == HP_OK, "hp_coulomb status", l, rho);
        // Wronskian F' G - F G' = 1
        const double wr = out[1] * out[2] - out[0] * out[3];
        check(std::fabs(wr - 1.0) < 1e-10, "Coulomb Wronskian", wr, eta);
        std::free(out);
      }
  double out[4];
  check(hp_coulomb(-1, 0.0, 1.0, out) == HP_ERR_ARG, "hp_coulomb l < 0");
  check(hp_coulomb(0, 0.0, 1.0, nullptr) == HP_ERR_ARG, "hp_coulomb null out");
}

// The kinetic inverse (binary128 elimination) against the matrix it inverts,
// and the Woodbury-kinetic and deep-Coulomb host paths.
static void woodbury_and_range_checks() {
  const int nrs[] = {1, 7, 40};
  for (int nr : nrs) {
    double *tl = exact<double>((size_t)nr * nr), *ki = exact<double>((size_t)nr * nr);
    check(hp_mesh(nr, 10.0, nullptr, nullptr, nullptr, tl) == HP_OK, "mesh for the inverse", nr);
    check(hp_kinetic_inverse(nr, 10.0, ki) == HP_OK, "hp_kinetic_inverse status", nr);
    double worst = 0.0;
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nr; ++j) {
        long double s = 0.0L;
        for (int k = 0; k < nr; ++k) s += (long double)tl[(size_t)i * nr + k] * ki[(size_t)k * nr + j];
        worst = std::fmax(worst, std::fabs((double)(s - (i == j ? 1.0L : 0.0L))));
      }
    check(worst < 1e-6, "tl * kinv = I", worst, nr);
    std::free(tl);
    std::free(ki);
  }
  check(hp_kinetic_inverse(0, 1.0, nullptr) == HP_ERR_ARG, "kinetic_inverse nr = 0");
  check(hp_schur_workspace_bytes(6, 4, HP_C64) == 0, "schur workspace n % nrhs");
  check(hp_schur_workspace_bytes(600, 6, HP_C64) > hp_workspace_bytes(600, 6, HP_C64), "schur workspace extra");
  double out[4];
  check(hp_coulomb(2, 322.0, 0.33, out) == HP_ERR_NOCONV, "coulomb far below the barrier reported");
  check(hp_coulomb(0, 100.0, 3.0, out) == HP_OK, "coulomb deep but in range");
}

static void workspace_checks() {
  const int ns[] = {1, 2, 127, 128, 129, 1000, 4000, 25600, 60000};
  const int nrhs[] = {0, 1, 64, 256};
  const int precs[] = {HP_C64, HP_C128, HP_C64H};
  for (int prec : precs)
    for (int k : nrhs) {
      size_t prev = 0;
      for (int n : ns) {
        const size_t b = hp_workspace_bytes(n, k, prec);
        check(b > 0 && b >= prev, "workspace grows with n", (double)n, (double)b);
        prev = b;
      }
    }
  check(hp_workspace_bytes(0, 1, HP_C128) == 0, "workspace n = 0");
  check(hp_workspace_bytes(10, -1, HP_C128) == 0, "workspace nrhs < 0");
  check(hp_workspace_bytes(10, 2, 7) == 0, "workspace bad precision");
  check(hp_batch_workspace_bytes(16, 160, 16000, 4000, HP_C64) > 0, "batch workspace");
  check(hp_batch_workspace_bytes(1024, 8192, 1 << 20, 3871, HP_C128) > 0, "batch workspace large");
  check(hp_batch_workspace_bytes(0, 1, 1, 1, HP_C64) == 0, "batch workspace count = 0");
  check(hp_batch_workspace_bytes(4, 4, 4, 4, HP_C64H) == 0, "batch workspace FP16 variant");
}

static void argument_checks() {
  int dummy_i[4] = {0, 0, 0, 0};
  double dummy_d[4] = {0, 0, 0, 0};
  void *p = dummy_d;
  check(hp_build_matrix(nullptr, 1.0, HP_C128, nullptr, 10, nullptr) == HP_ERR_ARG, "build null");
  check(hp_factor(0, HP_C128, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == HP_ERR_ARG,
        "factor n = 0");
  check(hp_factor(4, 9, p, 4, dummy_i, dummy_i, dummy_i, p, 1 << 20, nullptr) == HP_ERR_ARG, "factor bad prec");
  check(hp_factor(4, HP_C128, p, 3, dummy_i, dummy_i, dummy_i, p, 1 << 20, nullptr) == HP_ERR_ARG, "factor lda < n");
  check(hp_factor(64, HP_C128, p, 64, dummy_i, dummy_i, dummy_i, p, 16, nullptr) == HP_ERR_WORKSPACE,
        "factor small workspace");
  check(hp_lu_solve(4, 1, HP_C64, nullptr, 4, nullptr, nullptr, 1, nullptr, 0, nullptr) == HP_ERR_ARG,
        "lu_solve null");
  check(hp_lu_solve(4, 2, HP_C64, p, 4, dummy_i, p, 1, p, 1 << 20, nullptr) == HP_ERR_ARG, "lu_solve ldx < nrhs");
  check(hp_rmatrix(nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "rmatrix null");
  hp_system sys;
  std::memset(&sys, 0, sizeof(sys));
  sys.nc = 0;
  sys.nr = 4;
  check(hp_solve(&sys, 1.0, HP_C64, p, 4, dummy_i, dummy_i, dummy_d, 1, 0.0, p, 1, nullptr, nullptr) == HP_ERR_ARG,
        "solve nc = 0");
  check(hp_smatrix(&sys, 1.0, dummy_d, dummy_d, dummy_i, p, 1, nullptr) == HP_ERR_ARG, "smatrix nc = 0");
  check(hp_smatrix_noalloc(&sys, 1.0, dummy_d, dummy_d, dummy_i, nullptr) == HP_ERR_ARG, "smatrix_noalloc nc = 0");
  check(hp_gemm_sub(-1, 4, 4, HP_C64, p, 4, p, 4, p, 4, nullptr) == HP_ERR_ARG, "gemm_sub M < 0");
  check(hp_gemm_sub(4, 4, 4, HP_C64, p, 3, p, 4, p, 4, nullptr) == HP_ERR_ARG, "gemm_sub lda < K");
  check(hp_gemm_h3_sub(4, 4, 32, p, 32, p, 4, p, 4, p, 0, nullptr) == HP_ERR_WORKSPACE, "gemm_h3_sub no workspace");
  check(hp_gemm_h3_sub(4, 4, 16, p, 16, p, 4, p, 4, p, 1 << 20, nullptr) == HP_ERR_UNSUPPORTED, "gemm_h3_sub K = 16");
  check(hp_coulomb_device(-1, nullptr, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "coulomb_device n < 0");
  check(hp_coulomb_device(0, nullptr, nullptr, nullptr, nullptr, nullptr) == HP_OK, "coulomb_device n = 0");
  check(hp_batch_build(0, nullptr, HP_C64, p, nullptr) == HP_ERR_ARG, "batch_build count = 0");
  check(hp_batch_factor(1, nullptr, HP_C64, p, dummy_i, dummy_i, dummy_i, 8, 1, p, 1024, nullptr) == HP_ERR_ARG,
        "batch_factor null items");
  const int n_bad[2] = {10, 20};  // must be largest first
  hp_batch_item item;
  std::memset(&item, 0, sizeof(item));
  hp_batch_item items2[2] = {item, item};
  check(hp_batch_factor_stepped(2, items2, n_bad, HP_C64, p, dummy_i, dummy_i, dummy_i, 8, 64, p, 1 << 20,
                                nullptr) == HP_ERR_ARG,
        "batch_factor_stepped order");
  const int n_ok[1] = {100};
  check(hp_batch_factor_stepped(1, items2, n_ok, HP_C64, p, dummy_i, dummy_i, dummy_i, 8, 12, p, 1 << 20,
                                nullptr) == HP_ERR_ARG,
        "batch_factor_stepped block not a multiple of panel");
  check(hp_batch_factor_stepped(1, items2, n_ok, HP_C64, p, dummy_i, dummy_i, dummy_i, 8, 64, p, 16, nullptr) ==
            HP_ERR_WORKSPACE,
        "batch_factor_stepped small workspace");
  check(hp_batch_rmatrix(0, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "batch_rmatrix count = 0");
  check(hp_batch_smatrix(0, nullptr, nullptr, nullptr, nullptr, 0, 0, nullptr, 0, nullptr) == HP_ERR_ARG,
        "batch_smatrix count = 0");
  check(hp_batch_status(0, nullptr, nullptr, nullptr, nullptr) == HP_ERR_ARG, "batch_status count = 0");
  check(hp_set_concurrency(0) == HP_ERR_ARG && hp_set_concurrency(257) == HP_ERR_ARG, "concurrency range");
  const int prev = hp_set_concurrency(3);
  check(hp_set_concurrency(prev) == 3, "concurrency round trip", prev);
  for (int code = -12; code <= 12; ++code) check(hp_strerror(code) != nullptr, "strerror", code);
  check(hp_last_error() != nullptr, "last_error");
  check(std::strlen(hp_build_info()) > 20, "build_info");
}

int main() {
  mesh_checks();
  coulomb_checks();
  woodbury_and_range_checks();
  workspace_checks();
  argument_checks();
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
