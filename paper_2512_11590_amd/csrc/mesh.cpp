// Lagrange-Legendre mesh and kinetic + Bloch matrix (host precompute).
//
// Mesh (Sec. 2): x_i are the zeros of P_N(2x - 1) on (0, 1) with Gauss
// weights lambda_i; r_i = a x_i.  The basis functions are the shifted
// Legendre Lagrange functions regularised by r (they vanish at r = 0), whose
// value at the channel radius is q_i = f_i(a) = (-1)^(N+i) / sqrt(a x_i (1 - x_i)).
//
// Kinetic + Bloch block, (T + L)_ij / (hbar^2/2mu) = integral_0^a f_i' f_j' dr
// (integration by parts with the Bloch operator at r = a), in the closed
// form of the Lagrange-mesh literature the paper cites for its matrix
// elements (Baye, Phys. Rep. 565 (2015); Descouvemont, CPC 200 (2016)):
//   i == j : [(4N^2 + 4N + 3) x_i (1 - x_i) - 6 x_i + 1] / [3 x_i^2 (1 - x_i)^2 a^2]
//   i != j : (-1)^(i+j) / sqrt(x_i (1-x_i) x_j (1-x_j)) / a^2
//            * [N^2 + N + 1 + (x_i + x_j - 2 x_i x_j) / (x_i - x_j)^2
//               - 1/(1 - x_i) - 1/(1 - x_j)]
//
// Its inverse (the kinetic block of the Woodbury-kinetic form, Sec. 3.3,
// step 1) is formed here too, once per mesh: the inverse of the rounded
// matrix that hp_mesh returns (the one every kernel uses), by Gauss-Jordan
// elimination in binary128 arithmetic (the matrix's condition number, ~1e8
// at 100 points, would cost eight digits in double), rounded once.
#include <cmath>
#include <utility>
#include <vector>

#include "hprmat.h"

namespace {

typedef long double xr;  // x86-64 extended precision for the host precompute

// Gauss-Legendre nodes t (ascending) and weights on (-1, 1): Newton iteration
// on P_N in extended precision from the usual cosine starting guesses, P_N and
// P_N' by the three-term recurrence; results rounded once to double.
void gauss_legendre(int n, std::vector<xr> &t, std::vector<xr> &w) {
  t.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const xr pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    xr z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    xr dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      xr p0 = 1.0L, p1 = z;
      for (int m = 2; m <= n; ++m) {
        xr p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      const xr dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-19L * std::fabs(z) + 1e-300L && it > 1) break;
    }
    xr p0 = 1.0L, p1 = z;
    for (int m = 2; m <= n; ++m) {
      xr p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0L);
    const xr wi = 2.0L / ((1.0L - z * z) * dp * dp);
    // z is the (i+1)-th largest node; mirror for the symmetric partner
    t[n - 1 - i] = z;
    t[i] = -z;
    w[n - 1 - i] = wi;
    w[i] = wi;
  }
  if (n % 2 == 1) t[n / 2] = 0.0L;
}

// (T + L) / (hbar^2/2mu) on the nodes x (0, 1) of a mesh of radius A, unrounded.
std::vector<xr> kinetic_extended(int nr, const std::vector<xr> &x, xr A) {
  std::vector<xr> m((size_t)nr * nr);
  const xr N = nr;
  const xr a2 = A * A;
  for (int i = 0; i < nr; ++i) {
    const xr xi = x[i];
    m[(size_t)i * nr + i] =
        ((4.0L * N * N + 4.0L * N + 3.0L) * xi * (1.0L - xi) - 6.0L * xi + 1.0L) / (3.0L * xi * xi * (1.0L - xi) * (1.0L - xi) * a2);
    for (int j = i + 1; j < nr; ++j) {
      const xr xj = x[j];
      const xr sgn = ((i + j) % 2 == 0) ? 1.0L : -1.0L;
      const xr d = xi - xj;
      const xr br = N * N + N + 1.0L + (xi + xj - 2.0L * xi * xj) / (d * d) - 1.0L / (1.0L - xi) - 1.0L / (1.0L - xj);
      const xr val = sgn * br / (std::sqrt(xi * (1.0L - xi) * xj * (1.0L - xj)) * a2);
      m[(size_t)i * nr + j] = val;
      m[(size_t)j * nr + i] = val;
    }
  }
  return m;
}

std::vector<xr> mesh_nodes(int nr) {
  std::vector<xr> t, wt;
  gauss_legendre(nr, t, wt);
  std::vector<xr> x(nr);
  for (int i = 0; i < nr; ++i) x[i] = 0.5L * (t[i] + 1.0L);
  return x;
}

}  // namespace

extern "C" int hp_kinetic_inverse(int nr, double a, double *kinv) {
  if (nr < 1 || !(a > 0.0) || !kinv) return HP_ERR_ARG;
  typedef __float128 qr;
  const std::vector<xr> x = mesh_nodes(nr);
  const std::vector<xr> mx = kinetic_extended(nr, x, (xr)a);
  std::vector<qr> m(mx.size());
  for (size_t e = 0; e < mx.size(); ++e) m[e] = (qr)(double)mx[e];  // hp_mesh's rounded values
  auto qabs = [](qr v) { return v < 0 ? -v : v; };
  // Gauss-Jordan with partial pivoting on [m | I]
  std::vector<qr> inv((size_t)nr * nr, (qr)0);
  for (int i = 0; i < nr; ++i) inv[(size_t)i * nr + i] = (qr)1;
  for (int k = 0; k < nr; ++k) {
    int p = k;
    for (int i = k + 1; i < nr; ++i)
      if (qabs(m[(size_t)i * nr + k]) > qabs(m[(size_t)p * nr + k])) p = i;
    if (m[(size_t)p * nr + k] == (qr)0) return HP_ERR_SINGULAR;
    if (p != k)
      for (int j = 0; j < nr; ++j) {
        std::swap(m[(size_t)p * nr + j], m[(size_t)k * nr + j]);
        std::swap(inv[(size_t)p * nr + j], inv[(size_t)k * nr + j]);
      }
    const qr piv = (qr)1 / m[(size_t)k * nr + k];
    for (int j = 0; j < nr; ++j) {
      m[(size_t)k * nr + j] *= piv;
      inv[(size_t)k * nr + j] *= piv;
    }
    for (int i = 0; i < nr; ++i) {
      if (i == k) continue;
      const qr f = m[(size_t)i * nr + k];
      if (f == (qr)0) continue;
      for (int j = 0; j < nr; ++j) {
        m[(size_t)i * nr + j] -= f * m[(size_t)k * nr + j];
        inv[(size_t)i * nr + j] -= f * inv[(size_t)k * nr + j];
      }
    }
  }
  for (size_t e = 0; e < inv.size(); ++e) kinv[e] = (double)inv[e];
  return HP_OK;
}

extern "C" int hp_mesh(int nr, double a, double *r, double *w, double *q, double *tl) {
  if (nr < 1 || !(a > 0.0)) return HP_ERR_ARG;
  std::vector<xr> t, wt;
  gauss_legendre(nr, t, wt);
  // everything is computed from the extended-precision nodes and rounded once
  std::vector<xr> x(nr);
  for (int i = 0; i < nr; ++i) x[i] = 0.5L * (t[i] + 1.0L);
  const xr A = a;
  for (int i = 0; i < nr; ++i) {
    if (r) r[i] = (double)(A * x[i]);
    if (w) w[i] = (double)(0.5L * A * wt[i]);
    if (q) {
      const xr s = ((nr + i + 1) % 2 == 0) ? 1.0L : -1.0L;  // (-1)^(N+i), i 1-based
      q[i] = (double)(s / std::sqrt(A * x[i] * (1.0L - x[i])));
    }
  }
  if (tl) {
    const std::vector<xr> m = kinetic_extended(nr, x, A);
    for (size_t e = 0; e < m.size(); ++e) tl[e] = (double)m[e];
  }
  return HP_OK;
}
