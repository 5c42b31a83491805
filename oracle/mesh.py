"""Lagrange-Legendre mesh and basis (oracle; test infrastructure only).

Sec. 2: the internal wave function is expanded in n_lag Lagrange functions
f_i(r) built on Gauss-Legendre points r_i with weights lambda_i on (0, a),
with the Lagrange property f_i(r_j) = delta_ij / sqrt(lambda_j).  The paper
does not print the functions; this module uses the standard shifted-Legendre
functions regularised by r (they vanish at r = 0):

    x_i   : zeros of P_N(2x - 1) on (0, 1),   lambda_i : their weights (sum 1)
    r_i   = a x_i,  and the weights on (0, a) are a lambda_i
    f_i(r) = (-1)^(N+i) (r / r_i) sqrt(a x_i (1 - x_i)) P_N(2r/a - 1) / (r - r_i)

with i = 1..N.  Each f_i is a polynomial of degree N with f_i(0) = 0, so
f_i(r_j) = delta_ij / sqrt(a lambda_j).  It is evaluated without the
division, through the divided difference of P_N (see
:func:`_divided_difference`).

Kinetic + Bloch block (Eq. block_structure, K_alpha without the centrifugal
and potential terms): with T = -(hbar^2/2mu) d^2/dr^2 and the Bloch operator
L = (hbar^2/2mu) delta(r - a) d/dr, integration by parts gives

    <f_i | T + L | f_j> = (hbar^2/2mu) * integral_0^a f_i'(r) f_j'(r) dr,

which is what :func:`kinetic_bloch` returns (divided by hbar^2/2mu),
computed by Gauss quadrature of the derivative product (a polynomial of
degree 2N - 2, integrated exactly by any rule with at least N points).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_points(nr: int) -> tuple[np.ndarray, np.ndarray]:
    """x_i (ascending) and lambda_i on (0, 1), rounded once to FP64 from an
    extended-precision Gauss rule."""
    t, w = _gauss_rule_extended(nr)
    return ((t + 1) / 2).astype(np.float64), (w / 2).astype(np.float64)


def mesh(nr: int, a: float) -> tuple[np.ndarray, np.ndarray]:
    """Mesh points r_i and weights a*lambda_i on (0, a)."""
    x, lam = gauss_points(nr)
    return a * x, a * lam


def _legendre(n: int, s: np.ndarray) -> list[np.ndarray]:
    """[P_0(s), ..., P_n(s)] by the three-term recurrence (in the dtype of s)."""
    s = np.asarray(s)
    out = [np.ones_like(s), s.copy()]
    for m in range(1, n):
        out.append(((2 * m + 1) * s * out[m] - m * out[m - 1]) / (m + 1))
    return out[: n + 1]


def _divided_difference(n: int, t: np.ndarray, s: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """D(t, s) = (P_n(t) - P_n(s)) / (t - s) and dD/dt, broadcast over t and s.

    From the Legendre recurrence, with D_0 = 0 and D_1 = 1:
      D_{m+1} = [(2m+1) (t D_m + P_m(s)) - m D_{m-1}] / (m+1),
    which contains no division by t - s, so it stays accurate when t is close
    to s.  Since P_n(t_i) = 0 at a mesh point, D(t, t_i) = P_n(t) / (t - t_i).
    """
    t = np.asarray(t)
    s = np.asarray(s)
    t, s = np.broadcast_arrays(t, s)
    ps = _legendre(n, s)
    d_prev, d = np.zeros_like(t), np.ones_like(t)
    dd_prev, dd = np.zeros_like(t), np.zeros_like(t)
    if n == 0:
        return d_prev, dd_prev
    for m in range(1, n):
        d_new = ((2 * m + 1) * (t * d + ps[m]) - m * d_prev) / (m + 1)
        dd_new = ((2 * m + 1) * (d + t * dd) - m * dd_prev) / (m + 1)
        d_prev, d = d, d_new
        dd_prev, dd = dd, dd_new
    return d, dd


def _prefactor(nr: int, a: float, dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """Mesh points t_i = 2 x_i - 1 and c_i with f_i(r) = c_i r D(2r/a - 1, t_i).

    In long double the nodes are the extended-precision zeros (not their FP64
    rounding), so that D(t, t_i) is P_N(t)/(t - t_i) to extended accuracy."""
    if dtype == np.longdouble:
        t_ext, _ = _gauss_rule_extended(nr)
        x = (t_ext + 1) / 2
    else:
        x, _ = gauss_points(nr)
    x = x.astype(dtype)
    a = dtype(a)
    i = np.arange(1, nr + 1)
    sign = np.where((nr + i) % 2 == 0, 1.0, -1.0).astype(dtype)
    # f_i = sign sqrt(a x_i (1-x_i)) / (a x_i) * r * P_N(t) / (r - r_i),  r - r_i = (a/2)(t - t_i)
    c = sign * np.sqrt(a * x * (1 - x)) / (a * x) * (2 / a)
    return 2 * x - 1, c


def basis(nr: int, a: float, r: np.ndarray) -> np.ndarray:
    """f_i(r) for every i: shape (len(r), nr) (evaluated in long double)."""
    r = np.asarray(r).astype(np.longdouble)
    ti, c = _prefactor(nr, a, np.longdouble)
    d, _ = _divided_difference(nr, (2 * r / np.longdouble(a) - 1)[:, None], ti[None, :])
    return (c[None, :] * r[:, None] * d).astype(np.float64)


def basis_derivative(nr: int, a: float, r: np.ndarray, dtype=np.float64) -> np.ndarray:
    """f_i'(r): shape (len(r), nr).  d/dr [r D(t)] = D + r (2/a) dD/dt."""
    r = np.asarray(r).astype(dtype)
    ti, c = _prefactor(nr, a, dtype)
    a = dtype(a)
    d, dd = _divided_difference(nr, (2 * r / a - 1)[:, None], ti[None, :])
    return c[None, :] * (d + r[:, None] * (2 / a) * dd)


def _gauss_rule_extended(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre rule on (-1, 1) in extended precision: numpy's nodes
    polished by Newton steps on P_n in long double, weights 2/((1-t^2) P_n'^2)."""
    t0, _ = npleg.leggauss(n)
    t = t0.astype(np.longdouble)
    for _ in range(3):
        p = _legendre(n, t)
        dp = n * (p[n - 1] - t * p[n]) / (1 - t * t)
        t = t - p[n] / dp
    p = _legendre(n, t)
    dp = n * (p[n - 1] - t * p[n]) / (1 - t * t)
    return t, 2 / ((1 - t * t) * dp * dp)


def surface_values(nr: int, a: float) -> np.ndarray:
    """q_i = f_i(a), the boundary values that fill the right-hand sides."""
    return basis(nr, a, np.array([a]))[0]


def kinetic_bloch(nr: int, a: float) -> np.ndarray:
    """(T + L)_ij / (hbar^2/2mu) = integral_0^a f_i' f_j' dr, shape (nr, nr).

    Quadrature with an (N+1)-point Gauss rule on (0, a); exact for the
    degree-(2N-2) integrand.  Evaluated in long double (x86 extended
    precision) and rounded once to FP64, so the matrix is accurate to the last
    bit and does not add its own error to the parity comparisons.
    """
    t, w = _gauss_rule_extended(nr + 1)
    al = np.longdouble(a)
    rq = al * (t + 1) / 2
    wq = al * w / 2
    d = basis_derivative(nr, a, rq, dtype=np.longdouble)  # (nr+1, nr)
    g = np.einsum("q,qi,qj->ij", wq, d, d)
    # the sum is symmetric in exact arithmetic; average the two summation orders
    return (0.5 * (g + g.T)).astype(np.float64)
