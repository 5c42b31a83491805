"""Pins of the CPU oracle against results that do not come from the oracle.

Every test here checks the oracle against mathematics or the paper: closed
forms, textbook special cases, library routines on special cases, invariants
and brute force.  They run on the CPU (no GPU marker).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special as sps
import mpmath

from oracle import ge, mesh, pipeline, rmatrix, system
from tests.helpers import (CustomSystem, diagonal_potential, relerr, separable_kmatrix,
                           separable_nonlocal)
from workload import make_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


# ---------------------------------------------------------------- mesh ----

@pytest.mark.parametrize("nr", [1, 2, 7, 40, 100])
def test_gauss_points_are_legendre_zeros(nr):
    x, lam = mesh.gauss_points(nr)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < 1
    assert abs(lam.sum() - 1.0) < 1e-14
    # zeros of P_N(2x - 1), checked with scipy's Legendre evaluation
    assert np.max(np.abs(sps.eval_legendre(nr, 2 * x - 1))) < 1e-12
    # exact for monomials of degree <= 2N - 1 on (0, 1)
    for d in range(0, 2 * nr):
        assert abs(np.dot(lam, x ** d) - 1.0 / (d + 1)) < 1e-13 * max(1, d)


@pytest.mark.parametrize("nr,a", [(10, 5.0), (40, 15.0), (100, 30.0)])
def test_lagrange_property(nr, a):
    r, w = mesh.mesh(nr, a)
    F = mesh.basis(nr, a, r)
    assert np.max(np.abs(F * np.sqrt(w)[:, None] - np.eye(nr))) < 1e-11
    # basis vanishes at r = 0
    assert np.max(np.abs(mesh.basis(nr, a, np.array([0.0])))) == 0.0


@pytest.mark.parametrize("nr,a", [(10, 5.0), (40, 15.0), (60, 20.0), (100, 30.0)])
def test_kinetic_bloch_acts_exactly_on_polynomials(nr, a):
    """For u = (r/a)^k, 1 <= k <= N (inside the span of the f_i):
    sum_j TL_ij c_j = f_i(a) u'(a) - integral f_i u'' dr, and the last integral is
    sqrt(a lambda_i) u''(r_i) by the Gauss rule (exact for degree <= 2N-1)."""
    r, w = mesh.mesh(nr, a)
    TL = mesh.kinetic_bloch(nr, a)
    q = mesh.surface_values(nr, a)
    for k in sorted({1, 2, 3, 5, nr // 2, nr}):
        c = np.sqrt(w) * (r / a) ** k
        upp = k * (k - 1) / a ** 2 * (r / a) ** (k - 2) if k >= 2 else 0.0 * r
        rhs = (k / a) * q - np.sqrt(w) * upp
        scale = np.abs(TL) @ np.abs(c) + np.abs(rhs)
        assert np.max(np.abs(TL @ c - rhs) / scale) < 5e-12, k


@pytest.mark.parametrize("nr,a", [(12, 6.0), (60, 20.0)])
def test_kinetic_bloch_is_a_gram_matrix(nr, a):
    TL = mesh.kinetic_bloch(nr, a)
    assert np.max(np.abs(TL - TL.T)) <= 1e-14 * np.max(np.abs(TL))
    assert np.linalg.eigvalsh(TL).min() > 0


def test_surface_values_closed_form():
    # f_i(a) = (-1)^(N+i) / sqrt(a x_i (1 - x_i)) follows from P_N(1) = 1
    for nr, a in [(5, 3.0), (40, 15.0), (100, 30.0)]:
        x, _ = mesh.gauss_points(nr)
        i = np.arange(1, nr + 1)
        ref = (-1.0) ** (nr + i) / np.sqrt(a * x * (1 - x))
        assert relerr(mesh.surface_values(nr, a), ref) < 1e-12


# ------------------------------------------------------------ assembly ----

def test_paper_sparsity_fraction():
    """Sec. 2: about 3% non-zero elements for n_ch ~ 50, n_lag ~ 100."""
    g = json.load(open(GOLDEN))["sparsity"]
    sp = make_system("small", nc=g["nc"], nr=g["nr"])
    M, B = system.assemble(sp, 12.0)
    frac = np.count_nonzero(M) / M.size
    assert abs(frac - g["fraction_approx"]) < 0.005
    # exactly: dense diagonal blocks + one diagonal per off-diagonal block
    nc, nr = g["nc"], g["nr"]
    assert np.count_nonzero(M) == nc * nr * nr + nc * (nc - 1) * nr


def test_assembly_symmetric_and_structured_apply():
    sp = make_system("small")
    M, B = system.assemble(sp, sp.energies[3])
    assert np.array_equal(M, M.T)  # complex symmetric, exactly
    rng = np.random.default_rng(0)
    X = rng.standard_normal((sp.n, 3)) + 1j * rng.standard_normal((sp.n, 3))
    assert relerr(system.apply(sp, sp.energies[3], X), M @ X) < 1e-13
    # B: column c holds q in block c only
    md = system.MeshData(sp.nr, sp.a)
    for c in range(sp.nc):
        col = np.zeros(sp.n, complex)
        col[c * sp.nr:(c + 1) * sp.nr] = md.q
        assert np.array_equal(B[:, c], col)


def test_assembly_entries_by_hand():
    """Spot entries of M against Eq. block_structure written out directly."""
    sp = make_system("small")
    E = 7.0
    md = system.MeshData(sp.nr, sp.a)
    M, _ = system.assemble(sp, E, md)
    v = sp.potential(md.r)
    nr = sp.nr
    c, cp, i, j = 2, 0, 5, 9
    assert M[c * nr + i, cp * nr + j] == 0  # off-diagonal block, i != j
    assert M[c * nr + i, cp * nr + i] == v[i, c, cp]
    h = sp.hbar2_2mu
    lc = sp.l[c]
    diag = h * md.tl[i, i] + h * lc * (lc + 1) / md.r[i] ** 2 + sp.eps[c] - E + v[i, c, c]
    assert abs(M[c * nr + i, c * nr + i] - diag) < 1e-12 * abs(diag)
    assert M[c * nr + i, c * nr + j] == h * md.tl[i, j]


# ------------------------------------------------------ linear solve ----

@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_ge_matches_inverse_and_lapack_pivots(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    X, LU, ipiv = ge.solve(A, B)
    assert relerr(X, np.linalg.inv(A) @ B) < 1e-11
    # same pivot rule as LAPACK getrf (largest |Re|+|Im|, first on ties)
    _, piv = scipy.linalg.lu_factor(A)
    assert np.array_equal(ipiv, piv)
    # P A = L U
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    PA = A.copy()
    for k in range(n):
        PA[[k, ipiv[k]]] = PA[[ipiv[k], k]]
    assert relerr(L @ U, PA) < 1e-14 * n


def test_ge_manufactured_solution():
    """Sec. 6 (Table mgpu): x = 1, b = A 1, 64 right-hand sides."""
    g = json.load(open(GOLDEN))["manufactured_solution"]
    rng = np.random.default_rng(7)
    n = 300
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 30 * np.eye(n)
    X1 = np.ones((n, g["nrhs"]), complex)
    X, _, _ = ge.solve(A, A @ X1)
    assert np.max(np.abs(X - 1)) < g["max_forward_error"]


def test_ge_zero_pivot_reported():
    A = np.zeros((4, 4), complex)
    A[0, 0] = 1
    with pytest.raises(ZeroDivisionError):
        ge.solve(A, np.ones((4, 1), complex))


def test_ge_partial_steps_match_full_elimination():
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.ones((n, 2), complex)
    A1, B1 = A.copy(), B.copy()
    ge.eliminate_steps(A1, B1, 10)
    ge.eliminate_steps(A1, B1, 0)
    _, LU, _ = ge.solve(A, B)
    # the first 10 rows of U are final after 10 steps
    assert relerr(np.triu(A1[:10, :]), np.triu(LU[:10, :])) < 1e-14


# ----------------------------------------------------- Coulomb functions ----

@pytest.mark.parametrize("l,eta,rho", [(0, 0.0, 3.0), (4, 0.0, 12.5), (2, 1.5, 9.0),
                                       (0, 18.2, 11.9), (20, 25.8, 11.2), (20, 0.4, 116.0)])
def test_coulomb_wronskian(l, eta, rho):
    F, Fp, G, Gp = rmatrix.coulomb(l, eta, rho)
    assert abs(Fp * G - F * Gp - 1.0) < 1e-12


@pytest.mark.parametrize("l", [0, 1, 3, 8])
def test_coulomb_eta0_is_riccati_bessel(l):
    rho = 7.3
    F, Fp, G, Gp = rmatrix.coulomb(l, 0.0, rho)
    jl, yl = sps.spherical_jn(l, rho), sps.spherical_yn(l, rho)
    jp, yp = sps.spherical_jn(l, rho, derivative=True), sps.spherical_yn(l, rho, derivative=True)
    assert abs(F - rho * jl) < 1e-13
    assert abs(G + rho * yl) < 1e-13
    assert abs(Fp - (jl + rho * jp)) < 1e-13
    assert abs(Gp + (yl + rho * yp)) < 1e-13


def test_coulomb_derivative_numerical():
    l, eta, rho = 3, 4.2, 14.0
    F, Fp, G, Gp = rmatrix.coulomb(l, eta, rho)
    with mpmath.workdps(40):
        dF = mpmath.diff(lambda x: mpmath.coulombf(l, eta, x), rho)
        dG = mpmath.diff(lambda x: mpmath.coulombg(l, eta, x), rho)
    assert abs(Fp - float(dF)) < 1e-13 * max(1, abs(Fp))
    assert abs(Gp - float(dG)) < 1e-13 * max(1, abs(Gp))


# --------------------------------------------------- physics special cases ----

@pytest.mark.parametrize("z1z2", [0, 20])
def test_zero_nuclear_potential_gives_unit_S(z1z2):
    """V = 0 (or pure point Coulomb, matched with the same Coulomb functions): U = 1."""
    nc = 5
    l = np.array([0, 1, 3, 6, 10])
    sp = CustomSystem(nc=nc, nr=60, a=15.0, l=l, eps=np.array([0.0, 0.5, 1.0, 2.0, 3.0]),
                      z1z2=z1z2,
                      pot=diagonal_potential(nc, lambda r: z1z2 * 1.44 / r + 0j))
    out = pipeline.solve_energy(sp, 12.0)
    assert np.max(np.abs(out["S"] - np.eye(nc))) < 1e-11


@pytest.mark.parametrize("E", [0.7, 5.0, 23.0])
def test_square_well_s_wave_textbook_phase(E):
    """Square well of radius a (the channel radius), l = 0:
    tan(ka + delta) = (k/K) tan(Ka), K = sqrt((E + V0)/h)."""
    V0, a, h = 30.0, 8.0, 2.0
    sp = CustomSystem(nc=1, nr=40, a=a, l=np.array([0]), eps=np.zeros(1), hbar2_2mu=h,
                      pot=diagonal_potential(1, lambda r: np.full(len(r), -V0 + 0j)))
    out = pipeline.solve_energy(sp, E)
    k, K = np.sqrt(E / h), np.sqrt((E + V0) / h)
    delta = np.arctan(k / K * np.tan(K * a)) - k * a
    assert abs(out["S"][0, 0] - np.exp(2j * delta)) < 1e-11


@pytest.mark.parametrize("l", [0, 2, 5, 9])
def test_square_well_R_analytic(l):
    """Internal solution K r j_l(K r): R = u(a) / (a u'(a)) exactly."""
    V0, a, h, E = 30.0, 8.0, 2.0, 5.0
    sp = CustomSystem(nc=1, nr=40, a=a, l=np.array([l]), eps=np.zeros(1), hbar2_2mu=h,
                      pot=diagonal_potential(1, lambda r: np.full(len(r), -V0 + 0j)))
    out = pipeline.solve_energy(sp, E, with_smatrix=False)
    K = np.sqrt((E + V0) / h)
    x = K * a
    u = x * sps.spherical_jn(l, x)
    up = K * (sps.spherical_jn(l, x) + x * sps.spherical_jn(l, x, derivative=True))
    assert abs(out["R"][0, 0] - u / (a * up)) < 1e-11 * abs(u / (a * up))


def test_coupled_square_well_rotates_to_uncoupled():
    """Constant real symmetric coupling W for r < a, equal thresholds, l = 0:
    with W = Q D Q^T the channels decouple, U = Q diag(exp(2 i delta_d)) Q^T."""
    a, h, E = 7.0, 2.0, 4.0
    W = np.array([[-25.0, 4.0, -2.5], [4.0, -18.0, 3.0], [-2.5, 3.0, -31.0]])
    nc = 3
    sp = CustomSystem(nc=nc, nr=45, a=a, l=np.zeros(nc, int), eps=np.zeros(nc), hbar2_2mu=h,
                      pot=lambda r: np.broadcast_to(W.astype(complex), (len(r), nc, nc)).copy())
    out = pipeline.solve_energy(sp, E)
    d, Q = np.linalg.eigh(W)
    k = np.sqrt(E / h)
    K = np.sqrt((E - d) / h)
    delta = np.arctan(k / K * np.tan(K * a)) - k * a
    ref = Q @ np.diag(np.exp(2j * delta)) @ Q.T
    assert relerr(out["S"], ref) < 1e-11


def _real_family(nc=6, nr=70, a=15.0):
    sp = make_system("small", nc=nc, nr=nr, a=a)
    sp.w0 = 0.0
    return sp


def test_real_potential_S_unitary_and_symmetric():
    sp = _real_family()
    out = pipeline.solve_energy(sp, 14.0)
    S = out["S"]
    assert np.max(np.abs(S.conj().T @ S - np.eye(sp.nc))) < 1e-10
    assert np.max(np.abs(S - S.T)) < 1e-10


def test_absorptive_potential_S_symmetric_and_contracting():
    sp = make_system("small", nr=70)
    out = pipeline.solve_energy(sp, 14.0)
    S = out["S"]
    assert np.max(np.abs(S - S.T)) < 1e-10
    assert np.linalg.eigvalsh(S.conj().T @ S).max() < 1.0


def test_rmatrix_pole_expansion():
    """Real potential: R = (h/a) sum_n g_n g_n^T / (E_n - E) from the eigenpairs
    of the real symmetric internal Hamiltonian (with Bloch term)."""
    sp = _real_family(nc=4, nr=30)
    E = 9.3
    md = system.MeshData(sp.nr, sp.a)
    M0, B = system.assemble(sp, 0.0, md)
    H = M0.real
    assert np.max(np.abs(M0.imag)) == 0
    En, V = np.linalg.eigh(H)
    g = B.real.T @ V  # (nc, n)
    Rpole = (sp.hbar2_2mu / sp.a) * (g / (En - E)) @ g.T
    out = pipeline.solve_energy(sp, E, md, with_smatrix=False)
    assert relerr(out["R"], Rpole) < 1e-10


def test_real_potential_optical_relation():
    """Unitarity => sum_c sigma_{c<-c'} = (2 pi / k_c'^2) (1 - Re U_c'c')."""
    sp = _real_family(nc=4, nr=60)
    out = pipeline.solve_energy(sp, 11.0)
    tot = out["sigma"].sum(axis=0)
    ref = 2 * np.pi / out["k"] ** 2 * (1 - np.real(np.diag(out["S"])))
    assert relerr(tot, ref) < 1e-9


def test_solution_satisfies_system_structured_residual():
    sp = make_system("small")
    E = sp.energies[0]
    md = system.MeshData(sp.nr, sp.a)
    out = pipeline.solve_energy(sp, E, md, with_smatrix=False)
    M, B = system.assemble(sp, E, md)
    res = B - system.apply(sp, E, out["X"], md)
    assert np.max(np.abs(res)) / (np.abs(M).sum(axis=1).max() * np.max(np.abs(out["X"]))) < 1e-14


# ---------------------------------------------------------- closed channels --

@pytest.mark.parametrize("l,x", [(0, 0.3), (0, 4.0), (1, 0.5), (1, 2.0), (2, 0.7), (2, 5.0)])
def test_closed_logderiv_bessel_closed_forms(l, x):
    """eta = 0: W_{0, l+1/2}(2x) is e^-x times 1, 1 + 1/x, 1 + 3/x + 3/x^2
    (modified spherical Bessel), so x W'/W = -x, -x - 1/(x+1),
    -x - (3x + 6)/(x^2 + 3x + 3)."""
    ref = {0: -x, 1: -x - 1.0 / (x + 1.0), 2: -x - (3 * x + 6.0) / (x * x + 3 * x + 3.0)}[l]
    assert abs(rmatrix.closed_logderiv(l, 0.0, x) - ref) < 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("l,eta,x", [(0, 0.8, 1.5), (3, 2.5, 2.0), (6, 0.3, 4.0)])
def test_closed_logderiv_solves_the_equation_and_decays(l, eta, x):
    """With Coulomb (eta != 0), without trusting the library's Whittaker
    routine: y = W'/W satisfies the Riccati form y' = f - y^2 of
    u'' = (1 + l(l+1)/x^2 + 2 eta/x) u, and far out y -> -1 - eta/x (the
    decaying solution, W ~ e^-x (2x)^-eta), not +1 (the growing one)."""
    f = 1.0 + l * (l + 1) / x ** 2 + 2.0 * eta / x
    h = 1e-4
    y = lambda t: rmatrix.closed_logderiv(l, eta, t) / t  # noqa: E731
    dy = (y(x + h) - y(x - h)) / (2 * h)
    assert abs(dy - (f - y(x) ** 2)) < 1e-6
    X = 60.0 + l
    assert abs(y(X) - (-1.0 - eta / X)) < 2.0 * (l * (l + 1) + eta * eta + 1.0) / X ** 2


def _well_with_closed_channel():
    a, h, E = 7.0, 2.0, 4.0
    W = np.array([[-25.0, 4.0, -2.5], [4.0, -18.0, 3.0], [-2.5, 3.0, -31.0]])
    eps = np.array([0.0, 1.0, 6.0])  # channel 2 closed at E = 4
    nc = 3
    sp = CustomSystem(nc=nc, nr=45, a=a, l=np.zeros(nc, int), eps=eps, hbar2_2mu=h,
                      pot=lambda r: np.broadcast_to(W.astype(complex), (len(r), nc, nc)).copy())
    return sp, W, E


def test_square_well_with_closed_channel_direct_matching():
    """Constant real coupling W for r < a, l = 0, no Coulomb, one closed
    channel: inside u = P diag(s_n(r)) A with M = (W + eps - E)/h = P m P^T
    (s = sinh or sin of sqrt|m| r); outside e^-ikr - U e^ikr in the open
    channels and C e^-kappa r in the closed one.  Matching u and u' at r = a
    directly (2 nc equations per entrance channel) must give the oracle's
    U over the open channels."""
    sp, W, E = _well_with_closed_channel()
    out = pipeline.solve_energy(sp, E)
    o = list(out["open"])
    assert o == [0, 1]
    a, h, eps = sp.a, sp.hbar2_2mu, sp.eps
    m, P = np.linalg.eigh((W + np.diag(eps) - E * np.eye(3)) / h)
    q = np.sqrt(np.abs(m))
    s = np.where(m > 0, np.sinh(q * a), np.sin(q * a))
    sp_ = np.where(m > 0, q * np.cosh(q * a), q * np.cos(q * a))
    k = np.sqrt((E - eps[:2]) / h)
    kap = np.sqrt((eps[2] - E) / h)
    U = np.zeros((2, 2), dtype=complex)
    for c0 in range(2):
        Mx = np.zeros((6, 6), dtype=complex)
        rhs = np.zeros(6, dtype=complex)
        for c in range(3):
            Mx[c, :3] = P[c] * s
            Mx[3 + c, :3] = P[c] * sp_
            if c < 2:
                Mx[c, 3 + c] = np.exp(1j * k[c] * a) / np.sqrt(k[c])
                Mx[3 + c, 3 + c] = 1j * k[c] * np.exp(1j * k[c] * a) / np.sqrt(k[c])
                if c == c0:
                    rhs[c] = np.exp(-1j * k[c] * a) / np.sqrt(k[c])
                    rhs[3 + c] = -1j * k[c] * np.exp(-1j * k[c] * a) / np.sqrt(k[c])
            else:
                Mx[c, 5] = -np.exp(-kap * a)
                Mx[3 + c, 5] = kap * np.exp(-kap * a)
        x = np.linalg.solve(Mx, rhs)
        U[:, c0] = x[3:5]
    assert relerr(out["S"], U) < 1e-10


def test_uncoupled_closed_channel_drops_out():
    """A closed channel with no coupling to the others (Coulomb in every
    channel, l > 0 in the closed one) leaves the open channels' U equal to
    that of the system without it."""
    nc, nr, a, h, E = 3, 50, 12.0, 2.0, 6.0
    Wt = np.array([[-30.0, 5.0, 0.0], [5.0, -22.0, 0.0], [0.0, 0.0, -27.0]])

    def pot(r):
        f = 1.0 / (1.0 + np.exp((r - 5.0) / 0.6))
        return (Wt[None, :, :] * f[:, None, None]).astype(complex)

    sp = CustomSystem(nc=nc, nr=nr, a=a, l=np.array([0, 2, 3]), eps=np.array([0.0, 2.0, 9.0]), hbar2_2mu=h,
                      pot=pot, z1z2=6)
    sub = CustomSystem(nc=2, nr=nr, a=a, l=np.array([0, 2]), eps=np.array([0.0, 2.0]), hbar2_2mu=h,
                       pot=lambda r: pot(r)[:, :2, :2].copy(), z1z2=6)
    full = pipeline.solve_energy(sp, E)
    ref = pipeline.solve_energy(sub, E)
    assert list(full["open"]) == [0, 1]
    assert relerr(full["S"], ref["S"]) < 1e-12


def test_real_potential_with_closed_channels_unitary_and_symmetric():
    """Real coupled potential with two closed channels: flux stays in the
    open ones (U unitary there) and U is symmetric."""
    sp = _real_family(nc=6, nr=70, a=15.0)
    E = 0.5 * (np.sort(sp.eps)[3] + np.sort(sp.eps)[4])  # four open, two closed
    out = pipeline.solve_energy(sp, E)
    S = out["S"]
    assert len(out["open"]) == 4
    assert np.max(np.abs(S.conj().T @ S - np.eye(4))) < 1e-10
    assert np.max(np.abs(S - S.T)) < 1e-10


# ---------------------------------------------------------------- non-local --
# Sec. 2: with a non-local potential the coupling blocks are full matrices.
# The separable kernel -lam g_c(r) g_c'(r') has a closed-form K matrix
# (derived in tests/helpers.py), which pins the quadrature factor
# sqrt(w_i w_j), the (r_i, r_j) orientation inside each block and the
# channel placement of the blocks.

_NL_H = 20.736  # hbar^2 / 2mu of two nucleons (MeV fm^2)


def _zero_local(nc):
    return lambda r: np.zeros((len(r), nc, nc), dtype=complex)


@pytest.mark.parametrize("E", [1.0, 10.0, 50.0])
def test_separable_single_channel_phase_shift(E):
    """One s-wave channel, kernel -lam exp(-b r) exp(-b r'): S = exp(2 i delta)
    with tan(delta) = lam I^2 / (h k - lam J)."""
    lam, b = 120.0, 1.4
    sp = CustomSystem(nc=1, nr=60, a=20.0, l=np.array([0]), eps=np.array([0.0]), pot=_zero_local(1),
                      hbar2_2mu=_NL_H, nlpot=separable_nonlocal(lam, b))
    S = pipeline.solve_energy(sp, E)["S"][0, 0]
    K = separable_kmatrix(lam, b, np.sqrt(E / _NL_H), _NL_H)[0, 0]
    assert abs(S - (1 + 1j * K) / (1 - 1j * K)) < 1e-10
    assert abs(abs(S) - 1.0) < 1e-12  # a real kernel conserves flux


@pytest.mark.parametrize("E", [7.0, 15.0, 40.0])
def test_separable_coupled_channels_kmatrix(E):
    """Three s-wave channels with thresholds 0, 2.5, 6 MeV coupled only by a
    rank-one separable kernel with a different range per channel: the
    oracle's S equals (1 + iK)(1 - iK)^-1 of the closed-form K."""
    lam = 60.0
    beta = np.array([1.4, 0.9, 1.8])
    eps = np.array([0.0, 2.5, 6.0])
    sp = CustomSystem(nc=3, nr=80, a=30.0, l=np.zeros(3, dtype=int), eps=eps, pot=_zero_local(3),
                      hbar2_2mu=_NL_H, nlpot=separable_nonlocal(lam, beta))
    S = pipeline.solve_energy(sp, E)["S"]
    K = separable_kmatrix(lam, beta, np.sqrt((E - eps) / _NL_H), _NL_H)
    Sa = (np.eye(3) + 1j * K) @ np.linalg.inv(np.eye(3) - 1j * K)
    assert np.max(np.abs(S - Sa)) < 5e-11
    assert np.max(np.abs(Sa - np.eye(3))) > 0.5  # strong coupling, not a near-identity S


def test_nonlocal_assembly_and_apply_agree():
    """The structured product (apply) equals the assembled matrix times X for
    a system with local and non-symmetric complex non-local parts, and a zero
    kernel reproduces the local matrix exactly."""
    rng = np.random.default_rng(11)
    nc, nr = 3, 9
    V = rng.normal(size=(nr, nc, nc)) + 1j * rng.normal(size=(nr, nc, nc))
    W = rng.normal(size=(nc, nr, nc, nr)) + 1j * rng.normal(size=(nc, nr, nc, nr))
    kw = dict(nc=nc, nr=nr, a=8.0, l=np.array([0, 1, 3]), eps=np.array([0.0, 1.0, 2.0]),
              pot=lambda r: V, hbar2_2mu=2.0)
    sp = CustomSystem(**kw, nlpot=lambda r: W)
    md = system.MeshData(nr, 8.0)
    M, _ = system.assemble(sp, 3.0, md)
    X = rng.normal(size=(nc * nr, 2)) + 1j * rng.normal(size=(nc * nr, 2))
    assert relerr(system.apply(sp, 3.0, X, md), M @ X) < 1e-13
    # element (c, i), (c', j) off the local pattern is sqrt(w_i w_j) W
    c, i, cp, j = 2, 4, 0, 7
    assert M[c * nr + i, cp * nr + j] == pytest.approx(np.sqrt(md.w[i] * md.w[j]) * W[c, i, cp, j], rel=1e-15)
    Ml, _ = system.assemble(CustomSystem(**kw), 3.0, md)
    M0, _ = system.assemble(CustomSystem(**kw, nlpot=lambda r: np.zeros((nc, nr, nc, nr))), 3.0, md)
    assert np.array_equal(Ml, M0)


# ------------------------------------------------------- Woodbury-kinetic --
# Sec. 3.3 (Type 3): S = I + K^-1 V in radial-major order.  Its definition is
# pinned to the (already pinned) assembled M: (K (x) I_nc) S = M with M's
# unknowns reordered radial-major, and the Schur solution is the direct one.

def _radial_major(nc, nr):
    """Channel-major index of radial-major position k = i*nc + a."""
    return np.array([a * nr + i for i in range(nr) for a in range(nc)])


@pytest.mark.parametrize("cfg,kw", [("small", {}), ("small", dict(nc=3, nr=17)), ("mid", dict(nc=6))])
def test_woodbury_schur_matrix_reassembles_M(cfg, kw):
    from oracle import woodbury
    sp = make_system(cfg, **kw)
    md = system.MeshData(sp.nr, sp.a)
    E = float(sp.energies[3])
    S, bt = woodbury.schur_system(sp, E, md)
    M, B = system.assemble(sp, E, md)
    p = _radial_major(sp.nc, sp.nr)
    KI = np.kron(sp.hbar2_2mu * md.tl, np.eye(sp.nc))
    assert relerr(KI @ S, M[np.ix_(p, p)]) < 1e-13
    assert relerr(KI @ bt, B[p]) < 1e-10
    # the identity part and the coupling: S - I has the radial-diagonal V in every (i, j) block
    Ki = woodbury.kinetic_inverse(sp, md)
    V = woodbury.radial_diagonal(sp, E, md)
    i, j, a, b = 2, 5, 1, 0
    assert S[i * sp.nc + a, j * sp.nc + b] == pytest.approx(Ki[i, j] * V[j, a, b], rel=1e-15)


@pytest.mark.parametrize("cfg,kw", [("small", {}), ("small", dict(nc=3, nr=17)), ("mid", dict(nc=6))])
def test_woodbury_solution_equals_direct(cfg, kw):
    from oracle import woodbury
    sp = make_system(cfg, **kw)
    md = system.MeshData(sp.nr, sp.a)
    for e in (0, 7):
        E = float(sp.energies[e])
        w = woodbury.solve(sp, E, md)
        o = pipeline.solve_energy(sp, E, md, with_smatrix=False)
        assert relerr(w["X"], o["X"]) < 1e-10 and relerr(w["R"], o["R"]) < 1e-10


def test_woodbury_refuses_nonlocal_systems():
    from oracle import woodbury
    sp = CustomSystem(nc=1, nr=8, a=10.0, l=np.array([0]), eps=np.array([0.0]), pot=_zero_local(1),
                      nlpot=separable_nonlocal(1.0, 1.0))
    with pytest.raises(ValueError, match="local"):
        woodbury.schur_system(sp, 1.0)


# -------------------------------------------- far below a Coulomb barrier --
# An open channel a few keV above its threshold under a Coulomb field of
# Z1Z2 = 40 (eta ~ 300): F ~ 1e-300 and G ~ 1e+300 leave double range, and
# the oracle evaluates the matching in mpmath (smatrix_mp).

def _deep_system(coupled: bool):
    nc, nr, a, h = 3, 40, 15.0, 2.0
    Wt = np.array([[-30.0, 4.0, 3.0], [4.0, -22.0, 2.5], [3.0, 2.5, -27.0]])
    if not coupled:
        Wt[2, :2] = Wt[:2, 2] = 0.0

    def pot(r):
        f = 1.0 / (1.0 + np.exp((r - 5.0) / 0.6))
        v = (Wt[None, :, :] * f[:, None, None]).astype(complex)
        v[:, range(nc), range(nc)] += -4j * f[:, None]
        return v
    E = 12.0
    return CustomSystem(nc=nc, nr=nr, a=a, l=np.array([0, 1, 2]), eps=np.array([0.0, 1.5, E - 0.005]),
                        hbar2_2mu=h, pot=pot, z1z2=40), E


def test_mp_matching_equals_double_matching_in_range():
    sp = make_system("small")
    E = float(sp.energies[3])
    o = pipeline.solve_energy(sp, E)
    k, eta = rmatrix.wave_numbers(E, sp.eps, sp.hbar2_2mu, sp.z1z2)
    U = rmatrix.smatrix_mp(o["R"], k, sp.a, sp.l, eta)
    assert relerr(U, o["S"]) < 1e-13


def test_deep_channel_values_leave_double_range_and_keep_the_wronskian():
    sp, E = _deep_system(True)
    k, eta = rmatrix.wave_numbers(E, sp.eps, sp.hbar2_2mu, sp.z1z2)
    assert eta[2] > 250
    F, Fp, G, Gp = rmatrix.coulomb_mp(2, eta[2], k[2] * sp.a)
    assert float(mpmath.log10(G)) > 300 and float(mpmath.log10(F)) < -300
    assert abs(float(Fp * G - F * Gp) - 1.0) < 1e-20
    fg = rmatrix.coulomb_table(sp.l, eta, k * sp.a)
    assert not rmatrix.in_double_range(fg)


def test_uncoupled_deep_channel_is_identity_and_leaves_the_rest():
    """The deep channel coupled to nothing: its U row and column are those
    of the identity (its nuclear phase is suppressed far beyond double
    precision), and the other channels' U is that of the system without it."""
    sp, E = _deep_system(False)
    U = pipeline.solve_energy(sp, E)["S"]
    sub = CustomSystem(nc=2, nr=sp.nr, a=sp.a, l=sp.l[:2], eps=sp.eps[:2], hbar2_2mu=sp.hbar2_2mu,
                       pot=lambda r: sp.pot(r)[:, :2, :2].copy(), z1z2=sp.z1z2)
    ref = pipeline.solve_energy(sub, E)["S"]
    assert abs(U[2, 2] - 1.0) < 1e-12 and np.max(np.abs(U[2, :2])) < 1e-12 and np.max(np.abs(U[:2, 2])) < 1e-12
    assert relerr(U[:2, :2], ref) < 1e-12


def test_coupled_deep_channel_acts_through_its_log_derivative():
    """A coupled deep channel carries no flux in double precision: over the
    other channels U equals the matching with the effective R-matrix that
    eliminates it with L = rho G'/G (its regular part F is negligible), the
    closed-channel elimination of reading R12 with the irregular Coulomb
    function in place of the Whittaker function."""
    sp, E = _deep_system(True)
    o = pipeline.solve_energy(sp, E)
    U = o["S"]
    k, eta = rmatrix.wave_numbers(E, sp.eps, sp.hbar2_2mu, sp.z1z2)
    F, Fp, G, Gp = rmatrix.coulomb_mp(2, eta[2], k[2] * sp.a)
    Ld = float(k[2] * sp.a * Gp / G)
    R = o["R"]
    Reff = R[:2, :2] + R[:2, 2:] * Ld @ np.linalg.inv(np.eye(1) - R[2:, 2:] * Ld) @ R[2:, :2]
    fg = rmatrix.coulomb_table(sp.l[:2], eta[:2], k[:2] * sp.a)
    ref = rmatrix.smatrix(Reff, k[:2], sp.a, fg)
    assert relerr(U[:2, :2], ref) < 1e-10
    assert np.max(np.abs(U[2, :2])) < 1e-12 and abs(U[2, 2] - 1.0) < 1e-12
