"""R-matrix, Coulomb functions, collision matrix (oracle; test infrastructure only).

R-matrix (Sec. 3.1, step 4, with the factor hbar^2/(2 mu a) that turns the
sum into the dimensionless R-matrix of the Bloch-operator formalism):

    R_cc' = (hbar^2 / 2 mu a) sum_i q_i X[(c, i), c'],   X = M^-1 B.

Collision matrix (the matching to Coulomb functions at r = a that the paper
delegates to its Coulomb routine, Sec. 4.1): in every open channel the
external solution is u_c = k_c^(-1/2) [I_c delta_cc0 - U_cc0 O_c] with
I = G - iF, O = G + iF evaluated at rho_c = k_c a.  Imposing
u(a) = R a u'(a) gives

    U = (O - Rt O')^-1 (I - Rt I'),   Rt = rho^(1/2) R rho^(1/2),

where O, O', I, I' are diagonal and ' is d/drho.

Coulomb functions come from mpmath (arbitrary precision); derivatives use
Abramowitz & Stegun 14.2.2,
    (l+1) u_l' = ((l+1)^2/rho + eta) u_l - sqrt((l+1)^2 + eta^2) u_{l+1}.

Closed channels (E < eps_c; the Whittaker functions of the paper's special-
function set, Sec. 4.1): the external solution decays,
u_c(r) = C_c W_{-eta_c, l_c + 1/2}(2 kappa_c r) with kappa_c = sqrt((eps_c - E)/h)
and eta_c = Z1Z2 e^2 / (2 h kappa_c), so a u_c'(a) = L_c u_c(a) with
L_c = x W'(x) / W(x) at x = kappa_c a (W as a function of x).  Splitting
u(a) = R a u'(a) into open (o) and closed (c) channels and eliminating the
closed ones gives the open channels' effective R-matrix

    R_eff = R_oo + R_oc L (I - R_cc L)^-1 R_co,   L = diag(L_c),

from which U (open channels only) follows as above (reading R12).
Whittaker values come from mpmath; the derivative by mpmath's numerical
differentiation at the working precision.

Open channels far below their Coulomb barrier (large eta, rho well inside
the turning point): F underflows and G overflows double range, so the same
matching formula is evaluated with mpmath values and an mpmath solve
(:func:`smatrix_mp`).
"""
from __future__ import annotations

import numpy as np
import mpmath

E2 = 1.44  # MeV fm


def rmatrix(X: np.ndarray, q: np.ndarray, nc: int, nr: int, hbar2_2mu: float, a: float) -> np.ndarray:
    """R[c, c'] from the solution X (N x nc)."""
    R = np.zeros((nc, nc), dtype=np.complex128)
    for c in range(nc):
        for cp in range(nc):
            s = 0.0 + 0.0j
            for i in range(nr):
                s += q[i] * X[c * nr + i, cp]
            R[c, cp] = s
    return (hbar2_2mu / a) * R


def wave_numbers(E: float, eps: np.ndarray, hbar2_2mu: float, z1z2: int) -> tuple[np.ndarray, np.ndarray]:
    """k_c = sqrt((E - eps_c)/h) and eta_c = Z1Z2 e^2 / (2 h k_c) (open channels)."""
    ec = E - np.asarray(eps, dtype=np.float64)
    if np.any(ec <= 0):
        raise ValueError("closed channel")
    k = np.sqrt(ec / hbar2_2mu)
    eta = z1z2 * E2 / (2.0 * hbar2_2mu * k)
    return k, eta


def coulomb_mp(l: int, eta: float, rho: float, dps: int = 30):
    """(F, F', G, G') at (l, eta, rho) as mpmath numbers (no range limit),
    derivatives with respect to rho."""
    with mpmath.workdps(dps):
        L = mpmath.mpf(l)
        et = mpmath.mpf(eta)
        rh = mpmath.mpf(rho)
        F0 = mpmath.coulombf(L, et, rh)
        F1 = mpmath.coulombf(L + 1, et, rh)
        G0 = mpmath.coulombg(L, et, rh)
        G1 = mpmath.coulombg(L + 1, et, rh)
        s = ((L + 1) ** 2 / rh + et)
        r = mpmath.sqrt((L + 1) ** 2 + et ** 2)
        Fp = (s * F0 - r * F1) / (L + 1)
        Gp = (s * G0 - r * G1) / (L + 1)
        return F0, Fp, G0, Gp


def coulomb(l: int, eta: float, rho: float, dps: int = 30) -> tuple[float, float, float, float]:
    """(F, F', G, G') at (l, eta, rho), derivatives with respect to rho."""
    return tuple(float(x) for x in coulomb_mp(l, eta, rho, dps))


def coulomb_table(l: np.ndarray, eta: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """Array (nc, 4) of (F, F', G, G') per channel."""
    out = np.zeros((len(l), 4))
    for c in range(len(l)):
        out[c] = coulomb(int(l[c]), float(eta[c]), float(rho[c]))
    return out


def smatrix(R: np.ndarray, k: np.ndarray, a: float, fg: np.ndarray) -> np.ndarray:
    """Collision matrix U from R and the channel Coulomb values fg (nc, 4)."""
    rho = k * a
    F, Fp, G, Gp = fg[:, 0], fg[:, 1], fg[:, 2], fg[:, 3]
    O, Op = G + 1j * F, Gp + 1j * Fp
    I, Ip = G - 1j * F, Gp - 1j * Fp
    sq = np.sqrt(rho)
    Rt = sq[:, None] * R * sq[None, :]
    ZO = np.diag(O) - Rt * Op[None, :]
    ZI = np.diag(I) - Rt * Ip[None, :]
    return np.linalg.solve(ZO, ZI)


def in_double_range(fg: np.ndarray) -> bool:
    """Whether every channel's Coulomb values are finite doubles with F != 0
    (far below a Coulomb barrier F underflows and G overflows)."""
    return bool(np.all(np.isfinite(fg)) and np.all(fg[:, 0] != 0.0))


def smatrix_mp(R: np.ndarray, k: np.ndarray, a: float, l: np.ndarray, eta: np.ndarray,
               dps: int = 30) -> np.ndarray:
    """The collision matrix of :func:`smatrix`, U = (O - Rt O')^-1 (I - Rt I'),
    with the Coulomb values and the solve in mpmath arithmetic (for open
    channels whose F and G leave double range); U rounded to complex128."""
    nc = len(l)
    with mpmath.workdps(dps):
        fg = [coulomb_mp(int(l[c]), float(eta[c]), float(k[c] * a), dps) for c in range(nc)]
        sq = [mpmath.sqrt(mpmath.mpf(float(k[c] * a))) for c in range(nc)]
        ZO = mpmath.matrix(nc, nc)
        ZI = mpmath.matrix(nc, nc)
        for c in range(nc):
            for cp in range(nc):
                F, Fp, G, Gp = fg[cp]
                rt = sq[c] * mpmath.mpc(complex(R[c, cp])) * sq[cp]
                ZO[c, cp] = -rt * mpmath.mpc(Gp, Fp)
                ZI[c, cp] = -rt * mpmath.mpc(Gp, -Fp)
            F, Fp, G, Gp = fg[c]
            ZO[c, c] += mpmath.mpc(G, F)
            ZI[c, c] += mpmath.mpc(G, -F)
        # columns scaled by d_c = 1/|G_c| (the solver's singularity test is
        # relative to the matrix norm, which one G_c ~ 1e300 would dominate):
        # U = D (ZO D)^-1 (ZI D) D^-1, an identity
        d = [1 / abs(fg[c][2]) for c in range(nc)]
        for c in range(nc):
            for cp in range(nc):
                ZO[c, cp] *= d[cp]
                ZI[c, cp] *= d[cp]
        U = np.zeros((nc, nc), dtype=np.complex128)
        for j in range(nc):  # one right-hand column at a time
            col = mpmath.lu_solve(ZO, ZI.column(j))
            U[:, j] = [complex(d[i] * col[i] / d[j]) for i in range(nc)]
        return U


def closed_logderiv(l: int, eta: float, x: float, dps: int = 30) -> float:
    """x W'(x) / W(x) for W(x) = W_{-eta, l + 1/2}(2 x): the decaying solution of
    u'' = (1 + l(l+1)/x^2 + 2 eta/x) u, x = kappa r."""
    with mpmath.workdps(dps):
        kap = -mpmath.mpf(eta)
        mu = mpmath.mpf(l) + mpmath.mpf(1) / 2

        def w(xx):
            return mpmath.whitw(kap, mu, 2 * xx)

        X = mpmath.mpf(x)
        return float(X * mpmath.diff(w, X) / w(X))


def channels(E: float, eps: np.ndarray, hbar2_2mu: float, z1z2: int):
    """Open and closed channel indices, and per channel the wave number k
    (open) or decay constant kappa (closed) and its Sommerfeld parameter."""
    ec = E - np.asarray(eps, dtype=np.float64)
    if np.any(ec == 0.0):
        raise ValueError("energy at a threshold")
    kk = np.sqrt(np.abs(ec) / hbar2_2mu)
    eta = z1z2 * E2 / (2.0 * hbar2_2mu * kk)
    return np.where(ec > 0)[0], np.where(ec < 0)[0], kk, eta


def smatrix_closed(R: np.ndarray, E: float, eps: np.ndarray, l: np.ndarray, hbar2_2mu: float, z1z2: int,
                   a: float):
    """Collision matrix of the open channels with the closed ones eliminated
    through R_eff.  Returns (U, open indices, R_eff)."""
    o, c, kk, eta = channels(E, eps, hbar2_2mu, z1z2)
    if len(o) == 0:
        raise ValueError("no open channel")
    Reff = R[np.ix_(o, o)]
    if len(c):
        Lc = np.array([closed_logderiv(int(l[ci]), float(eta[ci]), float(kk[ci] * a)) for ci in c])
        Lm = np.diag(Lc)
        Y = np.linalg.solve(np.eye(len(c)) - R[np.ix_(c, c)] @ Lm, R[np.ix_(c, o)])
        Reff = Reff + R[np.ix_(o, c)] @ Lm @ Y
    fg = coulomb_table(np.asarray(l)[o], eta[o], kk[o] * a)
    if in_double_range(fg):
        return smatrix(Reff, kk[o], a, fg), o, Reff
    # an open channel far below its Coulomb barrier
    return smatrix_mp(Reff, kk[o], a, np.asarray(l)[o], eta[o]), o, Reff


def cross_sections(U: np.ndarray, k: np.ndarray) -> np.ndarray:
    """sigma[c, c'] = (pi / k_c'^2) |delta_cc' - U_cc'|^2 (fm^2), entrance channel c'."""
    d = np.eye(U.shape[0]) - U
    return np.pi / (k[None, :] ** 2) * np.abs(d) ** 2
