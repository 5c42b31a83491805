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


def coulomb(l: int, eta: float, rho: float, dps: int = 30) -> tuple[float, float, float, float]:
    """(F, F', G, G') at (l, eta, rho), derivatives with respect to rho."""
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
        return float(F0), float(Fp), float(G0), float(Gp)


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


def cross_sections(U: np.ndarray, k: np.ndarray) -> np.ndarray:
    """sigma[c, c'] = (pi / k_c'^2) |delta_cc' - U_cc'|^2 (fm^2), entrance channel c'."""
    d = np.eye(U.shape[0]) - U
    return np.pi / (k[None, :] ** 2) * np.abs(d) ** 2
