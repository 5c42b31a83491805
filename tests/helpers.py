"""Shared test helpers: hand-made systems with simple potentials, error metrics."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np


@dataclass
class CustomSystem:
    """Duck-typed stand-in for workload.SystemParams with an arbitrary potential."""
    nc: int
    nr: int
    a: float
    l: np.ndarray
    eps: np.ndarray
    pot: Callable[[np.ndarray], np.ndarray]
    z1z2: int = 0
    hbar2_2mu: float = 2.0
    energies: np.ndarray = field(default_factory=lambda: np.array([10.0]))
    nlpot: Callable[[np.ndarray], np.ndarray] | None = None  # W[c, i, c', j] = W_cc'(r_i, r_j)

    @property
    def n(self) -> int:
        return self.nc * self.nr

    def potential(self, r):
        return np.asarray(self.pot(np.asarray(r, dtype=np.float64)), dtype=np.complex128)

    def nonlocal_potential(self, r):
        if self.nlpot is None:
            return None
        return np.asarray(self.nlpot(np.asarray(r, dtype=np.float64)), dtype=np.complex128)


def separable_nonlocal(lam: float, beta):
    """Rank-one separable kernel W_cc'(r, r') = -lam g_c(r) g_c'(r') with
    g_c(r) = exp(-beta_c r) (the Yamaguchi form; one beta per channel)."""
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))

    def nl(r):
        g = np.exp(-beta[:, None] * r[None, :])  # (nc, nr)
        return (-lam * g[:, :, None, None] * g[None, None, :, :]).astype(np.complex128)
    return nl


def separable_kmatrix(lam: float, beta, k, h: float) -> np.ndarray:
    """Closed-form K matrix of the l = 0 channels coupled by the separable
    kernel above (no Coulomb field, no local potential, all channels open).

    Derivation: with k_c^2 = (E - eps_c)/h the radial equations read
    u_c'' + k_c^2 u_c = -(lam/h) g_c(r) C,  C = sum_c' int g_c' u_c'.  The
    standing-wave Green's function -sin(k r<) cos(k r>)/k gives
    u_c = A_c sin(k_c r) + (lam C / (h k_c)) int sin(k_c r<) cos(k_c r>) g_c,
    whose tail is A_c sin + (lam C I_c / (h k_c)) cos with
    I_c = int_0^inf g_c sin(k_c r) dr = k_c / (b^2 + k_c^2).  Closing for C
    with J_c = int int g_c(r) sin(k r<) cos(k r>) g_c(r')
             = k_c (b^2 - k_c^2) / (2 b (b^2 + k_c^2)^2)   (b = beta_c)
    gives C = sum_c A_c I_c / D, D = 1 - (lam/h) sum_c J_c / k_c, and in the
    flux-normalised form u_c ~ (a_c sin + b_c cos)/sqrt(k_c), b = K a with
    K_cc' = (lam/h) v_c v_c' / D,  v_c = I_c / sqrt(k_c).
    For one channel this is tan(delta) = lam I^2 / (h k - lam J)."""
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    b2k2 = beta ** 2 + k ** 2
    I = k / b2k2
    J = k * (beta ** 2 - k ** 2) / (2.0 * beta * b2k2 ** 2)
    D = 1.0 - (lam / h) * np.sum(J / k)
    v = I / np.sqrt(k)
    return (lam / h) * np.outer(v, v) / D


def diagonal_potential(nc: int, fn: Callable[[np.ndarray], np.ndarray]):
    def pot(r):
        v = np.zeros((len(r), nc, nc), dtype=np.complex128)
        vals = fn(r)
        for c in range(nc):
            v[:, c, c] = vals
        return v
    return pot


def relerr(x, ref) -> float:
    """max |x - ref| / max |ref| (the normwise relative error used throughout)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))
