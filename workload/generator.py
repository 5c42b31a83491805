"""Seeded synthetic coupled-channel systems (Woods-Saxon optical-potential family).

Every system is a set of drawn parameters plus the potential V_cc'(r) they
define.  The potential is the user-supplied input of the coupled-channel
radial equation (Sec. 2, Eq. cc_schrodinger); the R-matrix solver evaluates it
at its own mesh points by calling :meth:`SystemParams.potential`.

Potential family (readings of the workload description are listed in the
design notes):

* one complex central nuclear potential per system,
  U(r) = -(V0 + i W0) / (1 + exp((r - R) / d)),  R = 1.2 A^(1/3), d = 0.65 fm;
* the Coulomb potential of a uniformly charged sphere of radius R,
  Z1Z2 e^2 / r outside and Z1Z2 e^2 (3 - r^2/R^2) / (2R) inside;
* diagonal channel potential V_cc = U + V_Coulomb;
* all-pairs couplings V_cc' = -beta_cc' R dU/dr (deformation-length form
  factor), beta symmetric so that the coupling matrix is symmetric.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

HBAR2_2MU = 2.0  # MeV fm^2, common to all channels
E2 = 1.44  # e^2 in MeV fm
DIFFUSENESS = 0.65  # fm
E_LO, E_HI = 5.0, 30.0  # MeV, energy window of every configuration

# name -> (nc, nr, a [fm], l_max, number of energies, seed)
CONFIGS = {
    "small": dict(nc=4, nr=40, a=15.0, lmax=6, n_energies=10, seed=1159001),
    "mid": dict(nc=100, nr=60, a=20.0, lmax=20, n_energies=20, seed=1159002),
    "large": dict(nc=256, nr=100, a=30.0, lmax=20, n_energies=10, seed=1159003),
}


def energies(n_energies: int, lo: float = E_LO, hi: float = E_HI) -> np.ndarray:
    """Total energies: midpoints of n equal sub-intervals of [lo, hi] (MeV)."""
    j = np.arange(n_energies, dtype=np.float64)
    return lo + (hi - lo) * (j + 0.5) / n_energies


@dataclass
class SystemParams:
    nc: int
    nr: int
    a: float
    l: np.ndarray  # int64 [nc]
    eps: np.ndarray  # float64 [nc], channel thresholds (MeV)
    z1z2: int
    v0: float
    w0: float
    mass_a: float
    beta: np.ndarray  # float64 [nc, nc], symmetric, zero diagonal
    energies: np.ndarray  # float64 [n_E]
    hbar2_2mu: float = HBAR2_2MU
    diffuseness: float = DIFFUSENESS
    label: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nc * self.nr

    @property
    def radius(self) -> float:
        return 1.2 * self.mass_a ** (1.0 / 3.0)

    def central(self, r: np.ndarray) -> np.ndarray:
        """U(r), complex, MeV."""
        x = (np.asarray(r, dtype=np.float64) - self.radius) / self.diffuseness
        f = 1.0 / (1.0 + np.exp(x))
        return -(self.v0 + 1j * self.w0) * f

    def coupling_form(self, r: np.ndarray) -> np.ndarray:
        """-R dU/dr (complex, MeV); multiplied by beta_cc' it gives V_cc'."""
        x = (np.asarray(r, dtype=np.float64) - self.radius) / self.diffuseness
        f = 1.0 / (1.0 + np.exp(x))
        du_dr = (self.v0 + 1j * self.w0) * f * (1.0 - f) / self.diffuseness
        return -self.radius * du_dr

    def coulomb(self, r: np.ndarray) -> np.ndarray:
        r = np.asarray(r, dtype=np.float64)
        rc = self.radius
        zz = self.z1z2 * E2
        out = np.where(r >= rc, zz / np.maximum(r, 1e-300),
                       zz * (3.0 - (r / rc) ** 2) / (2.0 * rc))
        return out

    def potential(self, r: np.ndarray) -> np.ndarray:
        """V[i, c, c'] = V_cc'(r_i), complex128, shape (len(r), nc, nc)."""
        r = np.asarray(r, dtype=np.float64)
        diag = self.central(r) + self.coulomb(r)
        form = self.coupling_form(r)
        v = form[:, None, None] * self.beta[None, :, :]
        idx = np.arange(self.nc)
        v[:, idx, idx] = diag[:, None]
        return v.astype(np.complex128)


def perey_buck_factors(sp: SystemParams, r: np.ndarray, strength: float = 0.4,
                       width: float = 0.85) -> tuple[np.ndarray, np.ndarray]:
    """A non-local optical kernel of Perey-Buck form on the system's channels
    (an input of the non-local coupled-channel equation, Sec. 2):

        W_cc'(r, r') = B_cc' s U((r + r')/2) exp(-((r - r')/width)^2) / (sqrt(pi) width),

    U the system's complex Woods-Saxon shape, s = `strength`, B = I + beta
    (the system's coupling strengths off the diagonal).  Returned as the
    factors (B [nc, nc] float64, K [nr, nr] complex128 at the points r), so
    that the kernel values in channel-major order are kron(B, K)."""
    r = np.asarray(r, dtype=np.float64)
    rbar = 0.5 * (r[:, None] + r[None, :])
    h = np.exp(-((r[:, None] - r[None, :]) / width) ** 2) / (math.sqrt(math.pi) * width)
    K = strength * sp.central(rbar.ravel()).reshape(rbar.shape) * h
    B = np.eye(sp.nc) + np.asarray(sp.beta, dtype=np.float64)
    return B, K.astype(np.complex128)


def with_perey_buck(sp: SystemParams, strength: float = 0.4) -> SystemParams:
    """The same system with the Perey-Buck kernel added: sets its
    ``nonlocal_potential(r)`` (shape (nc, nr, nc, nr)); for small systems, as
    the values are held on the host."""
    def nonlocal_potential(r):
        B, K = perey_buck_factors(sp, r, strength)
        n = len(r)
        return np.kron(B, K).reshape(sp.nc, n, sp.nc, n)
    sp.nonlocal_potential = nonlocal_potential
    sp.label += f" + Perey-Buck non-local x{strength}"
    return sp


def _draw(rng: np.random.Generator, nc: int, nr: int, a: float, lmax: int,
          n_energies: int, label: str) -> SystemParams:
    v0 = float(rng.uniform(40.0, 60.0))
    w0 = float(rng.uniform(5.0, 15.0))
    mass_a = float(rng.uniform(40.0, 60.0))
    z1z2 = int(rng.integers(0, 41))
    eps = rng.uniform(0.0, 5.0, size=nc)
    l = rng.integers(0, lmax + 1, size=nc).astype(np.int64)
    beta = np.zeros((nc, nc))
    iu = np.triu_indices(nc, k=1)
    beta[iu] = rng.uniform(0.05, 0.3, size=len(iu[0]))
    beta = beta + beta.T
    return SystemParams(nc=nc, nr=nr, a=a, l=l, eps=eps, z1z2=z1z2, v0=v0, w0=w0,
                        mass_a=mass_a, beta=beta, energies=energies(n_energies),
                        label=label)


def make_system(config: str = "small", seed: int | None = None, **override) -> SystemParams:
    """Draw the system of a named configuration ("small", "mid", "large").

    Keyword overrides (nc, nr, a, lmax, n_energies) resize it while keeping the
    same potential family and seed.
    """
    cfg = dict(CONFIGS[config])
    cfg.update(override)
    s = cfg.pop("seed") if seed is None else seed
    cfg.pop("seed", None)
    rng = np.random.default_rng(s)
    return _draw(rng, cfg["nc"], cfg["nr"], cfg["a"], cfg["lmax"], cfg["n_energies"],
                 label=f"{config}:seed={s}")


def batch_systems(count: int = 512, seed: int = 1159004, a: float = 20.0,
                  lmax: int = 20) -> list[SystemParams]:
    """Uneven batch: nc ~ U{5..80}, nr ~ U{40..50}, one energy label each."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        nc = int(rng.integers(5, 81))
        nr = int(rng.integers(40, 51))
        sp = _draw(rng, nc, nr, a, lmax, 1, label=f"batch[{b}]")
        sp.energies = np.array([float(rng.uniform(E_LO + 1.0, E_HI))])
        sp.extra["jpi"] = (int(rng.integers(0, 20)), int(rng.choice([-1, 1])))
        out.append(sp)
    return out


def served_requests(count: int, rate_hz: float, seed: int = 1159005,
                    a: float = 20.0, lmax: int = 20) -> list[tuple[float, SystemParams]]:
    """Poisson arrivals; N log-uniform in [500, 16000], nr in [40, 100], 1-8 energies."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        n_target = math.exp(rng.uniform(math.log(500.0), math.log(16000.0)))
        nr = int(rng.integers(40, 101))
        nc = max(1, int(round(n_target / nr)))
        ne = int(rng.integers(1, 9))
        sp = _draw(rng, nc, nr, a, lmax, ne, label=f"req[{q}]")
        out.append((t, sp))
    return out
