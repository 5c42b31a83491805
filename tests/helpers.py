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

    @property
    def n(self) -> int:
        return self.nc * self.nr

    def potential(self, r):
        return np.asarray(self.pot(np.asarray(r, dtype=np.float64)), dtype=np.complex128)


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
