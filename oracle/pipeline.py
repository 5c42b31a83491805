"""One energy end to end (oracle; test infrastructure only).

Sec. 3.1 (Type 1): build M and B, solve M X = B by Gaussian elimination with
partial pivoting, extract R; then the collision matrix and channel cross
sections by matching to Coulomb functions.
"""
from __future__ import annotations

import numpy as np

from . import ge, rmatrix, system


def solve_energy(params, E: float, md: system.MeshData | None = None,
                 with_smatrix: bool = True) -> dict:
    md = md or system.MeshData(params.nr, params.a)
    M, B = system.assemble(params, E, md)
    X, _, ipiv = ge.solve(M, B)
    R = rmatrix.rmatrix(X, md.q, params.nc, params.nr, params.hbar2_2mu, params.a)
    out = {"E": E, "X": X, "R": R, "ipiv": ipiv}
    if with_smatrix:
        if np.all(E > np.asarray(params.eps, dtype=np.float64)):
            k, eta = rmatrix.wave_numbers(E, params.eps, params.hbar2_2mu, params.z1z2)
            fg = rmatrix.coulomb_table(params.l, eta, k * params.a)
            if rmatrix.in_double_range(fg):
                U = rmatrix.smatrix(R, k, params.a, fg)
            else:  # a channel far below its Coulomb barrier
                U = rmatrix.smatrix_mp(R, k, params.a, np.asarray(params.l), eta)
            out.update(k=k, eta=eta, fg=fg, S=U, sigma=rmatrix.cross_sections(U, k),
                       open=np.arange(params.nc))
        else:
            # closed channels eliminated; S over the open channels only
            U, o, _ = rmatrix.smatrix_closed(R, E, np.asarray(params.eps), np.asarray(params.l),
                                             params.hbar2_2mu, params.z1z2, params.a)
            _, _, kk, eta = rmatrix.channels(E, params.eps, params.hbar2_2mu, params.z1z2)
            out.update(k=kk[o], eta=eta[o], S=U, sigma=rmatrix.cross_sections(U, kk[o]), open=o)
    return out
