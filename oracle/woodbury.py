"""Woodbury-kinetic solve, the paper's Type 3 solver (oracle; test
infrastructure only).

Sec. 3.3: split M = K_diag + V_coupling with K_diag block diagonal in the
channels and solve M c = b as (I + K_diag^-1 V_coupling) c = K_diag^-1 b.
The kinetic block K is real and the same in every channel (Sec. 3.3, step
1), so it is the kinetic + Bloch matrix alone, K = h (T + L); everything
else in M is diagonal in the radial index and goes into the n_c x n_c
matrices of step 2,

    V_aa'(r_j) = V_aa'(r_j) + delta_aa' (h l_a(l_a+1)/r_j^2 + eps_a - E),

which is M's element ((a,j),(a',j)) minus K_jj delta_aa' (reading R14).
Step 3, the Schur-type matrix in the paper's radial-major order
(index (i-1) n_ch + a, 0-based i*nc + a here):

    S[(i,a),(j,a')] = delta_ij delta_aa' + (K^-1)_ij V_aa'(r_j);

step 4, the right-hand side bt[(i,a), c] = sum_j (K^-1)_ij q_j delta_ac;
step 5, S ct = bt (here by the oracle's Gaussian elimination in FP64; the
paper uses single precision); step 6, c[(a,i)] = ct[(i,a)] and R from c as
for the other solvers.  In exact arithmetic c = M^-1 B.
"""
from __future__ import annotations

import numpy as np

from . import ge, rmatrix, system


def kinetic_inverse(params, md: system.MeshData) -> np.ndarray:
    """K^-1 for K = h (T + L) (Sec. 3.3, step 1); a library inverse."""
    return np.linalg.inv(params.hbar2_2mu * md.tl)


def radial_diagonal(params, E: float, md: system.MeshData) -> np.ndarray:
    """V(r_j) of step 2, shape (nr, nc, nc): the potential plus the
    centrifugal barrier, threshold and -E on the channel diagonal."""
    v = np.array(params.potential(md.r), dtype=np.complex128)
    h = params.hbar2_2mu
    for a in range(params.nc):
        la = params.l[a]
        v[:, a, a] += h * la * (la + 1) / md.r ** 2 + params.eps[a] - E
    return v


def schur_system(params, E: float, md: system.MeshData | None = None) -> tuple[np.ndarray, np.ndarray]:
    """(S, bt) of steps 3-4 in radial-major order: S is N x N, bt N x nc."""
    nc, nr = params.nc, params.nr
    md = md or system.MeshData(nr, params.a)
    if system.nonlocal_elements(params, md) is not None:
        raise ValueError("the Woodbury-kinetic form needs local potentials (Sec. 3.3)")
    Ki = kinetic_inverse(params, md)
    V = radial_diagonal(params, E, md)
    n = nc * nr
    S = np.zeros((n, n), dtype=np.complex128)
    for i in range(nr):
        for j in range(nr):
            S[i * nc:(i + 1) * nc, j * nc:(j + 1) * nc] = Ki[i, j] * V[j]
    S += np.eye(n)
    kq = Ki @ md.q
    bt = np.zeros((n, nc), dtype=np.complex128)
    for i in range(nr):
        for a in range(nc):
            bt[i * nc + a, a] = kq[i]
    return S, bt


def solve(params, E: float, md: system.MeshData | None = None) -> dict:
    """Steps 3-6: X (channel-major, N x nc) and R."""
    nc, nr = params.nc, params.nr
    md = md or system.MeshData(nr, params.a)
    S, bt = schur_system(params, E, md)
    ct, _, _ = ge.solve(S, bt)
    X = ct.reshape(nr, nc, nc).transpose(1, 0, 2).reshape(nc * nr, nc)
    R = rmatrix.rmatrix(X, md.q, nc, nr, params.hbar2_2mu, params.a)
    return {"E": E, "X": X, "R": R}
