"""Block matrix M and surface right-hand sides B (oracle; test infrastructure only).

Sec. 2, Eqs. linear_system and block_structure: M is N x N with
N = n_ch * n_lag, channel-major index (alpha - 1) n_lag + i (Sec. 3.1,
step 4).  Diagonal blocks are K_alpha + D_alpha,alpha, off-diagonal blocks
are the diagonal coupling matrices (D_alpha,alpha')_ij = V_alpha,alpha'(r_i)
delta_ij of local potentials.

K_alpha holds the kinetic energy with the Bloch term, the centrifugal
barrier of Eq. cc_schrodinger, the channel threshold and -E.  With the
Gauss approximation for the local terms (Lagrange property):

  M[(c,i),(c',j)] = delta_cc' [ h TL_ij + delta_ij ( h l_c (l_c+1) / r_i^2
                                                    + eps_c - E ) ]
                    + delta_ij V_cc'(r_i),           h = hbar^2 / 2 mu.

Non-local potentials (Sec. 2: the coupling blocks D become full matrices).
A system may carry a non-local kernel W_cc'(r, r') besides the local V.  Its
Lagrange-mesh matrix element, with the same Gauss quadrature as the local
terms and f_i(r_k) = delta_ik / sqrt(w_i), is

  <f_i | W_cc' | f_j> = sqrt(w_i w_j) W_cc'(r_i, r_j),      w_i = a lambda_i,

added to every element of block (c, c').  The system supplies the kernel at
the mesh-point pairs through ``nonlocal_potential(r)`` (shape
(nc, nr, nc, nr): W[c, i, c', j] = W_cc'(r_i, r_j), MeV/fm); a system
without that method, or returning None, is local.

B (Sec. 3.1, step 2) is N x n_ch; column c holds q_i = f_i(a) in block c.
"""
from __future__ import annotations

import numpy as np

from . import mesh


class MeshData:
    """Mesh, kinetic+Bloch matrix and surface values for one (n_lag, a)."""

    def __init__(self, nr: int, a: float):
        self.nr = nr
        self.a = a
        self.r, self.w = mesh.mesh(nr, a)
        self.tl = mesh.kinetic_bloch(nr, a)
        self.q = mesh.surface_values(nr, a)


def nonlocal_elements(params, md: MeshData) -> np.ndarray | None:
    """The N x N non-local matrix elements sqrt(w_i w_j) W_cc'(r_i, r_j) in
    channel-major order, or None for a local system."""
    fn = getattr(params, "nonlocal_potential", None)
    W = fn(md.r) if fn is not None else None
    if W is None:
        return None
    nc, nr = params.nc, params.nr
    W = np.asarray(W, dtype=np.complex128).reshape(nc, nr, nc, nr)
    sw = np.sqrt(md.w)
    return (sw[None, :, None, None] * W * sw[None, None, None, :]).reshape(nc * nr, nc * nr)


def assemble(params, E: float, md: MeshData | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Return (M, B) as complex128 arrays, M row-major N x N, B N x nc."""
    nc, nr = params.nc, params.nr
    md = md or MeshData(nr, params.a)
    h = params.hbar2_2mu
    v = params.potential(md.r)  # (nr, nc, nc)
    n = nc * nr
    M = np.zeros((n, n), dtype=np.complex128)
    for c in range(nc):
        blk = slice(c * nr, (c + 1) * nr)
        K = h * md.tl.astype(np.complex128)
        K[np.arange(nr), np.arange(nr)] += (h * params.l[c] * (params.l[c] + 1) / md.r ** 2
                                            + params.eps[c] - E)
        M[blk, blk] = K
    for c in range(nc):
        for cp in range(nc):
            rows = c * nr + np.arange(nr)
            cols = cp * nr + np.arange(nr)
            M[rows, cols] += v[:, c, cp]
    Wm = nonlocal_elements(params, md)
    if Wm is not None:
        M += Wm
    B = np.zeros((n, nc), dtype=np.complex128)
    for c in range(nc):
        B[c * nr:(c + 1) * nr, c] = md.q
    return M, B


def apply(params, E: float, X: np.ndarray, md: MeshData | None = None) -> np.ndarray:
    """M @ X using the block structure (no N x N array), X of shape (N, k).

    Row (c, i): sum_j h TL_ij X[(c, j)] + (h l_c(l_c+1)/r_i^2 + eps_c - E) X[(c, i)]
                + sum_c' V_cc'(r_i) X[(c', i)]
                + sum_c',j sqrt(w_i w_j) W_cc'(r_i, r_j) X[(c', j)]   (non-local systems).
    """
    nc, nr = params.nc, params.nr
    md = md or MeshData(nr, params.a)
    h = params.hbar2_2mu
    v = params.potential(md.r)
    Xb = X.reshape(nc, nr, -1)
    out = np.empty_like(Xb, dtype=np.complex128)
    for c in range(nc):
        diag = h * params.l[c] * (params.l[c] + 1) / md.r ** 2 + params.eps[c] - E
        out[c] = h * (md.tl @ Xb[c]) + diag[:, None] * Xb[c]
    # sum over c' of V_cc'(r_i) X[(c', i)], for every i
    out += np.einsum("icd,dik->cik", v, Xb)
    out = out.reshape(nc * nr, -1)
    Wm = nonlocal_elements(params, md)
    if Wm is not None:
        out += Wm @ X
    return out
