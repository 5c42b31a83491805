"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (normwise relative, max|x - ref| / max|ref|):
  * assembly FP64: 1e-12 (the library's closed-form kinetic matrix and the
    oracle's quadrature of its definition agree to 1 ulp; 1e-12 leaves room
    for the FP64 potential evaluation at mesh points that differ by 1 ulp);
  * LU factors / solutions of random well-conditioned matrices: 1e-12 (FP64),
    1e-4 (FP32);
  * R and S of the small workload: 1e-10 (FP64 LU; FP32 LU + FP64 refinement).
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import ge, pipeline as opipe, rmatrix as ormat, system as osys  # noqa: E402
from tests.helpers import CustomSystem, diagonal_potential, relerr  # noqa: E402
from workload import make_system  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat
    hprmat.lib()
    return hprmat


@pytest.fixture(scope="module")
def P(H):
    from paper_2512_11590_amd import pipeline
    return pipeline


def rand_matrix(n, seed, diag=0.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A + diag * np.eye(n)


def device_factor(H, A, prec):
    n = A.shape[0]
    ct = torch.complex64 if prec == H.HP_C64 else torch.complex128
    dA = torch.from_numpy(A.astype(np.complex64 if prec == H.HP_C64 else np.complex128)).to("cuda")
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = torch.empty(H.hp_workspace_bytes(n, 256, prec), dtype=torch.uint8, device="cuda")
    H.hp_factor(n, prec, dA, n, ipiv, perm, info, work)
    torch.cuda.synchronize()
    assert dA.dtype == ct
    return dA, ipiv, perm, info, work


# ------------------------------------------------------------ factorization --

@pytest.mark.parametrize("n", [1, 7, 32, 33, 100, 255, 256, 257, 300, 600])
def test_lu_fp64_matches_oracle_elimination(H, n):
    say("lu fp64", n)
    A = rand_matrix(n, n)
    dA, ipiv, perm, info, _ = device_factor(H, A, H.HP_C128)
    assert int(info.item()) == 0
    _, LU, ipiv_o = ge.solve(A, np.ones((n, 1), complex))
    # same pivot rule, same pivots on random data
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    assert relerr(dA.cpu().numpy(), LU) < 1e-12
    # perm is the composition of the interchanges
    pr = np.arange(n)
    for k in range(n):
        pr[[k, ipiv_o[k]]] = pr[[ipiv_o[k], k]]
    assert np.array_equal(perm.cpu().numpy(), pr)


def row_scrambled(n, seed, kind):
    """A diagonally dominant matrix with its rows moved, so that partial
    pivoting has to fetch every pivot row from elsewhere: `reverse` puts row
    j at n-1-j (pivots from far below the block); `shift` moves every row up
    by one (the pivot of every column is the row the previous interchange
    sent to the bottom, so one row is chosen many times within a panel)."""
    B = rand_matrix(n, seed, diag=10.0 * np.sqrt(n))
    if kind == "reverse":
        return B[::-1].copy()
    return np.roll(B, -1, axis=0)


@pytest.mark.parametrize("kind", ["reverse", "shift"])
@pytest.mark.parametrize("n", [45, 300, 600])
def test_lu_interchanges_from_below(H, n, kind):
    say("lu interchanges", kind, n)
    A = row_scrambled(n, 3 * n + len(kind), kind)
    _, LU, ipiv_o = ge.solve(A, np.ones((n, 1), complex))
    if kind == "shift":  # the pivot rows repeat: every column takes row n-1
        assert np.all(ipiv_o[:-1] == n - 1)
    dA, ipiv, perm, info, _ = device_factor(H, A, H.HP_C128)
    assert int(info.item()) == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    assert relerr(dA.cpu().numpy(), LU) < 1e-12
    dA, ipiv, perm, info, _ = device_factor(H, A, H.HP_C64)
    assert int(info.item()) == 0
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_o)
    LU32 = dA.cpu().numpy().astype(np.complex128)
    L = np.tril(LU32, -1) + np.eye(n)
    U = np.triu(LU32)
    assert relerr(L @ U, A[perm.cpu().numpy()]) < 1e-5


@pytest.mark.parametrize("n", [5, 64, 257, 513])
def test_lu_fp32_backward_error(H, n):
    say("lu fp32", n)
    A = rand_matrix(n, 100 + n)
    dA, ipiv, perm, info, _ = device_factor(H, A, H.HP_C64)
    assert int(info.item()) == 0
    LU = dA.cpu().numpy().astype(np.complex128)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    p = perm.cpu().numpy()
    # backward error of an LU factorization in unit roundoff u, elementwise:
    # |P A - L U| <= gamma_n |L||U|, gamma_n = n u / (1 - n u) (u = 2^-24 for
    # the FP32 factors, counting the complex product's few extra roundings in
    # a factor 4); the input is rounded to FP32 first
    A32 = A.astype(np.complex64).astype(np.complex128)
    nu = 4 * n * 2.0 ** -24
    bound = nu / (1 - nu) * (np.abs(L) @ np.abs(U))
    assert np.all(np.abs(L @ U - A32[p]) <= bound)
    assert relerr(L @ U, A[p]) < 1e-4
    # partial pivoting (largest |Re| + |Im| in the column, reading of Sec. 3.1):
    # l_ij u_jj is the entry of column j at step j before the division, so
    # no entry below the pivot may exceed the pivot in |Re| + |Im| (the
    # product recovers that entry to a few FP32 roundings)
    def cabs1(z):
        return np.abs(z.real) + np.abs(z.imag)
    d = np.diag(U)
    below = np.tril(cabs1(np.tril(LU, -1) * d[None, :]), -1)
    assert np.all(below <= cabs1(d)[None, :] * (1 + 1e-5))
    assert np.max(np.abs(np.tril(LU, -1))) <= np.sqrt(2.0) * (1 + 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (40, 3), (300, 17), (700, 64), (1025, 9), (384, 256)])
def test_lu_solve_general_rhs(H, prec, n, nrhs):
    say("lu_solve", prec, n, nrhs)
    A = rand_matrix(n, 7 * n + nrhs, diag=2.0 * np.sqrt(n))
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    dA, ipiv, perm, info, work = device_factor(H, A, prec)
    ct = np.complex64 if prec == H.HP_C64 else np.complex128
    dX = torch.from_numpy(B.astype(ct)).to("cuda")
    H.hp_lu_solve(n, nrhs, prec, dA, n, perm, dX, nrhs, work)
    X = dX.cpu().numpy()
    Xo, _, _ = ge.solve(A, B)
    assert relerr(X, Xo) < (1e-12 if prec == H.HP_C128 else 1e-4)


def test_manufactured_solution_fp64(H):
    """x = 1, b = A 1 with 64 right-hand sides (the paper's Table mgpu test)."""
    say("manufactured")
    n = 1000
    A = rand_matrix(n, 11, diag=60.0)
    X1 = np.ones((n, 64), complex)
    dA, ipiv, perm, info, work = device_factor(H, A, H.HP_C128)
    dX = torch.from_numpy(A @ X1).to("cuda")
    H.hp_lu_solve(n, 64, H.HP_C128, dA, n, perm, dX, 64, work)
    assert np.max(np.abs(dX.cpu().numpy() - 1)) < 7e-14


def test_zero_pivot_reported(H):
    say("singular")
    n = 40
    A = rand_matrix(n, 5)
    A[:, 17] = 0
    dA, ipiv, perm, info, _ = device_factor(H, A, H.HP_C128)
    assert int(info.item()) == 18


# ---------------------------------------------------------------- assembly --

@pytest.mark.parametrize("prec", [0, 1])
def test_build_matrix_matches_oracle(H, P, prec):
    say("assembly", prec)
    sp = make_system("small")
    E = float(sp.energies[2])
    d = P.DeviceSystem(sp)
    n = d.n
    ld = n + 3
    ct = torch.complex64 if prec == H.HP_C64 else torch.complex128
    C = torch.full((n, ld), 7 + 7j, dtype=ct, device="cuda")
    H.hp_build_matrix(d.sys, E, prec, C, ld)
    Cd = C.cpu().numpy()
    assert np.all(Cd[:, n:] == 7 + 7j)  # padding untouched
    Mo, _ = osys.assemble(sp, E)
    if prec == H.HP_C128:
        assert relerr(Cd[:, :n], Mo) < 1e-12
        assert np.array_equal(Cd[:, :n], Cd[:, :n].T)
    else:
        assert relerr(Cd[:, :n], Mo) < 1e-7
    # structure: exact zeros where the block structure has them
    assert np.array_equal(Cd[:, :n] == 0, Mo == 0)


# ---------------------------------------------------------------- pipeline --

def compare_energy(P, H, sp, idx, prec, tol_r, tol_s, dsys=None, solver=None):
    d = dsys or P.DeviceSystem(sp)
    s = solver or P.Solver(d, prec)
    md = osys.MeshData(sp.nr, sp.a)
    for e in idx:
        E = float(sp.energies[e])
        say("pipeline", sp.label, "prec", prec, "E", E)
        res = s.run(E)
        o = opipe.solve_energy(sp, E, md)
        er = relerr(res.R.cpu().numpy(), o["R"])
        es = relerr(res.S.cpu().numpy(), o["S"])
        print(f"   R err {er:.2e}  S err {es:.2e}  it {res.iterations} fb {res.fallback}", flush=True)
        assert er < tol_r and es < tol_s
        assert not res.fallback  # an FP32 result must come from the FP32 factors
        assert res.nopen == sp.nc
    return d, s


def test_pipeline_small_fp64(H, P):
    sp = make_system("small")
    compare_energy(P, H, sp, range(10), H.HP_C128, 1e-10, 1e-10)


def test_pipeline_small_fp32_refined(H, P):
    sp = make_system("small")
    compare_energy(P, H, sp, range(10), H.HP_C64, 1e-10, 1e-10)


@pytest.mark.parametrize("nc,nr", [(1, 7), (1, 40), (3, 97), (5, 52), (9, 33)])
def test_pipeline_edge_shapes(H, P, nc, nr):
    sp = make_system("small", nc=nc, nr=nr, lmax=8)
    compare_energy(P, H, sp, [0, 9], H.HP_C128, 1e-10, 1e-10)
    compare_energy(P, H, sp, [4], H.HP_C64, 1e-10, 1e-10)


def test_zero_potential_unit_S_on_device(H, P):
    nc = 4
    sp = CustomSystem(nc=nc, nr=60, a=15.0, l=np.array([0, 2, 5, 9]), eps=np.array([0.0, 1.0, 2.0, 3.0]),
                      z1z2=12, pot=diagonal_potential(nc, lambda r: 12 * 1.44 / r + 0j))
    sp.energies = np.array([12.0])
    say("zero potential")
    d = P.DeviceSystem(sp)
    res = P.Solver(d, H.HP_C128).run(12.0)
    assert np.max(np.abs(res.S.cpu().numpy() - np.eye(nc))) < 1e-11


def test_smatrix_from_oracle_R(H, P):
    """hp_smatrix alone: same R in, same U out as the oracle's matching."""
    sp = make_system("small", nc=6, nr=50)
    E = 13.0
    o = opipe.solve_energy(sp, E)
    d = P.DeviceSystem(sp)
    R = torch.from_numpy(o["R"]).to("cuda")
    S = torch.empty_like(R)
    work = torch.empty(H.hp_workspace_bytes(sp.nc, sp.nc, H.HP_C128), dtype=torch.uint8, device="cuda")
    say("smatrix")
    nopen = H.hp_smatrix(d.sys, E, R, S, work)
    assert nopen == sp.nc
    assert relerr(S.cpu().numpy(), o["S"]) < 1e-12


def test_coulomb_device_matches_host(H):
    cases = [(l, eta, rho) for l in (0, 3, 20) for eta in (0.0, 7.5, 25.8) for rho in (11.2, 40.0, 116.0)]
    say("coulomb device")
    l = torch.tensor([c[0] for c in cases], dtype=torch.int32, device="cuda")
    eta = torch.tensor([c[1] for c in cases], dtype=torch.float64, device="cuda")
    rho = torch.tensor([c[2] for c in cases], dtype=torch.float64, device="cuda")
    out = torch.empty(len(cases) * 4, dtype=torch.float64, device="cuda")
    H.hp_coulomb_device(l, eta, rho, out)
    got = out.cpu().numpy().reshape(-1, 4)
    for k, (L, e, r) in enumerate(cases):
        ref = np.array(ormat.coulomb(L, e, r))
        assert np.max(np.abs(got[k] - ref) / np.abs(ref)) < 1e-12


def test_repeat_is_bitwise_deterministic(H, P):
    sp = make_system("small", nc=8, nr=45)
    d = P.DeviceSystem(sp)
    s = P.Solver(d, H.HP_C64)
    say("determinism")
    a = s.run(9.0)
    R1, S1 = a.R.cpu().numpy().copy(), a.S.cpu().numpy().copy()
    b = s.run(9.0)
    assert np.array_equal(R1, b.R.cpu().numpy()) and np.array_equal(S1, b.S.cpu().numpy())


# ------------------------------------------------------------- GEMM kernel --

@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (63, 65, 17), (130, 129, 33), (300, 256, 256),
                                   (2100, 700, 256), (129, 4000, 32), (65, 67, 8), (191, 193, 48)])
def test_gemm_sub_matches_numpy(H, prec, M, N, K):
    say("gemm", prec, M, N, K)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    ct = np.complex64 if prec == H.HP_C64 else np.complex128
    A = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))).astype(ct)
    B = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))).astype(ct)
    C = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))).astype(ct)
    ref = C.astype(np.complex128) - A.astype(np.complex128) @ B.astype(np.complex128)
    dA, dB, dC = (torch.from_numpy(x).to("cuda") for x in (A, B, C))
    H.hp_gemm_sub(M, N, K, prec, dA, K, dB, N, dC, N)
    got = dC.cpu().numpy().astype(np.complex128)
    scale = np.abs(C).max() + np.abs(A).max() * np.abs(B).max() * K
    tol = 1e-14 if prec == H.HP_C128 else 2e-6
    assert np.max(np.abs(got - ref)) / scale < tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("K", [37, 40])
def test_gemm_sub_offset_views(H, prec, K):
    """Sub-matrix views with odd leading dimensions and offsets (FP32: the
    scalar-load path; FP64 with K a multiple of 8: the direct-staged kernel)."""
    say("gemm views", prec, K)
    rng = np.random.default_rng(5)
    ct = np.complex64 if prec == H.HP_C64 else np.complex128
    big = (rng.standard_normal((301, 303)) + 1j * rng.standard_normal((301, 303))).astype(ct)
    d = torch.from_numpy(big).to("cuda")
    M, N = 150, 140
    A = big[1:1 + M, 3:3 + K]
    B = big[200:200 + K, 5:5 + N]
    C = big[151:151 + M, 150:150 + N].astype(np.complex128) - A.astype(np.complex128) @ B.astype(np.complex128)
    base = d.data_ptr()
    es = d.element_size()
    Ap = base + (1 * 303 + 3) * es
    Bp = base + (200 * 303 + 5) * es
    Cp = base + (151 * 303 + 150) * es
    code = H.lib().hp_gemm_sub(M, N, K, prec, Ap, 303, Bp, 303, Cp, 303, H._stream(None))
    assert code == 0
    got = d.cpu().numpy()[151:151 + M, 150:150 + N].astype(np.complex128)
    tol = 1e-13 if prec == H.HP_C128 else 1e-5
    assert np.max(np.abs(got - C)) / np.max(np.abs(C)) < tol
