"""GPU tests of the FP16 variant (HP_C64H): complex FP32 factors whose
trailing updates run on the FP16 matrix cores with split operands under row
and column scaling (Sec. 3.2 / 3.4 mixed precision, the optional FP16
variant).

* factorization of random matrices: no zero pivot, the partial-pivoting
  invariant, and the backward error |PA - LU| <= gamma |L||U| with the
  update's unit roundoff 2^-22 (the split-FP16 product) in place of 2^-24;
* row-scrambled matrices (pivots unique): the same pivot sequence as the
  oracle's elimination;
* the pipeline (assembly, factorization, FP64 refinement, R, S) against the
  oracle at sizes with several trailing updates: R and S within 1e-10, no
  fallback to FP64.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import ge, pipeline as opipe, system as osys  # noqa: E402
from tests.helpers import relerr  # noqa: E402
from workload import make_system  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat, pipeline
    hprmat.lib()
    return hprmat, pipeline


def rand_matrix(n, seed, diag=0.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + diag * np.eye(n)


def factor_h3(H, A):
    n = A.shape[0]
    dA = torch.from_numpy(A.astype(np.complex64)).to("cuda")
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = torch.empty(H.hp_workspace_bytes(n, 0, H.HP_C64H), dtype=torch.uint8, device="cuda")
    H.hp_factor(n, H.HP_C64H, dA, n, ipiv, perm, info, work)
    torch.cuda.synchronize()
    return dA.cpu().numpy().astype(np.complex128), ipiv.cpu().numpy(), perm.cpu().numpy(), int(info.item())


@pytest.mark.parametrize("n", [300, 600, 1025, 2100])
def test_lu_h3_backward_error(mods, n):
    H, P = mods
    say("lu fp16x3", n)
    A = rand_matrix(n, 300 + n)
    LU, ipiv, p, info = factor_h3(H, A)
    assert info == 0
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    A32 = A.astype(np.complex64).astype(np.complex128)
    nu = 4 * n * 2.0 ** -22
    bound = nu / (1 - nu) * (np.abs(L) @ np.abs(U))
    assert np.all(np.abs(L @ U - A32[p]) <= bound)

    def cabs1(z):
        return np.abs(z.real) + np.abs(z.imag)
    d = np.diag(U)
    below = np.tril(cabs1(np.tril(LU, -1) * d[None, :]), -1)
    assert np.all(below <= cabs1(d)[None, :] * (1 + 1e-5))


@pytest.mark.parametrize("n", [600, 1300])
def test_lu_h3_pivots_match_oracle(mods, n):
    H, P = mods
    say("lu fp16x3 scrambled", n)
    B = rand_matrix(n, 7 * n, diag=10.0 * np.sqrt(n))
    A = B[::-1].copy()
    _, _, ipiv_o = ge.solve(A, np.ones((n, 1), complex))
    LU, ipiv, p, info = factor_h3(H, A)
    assert info == 0
    assert np.array_equal(ipiv, ipiv_o)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    assert relerr(L @ U, A[p]) < 1e-5


@pytest.mark.parametrize("nc,nr", [(8, 60), (13, 47), (24, 50)])
def test_pipeline_h3_against_oracle(mods, nc, nr):
    H, P = mods
    sp = make_system("small", nc=nc, nr=nr, lmax=12)
    d = P.DeviceSystem(sp)
    s = P.Solver(d, H.HP_C64H)
    md = osys.MeshData(sp.nr, sp.a)
    for e in (0, 5, 9):
        E = float(sp.energies[e])
        say("pipeline fp16x3 N", sp.n, "E", E)
        res = s.run(E)
        o = opipe.solve_energy(sp, E, md)
        er = relerr(res.R.cpu().numpy(), o["R"])
        es = relerr(res.S.cpu().numpy(), o["S"])
        print(f"   R err {er:.2e}  S err {es:.2e}  refinement {res.iterations}  fallback {res.fallback}", flush=True)
        assert er < 1e-10 and es < 1e-10
        assert not res.fallback


@pytest.mark.parametrize("M,N,K", [(1, 1, 32), (64, 128, 32), (300, 260, 64), (1000, 777, 256), (129, 4000, 256)])
def test_gemm_h3_matches_fp64_product(mods, M, N, K):
    """The split-FP16 product against the FP64 product of the same FP32
    operands: |error| <= 2^-20 (|A||B|) elementwise, rows and columns of very
    different magnitudes (the power-of-two scaling keeps them in range)."""
    H, P = mods
    say("gemm h3", M, N, K)
    rng = np.random.default_rng(M + 7 * N + K)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    A *= 2.0 ** rng.integers(-30, 30, size=(M, 1))
    B *= 2.0 ** rng.integers(-30, 30, size=(1, N))
    C = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    A, B, C = (x.astype(np.complex64) for x in (A, B, C))
    ref = C.astype(np.complex128) - A.astype(np.complex128) @ B.astype(np.complex128)
    dA, dB, dC = (torch.from_numpy(x.copy()).to("cuda") for x in (A, B, C))
    work = torch.empty(8 * K * (M + N) + 4 * (M + N) + 1024, dtype=torch.uint8, device="cuda")
    H.hp_gemm_h3_sub(M, N, K, dA, K, dB, N, dC, N, work)
    got = dC.cpu().numpy().astype(np.complex128)
    mag = np.abs(A.astype(np.complex128)) @ np.abs(B.astype(np.complex128)) + np.abs(C)
    err = np.max(np.abs(got - ref) / mag)
    print(f"   max |err| / (|A||B| + |C|) = {err:.2e}", flush=True)
    assert err < 2.0 ** -20
