"""GPU parity for non-local potentials (Sec. 2: the coupling blocks become
full matrices): the assembled C(E) with the quadrature-weighted kernel
values, and R and S from FP64 LU, FP32 LU + FP64 refinement (whose residual
then carries one FP64 product with the n x n kernel) and the split-FP16
variant, against the oracle; a separable kernel against its closed-form K
matrix, up to N = 25600 (256 s-wave channels, 100 points each)."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe  # noqa: E402
from oracle import system as osys  # noqa: E402
from tests.helpers import CustomSystem, relerr, separable_kmatrix, separable_nonlocal  # noqa: E402
from workload import make_system, with_perey_buck  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat, pipeline
    hprmat.lib()
    return hprmat, pipeline


def gaussian_nonlocal(nc: int, seed: int, strength: float = 20.0, width: float = 0.85):
    """A non-symmetric complex kernel of Gaussian non-locality:
    W_cc'(r, r') = s A_cc' exp(-((r - r')/width)^2) exp(-(r + r')/8)
    plus a small dense random part (fixed by the seed and the mesh size)."""
    g = np.random.default_rng(seed)
    A = g.normal(size=(nc, nc)) + 1j * g.normal(size=(nc, nc))
    A[np.diag_indices(nc)] = -np.abs(A[np.diag_indices(nc)]) * (1.0 + 0.3j) - 1.0

    def nl(r):
        d = r[:, None] - r[None, :]
        f = np.exp(-(d / width) ** 2) * np.exp(-(r[:, None] + r[None, :]) / 8.0)
        W = strength * A[:, None, :, None] * f[None, :, None, :]
        z = np.random.default_rng(seed + len(r))
        W = W + 0.05 * (z.normal(size=W.shape) + 1j * z.normal(size=W.shape))
        return W.astype(np.complex128)
    return nl


def with_nonlocal(sp, nl):
    sp.nonlocal_potential = nl
    return sp


@pytest.mark.parametrize("prec", [0, 1])
def test_build_matrix_nonlocal_matches_oracle(mods, prec):
    H, P = mods
    sp = with_nonlocal(make_system("small", nc=5, nr=37), gaussian_nonlocal(5, 3))
    E = float(sp.energies[3])
    d = P.DeviceSystem(sp)
    assert d.vnl is not None
    n = d.n
    ld = n + 5
    ct = torch.complex64 if prec == H.HP_C64 else torch.complex128
    C = torch.full((n, ld), 7 + 7j, dtype=ct, device="cuda")
    say("non-local assembly, prec", prec)
    H.hp_build_matrix(d.sys, E, prec, C, ld)
    Cd = C.cpu().numpy()
    assert np.all(Cd[:, n:] == 7 + 7j)  # padding untouched
    Mo, _ = osys.assemble(sp, E)
    assert relerr(Cd[:, :n], Mo) < (1e-14 if prec == H.HP_C128 else 1e-7)


def test_zero_kernel_builds_the_local_matrix(mods):
    """An all-zero kernel leaves C(E) bitwise equal to the local assembly."""
    H, P = mods
    sp = make_system("small", nc=4, nr=30)
    E = float(sp.energies[1])
    dl = P.DeviceSystem(sp)
    dz = P.DeviceSystem(sp, vnl=torch.zeros((dl.n, dl.n), dtype=torch.complex128, device="cuda"))
    Cl = torch.empty((dl.n, dl.n), dtype=torch.complex128, device="cuda")
    Cz = torch.empty_like(Cl)
    say("zero kernel")
    H.hp_build_matrix(dl.sys, E, H.HP_C128, Cl, dl.n)
    H.hp_build_matrix(dz.sys, E, H.HP_C128, Cz, dz.n)
    assert torch.equal(Cl, Cz)


@pytest.mark.parametrize("nc,nr", [(3, 20), (5, 37), (6, 70)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_nonlocal_pipeline_matches_oracle(mods, nc, nr, prec):
    """Local coupled potential (Coulomb, l up to 6) plus a non-symmetric
    complex non-local kernel; R and S against the oracle's Gaussian
    elimination, with every precision's result from its own factors."""
    H, P = mods
    sp = with_nonlocal(make_system("small", nc=nc, nr=nr, lmax=6), gaussian_nonlocal(nc, 17 + nc))
    s = P.Solver(P.DeviceSystem(sp), prec)
    md = osys.MeshData(nr, sp.a)
    for e in (0, 6):
        E = float(sp.energies[e])
        say("non-local pipeline nc", nc, "nr", nr, "prec", prec, "E", E)
        res = s.run(E)
        o = opipe.solve_energy(sp, E, md)
        er = relerr(res.R.cpu().numpy(), o["R"])
        es = relerr(res.S.cpu().numpy(), o["S"])
        print(f"   R err {er:.2e}  S err {es:.2e}  it {res.iterations} fb {res.fallback}", flush=True)
        assert er < 1e-10 and es < 1e-10
        assert not res.fallback
        if prec != H.HP_C128:
            assert res.iterations >= 1 and 0 <= res.backward_error < 1e-14


@pytest.mark.parametrize("prec", [0, 1])
def test_perey_buck_system_matches_oracle(mods, prec):
    """N = 2400 (40 channels of the mid family, Coulomb, l up to 20) with the
    Perey-Buck-form kernel coupled across channels: R and S against the
    oracle.  (The family's all-pairs couplings make the potential neither
    absorptive nor flux-conserving, so no unitarity bound applies.)"""
    H, P = mods
    sp = with_perey_buck(make_system("mid", nc=40))
    md = osys.MeshData(sp.nr, sp.a)
    E = float(sp.energies[2 if prec == 0 else 15])
    say("Perey-Buck N", sp.n, "prec", prec, "E", E)
    res = P.Solver(P.DeviceSystem(sp), prec).run(E)
    o = opipe.solve_energy(sp, E, md)
    S = res.S.cpu().numpy()
    assert relerr(res.R.cpu().numpy(), o["R"]) < 1e-10 and relerr(S, o["S"]) < 1e-10
    assert not res.fallback


_NL_H = 20.736


@pytest.mark.parametrize("prec", [0, 1])
def test_separable_kernel_closed_form_on_device(mods, prec):
    """Three s-wave channels coupled only by a rank-one separable kernel:
    S = (1 + iK)(1 - iK)^-1 with the closed-form K."""
    H, P = mods
    lam, beta, eps = 60.0, np.array([1.4, 0.9, 1.8]), np.array([0.0, 2.5, 6.0])
    sp = CustomSystem(nc=3, nr=80, a=30.0, l=np.zeros(3, dtype=int), eps=eps,
                      pot=lambda r: np.zeros((len(r), 3, 3), dtype=complex), hbar2_2mu=_NL_H,
                      nlpot=separable_nonlocal(lam, beta))
    s = P.Solver(P.DeviceSystem(sp), prec)
    for E in (7.0, 15.0, 40.0):
        say("separable closed form, prec", prec, "E", E)
        S = s.run(E).S.cpu().numpy()
        K = separable_kmatrix(lam, beta, np.sqrt((E - eps) / _NL_H), _NL_H)
        Sa = (np.eye(3) + 1j * K) @ np.linalg.inv(np.eye(3) - 1j * K)
        assert np.max(np.abs(S - Sa)) < 5e-11


@pytest.mark.parametrize("form", ["persistent", "stepped"])
@pytest.mark.parametrize("prec", [0, 1])
def test_batched_nonlocal_systems_against_oracle(mods, prec, form):
    """A bucket mixing local systems and systems with non-local kernels
    (Gaussian non-locality, Perey-Buck form): the batched assembly takes the
    kernel, the batched FP32 refinement its product; R and S of every system
    against the oracle."""
    H, P = mods
    from paper_2512_11590_amd import batch as B
    sps = [make_system("small", nc=nc, nr=nr, seed=sd) for nc, nr, sd in ((4, 30, 5), (3, 41, 6), (6, 25, 7),
                                                                         (5, 36, 8))]
    with_nonlocal(sps[0], gaussian_nonlocal(4, 31))
    with_perey_buck(sps[2])
    with_nonlocal(sps[3], gaussian_nonlocal(5, 33))
    energies = [float(s.energies[2 + k]) for k, s in enumerate(sps)]
    bt = B.Batch(sps, energies, prec)
    for b in bt.buckets:
        bt.tuning[b.key] = B.BucketTuning(8, 2 * bt.cus if form == "persistent" else 0, 0.0, 8)
    say("batched non-local, prec", prec, form)
    bt.run()
    st, it = bt.status()
    assert np.all(st == 1), (st, it)
    for k, (R, S) in enumerate(bt.results(fallback=False)):
        o = opipe.solve_energy(sps[k], energies[k])
        er, es = relerr(R, o["R"]), relerr(S, o["S"])
        print(f"   system {k} R err {er:.2e}  S err {es:.2e}  corrections {it[k]}", flush=True)
        assert er < 1e-10 and es < 1e-10


def test_full_size_separable_kernel(mods):
    """N = 25600: 256 s-wave channels (thresholds 0-10 MeV, all open at
    20 MeV, 100 points on a = 30 fm) coupled by a separable kernel with a
    range per channel, FP32 LU + FP64 refinement: every element of the
    256 x 256 S against the closed form (a property at any size)."""
    H, P = mods
    nc, nr, a, E, lam = 256, 100, 30.0, 20.0, 0.8
    g = np.random.default_rng(2512)
    eps = np.sort(g.uniform(0.0, 10.0, size=nc))
    beta = g.uniform(0.9, 1.8, size=nc)
    sp = CustomSystem(nc=nc, nr=nr, a=a, l=np.zeros(nc, dtype=int), eps=eps,
                      pot=lambda r: np.zeros((len(r), nc, nc), dtype=complex), hbar2_2mu=_NL_H)
    r = H.hp_mesh(nr, a)[0]
    gv = torch.from_numpy(np.exp(-beta[:, None] * r[None, :]).ravel()).to("cuda")  # g_c(r_i), channel-major
    W = (-lam) * torch.outer(gv, gv).to(torch.complex128)
    say("full-size separable kernel N", nc * nr)
    d = P.DeviceSystem(sp, vnl=W)
    res = P.Solver(d, H.HP_C64).run(E)
    assert not res.fallback and res.nopen == nc
    K = separable_kmatrix(lam, beta, np.sqrt((E - eps) / _NL_H), _NL_H)
    Sa = np.linalg.solve((np.eye(nc) - 1j * K).T, (np.eye(nc) + 1j * K).T).T
    err = np.max(np.abs(res.S.cpu().numpy() - Sa))
    print(f"   max |S - S_closed| {err:.2e}  it {res.iterations}", flush=True)
    # rank-one K: one eigenphase (about 74 degrees here) carries the coupling
    assert np.linalg.norm(Sa - np.eye(nc), 2) > 1.0
    assert err < 1e-9
