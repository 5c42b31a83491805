"""GPU parity of the Woodbury-kinetic form (the paper's Type 3 solver,
Sec. 3.3): S(E) = I + K_diag^-1 V assembled on the device against the
oracle's Schur matrix (the paper's radial-major order, permuted to the
library's channel-major order), and R and S of the whole solve, with FP64 or
FP32 factors of S and FP64 refinement on C(E)'s residual, against the
oracle's direct solve, up to N = 25600 against the stored oracle values."""
from __future__ import annotations

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe  # noqa: E402
from oracle import system as osys  # noqa: E402
from oracle import woodbury as owb  # noqa: E402
from tests.helpers import relerr  # noqa: E402
from workload import make_system  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat, pipeline
    hprmat.lib()
    return hprmat, pipeline


def radial_position(nc, nr):
    """Radial-major position of every channel-major index a*nr + i."""
    return np.array([i * nc + a for a in range(nc) for i in range(nr)])


@pytest.mark.parametrize("nc,nr", [(4, 40), (3, 17), (11, 9)])
@pytest.mark.parametrize("prec", [0, 1])
def test_build_schur_matches_oracle(mods, nc, nr, prec):
    H, P = mods
    sp = make_system("small", nc=nc, nr=nr)
    E = float(sp.energies[4])
    d = P.DeviceSystem(sp)
    n = d.n
    ld = n + 3
    ct = torch.complex64 if prec == H.HP_C64 else torch.complex128
    S = torch.full((n, ld), 7 + 7j, dtype=ct, device="cuda")
    say("schur build nc", nc, "nr", nr, "prec", prec)
    H.hp_build_schur(d.sys, E, prec, d.kinv, S, ld)
    Sd = S.cpu().numpy()
    assert np.all(Sd[:, n:] == 7 + 7j)  # padding untouched
    md = osys.MeshData(nr, sp.a)
    So, _ = owb.schur_system(sp, E, md)
    p = radial_position(nc, nr)
    # the oracle inverts K in FP64 (numpy), the library in binary128: the two
    # K^-1 differ by the oracle's inversion error, at most ~cond(K) u64
    tol64 = max(1e-14, 10 * np.linalg.cond(md.tl) * np.finfo(float).eps)
    err = relerr(Sd[:, :n], So[np.ix_(p, p)])
    print(f"   S(E) err {err:.2e} (tol {tol64:.1e})", flush=True)
    assert err < (tol64 if prec == H.HP_C128 else 1e-7)


@pytest.mark.parametrize("nc,nr", [(4, 40), (3, 17), (6, 70)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_schur_solve_matches_oracle(mods, nc, nr, prec):
    """R and S through the factors of S(E) with refinement on C(E)'s residual
    against the oracle's direct solve; the answer comes from these factors."""
    H, P = mods
    sp = make_system("small", nc=nc, nr=nr, lmax=8)
    s = P.Solver(P.DeviceSystem(sp), prec, schur=True)
    md = osys.MeshData(nr, sp.a)
    for e in (1, 8):
        E = float(sp.energies[e])
        say("schur solve nc", nc, "nr", nr, "prec", prec, "E", E)
        res = s.run(E)
        o = opipe.solve_energy(sp, E, md)
        er = relerr(res.R.cpu().numpy(), o["R"])
        es = relerr(res.S.cpu().numpy(), o["S"])
        print(f"   R err {er:.2e}  S err {es:.2e}  it {res.iterations}", flush=True)
        assert er < 1e-10 and es < 1e-10
        assert not res.fallback and res.iterations >= 1
        assert 0 <= res.backward_error < 1e-14


def test_unrefined_type3_solve(mods):
    """The paper's Type 3 as printed: FP32 factors of S, no refinement.
    R within the paper's single-precision level of the oracle; one
    refinement pass then lands at the FP64 level."""
    H, P = mods
    sp = make_system("mid", nc=20)
    E = float(sp.energies[5])
    o = opipe.solve_energy(sp, E)
    s = P.Solver(P.DeviceSystem(sp), H.HP_C64, schur=True, fallback=False)
    say("type 3 unrefined N", sp.n)
    r0 = relerr(s.run(E, max_refine=0).R.cpu().numpy(), o["R"])
    r1 = relerr(s.run(E).R.cpu().numpy(), o["R"])
    print(f"   R err unrefined {r0:.2e}  refined {r1:.2e}", flush=True)
    assert r0 < 1e-3 and r1 < 1e-10


def test_schur_full_size_against_oracle(mods):
    """N = 25600 (the large workload), FP32 factors of S + FP64 refinement:
    R and S against the stored oracle values at every stored energy, with
    the same bars as the direct path."""
    H, P = mods
    path = os.path.join(GOLD, "large_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("large_oracle.npz not generated")
    g = np.load(path)
    sp = make_system("large")
    s = P.Solver(P.DeviceSystem(sp), H.HP_C64, schur=True)
    for e in sorted(int(k[2:]) for k in g.files if k.startswith("S_")):
        E = float(g[f"E_{e}"])
        say("schur large N", sp.n, "E", E)
        res = s.run(E)
        er = relerr(res.R.cpu().numpy(), g[f"R_{e}"])
        es = relerr(res.S.cpu().numpy(), g[f"S_{e}"])
        rfloor = float(g[f"Rfloor_{e}"]) if f"Rfloor_{e}" in g.files else float("nan")
        tol_r = max(1e-10, 3 * rfloor) if rfloor == rfloor else 1e-10
        print(f"   R err {er:.2e} (tol {tol_r:.1e})  S err {es:.2e}  refinement {res.iterations}", flush=True)
        assert es < 1e-10 and er < tol_r
        assert not res.fallback
