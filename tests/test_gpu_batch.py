"""Batched uneven systems on the GPU (one workgroup per system).

* small systems of the batch family (N <= 600) against the oracle: R and S
  (batched collision-matrix kernel) within 1e-10, FP64 and FP32 +
  refinement, for every panel width, in the persistent form and the stepped
  form in one and two levels (outer blocks of 64 columns) of blocking;
* larger systems (N up to ~2500) against the single-system path of the
  library: S within 1e-10;
* refinement steps replayed from a captured graph give bit-identical X to
  the same steps launched one by one; whole buckets replayed from a graph
  give bit-identical R and S to the eager run, replay after replay;
* every system reports convergence; forced non-convergence sends every
  system to the FP64 single-system path, whose R and S match the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe, system as osys  # noqa: E402
from tests.helpers import relerr  # noqa: E402
from workload import batch_systems  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import batch, hprmat, pipeline
    hprmat.lib()
    return hprmat, batch, pipeline


def family(count, seed, nmax):
    out = [sp for sp in batch_systems(count, seed=seed) if sp.nc * sp.nr <= nmax]
    return out


@pytest.fixture(scope="module")
def small():
    sps = family(96, 1159201, 600)[:8]
    refs = []
    for sp in sps:
        md = osys.MeshData(sp.nr, sp.a)
        refs.append(opipe.solve_energy(sp, float(sp.energies[0]), md))
    return sps, refs


@pytest.mark.parametrize("form", ["persistent", "stepped", "stepped-blocked"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("panel", [8, 16, 32])
def test_small_batch_against_oracle(mods, small, prec, panel, form):
    """Persistent form; stepped form in one level (outer block = panel) and
    in two levels (outer blocks of 64 columns, ragged last block)."""
    H, B, P = mods
    sps, refs = small
    say("batch vs oracle", "prec", prec, "panel", panel, form, [sp.nc * sp.nr for sp in sps])
    bt = B.Batch(sps, [sp.energies[0] for sp in sps], prec)
    for b in bt.buckets:
        bt.tuning[b.key] = B.BucketTuning(panel, 2 * bt.cus if form == "persistent" else 0, 0.0,
                                          64 if form == "stepped-blocked" else panel)
    bt.run()
    st, it = bt.status()
    assert np.all(st == 1), (st, it)
    for (R, S), o in zip(bt.results(), refs):
        assert relerr(R, o["R"]) < 1e-10
        assert relerr(S, o["S"]) < 1e-10


def test_larger_systems_match_single_path(mods):
    H, B, P = mods
    sps = [sp for sp in batch_systems(64, seed=1159202) if 1200 <= sp.nc * sp.nr <= 2600][:4]
    say("batch vs single path", [sp.nc * sp.nr for sp in sps])
    bt = B.Batch(sps, [sp.energies[0] for sp in sps], H.HP_C64)
    bt.tune()
    bt.run()
    st, _ = bt.status()
    assert np.all(st == 1)
    for (R, S), sp in zip(bt.results(), sps):
        d = P.DeviceSystem(sp)
        s = P.Solver(d, H.HP_C128)
        res = s.run(float(sp.energies[0]))
        assert relerr(S, res.S.cpu().numpy()) < 1e-10


def test_graph_replay_matches_eager(mods):
    """Refinement steps replayed from a captured step give bit for bit the X
    of the same steps launched one by one (same factors, same solve form);
    the persistent and the stepped factorization forms agree to rounding."""
    H, B, P = mods
    sps = family(64, 1159203, 1500)[:6]
    say("graph vs eager", [sp.nc * sp.nr for sp in sps])
    xs = []
    for groups, use_graph in ((0, False), (0, True), (0, True), (512, False)):
        bk = B.Bucket(sps, [sp.energies[0] for sp in sps], list(range(len(sps))), H.HP_C64)
        bk.factor(16, groups, 16)
        steps = bk.solve(max_refine=30, use_graph=use_graph)
        torch.cuda.synchronize()
        xs.append((steps, bk.X.cpu().numpy().copy()))
    assert xs[0][0] == xs[1][0] == xs[2][0] and xs[0][0] >= 2
    assert np.array_equal(xs[0][1], xs[1][1]) and np.array_equal(xs[0][1], xs[2][1])
    assert relerr(xs[3][1], xs[0][1]) < 1e-12


def test_whole_bucket_graph_matches_eager(mods):
    """A bucket replayed from its captured graph (build, factor, solves,
    refinement steps, R, S) gives bit for bit the eager run's R and S, on
    several replays with eager work and synchronisations between them."""
    H, B, P = mods
    sps = family(64, 1159204, 2600)[:6]
    say("whole-bucket graph vs eager", [sp.nc * sp.nr for sp in sps])
    for prec in (H.HP_C64, H.HP_C128):
        bt = B.Batch(sps, [sp.energies[0] for sp in sps], prec, edges=())
        for b in bt.buckets:
            bt.tuning[b.key] = B.BucketTuning(16, 0, 0.0, 64)
        bt.run(use_graph=False)
        ref = [(R.copy(), S.copy()) for R, S in bt.results()]
        bt.run(use_graph=True)  # eager, then captured
        assert all(b.whole is not None for b in bt.buckets)
        for rep in range(3):
            bt.run(use_graph=True)  # replay
            torch.cuda.synchronize()
            got = bt.results()
            for (R0, S0), (R1, S1) in zip(ref, got):
                assert np.array_equal(R0, R1) and np.array_equal(S0, S1), (prec, rep)
            x = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
            assert x == x


def test_batched_fallback_to_fp64(mods, small):
    """Forced non-convergence (one refinement step, unreachable tolerance):
    every system reports status 2 and is solved again in FP64; R and S match
    the oracle.  With fallback disabled, results() raises."""
    H, B, P = mods
    sps, refs = small
    sps, refs = sps[:3], refs[:3]
    say("batched fallback", [sp.nc * sp.nr for sp in sps])
    bt = B.Batch(sps, [sp.energies[0] for sp in sps], H.HP_C64)
    for b in bt.buckets:
        bt.tuning[b.key] = B.BucketTuning(16, 0, 0.0, 64)
    bt.run(max_refine=1, tol=1e-300, use_graph=False)
    st, _ = bt.status()
    assert np.all(st == 2), st
    with pytest.raises(H.HprmatError):
        bt.results(fallback=False)
    out = bt.results()
    assert sorted(bt.fallbacks) == list(range(len(sps)))
    for (R, S), o in zip(out, refs):
        assert relerr(R, o["R"]) < 1e-10
        assert relerr(S, o["S"]) < 1e-10


def test_register_panel_matches_memory_panel(mods):
    """The FP32 stepped factorization with its 8-column panels held in
    registers (one 1024-thread workgroup per system; 1, 2 and 4 rows per
    thread) against the panels worked through memory: the same pivots, the
    factors equal up to FP32 rounding (the two kernels may contract the
    same products into fused multiply-adds differently), and R after
    refinement within 1e-10 of each other and of the oracle."""
    H, B, P = mods
    pool = batch_systems(200, seed=1159203)
    pick = []
    for lo, hi in ((300, 1000), (1100, 2000), (3000, 4000)):
        pick.append(next(sp for sp in pool if lo <= sp.nc * sp.nr <= hi))
    say("register panel N", [sp.nc * sp.nr for sp in pick])
    out = {}
    for on in (True, False):
        prev = H.hp_set_batch_reg_panel(on)
        try:
            bk = B.Bucket(pick, [float(sp.energies[0]) for sp in pick], list(range(3)), H.HP_C64)
            bk.factor(8, 0, 64)
            torch.cuda.synchronize()
            A = bk.A.cpu().numpy()
            facs = [A[int(bk.a_off[k]):int(bk.a_off[k]) + int(bk.n[k]) ** 2] for k in range(3)]
            piv = bk.ipiv.cpu().numpy()
            info = bk.info.cpu().numpy()
            bk.solve(30)
            bk.rmatrix()
            out[on] = (facs, piv, info, [bk.R_of(k) for k in range(3)], list(bk.index))
        finally:
            H.hp_set_batch_reg_panel(prev)
    reg, mem = out[True], out[False]
    assert np.array_equal(reg[1], mem[1]) and not reg[2].any() and not mem[2].any()
    for k in range(3):
        e = relerr(reg[0][k], mem[0][k])
        print(f"   system {k}: factors {e:.1e}  R {relerr(reg[3][k], mem[3][k]):.1e}", flush=True)
        assert e < 1e-4
        assert relerr(reg[3][k], mem[3][k]) < 1e-10
    k = reg[4].index(0)
    o = opipe.solve_energy(pick[0], float(pick[0].energies[0]))
    assert relerr(reg[3][k], o["R"]) < 1e-10
