"""Batched uneven systems on the GPU (one workgroup per system).

* small systems of the batch family (N <= 600) against the oracle: R and S
  within 1e-10, FP64 and FP32 + refinement, for every panel width, in the
  persistent and the stepped form of the factorization;
* larger systems (N up to ~2500) against the single-system path of the
  library: S within 1e-10;
* refinement steps replayed from a captured graph give bit-identical X to
  the same steps launched one by one;
* every system reports convergence.
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


@pytest.mark.parametrize("form", ["persistent", "stepped"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("panel", [8, 16, 32])
def test_small_batch_against_oracle(mods, small, prec, panel, form):
    H, B, P = mods
    sps, refs = small
    say("batch vs oracle", "prec", prec, "panel", panel, form, [sp.nc * sp.nr for sp in sps])
    bt = B.Batch(sps, [sp.energies[0] for sp in sps], prec)
    for b in bt.buckets:
        bt.tuning[b.key] = B.BucketTuning(panel, 2 * bt.cus if form == "persistent" else 0, 0.0)
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
    H, B, P = mods
    sps = family(64, 1159203, 1500)[:6]
    say("graph vs eager", [sp.nc * sp.nr for sp in sps])
    xs = []
    for use_graph in (False, True, True):
        bk = B.Bucket(sps, [sp.energies[0] for sp in sps], list(range(len(sps))), H.HP_C64)
        bk.factor(16, 0 if use_graph else 512)
        steps = bk.solve(max_refine=30, use_graph=use_graph)
        torch.cuda.synchronize()
        xs.append((steps, bk.X.cpu().numpy().copy()))
    assert xs[0][0] == xs[1][0] == xs[2][0] and xs[0][0] >= 2
    assert np.array_equal(xs[0][1], xs[1][1]) and np.array_equal(xs[0][1], xs[2][1])
