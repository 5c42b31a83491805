"""hp_solve's FP32 refinement solves replayed from a captured HIP graph.

The graph is replayed once per refinement step, with the eager FP64 residual,
the norms and a host synchronization between the replays; every replay must
do exactly what the launches did one by one.  Checked on the final iterate:
X, R and S bit-identical to the eager run and the same number of steps (a
replay that went wrong would change the iterate, which the following steps
would only correct to rounding).  Systems with a ragged last 256-row block
and an odd channel count are included.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("config,override", [("mid", {}), ("small", {}), ("small", {"nc": 7, "nr": 97})])
def test_graph_replays_match_eager(mods, config, override):
    H, P = mods
    sp = make_system(config, **override)
    E = float(sp.energies[len(sp.energies) // 2])
    say("graph vs eager", config, override, "N", sp.nc * sp.nr, "E", E)
    d = P.DeviceSystem(sp)
    out = []
    prev = H.hp_set_solve_graphs(True)
    try:
        for on in (False, True, True):
            H.hp_set_solve_graphs(on)
            s = P.Solver(d, H.HP_C64, fallback=False)
            res = s.run(E)
            torch.cuda.synchronize()
            out.append((res.iterations, s.X.cpu().numpy().copy(), res.R.cpu().numpy().copy(),
                        res.S.cpu().numpy().copy()))
            del s
    finally:
        H.hp_set_solve_graphs(prev)
    it0, X0, R0, S0 = out[0]
    assert it0 >= 2
    for it, X, R, S in out[1:]:
        assert it == it0
        assert np.array_equal(X, X0)
        assert np.array_equal(R, R0)
        assert np.array_equal(S, S0)


def test_setting_is_validated(mods):
    H, _ = mods
    assert H.lib().hp_set_solve_graphs(2) == H.HP_ERR_ARG
    prev = H.hp_set_solve_graphs(False)
    assert H.hp_set_solve_graphs(prev) is False
