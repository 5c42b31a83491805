"""GPU test of the energy scan with several solvers in flight: every energy's
R and S equal those of one solver running the energies one after another
(the factorizations are serialized on one device-wide stream and each slot
owns its buffers, so the arithmetic is the same), also when one energy's
refinement runs beside another's factorization."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workload import make_system  # noqa: E402


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat, pipeline
    hprmat.lib()
    return hprmat, pipeline


@pytest.mark.parametrize("prec", [1, 0])
def test_scan_equals_one_solver(mods, prec):
    H, P = mods
    sp = make_system("mid", nc=40)  # N = 2400: several outer blocks, look-ahead on
    d = P.DeviceSystem(sp)
    energies = [float(e) for e in sp.energies[:7]]
    print("[case] scan prec", prec, "N", sp.n, flush=True)
    one = P.Solver(d, prec)
    ref = []
    for E in energies:
        r = one.run(E)
        ref.append((r.R.cpu().numpy().copy(), r.S.cpu().numpy().copy(), r.fallback))
    scan = P.EnergyScan(d, prec, slots=3)
    got = scan.run(energies)
    assert H.hp_set_concurrency(1) == 1  # restored after the scan
    for (R, S, fb), g in zip(ref, got):
        assert g.fallback == fb
        assert np.max(np.abs(g.R.numpy() - R)) <= 1e-12 * np.max(np.abs(R))
        assert np.max(np.abs(g.S.numpy() - S)) <= 1e-12 * np.max(np.abs(S))


def test_scan_reraises_a_slot_error(mods, monkeypatch):
    """An error in one slot (planted on the host, no device work) stops the
    scan, is re-raised to the caller, and the concurrency setting is restored."""
    H, P = mods
    sp = make_system("small")
    d = P.DeviceSystem(sp)
    energies = [float(e) for e in sp.energies[:3]]
    scan = P.EnergyScan(d, H.HP_C64, slots=2)
    orig = P.Solver.run

    def planted(self, E, **kw):
        if E == energies[1]:
            raise RuntimeError("planted")
        return orig(self, E, **kw)

    monkeypatch.setattr(P.Solver, "run", planted)
    with pytest.raises(RuntimeError, match="planted"):
        scan.run(energies)
    assert H.hp_set_concurrency(1) == 1
