"""CPU tests of the served-stream scheduler (admission order, HBM budget,
overlap of slots, error capture, latency accounting) with a stand-in executor:
no device work is involved."""
from __future__ import annotations

import threading
import time
from types import SimpleNamespace

import numpy as np
import pytest

pytest.importorskip("torch")

from paper_2512_11590_amd import serve  # noqa: E402


def fake(nc, ne=2, fail=False):
    return SimpleNamespace(nc=nc, nr=10, energies=np.arange(ne, dtype=float) + 6.0, fail=fail)


class Recorder:
    def __init__(self, dt=0.03):
        self.dt = dt
        self.lock = threading.Lock()
        self.active = 0
        self.peak = 0
        self.order = []

    def __call__(self, req, params):
        with self.lock:
            self.active += 1
            self.peak = max(self.peak, self.active)
            self.order.append(req.rid)
        try:
            if params.fail:
                raise RuntimeError("planted failure")
            time.sleep(self.dt)
            for E in req.energies:
                req.S.append(np.eye(2) * E)
                req.R.append(np.eye(2))
                req.iterations.append(3)
                req.fallback.append(False)
        finally:
            with self.lock:
                self.active -= 1


def run(reqs, slots, budget, rec):
    srv = serve.Server(slots=slots, device="cpu", hbm_budget=budget, executor=rec,
                       bytes_of=lambda sp: sp.nc)
    return srv.run(reqs)


def test_slots_overlap_and_admit_in_arrival_order():
    rec = Recorder()
    reqs = [(0.001 * k, fake(10)) for k in range(8)]
    res = run(reqs, slots=3, budget=1000, rec=rec)
    assert all(r.error is None for r in res)
    assert rec.peak == 3
    assert rec.order[:3] == sorted(rec.order[:3]) and sorted(rec.order) == list(range(8))
    assert [r.admitted for r in res] == sorted(r.admitted for r in res)
    st = serve.summary(res)
    assert st["solves"] == 16 and st["failed"] == 0
    assert st["latency_p99_s"] >= st["latency_p50_s"] >= 0.03 - 1e-3


def test_budget_serializes_and_rejects_oversized():
    rec = Recorder(dt=0.02)
    reqs = [(0.0, fake(60)), (0.0, fake(60)), (0.0, fake(30)), (0.0, fake(500))]
    res = run(reqs, slots=3, budget=100, rec=rec)
    assert rec.peak == 2  # 60 + 60 does not fit 100, 60 + 30 does
    assert res[3].error is not None and "budget" in res[3].error and not res[3].S
    assert all(r.error is None for r in res[:3])
    # requests wait for memory rather than for a slot: the second 60 starts after the first ends
    assert res[1].admitted >= res[0].done - 1e-3


def test_failure_is_reported_and_the_stream_goes_on():
    rec = Recorder(dt=0.005)
    reqs = [(0.0, fake(5)), (0.0, fake(5, fail=True)), (0.01, fake(5))]
    res = run(reqs, slots=2, budget=100, rec=rec)
    assert res[1].error is not None and "planted" in res[1].error
    assert res[0].error is None and res[2].error is None
    st = serve.summary(res)
    assert st["failed"] == 1 and st["solves"] == 4


def test_arrivals_are_respected():
    rec = Recorder(dt=0.001)
    reqs = [(0.0, fake(5)), (0.15, fake(5))]
    res = run(reqs, slots=2, budget=100, rec=rec)
    assert res[1].admitted >= 0.15 - 1e-3
    assert res[1].latency < 0.1


# -- device-memory accounting of a request (host arithmetic only) -----------

def test_served_bytes_by_path():
    """A request's admitted bytes: one set of buffers per energy on the
    batched path (up to batched_max_n unknowns), one set on the
    single-system path; FP32 requests also hold the FP64 fallback's
    matrix; non-local requests take the single-system path at any size and
    hold their n x n kernel values too."""
    from paper_2512_11590_amd import hprmat as H
    from workload import make_system, with_perey_buck
    sp = make_system("small", nc=4, nr=40)
    n, ne = sp.nc * sp.nr, len(sp.energies)
    one = serve.request_bytes(sp.nc, sp.nr, H.HP_C64)
    assert not serve.is_nonlocal(sp)
    assert serve.served_bytes(sp, H.HP_C64, batched_max_n=n) == ne * one
    assert serve.served_bytes(sp, H.HP_C64, batched_max_n=n - 1) == one
    # FP32 factors: the FP32 matrix and the FP64 fallback's matrix at least
    assert one >= n * n * (8 + 16)
    assert serve.request_bytes(sp.nc, sp.nr, H.HP_C128) >= n * n * 16
    assert serve.request_bytes(sp.nc, sp.nr, H.HP_C128) < one
    nl = with_perey_buck(make_system("small", nc=4, nr=40))
    assert serve.is_nonlocal(nl)
    for bmax in (n, n - 1):
        assert serve.served_bytes(nl, H.HP_C64, batched_max_n=bmax) == one + n * n * 16
