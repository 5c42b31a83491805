"""Served stream (continuous batching) on the GPU.

* every request's S in the mix equals its S when it runs alone, within the
  S tolerance 1e-10 (the kernels are deterministic, so in practice bit for
  bit); the mix holds requests of both paths (the batched path up to 4000
  unknowns, the single-system path above);
* FP32 + refinement and FP64 agree on S within 1e-10 per request;
* a small request (N = 160, the small workload) served in the mix matches the
  oracle within 1e-10;
* admission respects the HBM budget: a budget that fits one request at a time
  serializes the stream, and a request larger than the budget is reported,
  not run.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe, system as osys  # noqa: E402
from tests.helpers import relerr  # noqa: E402
from workload import make_system, served_requests  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2512_11590_amd import hprmat, serve
    hprmat.lib()
    return hprmat, serve


def small_stream(count=8, rate=200.0, seed=1159105, nmax=2500):
    """Requests of the served family, kept small (N <= nmax) so the test runs in seconds."""
    reqs = []
    for t, sp in served_requests(4 * count, rate, seed=seed):
        if sp.nc * sp.nr <= nmax:
            sp.energies = sp.energies[:2]
            reqs.append((t, sp))
        if len(reqs) == count:
            break
    return reqs


def test_same_alone_and_in_mix(mods):
    H, S = mods
    reqs = small_stream()
    small = make_system("small")
    small.energies = small.energies[:2]
    reqs.insert(3, (reqs[3][0], small))
    # one request above the batched-path size, so both paths run in the mix
    big = make_system("small", nc=48, nr=100, lmax=12)
    big.energies = big.energies[:2]
    reqs.insert(1, (reqs[1][0], big))
    say("mix", [sp.nc * sp.nr for _, sp in reqs])
    mix = S.Server(slots=3, prec=H.HP_C64).run(reqs)
    assert all(r.error is None for r in mix), [r.error for r in mix]
    alone = S.Server(slots=1, prec=H.HP_C64).run([(0.0, sp) for _, sp in reqs])
    for a, b in zip(mix, alone):
        for sa, sb in zip(a.S, b.S):
            assert relerr(sa, sb) < 1e-10
    # the small workload against the oracle
    md = osys.MeshData(small.nr, small.a)
    for e, E in enumerate(small.energies):
        o = opipe.solve_energy(small, float(E), md)
        assert relerr(mix[4].S[e], o["S"]) < 1e-10
    st = S.summary(mix)
    say("summary", st)
    assert st["failed"] == 0 and st["latency_p99_s"] >= st["latency_p50_s"] > 0


def test_fp32_refined_matches_fp64_per_request(mods):
    H, S = mods
    reqs = small_stream(count=4, seed=1159106)
    r32 = S.Server(slots=2, prec=H.HP_C64).run(reqs)
    r64 = S.Server(slots=2, prec=H.HP_C128).run(reqs)
    for a, b in zip(r32, r64):
        assert a.error is None and b.error is None
        for sa, sb in zip(a.S, b.S):
            assert relerr(sa, sb) < 1e-10


def test_admission_by_memory(mods):
    H, S = mods
    t0, sp = small_stream(count=1, seed=1159107)[0]
    reqs = [(t0 + 0.001 * k, sp) for k in range(4)]  # four requests of one size
    need = S.served_bytes(sp, H.HP_C64, 4000)
    res = S.Server(slots=3, prec=H.HP_C64, hbm_budget=need).run(reqs)
    assert all(r.error is None for r in res)
    spans = sorted((r.admitted, r.done) for r in res)
    for (a0, d0), (a1, _) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-3  # one request on the device at a time
    big = S.Server(slots=2, prec=H.HP_C64, hbm_budget=need // 8).run(reqs[:1])
    assert big[0].error is not None and not big[0].S


def test_nonlocal_request_takes_the_single_system_path(mods):
    """A small non-local request (below the batched-path size) is served by
    the single-system solver, which takes the kernel: its S equals the
    oracle's, beside local requests in the same stream."""
    H, S = mods
    from workload import with_perey_buck
    nl = with_perey_buck(make_system("small"))
    nl.energies = nl.energies[:2]
    reqs = small_stream(count=3, seed=1159108)
    reqs.insert(1, (reqs[1][0], nl))
    say("non-local request in the mix")
    res = S.Server(slots=2, prec=H.HP_C64).run(reqs)
    assert all(r.error is None for r in res), [r.error for r in res]
    md = osys.MeshData(nl.nr, nl.a)
    for e, E in enumerate(nl.energies):
        o = opipe.solve_energy(nl, float(E), md)
        assert relerr(res[1].S[e], o["S"]) < 1e-10
