"""GPU parity of the collision matrix with closed channels (E below some
thresholds): the device log-derivatives of the decaying external solutions
(inward Taylor integration of the closed-channel equation) and the
elimination through the open channels' effective R-matrix, against the
oracle (whose Whittaker values come from mpmath and whose matching is pinned
to a directly matched coupled well on the CPU).  S over the open channels is
compared normwise; its closed rows and columns must be exactly zero."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe  # noqa: E402
from tests.helpers import CustomSystem, relerr  # noqa: E402
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


def _check_S(S: np.ndarray, o: dict, tol: float) -> None:
    op = np.asarray(o["open"])
    closed = np.setdiff1d(np.arange(S.shape[0]), op)
    assert relerr(S[np.ix_(op, op)], o["S"]) < tol
    assert not np.any(S[closed, :]) and not np.any(S[:, closed])


# Thresholds and energies with every channel at least 0.5 MeV from threshold:
# open channels right above threshold under a Coulomb barrier have
# sub-barrier Coulomb functions beyond double range (F ~ exp(-pi eta)), which
# no unscaled matching survives, open or closed.
CASES = [(np.array([0.0, 0.5, 1.0, 6.0, 7.0, 8.0]), 3.0, 3),
         (np.array([0.0, 3.0, 5.0, 5.5, 6.0, 9.0]), 4.0, 2),
         (np.array([0.0, 6.0, 6.5, 7.0, 8.0, 9.0]), 2.0, 1)]


def _small(eps):
    sp = make_system("small", nc=6, nr=50)
    sp.eps = eps.copy()
    return sp


@pytest.mark.parametrize("case", range(len(CASES)))
def test_smatrix_closed_from_oracle_R(mods, case):
    """hp_smatrix alone on the oracle's R: 6 channels with Coulomb and l up to
    4, some of them closed."""
    H, P = mods
    eps, E, k = CASES[case]
    sp = _small(eps)
    o = opipe.solve_energy(sp, E)
    assert len(o["open"]) == k
    d = P.DeviceSystem(sp)
    R = torch.from_numpy(o["R"]).to("cuda")
    S = torch.empty_like(R)
    work = torch.empty(H.hp_workspace_bytes(sp.nc, sp.nc, H.HP_C128), dtype=torch.uint8, device="cuda")
    say("smatrix closed, open", k)
    nopen = H.hp_smatrix(d.sys, E, R, S, work)
    assert nopen == k
    _check_S(S.cpu().numpy(), o, 1e-12)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_well_with_closed_channel(mods, prec):
    """The three-channel constant-coupling well with one closed channel (the
    oracle's U there equals the direct matching at r = a)."""
    H, P = mods
    a, h, E = 7.0, 2.0, 4.0
    W = np.array([[-25.0, 4.0, -2.5], [4.0, -18.0, 3.0], [-2.5, 3.0, -31.0]])
    sp = CustomSystem(nc=3, nr=45, a=a, l=np.zeros(3, int), eps=np.array([0.0, 1.0, 6.0]), hbar2_2mu=h,
                      pot=lambda r: np.broadcast_to(W.astype(complex), (len(r), 3, 3)).copy())
    o = opipe.solve_energy(sp, E)
    say("well with a closed channel, prec", prec)
    res = P.Solver(P.DeviceSystem(sp), prec).run(E)
    assert res.nopen == 2
    _check_S(res.S.cpu().numpy(), o, 1e-10)


@pytest.mark.parametrize("prec", [0, 1])
def test_closed_channels_end_to_end(mods, prec):
    """N = 2400 (40 channels, Coulomb, l up to 20) at 4 MeV with 12 channels
    closed (thresholds 6-11 MeV) and 28 open (thresholds 0-2 MeV): FP64 LU
    and FP32 LU + FP64 refinement."""
    H, P = mods
    sp = make_system("mid", nc=40)
    e = np.asarray(sp.eps, dtype=np.float64)
    sp.eps = np.where(np.arange(40) < 28, 0.4 * e, 6.0 + e)
    E = 4.0
    o = opipe.solve_energy(sp, E)
    assert len(o["open"]) == 28
    say("end to end N", sp.n, "open", len(o["open"]), "prec", prec)
    res = P.Solver(P.DeviceSystem(sp), prec).run(E)
    assert res.nopen == 28 and not res.fallback
    _check_S(res.S.cpu().numpy(), o, 1e-10)


def test_noalloc_form_with_closed_channels(mods):
    """hp_smatrix_noalloc takes the same path: same S as hp_smatrix."""
    H, P = mods
    eps, E, k = CASES[0]
    sp = _small(eps)
    o = opipe.solve_energy(sp, E)
    d = P.DeviceSystem(sp)
    R = torch.from_numpy(o["R"]).to("cuda")
    S1 = torch.empty_like(R)
    S2 = torch.empty_like(R)
    work = torch.empty(H.hp_workspace_bytes(sp.nc, sp.nc, H.HP_C128), dtype=torch.uint8, device="cuda")
    say("noalloc closed")
    n1 = H.hp_smatrix(d.sys, E, R, S1, work)
    n2 = H.hp_smatrix_noalloc(d.sys, E, R, S2)
    assert n1 == n2 == k
    assert torch.equal(S1, S2)


def test_threshold_and_no_open_channel_are_reported(mods):
    """An energy exactly at a threshold, or below every threshold, has no
    collision matrix: HP_ERR_UNSUPPORTED."""
    H, P = mods
    sp = make_system("small")
    d = P.DeviceSystem(sp)
    s = P.Solver(d, H.HP_C128)
    for E in (float(np.sort(sp.eps)[1]), float(np.min(sp.eps)) - 0.5):
        say("unsupported E", E)
        with pytest.raises(H.HprmatError) as ei:
            s.run(E)
        assert ei.value.code == H.HP_ERR_UNSUPPORTED


def test_full_size_with_closed_channels(mods):
    """N = 25600 (256 channels) at 16.25 MeV with the thresholds of every
    eighth channel raised to 22-27 MeV (32 closed): FP32 LU + FP64
    refinement end to end; the matching step at full size against the
    oracle's on the same R (its elimination and its Coulomb and Whittaker
    values for all 256 channels)."""
    H, P = mods
    from oracle import rmatrix as ormat
    sp = make_system("large")
    e = np.asarray(sp.eps, dtype=np.float64)
    sp.eps = np.where(np.arange(sp.nc) % 8 != 7, e, 22.0 + e)
    E = 16.25
    say("full size closed N", sp.n)
    res = P.Solver(P.DeviceSystem(sp), H.HP_C64).run(E)
    assert res.nopen == sp.nc - sp.nc // 8 and not res.fallback
    R = res.R.cpu().numpy()
    U, op, _ = ormat.smatrix_closed(R, E, sp.eps, np.asarray(sp.l), sp.hbar2_2mu, sp.z1z2, sp.a)
    _check_S(res.S.cpu().numpy(), {"open": op, "S": U}, 1e-12)


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_matching_with_closed_channels(mods, prec):
    """hp_batch_smatrix with closed channels: systems of the batch family
    (N <= 800) at 8 MeV with every second, third or no threshold raised above
    E, one with every channel closed (status 1); S over the open channels
    against the oracle, zero in the closed rows and columns."""
    H, P = mods
    from paper_2512_11590_amd import batch as B
    from workload import batch_systems
    E = 8.0
    sps = [sp for sp in batch_systems(200, seed=1159301) if sp.nc * sp.nr <= 800][:5]
    for k, sp in enumerate(sps):
        e = np.asarray(sp.eps, dtype=np.float64)
        step = (0, 2, 3, 2, 1)[k]
        if step:
            sp.eps = np.where(np.arange(sp.nc) % step == step - 1, E + 1.5 + e, e)
    assert np.all(sps[4].eps > E) and np.all(sps[0].eps < E - 0.5)
    bk = B.Bucket(sps, [E] * len(sps), list(range(len(sps))), prec)
    bk.factor(8, 0, 8)
    bk.solve(30)
    bk.rmatrix()
    bk.smatrix()
    st, _ = bk.status()
    sst = bk.sstat.cpu().numpy()
    say("batched closed, prec", prec, "open", [int(np.sum(sp.eps < E)) for sp in bk.systems])
    for k, sp in enumerate(bk.systems):
        if np.all(sp.eps > E):
            assert sst[k] == 1
            continue
        assert st[k] == 1 and sst[k] == 0
        o = opipe.solve_energy(sp, E)
        _check_S(bk.S_of(k), o, 1e-10)


def _deep_system(coupled: bool, closed: bool = False):
    """Three channels at 12 MeV, Z1Z2 = 40, the third 5 keV above its
    threshold (eta ~ 290: F ~ 1e-310, G ~ 1e+307), optionally a fourth,
    closed one."""
    nc = 4 if closed else 3
    Wt = np.full((nc, nc), 2.5)
    Wt[np.diag_indices(nc)] = [-30.0, -22.0, -27.0, -25.0][:nc]
    if not coupled:
        Wt[2, :] = Wt[:, 2] = 0.0
        Wt[2, 2] = -27.0

    def pot(r):
        f = 1.0 / (1.0 + np.exp((r - 5.0) / 0.6))
        v = (Wt[None, :, :] * f[:, None, None]).astype(complex)
        v[:, range(nc), range(nc)] += -4j * f[:, None]
        return v
    E = 12.0
    eps = [0.0, 1.5, E - 0.005, 14.0][:nc]
    return CustomSystem(nc=nc, nr=40, a=15.0, l=np.array([0, 1, 2, 1][:nc]), eps=np.array(eps), hbar2_2mu=2.0,
                        pot=pot, z1z2=40), E


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("coupled", [True, False])
def test_open_channel_far_below_its_coulomb_barrier(mods, prec, coupled):
    """An open channel whose F and G leave double range: the device carries
    them scaled by e^-+theta and matches with U = I - 2i E^-1 ZO~^-1 Q E^-1;
    S against the oracle's mpmath matching."""
    H, P = mods
    sp, E = _deep_system(coupled)
    o = opipe.solve_energy(sp, E)
    say("deep sub-barrier channel, coupled", coupled, "prec", prec)
    res = P.Solver(P.DeviceSystem(sp), prec).run(E)
    S = res.S.cpu().numpy()
    assert res.nopen == 3 and np.all(np.isfinite(S))
    assert relerr(S, o["S"]) < 1e-10
    assert abs(S[2, 2] - 1.0) < 1e-12


def test_deep_channel_with_closed_channels(mods):
    """A channel far below its Coulomb barrier together with a closed
    channel: the closed one eliminated through R_eff, the scaled matching
    over the open ones; S against the oracle."""
    H, P = mods
    sp, E = _deep_system(True, closed=True)
    o = opipe.solve_energy(sp, E)
    say("deep and closed channels")
    res = P.Solver(P.DeviceSystem(sp), H.HP_C128).run(E)
    assert res.nopen == 3
    _check_S(res.S.cpu().numpy(), o, 1e-10)


@pytest.mark.parametrize("closed", [False, True])
def test_noalloc_form_with_a_deep_channel(mods, closed):
    """hp_smatrix_noalloc on the scaled matching (and with a closed channel
    eliminated first): the same S as hp_smatrix, bit for bit, and the
    oracle's S."""
    H, P = mods
    sp, E = _deep_system(True, closed=closed)
    o = opipe.solve_energy(sp, E)
    d = P.DeviceSystem(sp)
    R = torch.from_numpy(o["R"]).to("cuda")
    S1 = torch.empty_like(R)
    S2 = torch.full_like(R, complex(np.nan, np.nan))
    work = torch.empty(H.hp_workspace_bytes(sp.nc, sp.nc, H.HP_C128), dtype=torch.uint8, device="cuda")
    say("noalloc deep channel, closed", closed)
    n1 = H.hp_smatrix(d.sys, E, R, S1, work)
    n2 = H.hp_smatrix_noalloc(d.sys, E, R, S2)
    assert n1 == n2 == 3
    assert torch.equal(S1, S2)
    _check_S(S2.cpu().numpy(), o, 1e-10)


@pytest.mark.parametrize("closed", [False, True])
def test_batched_matching_with_a_deep_channel(mods, closed):
    """The batched matching takes the same scaled form, with and without a
    closed channel; S against the oracle."""
    H, P = mods
    from paper_2512_11590_amd import batch as B
    sp, E = _deep_system(True, closed=closed)
    o = opipe.solve_energy(sp, E)
    bk = B.Bucket([sp], [E], [0], H.HP_C128)
    bk.factor(8, 0, 8)
    bk.solve(0)
    bk.rmatrix()
    bk.smatrix()
    say("batched deep channel, closed", closed)
    assert int(bk.sstat.cpu().numpy()[0]) == 0
    _check_S(bk.S_of(0), o, 1e-10)
