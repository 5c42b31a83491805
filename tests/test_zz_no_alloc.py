"""hp_smatrix_noalloc (workspace in a static device array) against hp_smatrix
(caller's workspace): the same kernels on the same R give the same S, bit for
bit, on two calls in a row, the second with fewer channels; and a channel
count beyond the array's limit is refused before any work is enqueued."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import pipeline as opipe  # noqa: E402
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


def test_smatrix_noalloc_matches_workspace_form(mods):
    H, P = mods
    # the larger call first, then a smaller one: the second must not see the
    # first one's leftovers in the shared array
    for nc, nr, E in ((200, 20, 13.0), (7, 30, 9.5)):
        sp = make_system("small", nc=nc, nr=nr, lmax=12)
        say("smatrix noalloc nc", nc, "E", E)
        d = P.DeviceSystem(sp)
        o = opipe.solve_energy(sp, E) if nc <= 16 else None
        # R from the solver (FP64 path), then S both ways from the same R
        res = P.Solver(d, H.HP_C128).run(E, smatrix=False)
        R = res.R.clone()
        work = torch.empty(H.hp_workspace_bytes(nc, nc, H.HP_C128), dtype=torch.uint8, device="cuda")
        S_ref = torch.empty((nc, nc), dtype=torch.complex128, device="cuda")
        S_new = torch.full((nc, nc), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
        n1 = H.hp_smatrix(d.sys, E, R, S_ref, work)
        n2 = H.hp_smatrix_noalloc(d.sys, E, R, S_new)
        assert n1 == n2 == nc
        a, b = S_ref.cpu().numpy(), S_new.cpu().numpy()
        assert np.array_equal(a, b)
        if o is not None:
            assert relerr(b, o["S"]) < 1e-10


def test_smatrix_noalloc_refuses_too_many_channels(mods):
    H, P = mods
    nc = 257
    sp = make_system("small", nc=nc, nr=2, lmax=4)
    d = P.DeviceSystem(sp)
    R = torch.zeros((nc, nc), dtype=torch.complex128, device="cuda")
    S = torch.empty_like(R)
    code = H.lib().hp_smatrix_noalloc(H.ctypes.byref(d.sys), 10.0, R.data_ptr(), S.data_ptr(), None,
                                      H._stream(None))
    assert code == H.HP_ERR_UNSUPPORTED
