"""Batched uneven systems: device layout, size buckets, autotuning, graphs.

Many independent systems (one per (J^pi, energy) label, N = nc*nr from a
few hundred to a few thousand) are laid out in shared device buffers and
solved by the batched entry points of the C ABI:

    hp_batch_build -> hp_batch_factor[_stepped] -> hp_batch_solve_init
        -> [hp_batch_refine_step]* (FP32 factors) -> hp_batch_rmatrix
        -> hp_batch_smatrix

Systems are split into size buckets; each bucket is one persistent
batched-LU launch (systems largest first, one workgroup per system) or the
stepped form (per step one launch over every system of the bucket: panel
column steps, block rows, and trailing updates with K up to 64 as tiles of
all systems).  The form, panel width, outer block and grid size of each
bucket are picked by `autotune` (timed on the bucket or its largest systems,
cached per bucket and precision).  After a first eager run, which also
counts the refinement steps the bucket needs, the whole bucket -- build,
factorization, solves, that many refinement steps, R and S -- is captured in
one HIP graph and replayed; a bucket that needs more steps than captured
continues eagerly.  Systems whose FP32 refinement does not converge, or
whose FP32 factor has an exactly zero pivot, are solved again in FP64
through the single-system path (the paper's fallback mechanism, Sec. 5.5).
All arithmetic runs in the HIP library; this module lays out memory and
sequences the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import hprmat as H

E2 = 1.44  # e^2 in MeV fm
BUCKET_EDGES = (1000, 2000)  # N boundaries of the size buckets
PANELS = (8, 16, 32)
GROUPS_PER_CU = (2, 3)
BLOCKS = (32, 64)  # outer blocks tried for the stepped form


@dataclass
class BucketTuning:
    panel: int
    groups: int  # workgroups of the persistent grid; 0: the stepped form
    ms: float
    block: int = 64  # outer block of the stepped form (a multiple of panel, <= 64)


_TUNED: dict = {}


class Bucket:
    """Systems of one size bucket in shared device buffers (largest first)."""

    def __init__(self, systems, energies, index, prec: int, device="cuda"):
        order = sorted(range(len(systems)), key=lambda k: -(systems[k].nc * systems[k].nr))
        self.index = [index[k] for k in order]
        self.systems = [systems[k] for k in order]
        self.energies = [float(energies[k]) for k in order]
        self.prec = prec
        self.count = len(self.systems)
        dev = torch.device(device)
        self.device = dev
        nc = np.array([s.nc for s in self.systems], dtype=np.int64)
        nr = np.array([s.nr for s in self.systems], dtype=np.int64)
        n = nc * nr
        self.n, self.nc, self.nr = n, nc, nr
        # each matrix starts on a 256-byte boundary (a multiple of 32 elements),
        # so the rows of every system with even n are 16-byte aligned (the
        # batched FP32 tile product then stages them by direct loads)
        slot = (n * n + 31) // 32 * 32
        self.a_off = np.concatenate([[0], np.cumsum(slot)[:-1]])
        self.x_off = np.concatenate([[0], np.cumsum(n * nc)[:-1]])
        self.p_off = np.concatenate([[0], np.cumsum(n)[:-1]])
        self.r_off = np.concatenate([[0], np.cumsum(nc * nc)[:-1]])
        self.c_off = np.concatenate([[0], np.cumsum(nc)[:-1]])
        self.sum_nc, self.sum_xn = int(nc.sum()), int((n * nc).sum())
        # per-system mesh, channel and potential data, concatenated
        r_h, q_h, tl_h, l_h, eps_h, v_h, w_h, nl_h = [], [], [], [], [], [], [], []
        for s in self.systems:
            r, w, q, tl = H.hp_mesh(int(s.nr), float(s.a))
            fn = getattr(s, "nonlocal_potential", None)
            W = fn(r) if fn is not None else None
            nl_h.append(None if W is None else
                        np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(-1)))
            w_h.append(w)
            r_h.append(r)
            q_h.append(q)
            tl_h.append(np.ascontiguousarray(tl).ravel())
            l_h.append(np.asarray(s.l, dtype=np.int32))
            eps_h.append(np.asarray(s.eps, dtype=np.float64))
            v_h.append(np.ascontiguousarray(s.potential(r), dtype=np.complex128).ravel())
        self.r = torch.from_numpy(np.concatenate(r_h)).to(dev)
        self.q = torch.from_numpy(np.concatenate(q_h)).to(dev)
        self.tl = torch.from_numpy(np.concatenate(tl_h)).to(dev)
        self.l = torch.from_numpy(np.concatenate(l_h)).to(dev)
        self.eps = torch.from_numpy(np.concatenate(eps_h)).to(dev)
        self.v = torch.from_numpy(np.concatenate(v_h)).to(dev)
        self.w = torch.from_numpy(np.concatenate(w_h)).to(dev)
        # non-local kernel values of the systems that have them (n x n each)
        nl_len = np.array([0 if W is None else W.size for W in nl_h], dtype=np.int64)
        off_nl = np.concatenate([[0], np.cumsum(nl_len)[:-1]])
        self.vnl = (torch.from_numpy(np.concatenate([W for W in nl_h if W is not None])).to(dev)
                    if nl_len.sum() else None)
        off_r = np.concatenate([[0], np.cumsum(nr)[:-1]])
        off_tl = np.concatenate([[0], np.cumsum(nr * nr)[:-1]])
        off_c = self.c_off
        off_v = np.concatenate([[0], np.cumsum(nr * nc * nc)[:-1]])
        self.sys = []
        items = (H.HpBatchItem * self.count)()
        for k, s in enumerate(self.systems):
            sy = H.HpSystem(int(nc[k]), int(nr[k]), float(s.a), float(s.hbar2_2mu), float(s.z1z2) * E2,
                            self.r.data_ptr() + 8 * int(off_r[k]), self.q.data_ptr() + 8 * int(off_r[k]),
                            self.tl.data_ptr() + 8 * int(off_tl[k]), self.l.data_ptr() + 4 * int(off_c[k]),
                            self.eps.data_ptr() + 8 * int(off_c[k]), self.v.data_ptr() + 16 * int(off_v[k]),
                            self.w.data_ptr() + 8 * int(off_r[k]),
                            (self.vnl.data_ptr() + 16 * int(off_nl[k])) if nl_len[k] else None)
            self.sys.append(sy)
            items[k] = H.HpBatchItem(sy, self.energies[k], int(self.a_off[k]), int(self.x_off[k]),
                                     int(self.p_off[k]), int(self.r_off[k]), int(self.c_off[k]))
        raw = np.frombuffer(bytes(items), dtype=np.uint8).copy()
        self.items = torch.from_numpy(raw).to(dev)
        ctype = torch.complex64 if prec == H.HP_C64 else torch.complex128
        self.A = torch.empty(int(slot.sum()), dtype=ctype, device=dev)
        self.ipiv = torch.empty(int(n.sum()), dtype=torch.int32, device=dev)
        self.perm = torch.empty(int(n.sum()), dtype=torch.int32, device=dev)
        self.info = torch.zeros(self.count, dtype=torch.int32, device=dev)
        self.X = torch.empty(self.sum_xn, dtype=torch.complex128, device=dev)
        self.R = torch.empty(int((nc * nc).sum()), dtype=torch.complex128, device=dev)
        self.work = torch.empty(H.hp_batch_workspace_bytes(self.count, self.sum_nc, self.sum_xn, int(n.max()),
                                                           prec), dtype=torch.uint8, device=dev)
        self.S = torch.empty_like(self.R)
        self.sstat = torch.zeros(self.count, dtype=torch.int32, device=dev)
        self.sum_nc2 = int((nc * nc).sum())
        self.zwork = torch.empty(32 * self.sum_nc2, dtype=torch.uint8, device=dev)
        self.shape = np.stack([n, nc], axis=1).astype(np.int32)  # (n, nc), largest n first
        self.stepped = False  # solves in the stepped form (set with the factorization form)
        self.graph = None  # captured refinement step
        self.whole = None  # captured bucket: (graph, key)
        self._steps = 0
        self.flops = float((8.0 / 3.0) * (n.astype(np.float64) ** 3).sum())

    @property
    def key(self):
        return (int(self.n.max()), int(self.n.min()), self.count, self.prec)

    def factor(self, panel: int, groups: int, block: int = 64) -> None:
        """Build and factor; groups > 0: persistent grid of that many
        workgroups, groups == 0: the stepped form with outer blocks of
        `block` columns (rounded down to a multiple of panel)."""
        H.hp_batch_build(self.count, self.items, self.prec, self.A)
        self.stepped = groups == 0
        if groups > 0:
            H.hp_batch_factor(self.count, self.items, self.prec, self.A, self.ipiv, self.perm, self.info, panel,
                              groups, self.work)
        else:
            block = max(panel, block // panel * panel)
            H.hp_batch_factor_stepped(self.count, self.items, self.n, self.prec, self.A, self.ipiv, self.perm,
                                      self.info, panel, block, self.work)

    def solve_init(self, max_refine: int = 30) -> bool:
        """Initial solve; True if FP32 refinement follows."""
        refine = self.prec == H.HP_C64 and max_refine > 0
        H.hp_batch_solve_init(self.count, self.items, self.shape if self.stepped else None, self.prec, self.A,
                              self.perm, self.info, self.X, refine, self.sum_nc, self.sum_xn, self.work)
        self._steps = 0
        return refine

    def refine_step(self, max_refine: int = 30, tol: float = 0.0, use_graph: bool = True) -> None:
        """Enqueue one refinement step (a graph replay after the first step)."""
        args = (self.count, self.items, self.shape if self.stepped else None, self.A, self.perm, self.X, max_refine,
                tol, self.sum_nc, self.sum_xn, self.work)
        if use_graph and self.graph is None and self._steps > 0:
            # capture one step (every kernel's launch attributes are set by now);
            # the capture runs nothing, the replay below does
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream(device=self.device)
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(g, stream=side):
                H.hp_batch_refine_step(*args)
            torch.cuda.current_stream().wait_stream(side)
            self.graph = (g, (max_refine, tol, self.stepped))
        if use_graph and self.graph is not None and self.graph[1] == (max_refine, tol, self.stepped):
            self.graph[0].replay()
        else:
            H.hp_batch_refine_step(*args)
        self._steps += 1

    def solve(self, max_refine: int = 30, tol: float = 0.0, use_graph: bool = True) -> int:
        """Initial solve, then (FP32) refinement steps until every system has
        stopped; returns the number of steps taken."""
        if not self.solve_init(max_refine):
            return 0
        while self._steps < max_refine:
            self.refine_step(max_refine, tol, use_graph)
            if H.hp_batch_active(self.work) == 0:
                break
        return self._steps

    def rmatrix(self) -> None:
        H.hp_batch_rmatrix(self.count, self.items, self.X, self.R)

    def smatrix(self) -> None:
        H.hp_batch_smatrix(self.count, self.items, self.R, self.S, self.sstat, self.sum_nc2, int(self.nc.max()),
                           self.zwork)

    def enqueue(self, t: BucketTuning, max_refine: int, tol: float, steps: int) -> None:
        """The whole bucket with a fixed number of refinement steps and no
        host synchronisation (capturable): build, factor, solve, `steps`
        refinement steps (systems that have stopped are skipped by the
        kernels), R, S."""
        self.factor(t.panel, t.groups, t.block)
        refine = self.solve_init(max_refine)
        args = (self.count, self.items, self.shape if self.stepped else None, self.A, self.perm, self.X, max_refine,
                tol, self.sum_nc, self.sum_xn, self.work)
        for _ in range(steps if refine else 0):
            H.hp_batch_refine_step(*args)
            self._steps += 1
        self.rmatrix()
        self.smatrix()

    def capture(self, t: BucketTuning, max_refine: int, tol: float, steps: int) -> None:
        """Capture enqueue(...) in a graph (after an eager run has set every
        kernel's launch attributes)."""
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            self.enqueue(t, max_refine, tol, steps)
        torch.cuda.current_stream().wait_stream(side)
        self.whole = (g, (t.panel, t.groups, t.block, max_refine, tol, steps))

    def status(self):
        return H.hp_batch_status(self.count, self.work)

    def R_of(self, k: int) -> np.ndarray:
        """R of the k-th system of this bucket (host copy)."""
        c = int(self.nc[k])
        o = int(self.r_off[k])
        return self.R[o:o + c * c].view(c, c).cpu().numpy()

    def S_of(self, k: int) -> np.ndarray:
        """S of the k-th system of this bucket (host copy; from hp_batch_smatrix)."""
        c = int(self.nc[k])
        o = int(self.r_off[k])
        return self.S[o:o + c * c].view(c, c).cpu().numpy()


def autotune(bucket: Bucket, cus: int, reps: int = 1, sample: int | None = None, panels=PANELS,
             groups_per_cu=GROUPS_PER_CU, blocks=BLOCKS) -> BucketTuning:
    """Time the factorization for each panel width and form (persistent
    grid sizes; stepped with each outer block), on the bucket itself or on a
    bucket of its `sample` largest systems; keep the fastest (cached per
    bucket shape and precision)."""
    if bucket.key in _TUNED:
        return _TUNED[bucket.key]
    probe = bucket
    if sample is not None and sample < bucket.count:
        probe = Bucket(bucket.systems[:sample], bucket.energies[:sample], list(range(sample)), bucket.prec,
                       bucket.device)
    best = None
    for panel in panels:
        shapes = [(gpc * cus, panel) for gpc in groups_per_cu] + [(0, b) for b in blocks if b % panel == 0]
        for groups, block in shapes:
            probe.factor(panel, groups, block)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                probe.factor(panel, groups, block)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            if best is None or ms < best.ms:
                best = BucketTuning(panel, groups, ms, block)
    _TUNED[bucket.key] = best
    return best


class Batch:
    """An uneven batch split into size buckets (one persistent launch each)."""

    def __init__(self, systems, energies, prec: int, device="cuda", edges=BUCKET_EDGES):
        self.prec = prec
        self.count = len(systems)
        n = np.array([s.nc * s.nr for s in systems])
        bounds = (0,) + tuple(edges) + (1 << 30,)
        self.buckets = []
        for lo, hi in zip(bounds, bounds[1:]):
            idx = [k for k in range(len(systems)) if lo <= n[k] < hi]
            if idx:
                self.buckets.append(Bucket([systems[k] for k in idx], [energies[k] for k in idx], idx, prec,
                                           device))
        props = torch.cuda.get_device_properties(torch.device(device))
        self.cus = int(props.multi_processor_count)
        self.tuning = {}
        self.flops = sum(b.flops for b in self.buckets)

    def tune(self, **kw) -> dict:
        for b in self.buckets:
            self.tuning[b.key] = autotune(b, self.cus, **kw)
        return {f"N {int(b.n.min())}-{int(b.n.max())} ({b.count})": vars(self.tuning[b.key]) for b in self.buckets}

    def run(self, max_refine: int = 30, tol: float = 0.0, use_graph: bool = True) -> dict:
        """Build, factor, solve (and refine), R and S for every system.  Each
        bucket has its own stream.  Eager form (the first run, or
        use_graph=False): all factorizations are enqueued first, then the
        refinement steps of the buckets still refining are interleaved, each
        step (after the first) replayed from a captured step.  With a captured
        bucket (use_graph, after an eager run), one graph replay per bucket;
        a bucket with systems still refining afterwards continues eagerly."""
        streams = [torch.cuda.Stream() for _ in self.buckets]
        cur = torch.cuda.current_stream()
        tun = {b.key: self.tuning.get(b.key) or BucketTuning(16, 2 * self.cus, 0.0) for b in self.buckets}
        refining = []
        for b, s in zip(self.buckets, streams):
            s.wait_stream(cur)
            t = tun[b.key]
            with torch.cuda.stream(s):
                key = (t.panel, t.groups, t.block, max_refine, tol)
                if use_graph and b.whole is not None and b.whole[1][:5] == key:
                    b.whole[0].replay()
                    b._steps = b.whole[1][5]
                    if self.prec == H.HP_C64:
                        refining.append((b, s))
                    continue
                b.factor(t.panel, t.groups, t.block)
                if b.solve_init(max_refine):
                    b.refine_step(max_refine, tol, use_graph)  # sets the count of systems still refining
                    refining.append((b, s))
        done_eager = set()
        while refining:
            still = []
            for b, s in refining:
                with torch.cuda.stream(s):
                    if H.hp_batch_active(b.work) > 0 and b._steps < max_refine:
                        still.append((b, s))
            for b, s in still:
                with torch.cuda.stream(s):
                    b.refine_step(max_refine, tol, use_graph)
                    done_eager.add(id(b))
            refining = still
        for b, s in zip(self.buckets, streams):
            t = tun[b.key]
            with torch.cuda.stream(s):
                replayed = use_graph and b.whole is not None and b.whole[1][:5] == (t.panel, t.groups, t.block,
                                                                                    max_refine, tol)
                if not replayed or id(b) in done_eager:  # X changed after the graph's R and S
                    b.rmatrix()
                    b.smatrix()
            cur.wait_stream(s)
        if use_graph:
            for b in self.buckets:
                t = tun[b.key]
                key = (t.panel, t.groups, t.block, max_refine, tol)
                if b.whole is None or b.whole[1][:5] != key or b.whole[1][5] < b._steps:
                    torch.cuda.synchronize()
                    b.capture(t, max_refine, tol, b._steps)
        return {f"N {int(b.n.min())}-{int(b.n.max())}": b._steps for b in self.buckets}

    def results(self, fallback: bool = True):
        """[(R, S)] in the original order of the systems (host arrays).  A
        system whose FP32 refinement did not converge (status 2), whose FP32
        factor met an exactly zero pivot (status 3) or that the batched
        refinement does not take (status 4: a non-local system on more than
        1024 mesh points) is solved again in FP64 through the single-system
        path when `fallback` is set (its index is then listed in
        self.fallbacks), else HprmatError is raised."""
        from . import pipeline as P
        out = [None] * self.count
        st, _ = self.status()
        self.fallbacks = []
        for b in self.buckets:
            sst = b.sstat.cpu().numpy()
            R_all = b.R.cpu().numpy()
            S_all = b.S.cpu().numpy()
            for k in range(b.count):
                g = b.index[k]
                if st[g] in (2, 3, 4):
                    if not fallback:
                        code = {2: H.HP_ERR_NOCONV, 3: H.HP_ERR_SINGULAR, 4: H.HP_ERR_UNSUPPORTED}[int(st[g])]
                        raise H.HprmatError(code, f"batched system {g}")
                    res = P.Solver(P.DeviceSystem(b.systems[k], device=str(b.device)), H.HP_C128).run(
                        b.energies[k])
                    out[g] = (res.R.cpu().numpy(), res.S.cpu().numpy())
                    self.fallbacks.append(g)
                    continue
                if sst[k] != 0:
                    code = H.HP_ERR_UNSUPPORTED if sst[k] in (1, 4) else (
                        H.HP_ERR_NOCONV if sst[k] == 2 else H.HP_ERR_SINGULAR)
                    raise H.HprmatError(code, f"hp_batch_smatrix, system {g}")
                c = int(b.nc[k])
                o = int(b.r_off[k])
                out[g] = (R_all[o:o + c * c].reshape(c, c), S_all[o:o + c * c].reshape(c, c))
        return out

    def status(self):
        st = np.zeros(self.count, dtype=np.int32)
        it = np.zeros(self.count, dtype=np.int32)
        for b in self.buckets:
            s, i = b.status()
            for k in range(b.count):
                st[b.index[k]] = s[k]
                it[b.index[k]] = i[k]
        return st, it
