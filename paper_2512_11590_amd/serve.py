"""A served stream of R-matrix solve requests on one GPU (continuous batching).

A request is one coupled-channel system (its potential, mesh and channel
data) with 1-8 energies; it arrives at a given time.  The server owns a fixed
number of slots, each a host thread with its own HIP stream.  A request is
admitted, in arrival order, as soon as a slot is free and its device memory
fits the HBM budget; requests that arrive while others are on the GPU are
therefore admitted as slots and memory free up, and the device work of the
slots overlaps (different streams).  Per request the slot uploads the system
once and runs, per energy, the five entry points of the C ABI
(hp_build_matrix -> hp_factor -> hp_solve -> hp_rmatrix -> hp_smatrix) in
FP32 + FP64 refinement or in FP64.  Factors are not shared between requests:
C(E) differs for every (system, energy).

The single-system factorization's panel grid must be resident as a whole,
so the server declares its number of slots to the library
(hp_set_concurrency), which then serializes those factorizations on one
device-wide stream and keeps panel workgroups small.  Requests of up to
`batched_max_n` unknowns take the batched path instead: all energies of the
request as one bucket of the stepped batched LU (hp_batch_*, no grid-wide
waits), with its solves, refinement, R and S, on the slot's own stream -- so
their factorizations overlap each other and the serialized large ones.
Everything else of the slots overlaps in either case.

Latency of a request = completion time - arrival time (host clock, the
request's S matrices copied back).  The summary reports p50 / p99 latency and
solves (energies) per second over the makespan.  All device arithmetic runs
in the HIP library; this module only schedules.
"""
from __future__ import annotations

import contextlib
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hprmat as H
from . import pipeline as P


def request_bytes(nc: int, nr: int, prec: int) -> int:
    """Device bytes one request holds while admitted (matrix, workspace, solution,
    potential values, small buffers); with FP32 factors also the FP64 matrix
    and workspace that a fallback to the FP64 solve allocates."""
    n = nc * nr
    elt = 16 if prec == H.HP_C128 else 8
    need = (n * n * elt + H.hp_workspace_bytes(n, nc, prec) + H.hp_workspace_bytes(nc, nc, H.HP_C128)
            + n * nc * 16 + 3 * nc * nc * 16 + nr * nc * nc * 16 + 64 * n)
    if prec != H.HP_C128:
        need += n * n * 16 + H.hp_workspace_bytes(n, nc, H.HP_C128) + n * nc * 16 + 3 * nc * nc * 16 + 64 * n
    return need


def is_nonlocal(params) -> bool:
    """Whether the system carries a non-local kernel (evaluated on its mesh)."""
    fn = getattr(params, "nonlocal_potential", None)
    return fn is not None and fn(H.hp_mesh(int(params.nr), float(params.a))[0]) is not None


def served_bytes(params, prec: int, batched_max_n: int) -> int:
    """Device bytes a request holds while admitted: one system's buffers, or,
    on the batched path, one per energy (a bound: the bucket holds each
    energy's matrix, solution and potential values).  Non-local systems take
    the single-system path and hold their n x n kernel values too."""
    nc, nr = int(params.nc), int(params.nr)
    if is_nonlocal(params):
        return request_bytes(nc, nr, prec) + (nc * nr) ** 2 * 16
    ne = len(params.energies) if nc * nr <= batched_max_n else 1
    return ne * request_bytes(nc, nr, prec)


@dataclass
class Served:
    rid: int
    n: int
    nc: int
    energies: np.ndarray
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    R: list = field(default_factory=list)
    S: list = field(default_factory=list)
    iterations: list = field(default_factory=list)
    fallback: list = field(default_factory=list)
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    def __init__(self, slots: int = 4, prec: int = H.HP_C64, hbm_budget: int | None = None,
                 max_refine: int = 30, tol: float = 0.0, device: str = "cuda", executor=None,
                 bytes_of=None, batched_max_n: int = 4000):
        """executor(req, params) runs one admitted request (default: the HIP
        pipeline on the slot's stream); bytes_of(params) its device bytes
        (default: request_bytes).  Both are replaceable so the scheduling can be
        tested without a device."""
        if slots < 1:
            raise ValueError("slots >= 1")
        self.slots = slots
        self.prec = prec
        self.batched_max_n = batched_max_n
        self.max_refine = max_refine
        self.tol = tol
        self._execute = executor or self._run_request
        self._bytes_of = bytes_of or (lambda sp: served_bytes(sp, self.prec, self.batched_max_n))
        dev = torch.device(device)
        self.gpu = dev.type == "cuda"
        if self.gpu:
            self.device = dev if dev.index is not None else torch.device(dev.type, torch.cuda.current_device())
            props = torch.cuda.get_device_properties(self.device)
            self.cus = int(props.multi_processor_count)
            total = props.total_memory
        else:
            if hbm_budget is None:
                raise ValueError("a budget is needed without a device")
            self.device, self.cus, total = dev, 256, hbm_budget
        self.budget = int(hbm_budget if hbm_budget is not None else total * 0.6)
        self._cv = threading.Condition()
        self._pending: deque = deque()
        self._in_use = 0
        self._closed = False

    # -- admission -----------------------------------------------------------
    def _admit(self):
        with self._cv:
            while True:
                if self._pending:
                    req, params, need = self._pending[0]
                    if need > self.budget:
                        self._pending.popleft()
                        req.error = f"needs {need} bytes, more than the HBM budget {self.budget}"
                        req.admitted = req.done = time.perf_counter() - self._t0
                        self._cv.notify_all()
                        continue
                    if self._in_use + need <= self.budget:
                        self._pending.popleft()
                        self._in_use += need
                        req.admitted = time.perf_counter() - self._t0
                        return req, params, need
                elif self._closed:
                    return None
                self._cv.wait(timeout=0.05)

    def _release(self, need: int) -> None:
        with self._cv:
            self._in_use -= need
            self._cv.notify_all()

    # -- one slot --------------------------------------------------------------
    def _run_request(self, req: Served, params) -> None:
        # a non-local request keeps one copy of its kernel values for all its
        # energies on the single-system path (a bucket holds one per energy)
        if req.n <= self.batched_max_n and not is_nonlocal(params):
            return self._run_request_batched(req, params)
        d = P.DeviceSystem(params, device=str(self.device))
        s = P.Solver(d, self.prec)
        for E in req.energies:
            r = s.run(float(E), max_refine=self.max_refine, tol=self.tol)
            req.R.append(r.R.cpu().numpy().copy())
            req.S.append(r.S.cpu().numpy().copy())
            req.iterations.append(r.iterations)
            req.fallback.append(r.fallback)

    def _run_request_batched(self, req: Served, params) -> None:
        """All energies of the request as one bucket of the batched path."""
        from . import batch as B
        ne = len(req.energies)
        bk = B.Bucket([params] * ne, [float(E) for E in req.energies], list(range(ne)), self.prec,
                      device=str(self.device))
        bk.factor(16, 0, 64)
        bk.solve(max_refine=self.max_refine, tol=self.tol, use_graph=False)
        bk.rmatrix()
        bk.smatrix()
        st, it = bk.status()
        sst = bk.sstat.cpu().numpy()
        R_all = bk.R.cpu().numpy()
        S_all = bk.S.cpu().numpy()
        out = [None] * ne
        for k in range(ne):
            if st[k] in (2, 3, 4):  # not converged / zero pivot / not taken: FP64 single-system solve
                r = P.Solver(P.DeviceSystem(params, device=str(self.device)), H.HP_C128).run(bk.energies[k])
                out[bk.index[k]] = (r.R.cpu().numpy().copy(), r.S.cpu().numpy().copy(), int(it[k]), True)
                continue
            if sst[k] != 0:
                code = H.HP_ERR_UNSUPPORTED if sst[k] in (1, 4) else (
                    H.HP_ERR_NOCONV if sst[k] == 2 else H.HP_ERR_SINGULAR)
                raise H.HprmatError(code, f"hp_batch_smatrix (request {req.rid})")
            c = int(bk.nc[k])
            o = int(bk.r_off[k])
            out[bk.index[k]] = (R_all[o:o + c * c].reshape(c, c).copy(), S_all[o:o + c * c].reshape(c, c).copy(),
                                int(it[k]), False)
        for R, S, its, fb in out:
            req.R.append(R)
            req.S.append(S)
            req.iterations.append(its)
            req.fallback.append(fb)

    def _slot(self, k: int, stream) -> None:
        if self.gpu:
            torch.cuda.set_device(self.device)
        with (torch.cuda.stream(stream) if self.gpu else contextlib.nullcontext()):
            while True:
                item = self._admit()
                if item is None:
                    return
                req, params, need = item
                try:
                    self._execute(req, params)
                except Exception as exc:  # reported per request, the stream goes on
                    req.error = f"{type(exc).__name__}: {exc}"
                finally:
                    if self.gpu:
                        stream.synchronize()
                    req.done = time.perf_counter() - self._t0
                    self._release(need)
                    if self._progress is not None:
                        self._progress(req)

    # -- the stream ----------------------------------------------------------
    def run(self, requests, progress=None) -> list[Served]:
        """requests: [(arrival_seconds, SystemParams)] in arrival order.  Blocks
        until every request is done; returns one Served per request.
        progress(req), if given, is called from a slot thread as each request
        completes."""
        self._progress = progress
        prev = H.hp_set_concurrency(self.slots) if self.gpu else None
        out: list[Served] = []
        streams = [torch.cuda.Stream(device=self.device) if self.gpu else None for _ in range(self.slots)]
        self._closed = False
        self._t0 = time.perf_counter()
        threads = [threading.Thread(target=self._slot, args=(k, streams[k]), daemon=True)
                   for k in range(self.slots)]
        for t in threads:
            t.start()
        try:
            for rid, (t_arr, params) in enumerate(requests):
                wait = t_arr - (time.perf_counter() - self._t0)
                if wait > 0:
                    time.sleep(wait)
                req = Served(rid=rid, n=int(params.nc) * int(params.nr), nc=int(params.nc),
                             energies=np.asarray(params.energies, dtype=np.float64), arrival=float(t_arr))
                out.append(req)
                with self._cv:
                    self._pending.append((req, params, int(self._bytes_of(params))))
                    self._cv.notify_all()
        finally:
            with self._cv:
                self._closed = True
                self._cv.notify_all()
            for t in threads:
                t.join()
            if prev is not None:
                H.hp_set_concurrency(prev)
        for req in out:
            if req.error is None and len(req.S) != len(req.energies):
                req.error = "not processed (no slot left)"
        return out


def summary(results: list[Served]) -> dict:
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    solves = sum(len(r.energies) for r in ok)
    span = max((r.done for r in results), default=0.0) - min((r.arrival for r in results), default=0.0)
    return {"requests": len(results), "failed": len(results) - len(ok), "solves": solves,
            "makespan_s": span, "solves_per_s": solves / span if span > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "refinement_steps_mean": float(np.mean([i for r in ok for i in r.iterations])) if ok else 0.0,
            "fp64_fallbacks": int(sum(f for r in ok for f in r.fallback))}
