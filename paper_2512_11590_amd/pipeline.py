"""Persistent device buffers and the per-energy call sequence of the C ABI.

A :class:`DeviceSystem` uploads one coupled-channel system (mesh, kinetic +
Bloch matrix, surface values, channel data and the potential values at the
mesh points) to the device once.  A :class:`Solver` owns the matrix, pivot,
solution and workspace buffers for that system, allocated once and reused for
every energy of a scan (persistent buffers as in the paper's GPU solver), and
runs the entry points in order:

    hp_build_matrix -> hp_factor -> hp_solve -> hp_rmatrix -> hp_smatrix

In FP32 mode a refinement that does not converge (or a zero FP32 pivot) is
followed by the FP64 path on the same system (the paper's fallback mechanism,
Sec. 5.5, Accuracy Validation), and the result says so.  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import hprmat as H

E2 = 1.44  # e^2 in MeV fm


class DeviceSystem:
    """`vnl`: optional device complex128 tensor (N, N) of non-local kernel
    values W_cc'(r_i, r_j) in channel-major order; without it, a
    ``nonlocal_potential(r)`` method of `params` (shape (nc, nr, nc, nr))
    supplies them, and a system with neither is local."""

    def __init__(self, params, device: str = "cuda", vnl: torch.Tensor | None = None):
        self.params = params
        self.nc, self.nr = int(params.nc), int(params.nr)
        self.n = self.nc * self.nr
        self.device = torch.device(device)
        r, w, q, tl = H.hp_mesh(self.nr, float(params.a))
        self.r_host, self.q_host, self.tl_host = r, q, tl
        v = np.ascontiguousarray(params.potential(r), dtype=np.complex128)  # user-supplied V(r_i)
        dev = self.device
        self.r = torch.from_numpy(r).to(dev)
        self.q = torch.from_numpy(q).to(dev)
        self.tl = torch.from_numpy(np.ascontiguousarray(tl)).to(dev)
        self.l = torch.from_numpy(np.asarray(params.l, dtype=np.int32)).to(dev)
        self.eps = torch.from_numpy(np.asarray(params.eps, dtype=np.float64)).to(dev)
        self.v = torch.from_numpy(v).to(dev)
        self.w = torch.from_numpy(w).to(dev)
        if vnl is None:
            fn = getattr(params, "nonlocal_potential", None)
            W = fn(r) if fn is not None else None
            if W is not None:
                W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(self.n, self.n))
                vnl = torch.from_numpy(W).to(dev)
        if vnl is not None:
            if (tuple(vnl.shape) != (self.n, self.n) or vnl.dtype != torch.complex128 or not vnl.is_contiguous()
                    or vnl.device != self.r.device):
                raise ValueError("vnl must be a contiguous complex128 (N, N) tensor on the system's device")
        self.vnl = vnl
        self._kinv = None
        self.sys = H.HpSystem(self.nc, self.nr, float(params.a), float(params.hbar2_2mu),
                              float(params.z1z2) * E2, self.r.data_ptr(), self.q.data_ptr(),
                              self.tl.data_ptr(), self.l.data_ptr(), self.eps.data_ptr(),
                              self.v.data_ptr(), self.w.data_ptr(),
                              vnl.data_ptr() if vnl is not None else None)


    @property
    def kinv(self) -> torch.Tensor:
        """The kinetic inverse of the Woodbury-kinetic form (device, made once)."""
        if self._kinv is None:
            self._kinv = torch.from_numpy(H.hp_kinetic_inverse(self.nr, float(self.params.a))).to(self.device)
        return self._kinv


@dataclass
class EnergyResult:
    E: float
    prec: int
    R: torch.Tensor
    S: torch.Tensor | None
    iterations: int
    correction: float
    fallback: bool
    nopen: int
    backward_error: float = -1.0


class Solver:
    """Buffers for one system in one working precision: HP_C128, HP_C64, or
    HP_C64H (FP32 factors whose trailing updates run on the FP16 matrix cores
    under row and column scaling).  With schur=True the factored matrix is
    the Woodbury-kinetic S(E) = I + K_diag^-1 V (the paper's Type 3, Sec. 3.3)
    instead of C(E); the refinement (both precisions) works on C(E)'s FP64
    residual, and max_refine=0 gives the paper's unrefined Type 3 solve."""

    def __init__(self, dsys: DeviceSystem, prec: int = H.HP_C64, ld: int | None = None,
                 fallback: bool = True, schur: bool = False):
        self.d = dsys
        self.prec = prec
        self.fallback = fallback
        self.schur = schur
        n, nc = dsys.n, dsys.nc
        self.ld = ld or n
        dev = dsys.device
        ctype = torch.complex128 if prec == H.HP_C128 else torch.complex64
        self.A = torch.empty((n, self.ld), dtype=ctype, device=dev)
        self.ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        self.perm = torch.empty(n, dtype=torch.int32, device=dev)
        self.info = torch.zeros(1, dtype=torch.int32, device=dev)
        self.X = torch.empty((n, nc), dtype=torch.complex128, device=dev)
        self.R = torch.empty((nc, nc), dtype=torch.complex128, device=dev)
        self.S = torch.empty((nc, nc), dtype=torch.complex128, device=dev)
        wb = H.hp_schur_workspace_bytes(n, nc, prec) if schur else H.hp_workspace_bytes(n, nc, prec)
        self.work = torch.empty(wb, dtype=torch.uint8, device=dev)
        self.swork = torch.empty(H.hp_workspace_bytes(nc, nc, H.HP_C128), dtype=torch.uint8, device=dev)
        self._fp64 = None

    def factor(self, E: float) -> None:
        if self.schur:
            H.hp_build_schur(self.d.sys, E, self.prec, self.d.kinv, self.A, self.ld)
        else:
            H.hp_build_matrix(self.d.sys, E, self.prec, self.A, self.ld)
        H.hp_factor(self.d.n, self.prec, self.A, self.ld, self.ipiv, self.perm, self.info, self.work)

    def solve(self, E: float, max_refine: int, tol: float):
        if self.schur:
            return H.hp_solve_schur(self.d.sys, E, self.prec, self.d.kinv, self.A, self.ld, self.perm, self.info,
                                    self.X, max_refine, tol, self.work)
        return H.hp_solve(self.d.sys, E, self.prec, self.A, self.ld, self.perm, self.info, self.X,
                          max_refine, tol, self.work)

    def run(self, E: float, max_refine: int = 30, tol: float = 0.0, smatrix: bool = True) -> EnergyResult:
        """max_refine applies to FP32 factors and to the Woodbury-kinetic form;
        a plain FP64 factorization is solved once."""
        self.factor(E)
        refine = max_refine if (self.prec != H.HP_C128 or self.schur) else 0
        code, info = self.solve(E, refine, tol)
        iterations, backward = info.iterations, info.residual
        used_fallback = False
        if code != H.HP_OK:
            if not (self.fallback and (self.prec != H.HP_C128 or self.schur)
                    and code in (H.HP_ERR_NOCONV, H.HP_ERR_SINGULAR)):
                raise H.HprmatError(code, "hp_solve")
            if self._fp64 is None:
                self._fp64 = Solver(self.d, H.HP_C128, fallback=False)
            self._fp64.factor(E)
            code, info = self._fp64.solve(E, 0, tol)
            if code != H.HP_OK:
                raise H.HprmatError(code, "hp_solve (FP64 fallback)")
            self.X.copy_(self._fp64.X)
            used_fallback = True
        H.hp_rmatrix(self.d.sys, self.X, self.R)
        nopen = 0
        S = None
        if smatrix:
            nopen = H.hp_smatrix(self.d.sys, E, self.R, self.S, self.swork)
            S = self.S
        return EnergyResult(E=E, prec=self.prec, R=self.R, S=S, iterations=iterations,
                            correction=info.correction, fallback=used_fallback, nopen=nopen,
                            backward_error=backward)


class EnergyScan:
    """An energy scan of one system with `slots` solvers in flight (the
    paper's steady-state energy scan, Sec. 5.3, with persistent buffers per
    slot): each slot owns a Solver (matrix, factors, workspace) and a stream,
    and takes the next energy as soon as its previous one is done.  The
    library serializes the slots' factorizations on one device-wide stream
    (hp_set_concurrency), so one slot's triangular solves, refinement, R and S
    run beside the next slot's assembly and factorization.  Results are
    returned in energy order (R and S copied to the host)."""

    def __init__(self, dsys: DeviceSystem, prec: int = H.HP_C64, slots: int = 2, fallback: bool = True,
                 schur: bool = False):
        if slots < 1:
            raise ValueError("slots >= 1")
        self.d = dsys
        self.prec = prec
        self.slots = [Solver(dsys, prec, fallback=fallback, schur=schur) for _ in range(slots)]
        self.streams = [torch.cuda.Stream(device=dsys.device) for _ in range(slots)]

    def run(self, energies, max_refine: int = 30, tol: float = 0.0) -> list[EnergyResult]:
        import threading
        energies = [float(E) for E in energies]
        out: list[EnergyResult | None] = [None] * len(energies)
        errors: list[BaseException] = []
        lock = threading.Lock()
        nxt = [0]
        dev = self.d.device
        index = dev.index if dev.index is not None else torch.cuda.current_device()
        cur = torch.cuda.current_stream(index)

        def slot(k: int) -> None:
            try:
                torch.cuda.set_device(index)
                st = self.streams[k]
                st.wait_stream(cur)
                with torch.cuda.stream(st):
                    while True:
                        with lock:
                            i = nxt[0]
                            if i >= len(energies) or errors:
                                return
                            nxt[0] = i + 1
                        r = self.slots[k].run(energies[i], max_refine=max_refine, tol=tol)
                        out[i] = EnergyResult(E=r.E, prec=r.prec, R=r.R.cpu().clone(),
                                              S=None if r.S is None else r.S.cpu().clone(),
                                              iterations=r.iterations, correction=r.correction,
                                              fallback=r.fallback, nopen=r.nopen,
                                              backward_error=r.backward_error)
            except BaseException as exc:  # stop the scan, re-raised below
                with lock:
                    errors.append(exc)

        prev = H.hp_set_concurrency(len(self.slots))
        try:
            threads = [threading.Thread(target=slot, args=(k,), daemon=True) for k in range(len(self.slots))]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
        finally:
            H.hp_set_concurrency(prev)
        for st in self.streams:
            cur.wait_stream(st)
        if errors:
            raise errors[0]
        return out
