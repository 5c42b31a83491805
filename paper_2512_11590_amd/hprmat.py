"""ctypes binding of libhprmat.so (the C ABI in include/hprmat.h).

Argument marshalling only: every function forwards to the entry point of the
same name.  Device buffers are torch tensors on the HIP device (PyTorch is
used for device memory and streams); their data pointers and the current
stream are passed through.  If the library has not been built, or the HIP
device is missing, calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhprmat.so")

HP_OK = 0
HP_ERR_ARG = -1
HP_ERR_HIP = -2
HP_ERR_SINGULAR = -3
HP_ERR_NOCONV = -4
HP_ERR_WORKSPACE = -5
HP_ERR_UNSUPPORTED = -6
HP_ERR_SYNC = -7

HP_C128 = 0
HP_C64 = 1
HP_C64H = 2  # complex FP32 factors, split-FP16 trailing updates under row/column scaling

c_int, c_long, c_double, c_void_p, c_size_t = (ctypes.c_int, ctypes.c_long, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_size_t)


class HpSystem(ctypes.Structure):
    _fields_ = [("nc", c_int), ("nr", c_int), ("a", c_double), ("hbar2_2mu", c_double),
                ("z1z2e2", c_double), ("r", c_void_p), ("q", c_void_p), ("tl", c_void_p),
                ("l", c_void_p), ("eps", c_void_p), ("v", c_void_p), ("w", c_void_p), ("vnl", c_void_p)]


class HpBatchItem(ctypes.Structure):
    _fields_ = [("sys", HpSystem), ("E", c_double), ("a_off", c_long), ("x_off", c_long),
                ("p_off", c_long), ("r_off", c_long), ("c_off", c_long)]


class HpTraceStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", c_long), ("ms", c_double), ("flops", c_double),
                ("bytes", c_double)]


HP_TRACE_STAGES = 11


class HpSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("converged", c_int), ("correction", c_double),
                ("residual", c_double)]


EXPORTS = ["hp_mesh", "hp_workspace_bytes", "hp_build_matrix", "hp_factor", "hp_solve",
           "hp_lu_solve", "hp_rmatrix", "hp_smatrix", "hp_smatrix_noalloc", "hp_coulomb", "hp_coulomb_device",
           "hp_build_info", "hp_strerror", "hp_trace_enable", "hp_trace_read", "hp_last_error",
           "hp_gemm_sub", "hp_gemm_h3_sub", "hp_set_concurrency", "hp_set_solve_graphs", "hp_batch_workspace_bytes", "hp_batch_build",
           "hp_batch_factor", "hp_batch_factor_stepped", "hp_batch_solve_init", "hp_batch_refine_step", "hp_batch_active",
           "hp_batch_status", "hp_batch_rmatrix", "hp_batch_smatrix", "hp_kinetic_inverse",
           "hp_schur_workspace_bytes", "hp_build_schur", "hp_solve_schur", "hp_set_batch_reg_panel"]

_lib = None


class HprmatError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = ""
        if code == HP_ERR_HIP:
            try:
                detail = " [" + lib().hp_last_error().decode() + "]"
            except ImportError:
                pass
        super().__init__(f"{where}: {strerror(code)} ({code}){detail}")


def lib() -> ctypes.CDLL:
    """Load libhprmat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.hp_mesh.argtypes = [c_int, c_double, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hp_mesh.restype = c_int
    L.hp_workspace_bytes.argtypes = [c_int, c_int, c_int]
    L.hp_workspace_bytes.restype = c_size_t
    L.hp_build_matrix.argtypes = [P(HpSystem), c_double, c_int, c_void_p, c_long, c_void_p]
    L.hp_build_matrix.restype = c_int
    L.hp_factor.argtypes = [c_int, c_int, c_void_p, c_long, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_size_t, c_void_p]
    L.hp_factor.restype = c_int
    L.hp_solve.argtypes = [P(HpSystem), c_double, c_int, c_void_p, c_long, c_void_p, c_void_p,
                           c_void_p, c_int, c_double, c_void_p, c_size_t, P(HpSolveInfo), c_void_p]
    L.hp_solve.restype = c_int
    L.hp_kinetic_inverse.argtypes = [c_int, c_double, c_void_p]
    L.hp_kinetic_inverse.restype = c_int
    L.hp_schur_workspace_bytes.argtypes = [c_int, c_int, c_int]
    L.hp_schur_workspace_bytes.restype = c_size_t
    L.hp_build_schur.argtypes = [P(HpSystem), c_double, c_int, c_void_p, c_void_p, c_long, c_void_p]
    L.hp_build_schur.restype = c_int
    L.hp_solve_schur.argtypes = [P(HpSystem), c_double, c_int, c_void_p, c_void_p, c_long, c_void_p, c_void_p,
                                 c_void_p, c_int, c_double, c_void_p, c_size_t, P(HpSolveInfo), c_void_p]
    L.hp_solve_schur.restype = c_int
    L.hp_set_batch_reg_panel.argtypes = [c_int]
    L.hp_set_batch_reg_panel.restype = c_int
    L.hp_lu_solve.argtypes = [c_int, c_int, c_int, c_void_p, c_long, c_void_p, c_void_p, c_long,
                              c_void_p, c_size_t, c_void_p]
    L.hp_lu_solve.restype = c_int
    L.hp_gemm_sub.argtypes = [c_int, c_int, c_int, c_int, c_void_p, c_long, c_void_p, c_long, c_void_p,
                              c_long, c_void_p]
    L.hp_gemm_sub.restype = c_int
    L.hp_gemm_h3_sub.argtypes = [c_int, c_int, c_int, c_void_p, c_long, c_void_p, c_long, c_void_p, c_long,
                                 c_void_p, c_size_t, c_void_p]
    L.hp_gemm_h3_sub.restype = c_int
    L.hp_rmatrix.argtypes = [P(HpSystem), c_void_p, c_void_p, c_void_p]
    L.hp_rmatrix.restype = c_int
    L.hp_smatrix.argtypes = [P(HpSystem), c_double, c_void_p, c_void_p, P(c_int), c_void_p,
                             c_size_t, c_void_p]
    L.hp_smatrix.restype = c_int
    L.hp_smatrix_noalloc.argtypes = [P(HpSystem), c_double, c_void_p, c_void_p, P(c_int), c_void_p]
    L.hp_smatrix_noalloc.restype = c_int
    L.hp_coulomb.argtypes = [c_int, c_double, c_double, c_void_p]
    L.hp_coulomb.restype = c_int
    L.hp_coulomb_device.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hp_coulomb_device.restype = c_int
    L.hp_batch_workspace_bytes.argtypes = [c_int, c_long, c_long, c_int, c_int]
    L.hp_batch_workspace_bytes.restype = c_size_t
    L.hp_batch_build.argtypes = [c_int, c_void_p, c_int, c_void_p, c_void_p]
    L.hp_batch_build.restype = c_int
    L.hp_batch_factor.argtypes = [c_int, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                  c_void_p, c_size_t, c_void_p]
    L.hp_batch_factor.restype = c_int
    L.hp_batch_factor_stepped.argtypes = [c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_int, c_int, c_void_p, c_size_t, c_void_p]
    L.hp_batch_factor_stepped.restype = c_int
    L.hp_batch_solve_init.argtypes = [c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_int, c_long, c_long, c_void_p, c_size_t, c_void_p]
    L.hp_batch_solve_init.restype = c_int
    L.hp_batch_refine_step.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double,
                                       c_long, c_long, c_void_p, c_size_t, c_void_p]
    L.hp_batch_refine_step.restype = c_int
    L.hp_batch_smatrix.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_long, c_int, c_void_p,
                                   c_size_t, c_void_p]
    L.hp_batch_smatrix.restype = c_int
    L.hp_batch_active.argtypes = [c_void_p, P(ctypes.c_uint), c_void_p]
    L.hp_batch_active.restype = c_int
    L.hp_batch_status.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hp_batch_status.restype = c_int
    L.hp_batch_rmatrix.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.hp_batch_rmatrix.restype = c_int
    L.hp_set_concurrency.argtypes = [c_int]
    L.hp_set_concurrency.restype = c_int
    L.hp_set_solve_graphs.argtypes = [c_int]
    L.hp_set_solve_graphs.restype = c_int
    L.hp_trace_enable.argtypes = [c_int]
    L.hp_trace_enable.restype = c_int
    L.hp_trace_read.argtypes = [ctypes.POINTER(HpTraceStat), c_int]
    L.hp_trace_read.restype = c_int
    L.hp_last_error.argtypes = []
    L.hp_last_error.restype = ctypes.c_char_p
    L.hp_build_info.argtypes = []
    L.hp_build_info.restype = ctypes.c_char_p
    L.hp_strerror.argtypes = [c_int]
    L.hp_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().hp_strerror(code).decode()
    except ImportError:
        return f"code {code}"


def _check(code: int, where: str) -> int:
    if code != HP_OK:
        raise HprmatError(code, where)
    return code


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


# ------------------------------------------------------------------ host --

def hp_mesh(nr: int, a: float):
    """(r, w, q, tl) as numpy arrays (closed-form Lagrange-Legendre mesh)."""
    r = np.zeros(nr)
    w = np.zeros(nr)
    q = np.zeros(nr)
    tl = np.zeros((nr, nr))
    _check(lib().hp_mesh(nr, a, r.ctypes.data, w.ctypes.data, q.ctypes.data, tl.ctypes.data), "hp_mesh")
    return r, w, q, tl


def hp_workspace_bytes(n: int, nrhs: int, prec: int) -> int:
    return int(lib().hp_workspace_bytes(n, nrhs, prec))


def hp_kinetic_inverse(nr: int, a: float) -> np.ndarray:
    """The inverse of hp_mesh's tl, nr x nr host array (binary128 elimination)."""
    out = np.zeros((nr, nr))
    _check(lib().hp_kinetic_inverse(nr, a, out.ctypes.data), "hp_kinetic_inverse")
    return out


def hp_schur_workspace_bytes(n: int, nrhs: int, prec: int) -> int:
    return int(lib().hp_schur_workspace_bytes(n, nrhs, prec))


def hp_coulomb(l: int, eta: float, rho: float) -> np.ndarray:
    out = np.zeros(4)
    _check(lib().hp_coulomb(int(l), float(eta), float(rho), out.ctypes.data), "hp_coulomb")
    return out


def hp_build_info() -> str:
    return lib().hp_build_info().decode()


# ---------------------------------------------------------------- device --

def hp_build_matrix(sys: HpSystem, E: float, prec: int, C, ldc: int, stream=None) -> None:
    _check(lib().hp_build_matrix(ctypes.byref(sys), float(E), prec, _ptr(C), ldc, _stream(stream)),
           "hp_build_matrix")


def hp_factor(n: int, prec: int, A, lda: int, ipiv, perm, info, work, stream=None) -> None:
    _check(lib().hp_factor(n, prec, _ptr(A), lda, _ptr(ipiv), _ptr(perm), _ptr(info), _ptr(work),
                           work.numel() * work.element_size(), _stream(stream)), "hp_factor")


def hp_solve(sys: HpSystem, E: float, prec: int, LU, lda: int, perm, info_factor, X,
             max_refine: int, tol: float, work, stream=None, check: bool = True):
    """Returns (code, HpSolveInfo); raises on errors other than HP_ERR_NOCONV unless check=False."""
    info = HpSolveInfo()
    code = lib().hp_solve(ctypes.byref(sys), float(E), prec, _ptr(LU), lda, _ptr(perm),
                          _ptr(info_factor), _ptr(X), int(max_refine), float(tol), _ptr(work),
                          work.numel() * work.element_size(), ctypes.byref(info), _stream(stream))
    if check and code not in (HP_OK, HP_ERR_NOCONV, HP_ERR_SINGULAR):
        raise HprmatError(code, "hp_solve")
    return code, info


def hp_build_schur(sys: HpSystem, E: float, prec: int, kinv, S, lds: int, stream=None) -> None:
    _check(lib().hp_build_schur(ctypes.byref(sys), float(E), prec, _ptr(kinv), _ptr(S), lds, _stream(stream)),
           "hp_build_schur")


def hp_solve_schur(sys: HpSystem, E: float, prec: int, kinv, LU, lda: int, perm, info_factor, X,
                   max_refine: int, tol: float, work, stream=None, check: bool = True):
    """As hp_solve, through the factors of the Woodbury-kinetic matrix."""
    info = HpSolveInfo()
    code = lib().hp_solve_schur(ctypes.byref(sys), float(E), prec, _ptr(kinv), _ptr(LU), lda, _ptr(perm),
                                _ptr(info_factor), _ptr(X), int(max_refine), float(tol), _ptr(work),
                                work.numel() * work.element_size(), ctypes.byref(info), _stream(stream))
    if check and code not in (HP_OK, HP_ERR_NOCONV, HP_ERR_SINGULAR):
        raise HprmatError(code, "hp_solve_schur")
    return code, info


def hp_lu_solve(n: int, nrhs: int, prec: int, LU, lda: int, perm, X, ldx: int, work, stream=None) -> None:
    _check(lib().hp_lu_solve(n, nrhs, prec, _ptr(LU), lda, _ptr(perm), _ptr(X), ldx, _ptr(work),
                             work.numel() * work.element_size(), _stream(stream)), "hp_lu_solve")


def hp_gemm_sub(M: int, N: int, K: int, prec: int, A, lda: int, B, ldb: int, C, ldc: int,
                stream=None) -> None:
    _check(lib().hp_gemm_sub(M, N, K, prec, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, _stream(stream)),
           "hp_gemm_sub")


def hp_gemm_h3_sub(M: int, N: int, K: int, A, lda: int, B, ldb: int, C, ldc: int, work, stream=None) -> None:
    _check(lib().hp_gemm_h3_sub(M, N, K, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, _ptr(work),
                                work.numel() * work.element_size(), _stream(stream)), "hp_gemm_h3_sub")


def hp_rmatrix(sys: HpSystem, X, R, stream=None) -> None:
    _check(lib().hp_rmatrix(ctypes.byref(sys), _ptr(X), _ptr(R), _stream(stream)), "hp_rmatrix")


def hp_smatrix(sys: HpSystem, E: float, R, S, work, stream=None) -> int:
    nopen = c_int(0)
    _check(lib().hp_smatrix(ctypes.byref(sys), float(E), _ptr(R), _ptr(S), ctypes.byref(nopen),
                            _ptr(work), work.numel() * work.element_size(), _stream(stream)),
           "hp_smatrix")
    return int(nopen.value)


def hp_smatrix_noalloc(sys: HpSystem, E: float, R, S, stream=None) -> int:
    nopen = c_int(0)
    _check(lib().hp_smatrix_noalloc(ctypes.byref(sys), float(E), _ptr(R), _ptr(S), ctypes.byref(nopen),
                                    _stream(stream)), "hp_smatrix_noalloc")
    return int(nopen.value)


def hp_coulomb_device(l, eta, rho, out, stream=None) -> None:
    _check(lib().hp_coulomb_device(int(l.numel()), _ptr(l), _ptr(eta), _ptr(rho), _ptr(out),
                                   _stream(stream)), "hp_coulomb_device")


# ---- batched uneven systems (device item array: a uint8 tensor of HpBatchItem records)

def hp_batch_workspace_bytes(count: int, sum_nc: int, sum_xn: int, nmax: int, prec: int) -> int:
    return int(lib().hp_batch_workspace_bytes(count, sum_nc, sum_xn, nmax, prec))


def hp_batch_build(count, items, prec, A, stream=None) -> None:
    _check(lib().hp_batch_build(count, _ptr(items), prec, _ptr(A), _stream(stream)), "hp_batch_build")


def hp_batch_factor(count, items, prec, A, ipiv, perm, info, panel, groups, work, stream=None) -> None:
    _check(lib().hp_batch_factor(count, _ptr(items), prec, _ptr(A), _ptr(ipiv), _ptr(perm), _ptr(info), panel,
                                 groups, _ptr(work), work.numel(), _stream(stream)), "hp_batch_factor")


def hp_batch_factor_stepped(count, items, n_host, prec, A, ipiv, perm, info, panel, block, work,
                            stream=None) -> None:
    n = np.ascontiguousarray(n_host, dtype=np.int32)
    _check(lib().hp_batch_factor_stepped(count, _ptr(items), n.ctypes.data, prec, _ptr(A), _ptr(ipiv), _ptr(perm),
                                         _ptr(info), panel, block, _ptr(work), work.numel(), _stream(stream)),
           "hp_batch_factor_stepped")


def _shape(shape):
    return None if shape is None else np.ascontiguousarray(shape, dtype=np.int32)


def hp_batch_solve_init(count, items, shape, prec, LU, perm, info, X, refine, sum_nc, sum_xn, work,
                        stream=None) -> None:
    sh = _shape(shape)
    _check(lib().hp_batch_solve_init(count, _ptr(items), None if sh is None else sh.ctypes.data, prec, _ptr(LU),
                                     _ptr(perm), _ptr(info), _ptr(X), int(bool(refine)), sum_nc, sum_xn, _ptr(work),
                                     work.numel(), _stream(stream)), "hp_batch_solve_init")


def hp_batch_refine_step(count, items, shape, LU, perm, X, max_refine, tol, sum_nc, sum_xn, work,
                         stream=None) -> None:
    sh = _shape(shape)
    _check(lib().hp_batch_refine_step(count, _ptr(items), None if sh is None else sh.ctypes.data, _ptr(LU),
                                      _ptr(perm), _ptr(X), max_refine, tol, sum_nc, sum_xn, _ptr(work), work.numel(),
                                      _stream(stream)), "hp_batch_refine_step")


def hp_batch_active(work, stream=None) -> int:
    v = ctypes.c_uint(0)
    _check(lib().hp_batch_active(_ptr(work), ctypes.byref(v), _stream(stream)), "hp_batch_active")
    return int(v.value)


def hp_batch_status(count, work, stream=None):
    st = np.zeros(count, dtype=np.int32)
    it = np.zeros(count, dtype=np.int32)
    _check(lib().hp_batch_status(count, _ptr(work), st.ctypes.data, it.ctypes.data, _stream(stream)),
           "hp_batch_status")
    return st, it


def hp_batch_rmatrix(count, items, X, R, stream=None) -> None:
    _check(lib().hp_batch_rmatrix(count, _ptr(items), _ptr(X), _ptr(R), _stream(stream)), "hp_batch_rmatrix")


def hp_batch_smatrix(count, items, R, S, status, sum_nc2, nc_max, work, stream=None) -> None:
    _check(lib().hp_batch_smatrix(count, _ptr(items), _ptr(R), _ptr(S), _ptr(status), int(sum_nc2), int(nc_max),
                                  _ptr(work), work.numel() * work.element_size(), _stream(stream)),
           "hp_batch_smatrix")


def hp_set_batch_reg_panel(on: bool) -> int:
    """FP32 batched panels held in registers (default) or through memory;
    returns the previous setting."""
    return int(lib().hp_set_batch_reg_panel(int(bool(on))))


def hp_set_concurrency(factorizations: int) -> int:
    """Factorizations that may run at once on the device; returns the previous value."""
    rc = lib().hp_set_concurrency(int(factorizations))
    if rc < 0:
        raise HprmatError(rc, "hp_set_concurrency")
    return rc


def hp_set_solve_graphs(on: bool) -> bool:
    """Replay hp_solve's FP32 refinement solves from a HIP graph (default) or
    launch them one by one; returns the previous setting."""
    rc = lib().hp_set_solve_graphs(1 if on else 0)
    if rc < 0:
        raise HprmatError(rc, "hp_set_solve_graphs")
    return bool(rc)


TRACE_STAGES = ("assemble", "panel", "laswp", "trsm", "gemm_c128", "gemm_c64", "residual", "refine",
                "rmatrix", "smatrix", "gemm_f16x3")


def hp_trace_enable(on: bool = True, stages=None) -> None:
    """Start (clearing the record) or stop the per-stage timers; `stages`
    names the stages to time (default: all)."""
    if not on:
        mask = 0
    elif stages is None:
        mask = -1
    else:
        mask = 0
        for s in stages:
            mask |= 1 << TRACE_STAGES.index(s)
    _check(lib().hp_trace_enable(mask), "hp_trace_enable")


def hp_trace_read() -> dict:
    """{stage: dict(launches, ms, flops, bytes)} for the launches since hp_trace_enable(1)."""
    arr = (HpTraceStat * HP_TRACE_STAGES)()
    n = lib().hp_trace_read(arr, HP_TRACE_STAGES)
    if n < 0:
        raise HprmatError(n, "hp_trace_read")
    return {arr[i].name.decode(): dict(launches=int(arr[i].launches), ms=float(arr[i].ms),
                                       flops=float(arr[i].flops), bytes=float(arr[i].bytes))
            for i in range(n)}
