"""ctypes binding of libdctplus.so (argument marshalling only).

Every function here has the name of the C-ABI entry point it wraps (see
include/dctplus.h).  Device buffers are passed as integer addresses
(``tensor.data_ptr()``) and streams as integer handles
(``torch.cuda.current_stream().cuda_stream``).  No arithmetic of the
transform happens in Python.  Loading fails loudly when the library has not
been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdctplus.so")

DCTPLUS_OK = 0
DCTPLUS_EINVAL = 1
DCTPLUS_ENOMEM = 2
DCTPLUS_EDEVICE = 3
DCTPLUS_EUNSUPPORTED = 4
DCTPLUS_ENOCONV = 5
DCTPLUS_EDEGENERATE = 6

DCTPLUS_F32, DCTPLUS_F64, DCTPLUS_BF16, DCTPLUS_F32_SPLIT = 0, 1, 2, 3
DCTPLUS_ROUTE_AUTO, DCTPLUS_ROUTE_FAST, DCTPLUS_ROUTE_DENSE, DCTPLUS_ROUTE_GFT = 0, 1, 2, 3

EXPORTED = (
    "dctplus_default_opts", "dctplus_plan", "dctplus_forward", "dctplus_adjoint", "dctplus_grad",
    "dctplus_plan_info", "dctplus_plan_table", "dctplus_plan_destroy", "dctplus_status_string",
    "dctplus_last_error", "dctplus_select_plan", "dctplus_select", "dctplus_select_factor",
    "dctplus_select_size", "dctplus_select_destroy", "dctplus_select_tune", "dctplus_grad_noalloc",
    "dctplus_plan_rank_k", "dctplus_plan_general", "dctplus_tune",
)


class dctplus_opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32),
        ("route", ctypes.c_int32),
        ("defl_tol", ctypes.c_double),
        ("nufft_width", ctypes.c_int32),
        ("direct_kappa", ctypes.c_double),
        ("device", ctypes.c_int32),
        ("factored", ctypes.c_int32),
    ]


class DctPlusError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status} ({message})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2409_08970_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.dctplus_default_opts.argtypes = [ctypes.POINTER(dctplus_opts)]
    lib.dctplus_default_opts.restype = None
    lib.dctplus_plan.argtypes = [i64, ctypes.c_double, dp, ctypes.POINTER(dctplus_opts), vp,
                                 ctypes.POINTER(vp)]
    lib.dctplus_plan.restype = ctypes.c_int
    lib.dctplus_plan_rank_k.argtypes = [i64, ctypes.c_int32, dp, dp, ctypes.POINTER(dctplus_opts), vp,
                                        ctypes.POINTER(vp)]
    lib.dctplus_plan_rank_k.restype = ctypes.c_int
    lib.dctplus_plan_general.argtypes = [i64, dp, dp, ctypes.c_double, dp, ctypes.POINTER(dctplus_opts), vp,
                                         ctypes.POINTER(vp)]
    lib.dctplus_plan_general.restype = ctypes.c_int
    lib.dctplus_tune.argtypes = [vp, vp, vp, i64, vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_float)]
    lib.dctplus_tune.restype = ctypes.c_int
    lib.dctplus_forward.argtypes = [vp, vp, vp, i64, vp]
    lib.dctplus_forward.restype = ctypes.c_int
    lib.dctplus_adjoint.argtypes = [vp, vp, vp, i64, vp]
    lib.dctplus_adjoint.restype = ctypes.c_int
    lib.dctplus_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    lib.dctplus_grad.restype = ctypes.c_int
    lib.dctplus_grad_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    lib.dctplus_grad_noalloc.restype = ctypes.c_int
    lib.dctplus_plan_info.argtypes = [vp, dp, dp, dp, i32p, i32p]
    lib.dctplus_plan_info.restype = ctypes.c_int
    lib.dctplus_plan_table.argtypes = [vp, ctypes.c_char_p, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.dctplus_plan_table.restype = ctypes.c_int
    lib.dctplus_plan_destroy.argtypes = [vp]
    lib.dctplus_plan_destroy.restype = None
    lib.dctplus_status_string.argtypes = [ctypes.c_int]
    lib.dctplus_status_string.restype = ctypes.c_char_p
    lib.dctplus_last_error.argtypes = []
    lib.dctplus_last_error.restype = ctypes.c_char_p
    lib.dctplus_select_plan.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, i32p, dp, vp, ctypes.POINTER(vp)]
    lib.dctplus_select_plan.restype = ctypes.c_int
    lib.dctplus_select.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, vp, vp, vp, vp]
    lib.dctplus_select.restype = ctypes.c_int
    lib.dctplus_select_tune.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, vp, vp, vp, vp,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
    lib.dctplus_select_tune.restype = ctypes.c_int
    lib.dctplus_select_factor.argtypes = [vp, i64, ctypes.c_int32, dp]
    lib.dctplus_select_factor.restype = ctypes.c_int
    lib.dctplus_select_size.argtypes = [vp]
    lib.dctplus_select_size.restype = i64
    lib.dctplus_select_destroy.argtypes = [vp]
    lib.dctplus_select_destroy.restype = None
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != DCTPLUS_OK:
        lib = load()
        msg = lib.dctplus_last_error().decode(errors="replace")
        raise DctPlusError(status, where, msg or lib.dctplus_status_string(status).decode())


def dctplus_default_opts() -> dctplus_opts:
    o = dctplus_opts()
    load().dctplus_default_opts(ctypes.byref(o))
    return o


def dctplus_plan(n: int, rho: float, v, opts: dctplus_opts | None = None, stream: int = 0,
                 check: bool = True):
    """Returns (status, handle).  v: sequence of n floats (copied to a host double array)."""
    import numpy as np
    varr = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    handle = ctypes.c_void_p()
    st = load().dctplus_plan(int(n), float(rho), varr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ctypes.byref(opts) if opts is not None else None, ctypes.c_void_p(stream),
                             ctypes.byref(handle))
    if check:
        _check(st, "dctplus_plan")
    return st, handle


def dctplus_plan_rank_k(n: int, rhos, V, opts: dctplus_opts | None = None, stream: int = 0,
                        check: bool = True):
    """Returns (status, handle).  rhos: k floats; V: k x n (row j = v_j), copied."""
    import numpy as np
    r = np.ascontiguousarray(np.asarray(rhos, dtype=np.float64).reshape(-1))
    Varr = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))   # k x n, row-major
    handle = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    st = load().dctplus_plan_rank_k(int(n), int(r.size), r.ctypes.data_as(dp), Varr.ctypes.data_as(dp),
                                    ctypes.byref(opts) if opts is not None else None, ctypes.c_void_p(stream),
                                    ctypes.byref(handle))
    if check:
        _check(st, "dctplus_plan_rank_k")
    return st, handle


def dctplus_plan_general(n: int, lam, U, rho: float, v, opts: dctplus_opts | None = None, stream: int = 0,
                         check: bool = True):
    """Returns (status, handle).  lam: n base eigenvalues; U: n x n base basis (columns)."""
    import numpy as np
    dp = ctypes.POINTER(ctypes.c_double)
    la = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(-1))
    Ua = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(-1))
    va = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    handle = ctypes.c_void_p()
    st = load().dctplus_plan_general(int(n), la.ctypes.data_as(dp), Ua.ctypes.data_as(dp), float(rho),
                                     va.ctypes.data_as(dp), ctypes.byref(opts) if opts is not None else None,
                                     ctypes.c_void_p(stream), ctypes.byref(handle))
    if check:
        _check(st, "dctplus_plan_general")
    return st, handle


def dctplus_tune(plan, x_ptr: int, y_ptr: int, batch: int, stream: int = 0, cache_path: str | None = None,
                 check: bool = True):
    """Returns (status, chosen [2] ints, ms [16] floats)."""
    chosen = (ctypes.c_int32 * 2)()
    ms = (ctypes.c_float * 16)()
    st = load().dctplus_tune(plan, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), int(batch),
                             ctypes.c_void_p(stream), cache_path.encode() if cache_path else None, chosen, ms)
    if check:
        _check(st, "dctplus_tune")
    return st, list(chosen), list(ms)


def dctplus_forward(plan, x_ptr: int, y_ptr: int, batch: int, stream: int = 0, check: bool = True) -> int:
    st = load().dctplus_forward(plan, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), int(batch),
                                ctypes.c_void_p(stream))
    if check:
        _check(st, "dctplus_forward")
    return st


def dctplus_adjoint(plan, y_ptr: int, x_ptr: int, batch: int, stream: int = 0, check: bool = True) -> int:
    st = load().dctplus_adjoint(plan, ctypes.c_void_p(y_ptr), ctypes.c_void_p(x_ptr), int(batch),
                                ctypes.c_void_p(stream))
    if check:
        _check(st, "dctplus_adjoint")
    return st


def dctplus_grad(plan, y_ptr: int, gy_ptr: int, batch: int, gx_ptr: int, grho_ptr: int, gv_ptr: int,
                 stream: int = 0, check: bool = True) -> int:
    st = load().dctplus_grad(plan, ctypes.c_void_p(y_ptr), ctypes.c_void_p(gy_ptr), int(batch),
                             ctypes.c_void_p(gx_ptr or None), ctypes.c_void_p(grho_ptr or None),
                             ctypes.c_void_p(gv_ptr or None), ctypes.c_void_p(stream))
    if check:
        _check(st, "dctplus_grad")
    return st


def dctplus_grad_noalloc(plan, y_ptr: int, gy_ptr: int, batch: int, gx_ptr: int, grho_ptr: int, gv_ptr: int,
                         stream: int = 0, check: bool = True) -> int:
    st = load().dctplus_grad_noalloc(plan, ctypes.c_void_p(y_ptr), ctypes.c_void_p(gy_ptr), int(batch),
                                     ctypes.c_void_p(gx_ptr or None), ctypes.c_void_p(grho_ptr or None),
                                     ctypes.c_void_p(gv_ptr or None), ctypes.c_void_p(stream))
    if check:
        _check(st, "dctplus_grad_noalloc")
    return st


def dctplus_plan_info(plan, n: int):
    """Host copies: dict(mu, a, z, kind, counts)."""
    import numpy as np
    mu = np.zeros(n)
    a = np.zeros(n)
    z = np.zeros(n)
    kind = np.zeros(n, dtype=np.int32)
    counts = np.zeros(4, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    st = load().dctplus_plan_info(plan, mu.ctypes.data_as(dp), a.ctypes.data_as(dp), z.ctypes.data_as(dp),
                                  kind.ctypes.data_as(ip), counts.ctypes.data_as(ip))
    _check(st, "dctplus_plan_info")
    return dict(mu=mu, a=a, z=z, kind=kind, counts=counts)


_INT_TABLES = {"origin", "kind", "ref", "m0", "rowOfBin", "rowOfK", "direct_row", "ntie"}


def dctplus_plan_table(plan, name: str):
    """Host copy of one named plan table (numpy array)."""
    import numpy as np
    lib = load()
    size = ctypes.c_int64(0)
    _check(lib.dctplus_plan_table(plan, name.encode(), None, ctypes.byref(size)), "dctplus_plan_table")
    dt = np.int8 if name == "tune" else (np.int32 if name in _INT_TABLES else np.float64)
    out = np.zeros(size.value // np.dtype(dt).itemsize, dtype=dt)
    if size.value:
        _check(lib.dctplus_plan_table(plan, name.encode(), ctypes.c_void_p(out.ctypes.data), ctypes.byref(size)),
               "dctplus_plan_table")
    return out


def dctplus_plan_destroy(plan) -> None:
    if plan:
        load().dctplus_plan_destroy(plan)


def dctplus_select_plan(n_blocks, K: int, S: int, cand, stream: int = 0, check: bool = True):
    """Returns (status, handle).  n_blocks: nblocks ints; cand: nblocks*K*4 doubles (kind, i, j, w)."""
    import numpy as np
    nb = np.ascontiguousarray(np.asarray(n_blocks, dtype=np.int32).reshape(-1))
    cd = np.ascontiguousarray(np.asarray(cand, dtype=np.float64).reshape(-1))
    handle = ctypes.c_void_p()
    st = load().dctplus_select_plan(int(nb.size), int(K), int(S),
                                    nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if nb.size else None,
                                    cd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if cd.size else None,
                                    ctypes.c_void_p(stream), ctypes.byref(handle))
    if check:
        _check(st, "dctplus_select_plan")
    return st, handle


def dctplus_select_tune(plan, x_ptr: int, c_p: int, prune_tau: float, best_ptr: int, cost_ptr: int, y_ptr: int,
                        stream: int = 0, check: bool = True):
    """Returns (status, chosen workgroups per CU, [ms per call of each candidate])."""
    chosen = ctypes.c_int32(0)
    ms = (ctypes.c_float * 4)()
    st = load().dctplus_select_tune(plan, ctypes.c_void_p(x_ptr), int(c_p), float(prune_tau), ctypes.c_void_p(best_ptr),
                                    ctypes.c_void_p(cost_ptr), ctypes.c_void_p(y_ptr), ctypes.c_void_p(stream),
                                    ctypes.byref(chosen), ms)
    if check:
        _check(st, "dctplus_select_tune")
    return st, chosen.value, list(ms)


def dctplus_select(plan, x_ptr: int, c_p: int, prune_tau: float, best_ptr: int, cost_ptr: int, y_ptr: int,
                   stream: int = 0, check: bool = True) -> int:
    st = load().dctplus_select(plan, ctypes.c_void_p(x_ptr), int(c_p), float(prune_tau), ctypes.c_void_p(best_ptr),
                               ctypes.c_void_p(cost_ptr), ctypes.c_void_p(y_ptr), ctypes.c_void_p(stream))
    if check:
        _check(st, "dctplus_select")
    return st


def dctplus_select_factor(plan, block: int, r: int, n: int):
    """Host copy (n x n numpy float64) of candidate r's stored factor of one block."""
    import numpy as np
    out = np.zeros((n, n))
    _check(load().dctplus_select_factor(plan, int(block), int(r), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "dctplus_select_factor")
    return out


def dctplus_select_size(plan) -> int:
    return int(load().dctplus_select_size(plan))


def dctplus_select_destroy(plan) -> None:
    if plan:
        load().dctplus_select_destroy(plan)


def dctplus_status_string(status: int) -> str:
    return load().dctplus_status_string(int(status)).decode()


def dctplus_last_error() -> str:
    return load().dctplus_last_error().decode(errors="replace")
