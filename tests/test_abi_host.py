"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dctplus.h, and rejects bad arguments before any device
work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dctplus.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dctplus_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_08970_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        from paper_2409_08970_amd import build
        build.build()
    return B.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("dctplus_plan", "dctplus_forward", "dctplus_adjoint", "dctplus_grad",
                     "dctplus_plan_destroy", "dctplus_plan_info", "dctplus_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2409_08970_amd import _binding as B
    names = _declared_functions()
    missing = [nm for nm in names if not hasattr(lib, nm)]
    assert not missing, missing
    assert set(names) == set(B.EXPORTED)


def test_status_strings_and_defaults(lib):
    from paper_2409_08970_amd import _binding as B
    assert B.dctplus_status_string(0) == "ok"
    assert B.dctplus_status_string(1) == "invalid argument"
    assert B.dctplus_status_string(99) == "unknown status"
    o = B.dctplus_default_opts()
    assert (o.dtype, o.route, o.nufft_width, o.device, o.factored) == (0, 0, 0, -1, 0)
    assert o.defl_tol == 1e-13 and o.direct_kappa == 0.0   # 0: chosen per dtype at plan time


@pytest.mark.parametrize("n,rho,vfill,expect", [
    (1, 1.0, 0.0, 1),            # n < 2: EINVAL
    (3, 1.0, 0.0, 4),            # not a power of two: EUNSUPPORTED
    (32768, 1.0, 0.0, 4),        # above 16384: EUNSUPPORTED
    (64, float("nan"), 0.0, 1),  # non-finite rho
    (64, 1.0, float("inf"), 1),  # non-finite v
])
def test_plan_rejects_bad_arguments_on_host(lib, n, rho, vfill, expect):
    from paper_2409_08970_amd import _binding as B
    v = np.full(max(n, 1), vfill)
    st, h = B.dctplus_plan(n, rho, v, check=False)
    assert st == expect
    assert not h.value
    assert B.dctplus_last_error()


def test_plan_rejects_bad_options_on_host(lib):
    from paper_2409_08970_amd import _binding as B
    v = np.ones(64)
    for field, value, expect in [("dtype", 7, 1), ("route", 9, 1), ("nufft_width", 5, 1), ("nufft_width", 20, 1)]:
        o = B.dctplus_default_opts()
        setattr(o, field, value)
        st, h = B.dctplus_plan(64, 1.0, v, o, check=False)
        assert st == expect, (field, value)
    o = B.dctplus_default_opts()
    o.dtype = B.DCTPLUS_BF16
    o.route = B.DCTPLUS_ROUTE_DENSE
    assert B.dctplus_plan(128, 1.0, np.ones(128), o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    o = B.dctplus_default_opts()
    o.dtype = B.DCTPLUS_F32_SPLIT
    assert B.dctplus_plan(8192, 1.0, np.ones(8192), o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    assert B.dctplus_plan(16, 1.0, np.ones(16), o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    o = B.dctplus_default_opts()
    o.dtype = B.DCTPLUS_BF16
    o.route = B.DCTPLUS_ROUTE_FAST
    assert B.dctplus_plan(64, 1.0, v, o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    # the factored form: 0 or 1, DENSE route, F32, BF16 or F32_SPLIT (split: n = 64 only)
    for route, dtype, fac, expect in [(B.DCTPLUS_ROUTE_DENSE, B.DCTPLUS_F32, 2, B.DCTPLUS_EINVAL),
                                      (B.DCTPLUS_ROUTE_GFT, B.DCTPLUS_F32, 1, B.DCTPLUS_EUNSUPPORTED),
                                      (B.DCTPLUS_ROUTE_DENSE, B.DCTPLUS_F64, 1, B.DCTPLUS_EUNSUPPORTED)]:
        o = B.dctplus_default_opts()
        o.route, o.dtype, o.factored = route, dtype, fac
        assert B.dctplus_plan(64, 1.0, v, o, check=False)[0] == expect, (route, dtype, fac)
    o = B.dctplus_default_opts()
    o.route, o.dtype, o.factored = B.DCTPLUS_ROUTE_DENSE, B.DCTPLUS_F32_SPLIT, 1
    assert B.dctplus_plan(32, 1.0, np.ones(32), o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    # null v and null output pointer
    assert lib.dctplus_plan(64, 1.0, None, None, None, ctypes.byref(ctypes.c_void_p())) == 1
    assert lib.dctplus_plan(64, 1.0, None, None, None, None) == 1


def test_calls_on_null_plan_are_rejected(lib):
    assert lib.dctplus_forward(None, ctypes.c_void_p(16), ctypes.c_void_p(32), 4, None) == 1
    assert lib.dctplus_adjoint(None, ctypes.c_void_p(16), ctypes.c_void_p(32), 4, None) == 1
    assert lib.dctplus_grad(None, None, None, 4, None, None, None, None) == 1
    assert lib.dctplus_grad_noalloc(None, None, None, 4, None, None, None, None) == 1
    assert lib.dctplus_plan_info(None, None, None, None, None, None) == 1
    lib.dctplus_plan_destroy(None)
    from paper_2409_08970_amd import _binding as B
    B.load()
    assert lib.dctplus_select(None, None, 0, 0.1, None, None, None, None) == 1
    assert lib.dctplus_select_tune(None, None, 0, 0.1, None, None, None, None, None, None) == 1
    assert lib.dctplus_select_size(None) == -1
    lib.dctplus_select_destroy(None)


@pytest.mark.parametrize("nb,K,S,cand_row,expect", [
    ([64], 0, 64, (0, 0, 0, 1.0), 1),          # K < 1
    ([64], 17, 64, (0, 0, 0, 1.0), 1),         # K > 16
    ([64], 2, 0, (0, 0, 0, 1.0), 1),           # S < 1
    ([64], 2, 65, (0, 0, 0, 1.0), 1),          # S > 64
    ([48], 2, 64, (0, 0, 0, 1.0), 4),          # block size outside {4, ..., 64}: EUNSUPPORTED
    ([128], 2, 64, (0, 0, 0, 1.0), 4),
    ([64], 2, 64, (2, 0, 0, 1.0), 1),          # unknown kind
    ([64], 2, 64, (1, 3, 3, 1.0), 1),          # edge with i == j
    ([64], 2, 64, (0, 64, 0, 1.0), 1),         # vertex out of range
    ([64], 2, 64, (0, 1.5, 0, 1.0), 1),        # non-integer vertex
    ([64], 2, 64, (0, 0, 0, 0.0), 1),          # weight <= 0
    ([64], 2, 64, (0, 0, 0, float("nan")), 1),
])
def test_select_plan_rejects_bad_arguments_on_host(lib, nb, K, S, cand_row, expect):
    from paper_2409_08970_amd import _binding as B
    cand = np.tile(np.asarray(cand_row, dtype=np.float64), (len(nb), max(K, 1), 1))
    st, h = B.dctplus_select_plan(nb, K, S, cand, check=False)
    assert st == expect
    assert not h.value
    assert B.dctplus_last_error()


def test_select_calls_on_null_plan_are_rejected(lib):
    assert lib.dctplus_select(None, ctypes.c_void_p(16), 0, 0.1, ctypes.c_void_p(16), ctypes.c_void_p(16),
                              ctypes.c_void_p(16), None) == 1
    out = np.zeros(16)
    assert lib.dctplus_select_factor(None, 0, 0, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 1
    assert lib.dctplus_select_size(None) == -1
    assert lib.dctplus_select_plan(1, 2, 64, None, None, None, ctypes.byref(ctypes.c_void_p())) == 1
    lib.dctplus_select_destroy(None)


def test_rank_k_plan_rejects_bad_arguments_on_host(lib):
    from paper_2409_08970_amd import _binding as B
    n = 64
    V = np.ones((2, n)) / 8.0
    assert B.dctplus_plan_rank_k(n, [], np.zeros((0, n)), check=False)[0] == B.DCTPLUS_EINVAL        # k = 0
    assert B.dctplus_plan_rank_k(n, np.ones(65), np.ones((65, n)), check=False)[0] == B.DCTPLUS_EINVAL
    bad = V.copy()
    bad[1, 3] = np.nan
    assert B.dctplus_plan_rank_k(n, [1.0, 1.0], bad, check=False)[0] == B.DCTPLUS_EINVAL
    assert B.dctplus_plan_rank_k(n, [1.0, np.inf], V, check=False)[0] == B.DCTPLUS_EINVAL
    assert B.dctplus_plan_rank_k(8192, [1.0, 1.0], np.ones((2, 8192)), check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    o = B.dctplus_default_opts()
    o.route = B.DCTPLUS_ROUTE_FAST
    assert B.dctplus_plan_rank_k(n, [1.0, 1.0], V, o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    assert lib.dctplus_plan_rank_k(n, 2, None, None, None, None, None) == B.DCTPLUS_EINVAL


def test_general_plan_rejects_bad_arguments_on_host(lib):
    from paper_2409_08970_amd import _binding as B
    n = 16
    lam = np.arange(n, dtype=np.float64)
    U = np.eye(n)
    v = np.ones(n) / 4.0
    lam_bad = lam.copy()
    lam_bad[5] = lam_bad[4]
    assert B.dctplus_plan_general(n, lam_bad, U, 1.0, v, check=False)[0] == B.DCTPLUS_EINVAL
    U_bad = U.copy()
    U_bad[2, 3] = np.nan
    assert B.dctplus_plan_general(n, lam, U_bad, 1.0, v, check=False)[0] == B.DCTPLUS_EINVAL
    assert B.dctplus_plan_general(12, np.arange(12.0), np.eye(12), 1.0, np.ones(12), check=False)[0] == \
        B.DCTPLUS_EUNSUPPORTED
    o = B.dctplus_default_opts()
    o.route = B.DCTPLUS_ROUTE_FAST
    assert B.dctplus_plan_general(n, lam, U, 1.0, v, o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    o = B.dctplus_default_opts()
    o.factored = 1
    assert B.dctplus_plan_general(n, lam, U, 1.0, v, o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    assert lib.dctplus_plan_general(n, None, None, ctypes.c_double(1.0), None, None, None, None) == B.DCTPLUS_EINVAL
