"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (FP32 signals): max over signals of ||y - y_ref|| / ||y_ref|| <= 1e-5,
the accuracy the paper reports for its fast transform (SNR above 100 dB,
Sec. 5 and Table 1).  FP64 signals: 1e-12.  BF16 operands: 2e-2 (an
8-bit-mantissa product; stated separately, never as 1e-5).

Reference: the Jacobi oracle (plain definition) where the spectrum is simple
and n <= 256; the secular semi-oracle (Thm 3.1 by bisection, itself pinned to
Jacobi in test_oracle_pins) for larger n and for the double eigenvalues some
added edges produce, where it fixes the canonical deflation basis.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
TOLBF16 = 2e-2


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def relerr(y, yref):
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    num = np.linalg.norm(y - yref, axis=-1)
    den = np.maximum(np.linalg.norm(yref, axis=-1), 1e-300)
    return float(np.max(num / den))


def case(n, kind, seed=0):
    g = np.random.default_rng(10_000 + 17 * n + seed)
    if kind == "dense":
        return float(g.uniform(0.1, 2.0)), workloads.unit_vector(g, n)
    if kind == "loop0":
        v = np.zeros(n); v[0] = 1.0
        return float(g.uniform(0.25, 2.0)), v
    if kind == "loopn":
        v = np.zeros(n); v[-1] = 1.0
        return float(g.uniform(0.25, 2.0)), v
    if kind == "edge":
        i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
        return 2.0, workloads.edge_vector(n, i, j)
    if kind == "negative":
        return -float(g.uniform(0.1, 1.0)), workloads.unit_vector(g, n)
    raise ValueError(kind)


_REF_CACHE = {}


def reference(n, rho, v):
    """(forward, adjoint) callables of the oracle for this (n, rho, v)."""
    key = (n, rho, v.tobytes())
    if key in _REF_CACHE:
        return _REF_CACHE[key]
    plan = oracle.semi_plan(n, rho, v) if rho != 0.0 else None
    simple = True
    if plan is not None:
        simple = np.min(np.diff(plan["mu"])) > 1e-9
    if n <= 256 and simple:
        _, X = oracle.basis(n, rho, v)
        fwd = lambda x: oracle.forward(X, x)
        adj = lambda y: oracle.adjoint(X, y)
    else:
        fwd = lambda x: oracle.semi_forward(n, rho, v, x, plan)
        adj = lambda y: oracle.semi_adjoint(n, rho, v, y, plan)
    _REF_CACHE[key] = (fwd, adj)
    return fwd, adj


def run(plan, arr, adjoint=False):
    torch = _torch()
    dt = torch.float64 if plan.dtype == "f64" else torch.float32
    t = torch.from_numpy(np.ascontiguousarray(arr)).to("cuda", dt)
    out = plan.adjoint(t) if adjoint else plan.forward(t)
    torch.cuda.synchronize()
    return out.cpu().double().numpy()


def make_plan(n, rho, v, route, dtype="f32", **kw):
    """route "dense-factored": the DENSE route with the two factors of Thm 3.1 kept
    apart (DCT-II on the GPU, then the Cauchy factor)."""
    _torch()
    from paper_2409_08970_amd import Plan
    if route == "dense-factored":
        return Plan(n, rho, v, route="dense", dtype=dtype, factored=True, **kw)
    return Plan(n, rho, v, route=route, dtype=dtype, **kw)


# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 64, 1024])
@pytest.mark.parametrize("kind", ["dense", "loop0", "edge", "negative"])
def test_plan_spectrum_matches_oracle(n, kind):
    rho, v = case(n, kind)
    p = make_plan(n, rho, v, "fast")
    sp = oracle.semi_plan(n, rho, v)
    info = p.info
    assert np.abs(info["mu"] - sp["mu"]).max() <= 1e-12 * max(1.0, np.abs(sp["mu"]).max())
    assert np.abs(info["z"] - sp["z"]).max() <= 1e-13
    lam = oracle.path_eigenvalues(n)
    a_ref = np.ones(n)
    for i in range(n):
        if sp["kind"][i] == 0:
            nz = sp["z"] != 0
            a_ref[i] = 1.0 / np.sqrt(np.sum(sp["z"][nz] ** 2 / (sp["mu"][i] - lam[nz]) ** 2))
    assert np.abs(info["a"] - a_ref).max() <= 1e-10 * np.abs(a_ref).max()
    assert int(info["counts"][0]) == int(np.sum(sp["kind"]))
    p.close()


ROUTE_SIZES = [("fast", n) for n in (4, 8, 16, 32, 64, 128, 256, 1024)] + \
              [("dense", n) for n in (4, 8, 16, 32, 64, 128, 256)] + \
              [("gft", n) for n in (4, 8, 16, 32, 64, 128, 256)] + \
              [("dense-factored", n) for n in (4, 8, 16, 32, 64, 128, 256, 1024)]


@pytest.mark.parametrize("route,n", ROUTE_SIZES)
@pytest.mark.parametrize("kind", ["dense", "loop0", "loopn", "edge", "negative"])
def test_forward_and_adjoint_parity(route, n, kind):
    rho, v = case(n, kind)
    batch = 301                     # several tiles plus a ragged tail
    g = np.random.default_rng(n + 7)
    x = workloads.ar1(g, batch, n, 0.95)
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, route)
    y = run(p, x)
    assert relerr(y, fwd(x.astype(np.float64))) <= TOL32, (route, n, kind)
    yin = g.standard_normal((batch, n)).astype(np.float32)
    xa = run(p, yin, adjoint=True)
    assert relerr(xa, adj(yin.astype(np.float64))) <= TOL32, (route, n, kind)
    p.close()


@pytest.mark.parametrize("route", ["fast", "dense"])
@pytest.mark.parametrize("n", [1024, 2048, 4096, 8192, 16384])
@pytest.mark.parametrize("kind", ["dense", "edge"])
def test_large_n_full_batch_sampled(route, n, kind):
    """Workload-3 shape (256 N(0,1) signals): the whole batch runs on the GPU,
    sampled signals are checked against the semi-oracle, and the intertwining
    property X^T (L s) = mu * X^T s and Parseval are checked on every signal."""
    torch = _torch()
    W = workloads.workload3(n, kind)
    rho, v, x = W["rho"], W["v"], W["x"]
    p = make_plan(n, rho, v, route)
    y = run(p, x)
    rows = [0, 77, 255]
    sp = oracle.semi_plan(n, rho, v)
    yref = oracle.semi_forward(n, rho, v, x[rows].astype(np.float64), sp)
    assert relerr(y[rows], yref) <= TOL32
    xr = run(p, y.astype(np.float32), adjoint=True)
    assert relerr(xr, x) <= 2 * TOL32
    # Parseval (X orthogonal)
    assert np.max(np.abs(np.linalg.norm(y, axis=1) / np.linalg.norm(x, axis=1) - 1)) <= TOL32
    # intertwining: L s for every signal (tridiagonal plus rank one, FP64 on the host)
    xd = x.astype(np.float64)
    Ls = 2 * xd
    Ls[:, 0] -= xd[:, 0]
    Ls[:, -1] -= xd[:, -1]
    Ls[:, 1:] -= xd[:, :-1]
    Ls[:, :-1] -= xd[:, 1:]
    Ls += rho * np.outer(xd @ v, v)
    yL = run(p, Ls.astype(np.float32))
    mu = p.info["mu"]
    assert relerr(yL, mu * y) <= 4 * TOL32
    p.close()
    del torch


@pytest.mark.parametrize("route", ["fast", "dense", "gft"])
def test_rho_zero_and_v_zero_give_dct2(route):
    import scipy.fft
    n = 64
    x = np.random.default_rng(3).standard_normal((130, n)).astype(np.float32)
    ref = scipy.fft.dct(x.astype(np.float64), type=2, norm="ortho", axis=-1)
    for rho, v in [(0.0, workloads.unit_vector(np.random.default_rng(1), n)), (1.5, np.zeros(n))]:
        p = make_plan(n, rho, v, route)
        assert relerr(run(p, x), ref) <= TOL32
        assert int(p.info["counts"][0]) == n      # every row deflated
        p.close()


@pytest.mark.parametrize("route", ["fast", "dense", "gft"])
@pytest.mark.parametrize("n", [16, 64, 256])
def test_double_eigenvalues_from_mirror_edge(route, n):
    """A mirror-symmetric added edge makes a secular root land on a deflated
    eigenvalue; the deflation basis is the canonical one (semi-oracle)."""
    v = workloads.edge_vector(n, 2, n - 3)
    rho = 2.0
    x = workloads.ar1(np.random.default_rng(5), 200, n, 0.9)
    sp = oracle.semi_plan(n, rho, v)
    assert np.min(np.diff(sp["mu"])) < 1e-9
    p = make_plan(n, rho, v, route)
    assert relerr(run(p, x), oracle.semi_forward(n, rho, v, x.astype(np.float64), sp)) <= TOL32
    p.close()


def test_auto_route_small_batches_at_1024():
    """AUTO at n = 1024 keeps the dense product for large batches and runs calls of fewer
    than 1,024 signals on the FAST route (measured faster there): bit-identical to an
    explicit FAST plan below the switch and to a DENSE plan at and above it, and within
    the FP32 bar of the semi-oracle on both sides."""
    n = 1024
    rho, v = case(n, "dense")
    sp = oracle.semi_plan(n, rho, v)
    g = np.random.default_rng(77)
    pa, pf, pd = make_plan(n, rho, v, "auto"), make_plan(n, rho, v, "fast"), make_plan(n, rho, v, "dense")
    assert pa.route == "dense"
    for batch, twin in [(1, pf), (300, pf), (1023, pf), (1024, pd), (1500, pd)]:
        x = g.standard_normal((batch, n)).astype(np.float32)
        ya = run(pa, x)
        assert np.array_equal(ya, run(twin, x)), batch
        xa = run(pa, x, adjoint=True)
        assert np.array_equal(xa, run(twin, x, adjoint=True)), batch
        rows = [0, batch // 2, batch - 1]
        assert relerr(ya[rows], oracle.semi_forward(n, rho, v, x[rows].astype(np.float64), sp)) <= TOL32
    pa.close(); pf.close(); pd.close()


@pytest.mark.parametrize("n,dtype,expect", [(64, "f32", "dense"), (1024, "f32", "dense"), (2048, "f32", "fast"),
                                            (4096, "f32", "fast"), (16384, "f32", "fast"), (4096, "f64", "dense"),
                                            (16384, "bf16", None), (64, "f64", "dense")])
def test_auto_route_choice(n, dtype, expect):
    """AUTO takes the route measured faster on this GPU for FP32 signals: the dense
    product up to n = 1024, the O(n log n) route from n = 2048.  FP64 plans keep the
    dense product (1e-12); BF16 operands exist on the dense route only, n in {32, 64}."""
    _torch()
    from paper_2409_08970_amd import Plan, _binding as B
    v = workloads.unit_vector(np.random.default_rng(n), n)
    if expect is None:
        with pytest.raises(B.DctPlusError):
            Plan(n, 0.5, v, route="auto", dtype=dtype)
        return
    p = Plan(n, 0.5, v, route="auto", dtype=dtype)
    assert p.route == expect
    p.close()


@pytest.mark.parametrize("route", ["fast", "dense", "gft", "auto"])
def test_fp64_self_loop_dst7(route):
    """Workload 1: n = 64, unit self-loop at vertex 0, 1024 N(0,1) signals in FP64;
    the basis is the DST-VII closed form."""
    W = workloads.workload1()
    n = W["n"]
    p = make_plan(n, W["rho"], W["v"], route, dtype="f64")
    y = run(p, W["x"])
    j = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    X = 2.0 / np.sqrt(2 * n + 1) * np.sin(np.pi * (2 * k + 1) * (j + 1) / (2 * n + 1))
    assert relerr(y, W["x"] @ X) <= TOL64
    _, Xj = oracle.basis(n, W["rho"], W["v"])
    assert relerr(y, oracle.forward(Xj, W["x"])) <= TOL64
    xr = run(p, y, adjoint=True)
    assert relerr(xr, W["x"]) <= TOL64
    p.close()


TOL_FAST64 = 1e-11


@pytest.mark.parametrize("n", [8192, 16384])
def test_fp64_fast_parity_buffer_in_global_memory(n):
    """FP64 signals on the FAST route where the per-signal buffer lives in global
    memory and the FFTs are staged through LDS (a 64 KiB stage at n = 8192, 16 KiB at
    n = 16384): the workload-3 graph (dense v, rho = 0.5) on two signals against the
    secular semi-oracle, forward and adjoint.  The bar grows with n: the h-scale of
    Alg. 1 step 4 divides by sin(pi j / n) >= sin(pi / n) ~ pi / n, so the rounding of
    the FP64 transforms after it, relative to the output, grows in proportion to n;
    1e-11 holds with a 5x margin up to n = 4096 (below), hence 1e-11 * n / 4096."""
    W = workloads.workload3(n, "dense", batch=2)
    rho, v = W["rho"], W["v"]
    x = W["x"].astype(np.float64)
    yin = np.random.default_rng(n + 1).standard_normal((2, n))
    p = make_plan(n, rho, v, "fast", dtype="f64")
    y = run(p, x)
    xa = run(p, yin, adjoint=True)
    p.close()
    sp = oracle.semi_plan(n, rho, v)
    tol = TOL_FAST64 * n / 4096
    assert relerr(y, oracle.semi_forward(n, rho, v, x, sp)) <= tol, n
    assert relerr(xa, oracle.semi_adjoint(n, rho, v, yin, sp)) <= tol, n


@pytest.mark.parametrize("n,batch", [(8, 75), (64, 75), (256, 75), (1024, 20), (4096, 4)])
@pytest.mark.parametrize("kind", ["dense", "loopn", "edge", "negative"])
def test_fp64_fast_parity(n, batch, kind):
    """FP64 signals on the FAST route.  Thm 3.3 is exact up to the NUFFT error: 16
    window taps leave ~1e-15 per interpolated value, and rows that would amplify it
    by more than 1e3 (small sin(n psi)) are summed exactly, so the bar is 1e-11
    against the secular semi-oracle (1e-12 for the dense routes)."""
    rho, v = case(n, kind)
    g = np.random.default_rng(5 * n + 3)
    x = g.standard_normal((batch, n))
    yin = g.standard_normal((batch, n))
    p = make_plan(n, rho, v, "fast", dtype="f64")
    y = run(p, x)
    xa = run(p, yin, adjoint=True)
    p.close()
    sp = oracle.semi_plan(n, rho, v)
    assert relerr(y, oracle.semi_forward(n, rho, v, x, sp)) <= TOL_FAST64, (n, kind)
    assert relerr(xa, oracle.semi_adjoint(n, rho, v, yin, sp)) <= TOL_FAST64, (n, kind)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL_FAST64), ("f32", TOL32)])
def test_fast_roots_past_their_origin_bin(dtype, tol):
    """Edge (16, 47) at n = 64 deflates lambda_k between some roots and their nearer
    non-deflated pole, so those roots lie one Chebyshev bin past the pole's: each NUFFT
    row's bin must be the bin (theta_b, theta_b+1) of its own root angle (with every
    window tap inside the aligned table), and the transform keeps its bar."""
    from paper_2409_08970_amd import dctplus_plan_table
    n = 64
    v = workloads.edge_vector(n, 16, 47)
    sp = oracle.semi_plan(n, 2.0, v)
    psi = 2.0 * np.arcsin(np.sqrt(np.clip(sp["mu"], 0.0, 4.0)) / 2.0)
    bins = np.floor(psi * n / np.pi).astype(int)
    lam_o = oracle.path_eigenvalues(n)[sp["origin"]]
    past = [i for i in range(n) if sp["kind"][i] == 0 and bins[i] != (sp["origin"][i] - (sp["tau"][i] < 0))]
    assert len(past) >= 4 and np.all(lam_o[past] > 0)
    p = make_plan(n, 2.0, v, "fast", dtype=dtype)
    kind = dctplus_plan_table(p.handle, "kind")
    ref = dctplus_plan_table(p.handle, "ref")
    nufft = np.nonzero(kind == 0)[0]
    assert set(past) & set(nufft.tolist())
    assert np.array_equal(ref[nufft], bins[nufft])
    g = np.random.default_rng(64)
    x = g.standard_normal((100, n))
    y = run(p, x.astype(np.float32) if dtype == "f32" else x)
    xa = run(p, x.astype(np.float32) if dtype == "f32" else x, adjoint=True)
    p.close()
    xin = x.astype(np.float32).astype(np.float64) if dtype == "f32" else x
    assert relerr(y, oracle.semi_forward(n, 2.0, v, xin, sp)) <= tol
    assert relerr(xa, oracle.semi_adjoint(n, 2.0, v, xin, sp)) <= tol


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 64, 1024])
def test_fast_spreading_is_the_transpose_of_the_interpolation(dtype, n):
    """The adjoint's spreading table (per grid point, folds merged in) against the
    forward's window table (per bin): <u, I G> = <S u, G> for random bin values u and
    grid values G_1..G_{2n-1}, the interpolation I reading the grid's odd extension
    (G(-p) = -G(p), G(4n - p) = -G(p), G_0 = G_2n = 0) at 2b + 1 - w/2 + k."""
    _torch()
    from paper_2409_08970_amd import dctplus_plan_table
    rho, v = case(n, "dense")
    p = make_plan(n, rho, v, "fast", dtype=dtype)
    w = int(p.info["counts"][2])                 # the plan's window width
    hw = w // 2
    taps = 18
    wina = dctplus_plan_table(p.handle, "wina").reshape(taps, n)
    wspr = dctplus_plan_table(p.handle, "wspr").reshape(10, 2 * n)
    p.close()
    g = np.random.default_rng(n)
    u = g.standard_normal(n)
    u[n - 1] = 0.0                               # bins are 0 .. n - 2
    Gin = np.zeros(2 * n + 1)
    Gin[1:2 * n] = g.standard_normal(2 * n - 1)

    def grid(q):                                 # odd extension, period 4n
        q %= 4 * n
        return Gin[q] if q <= 2 * n else -Gin[4 * n - q]
    lhs = 0.0
    for b in range(n - 1):
        t = sum(wina[k, b] * grid(2 * b + 1 - hw + k) for k in range(taps))
        lhs += u[b] * t
    rhs = 0.0
    for P in range(1, 2 * n):
        blo = max(0, ((P - hw - 3) >> 1) + 1)
        Sp = sum(wspr[k, P] * u[min(blo + k, n - 1)] for k in range(10))
        rhs += Sp * Gin[P]
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, np.abs(wina).sum() * np.abs(u).max() * np.abs(Gin).max())
    # no weight past the bins that reach a grid point at this width
    assert np.all(wspr[hw + 2:] == 0.0)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_fast_route_exact_row_threshold(n):
    """direct_kappa bounds the NUFFT error amplification a row may have before it is
    summed exactly.  At 1e-9 every row of these plans is exact, and the FAST route
    then reproduces the Cauchy product to FP64 rounding; a threshold that would need
    more exact rows than the kernels hold is refused at plan time."""
    _torch()
    from paper_2409_08970_amd import Plan, _binding as B
    rho, v = case(n, "dense")
    x = np.random.default_rng(n).standard_normal((40, n))
    p = make_plan(n, rho, v, "fast", dtype="f64", direct_kappa=1e-9)
    assert int(p.info["counts"][1]) == n               # every row exact (no deflation here)
    y = run(p, x)
    p.close()
    sp = oracle.semi_plan(n, rho, v)
    assert relerr(y, oracle.semi_forward(n, rho, v, x, sp)) <= TOL64
    with pytest.raises(B.DctPlusError):
        Plan(4096, rho, workloads.unit_vector(np.random.default_rng(1), 4096), route="fast", direct_kappa=1e-9)


@pytest.mark.parametrize("n,dtype", [(4096, "f32"), (8192, "f32"), (4096, "f64")])
def test_fast_many_exact_rows_one_signal_per_workgroup(n, dtype):
    """The FAST kernels that hold one signal per workgroup (n >= 4096) sum the exact
    rows a group of eight at a time, every thread taking its share of the samples.
    Lowering direct_kappa makes dozens of rows exact (several groups and a ragged
    last one); forward and adjoint against the semi-oracle."""
    _torch()
    from paper_2409_08970_amd import _binding as B
    rho, v = case(n, "dense")
    p, nd = None, 0
    for kappa in np.geomspace(1e3, 1.0, 25):
        try:
            q = make_plan(n, rho, v, "fast", dtype=dtype, direct_kappa=float(kappa))
        except B.DctPlusError:                     # more exact rows than the kernels hold
            break
        if p is not None:
            p.close()
        p, nd = q, int(q.info["counts"][1])
        if nd >= 17 and nd % 8 != 0:
            break
    assert p is not None and nd >= 17 and nd % 8 != 0, nd
    g = np.random.default_rng(n + 7)
    x = g.standard_normal((6, n))
    yin = g.standard_normal((6, n))
    tol = TOL32 if dtype == "f32" else TOL_FAST64 * n / 4096
    io = np.float32 if dtype == "f32" else np.float64
    y = run(p, x.astype(io))
    xa = run(p, yin.astype(io), adjoint=True)
    p.close()
    sp = oracle.semi_plan(n, rho, v)
    assert relerr(y, oracle.semi_forward(n, rho, v, x.astype(io).astype(np.float64), sp)) <= tol, nd
    assert relerr(xa, oracle.semi_adjoint(n, rho, v, yin.astype(io).astype(np.float64), sp)) <= tol, nd


@pytest.mark.parametrize("route", ["dense", "gft"])
@pytest.mark.parametrize("n", [4, 8, 16, 32, 64, 128, 256, 1024])
@pytest.mark.parametrize("kind", ["dense", "loopn", "edge", "negative"])
def test_fp64_dense_parity(route, n, kind):
    """FP64 signals: 1e-12 against the secular semi-oracle, and against the
    Jacobi eigenvectors (simple spectra, n <= 256) within their own conditioning,
    100 eps ||L|| / (smallest eigenvalue gap): the first-order error bound of a
    backward-stable eigensolver, which exceeds 1e-12 once gaps fall below ~1e-3."""
    rho, v = case(n, kind)
    batch = 75                      # one full 64-signal tile and a ragged tail
    g = np.random.default_rng(3 * n + 1)
    x = g.standard_normal((batch, n))
    yin = g.standard_normal((batch, n))
    p = make_plan(n, rho, v, route, dtype="f64")
    y = run(p, x)
    xa = run(p, yin, adjoint=True)
    p.close()
    sp = oracle.semi_plan(n, rho, v)
    assert relerr(y, oracle.semi_forward(n, rho, v, x, sp)) <= TOL64, (route, n, kind)
    assert relerr(xa, oracle.semi_adjoint(n, rho, v, yin, sp)) <= TOL64, (route, n, kind)
    mu = np.linalg.eigvalsh(oracle.laplacian(n, rho, v))
    gaps = np.diff(mu)
    if n <= 256 and gaps.min() > 1e-9:
        tol = max(TOL64, 100 * np.finfo(float).eps * (4 + abs(rho) * float(v @ v)) / gaps.min())
        _, X = oracle.basis(n, rho, v)
        assert relerr(y, oracle.forward(X, x)) <= tol, (route, n, kind, tol)
        assert relerr(xa, oracle.adjoint(X, yin)) <= tol, (route, n, kind, tol)


@pytest.mark.parametrize("route", ["dense", "gft", "dense-factored"])
@pytest.mark.parametrize("n", [32, 64])
def test_bf16_operands(route, n):
    rho, v = case(n, "dense")
    x = workloads.ar1(np.random.default_rng(2), 257, n, 0.95)
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, route, dtype="bf16")
    err = relerr(run(p, x), fwd(x.astype(np.float64)))
    assert err <= TOLBF16
    assert relerr(run(p, x, adjoint=True), adj(x.astype(np.float64))) <= TOLBF16
    print(f"bf16 {route} n={n}: {err:.2e}")
    p.close()


@pytest.mark.parametrize("route", ["dense", "gft"])
@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("kind", ["dense", "edge", "negative"])
def test_f32_split_bf16_products(route, n, kind):
    """FP32-accurate products from three-piece BF16 splits: held to the FP32 bar."""
    rho, v = case(n, kind)
    x = workloads.ar1(np.random.default_rng(4), 333, n, 0.95)
    x[5] *= 1e-30                        # tiny and huge signals keep relative accuracy
    x[6] *= 1e30
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, route, dtype="f32split")
    assert relerr(run(p, x), fwd(x.astype(np.float64))) <= TOL32
    assert relerr(run(p, x, adjoint=True), adj(x.astype(np.float64))) <= TOL32
    p.close()


@pytest.mark.parametrize("route", ["dense", "gft"])
@pytest.mark.parametrize("n,batch", [(128, 333), (256, 333), (1024, 130), (4096, 40)])
@pytest.mark.parametrize("kind", ["dense", "edge", "negative"])
def test_f32_split_gemm(route, n, batch, kind):
    """The split-BF16 product above n = 64 (64 x 64 tiles at these batches, a ragged
    last tile): FP32 bar, with tiny and huge signals keeping their relative accuracy."""
    rho, v = case(n, kind)
    x = workloads.ar1(np.random.default_rng(5), batch, n, 0.95)
    x[5] *= 1e-30
    x[6] *= 1e30
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, route, dtype="f32split")
    assert relerr(run(p, x), fwd(x.astype(np.float64))) <= TOL32, (route, n, kind)
    assert relerr(run(p, x, adjoint=True), adj(x.astype(np.float64))) <= TOL32, (route, n, kind)
    p.close()


@pytest.mark.parametrize("n,batch", [(256, 32768), (1024, 8192)])
def test_f32_split_gemm_large_tiles(n, batch):
    """Batches that take the 128 x 128 tiles of the split-BF16 product; sampled rows
    against the oracle (every row of the last, ragged tile included)."""
    torch = _torch()
    rho, v = case(n, "dense")
    x = workloads.ar1(np.random.default_rng(6), batch - 37, n, 0.95)
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, "dense", dtype="f32split")
    y = run(p, x)
    xa = run(p, x, adjoint=True)
    rows = np.r_[np.arange(0, x.shape[0], 97), np.arange(x.shape[0] - 150, x.shape[0])]
    assert relerr(y[rows], fwd(x[rows].astype(np.float64))) <= TOL32
    assert relerr(xa[rows], adj(x[rows].astype(np.float64))) <= TOL32
    p.close()


@pytest.mark.parametrize("kind", ["dense", "loop0", "loopn", "edge", "negative"])
def test_factored_split_n64(kind):
    """The factored form at n = 64 with split-BF16 products (DCT-II in registers, then
    the Cauchy factor on MFMA): held to the FP32 bar, on a ragged batch with tiny and
    huge signals."""
    n = 64
    rho, v = case(n, kind)
    x = workloads.ar1(np.random.default_rng(14), 333, n, 0.95)
    x[5] *= 1e-30
    x[6] *= 1e30
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, "dense-factored", dtype="f32split")
    assert relerr(run(p, x), fwd(x.astype(np.float64))) <= TOL32
    assert relerr(run(p, x, adjoint=True), adj(x.astype(np.float64))) <= TOL32
    p.close()


@pytest.mark.parametrize("dtype", ["f32", "f32split"])
def test_factored_n64_batch_edges_and_alignment(dtype):
    """Factored n = 64: batches around the 16-signal tile and the 4-tile grid
    granule; arrays that are only 4-byte aligned take the LDS-tile kernel (FP32) or
    are refused (split products need 16-byte alignment)."""
    torch = _torch()
    from paper_2409_08970_amd import _binding as B
    n = 64
    rho, v = case(n, "dense")
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, "dense-factored", dtype=dtype)
    for batch in (1, 15, 16, 17, 63, 64, 65, 1000):
        x = np.random.default_rng(batch).standard_normal((batch, n)).astype(np.float32)
        assert relerr(run(p, x), fwd(x.astype(np.float64))) <= TOL32, batch
        assert relerr(run(p, x, adjoint=True), adj(x.astype(np.float64))) <= TOL32, batch
    xs = np.random.default_rng(9).standard_normal((40, n)).astype(np.float32)
    buf = torch.zeros(40 * n + 2, device="cuda")
    buf[1:1 + 40 * n] = torch.from_numpy(xs.reshape(-1)).cuda()
    outb = torch.zeros(40 * n + 2, device="cuda")
    st = B.dctplus_forward(p.handle, buf.data_ptr() + 4, outb.data_ptr() + 4, 40, check=False)
    if dtype == "f32":
        assert st == B.DCTPLUS_OK
        torch.cuda.synchronize()
        yo = outb[1:1 + 40 * n].cpu().double().numpy().reshape(40, n)
        assert relerr(yo, fwd(xs.astype(np.float64))) <= TOL32
    else:
        assert st == B.DCTPLUS_EUNSUPPORTED
    # determinism: repeated calls give the same bits
    xt = torch.randn(517, n, device="cuda")
    a, b = p.forward(xt), p.forward(xt)
    c, d = p.adjoint(a), p.adjoint(a)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d)
    p.close()


@pytest.mark.parametrize("route", ["fast", "dense", "gft", "dense-f32split", "dense-factored-f32",
                                   "dense-factored-f32split"])
def test_full_size_workload2_sampled(route):
    """Workload-2 launch shape (2^20 AR(0.95) signals, n = 64): every output
    row runs on the GPU; 2048 sampled signals are checked against Jacobi."""
    torch = _torch()
    W = workloads.workload2(64)
    n, rho, v, x = W["n"], W["rho"], W["v"], W["x"]
    if route.startswith("dense-factored"):
        rt, dt = "dense-factored", route.rsplit("-", 1)[1]
    else:
        rt, _, dt = route.partition("-")
    p = make_plan(n, rho, v, rt, dtype=dt or "f32")
    xt = torch.from_numpy(x).cuda()
    y = p.forward(xt)
    xr = p.adjoint(y)
    torch.cuda.synchronize()
    rows = np.random.default_rng(0).choice(x.shape[0], 2048, replace=False)
    fwd, _ = reference(n, rho, v)
    ys = y[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    assert relerr(ys, fwd(x[rows].astype(np.float64))) <= TOL32
    xs = xr[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    assert relerr(xs, x[rows]) <= 2 * TOL32
    p.close()


@pytest.mark.parametrize("n,batch,route", [(128, 70001, "dense"), (256, 33001, "dense"),
                                           (256, 33001, "dense-factored"), (512, 301, "gft")])
def test_dense_product_large_batches(n, batch, route):
    """The FP32 dense product above n = 64 (our MFMA GEMM): batches that take its
    128 x 128 tiles (at least two workgroups per CU) with a ragged last tile, and a
    small batch on the 64 x 64 tiles; sampled rows against the oracle, every row in
    the round trip."""
    torch = _torch()
    rho, v = case(n, "dense")
    x = workloads.ar1(np.random.default_rng(n + batch), batch, n, 0.95)
    fwd, adj = reference(n, rho, v)
    p = make_plan(n, rho, v, route)
    xt = torch.from_numpy(x).cuda()
    y = p.forward(xt)
    xr = p.adjoint(y)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([np.random.default_rng(1).choice(batch, 300, replace=False),
                                     np.arange(batch - 40, batch)]))
    ri = torch.from_numpy(rows).cuda()
    assert relerr(y[ri].cpu().double().numpy(), fwd(x[rows].astype(np.float64))) <= TOL32
    assert relerr(xr.cpu().double().numpy(), x) <= 2 * TOL32
    p.close()


@pytest.mark.parametrize("route,n", [("fast", 8192), ("dense-factored", 256)])
def test_two_streams_on_one_plan(route, n):
    """Routes with scratch memory keep one workspace per stream: forward and adjoint
    calls on two streams at once on one plan give the bits of the same calls made
    one after the other on one stream."""
    torch = _torch()
    rho, v = case(n, "dense")
    p = make_plan(n, rho, v, route)
    g = torch.Generator(device="cuda").manual_seed(5)
    xa = torch.randn(64, n, device="cuda", generator=g)
    xb = torch.randn(96, n, device="cuda", generator=g)
    ya_ref, yb_ref = p.forward(xa), p.forward(xb)
    ra_ref, rb_ref = p.adjoint(ya_ref), p.adjoint(yb_ref)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(s1):
            ya = p.forward(xa, stream=s1)
            ra = p.adjoint(ya, stream=s1)
        with torch.cuda.stream(s2):
            yb = p.forward(xb, stream=s2)
            rb = p.adjoint(yb, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(ya, ya_ref) and torch.equal(yb, yb_ref)
        assert torch.equal(ra, ra_ref) and torch.equal(rb, rb_ref)
    p.close()


def test_batch_edge_cases_and_errors():
    torch = _torch()
    from paper_2409_08970_amd import _binding as B
    n = 64
    rho, v = case(n, "dense")
    fwd, _ = reference(n, rho, v)
    for route in ("dense", "gft"):
        p = make_plan(n, rho, v, route)
        for batch in (1, 63, 64, 65, 1000):
            x = np.random.default_rng(batch).standard_normal((batch, n)).astype(np.float32)
            assert relerr(run(p, x), fwd(x.astype(np.float64))) <= TOL32
        # 4-byte aligned but not 16-byte aligned arrays are valid input
        xs = np.random.default_rng(9).standard_normal((40, n)).astype(np.float32)
        buf = torch.zeros(40 * n + 2, device="cuda")
        buf[1:1 + 40 * n] = torch.from_numpy(xs.reshape(-1)).cuda()
        outb = torch.zeros(40 * n + 2, device="cuda")
        B.dctplus_forward(p.handle, buf.data_ptr() + 4, outb.data_ptr() + 4, 40)
        torch.cuda.synchronize()
        yo = outb[1:1 + 40 * n].cpu().double().numpy().reshape(40, n)
        assert relerr(yo, fwd(xs.astype(np.float64))) <= TOL32
        x = torch.zeros(4, n, device="cuda")
        assert B.dctplus_forward(p.handle, x.data_ptr(), x.data_ptr(), 0, check=False) == B.DCTPLUS_OK
        assert B.dctplus_forward(p.handle, x.data_ptr(), x.data_ptr(), 4, check=False) == B.DCTPLUS_EINVAL
        assert B.dctplus_forward(p.handle, x.data_ptr(), x[1:].data_ptr(), 2, check=False) == B.DCTPLUS_EINVAL
        assert B.dctplus_forward(p.handle, x.data_ptr() + 2, x[2:].data_ptr(), 1, check=False) == B.DCTPLUS_EINVAL
        assert B.dctplus_forward(p.handle, x.data_ptr(), x[2:].data_ptr(), -1, check=False) == B.DCTPLUS_EINVAL
        p.close()


@pytest.mark.parametrize("route,n", [("fast", 64),
                                     ("fast", 4096), ("dense", 64), ("gft", 64),
                                     ("dense", 1024), ("gft", 256)])
def test_bitwise_determinism(route, n):
    torch = _torch()
    rho, v = case(n, "dense")
    p = make_plan(n, rho, v, route)
    x = torch.randn(513 if n <= 64 else 64, n, device="cuda")
    a = p.forward(x)
    b = p.forward(x)
    c = p.adjoint(a)
    d = p.adjoint(a)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d)
    p.close()


# --------------------------------------------------------------------------
# gradients
#
# The oracle computes its own y = X^T x (Jacobi basis, or the secular semi-oracle's
# rows for n > 256) and gy = d loss / d y of loss = mean |y|; that gy, rounded to
# FP32, is the gy input of dctplus_grad (the gradient entry point takes gy as an
# argument), so both sides differentiate the same loss.  The GPU's y is its own
# forward.
#
# Tolerance (derived from the arithmetic): G = sum_b gy_b y_b^T is accumulated in
# FP32 over splits of at most 512 batch rows, the splits summed in FP64.  Rounding
# errors of a running FP32 sum of m terms of random sign have relative size about
# u32 sqrt(m / 2) against the sum (u32 = 2^-24): 1e-6 at m = 512; y enters with its
# forward error (<= 1e-6 relative on these workloads).  d rho and d v are linear in
# G with the same FP64 gap factors on both sides, so they inherit that relative error:
# the bar is 1e-5, ten times the estimate, against max(|d rho|, ||d v||_inf).
# dl/dx = X gy is an adjoint transform and has the forward's bar, 1e-5 per signal.
# --------------------------------------------------------------------------
TOLGRAD = 1e-5


def _oracle_basis(n, rho, v):
    if n <= 256:
        return oracle.basis(n, rho, v)
    plan = oracle.semi_plan(n, rho, v)
    X = oracle.dct2_matrix(n) @ oracle.semi_rows(plan, range(n)).T     # X = U M^T
    return plan["mu"], X


def _grad_case(n, rho, v, x, route, rows=None, dtype="f32"):
    """GPU (y, dx, drho, dv) and oracle (dx, drho, dv) for loss = mean |y|.

    rows: indices of the signals whose dl/dx is compared (all when None)."""
    torch = _torch()
    mu, X = _oracle_basis(n, rho, v)
    y_ref = oracle.forward(X, x.astype(np.float64))
    gy32 = oracle.loss_l1_grad(y_ref).astype(np.float32)
    gy = gy32.astype(np.float64)
    p = make_plan(n, rho, v, route, dtype=dtype)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = p.forward(xt)
    gx, grho, gv = p.grad(y, torch.from_numpy(gy32).cuda())
    torch.cuda.synchronize()
    sel = slice(None) if rows is None else rows
    gpu = dict(y=y.cpu().double().numpy(), dx=gx[sel].cpu().double().numpy(), drho=grho.item(),
               dv=gv.cpu().numpy())
    p.close()
    w = X.T @ v
    G = gy.T @ y_ref
    diff = mu[:, None] - mu[None, :]
    np.fill_diagonal(diff, 1.0)
    A = G / diff
    np.fill_diagonal(A, 0.0)
    ref = dict(drho=float(w @ A @ w), dv=rho * (X @ ((A + A.T) @ w)), dx=gy[sel] @ X.T, y=y_ref)
    # the same formula as oracle.grad_perturbation, restricted to the compared rows
    if rows is None:
        dx_o, drho_o, dv_o = oracle.grad_perturbation(mu, X, rho, v, y_ref, gy)
        assert abs(drho_o - ref["drho"]) <= 1e-12 * max(1.0, abs(drho_o))
    return gpu, ref


def _check_grad(gpu, ref):
    assert relerr(gpu["y"], ref["y"]) <= TOL32
    assert relerr(gpu["dx"], ref["dx"]) <= TOL32
    scale = max(abs(ref["drho"]), np.abs(ref["dv"]).max())
    e_rho = abs(gpu["drho"] - ref["drho"]) / scale
    e_v = np.abs(gpu["dv"] - ref["dv"]).max() / scale
    assert e_rho <= TOLGRAD and e_v <= TOLGRAD, (e_rho, e_v)
    return e_rho, e_v


@pytest.mark.parametrize("route", ["fast", "dense", "gft"])
def test_gradient_n16_vs_oracle(route):
    n = 16
    W = workloads.workload5(n=n, batch=512)
    rho, v, x = W["rho"], W["v"], W["x"]
    gpu, ref = _grad_case(n, rho, v, x, route)
    _check_grad(gpu, ref)
    # scale invariance of L in (rho, v): v . grad_v = 2 rho d/drho
    assert abs(v @ gpu["dv"] - 2 * rho * gpu["drho"]) <= TOLGRAD * np.abs(ref["dv"]).max()


def _edge_without_double_eigenvalues(n, seed):
    """An added edge (weight 1, rho = 2) whose spectrum is simple (no secular root on
    a deflated lambda), found by scanning seeded vertex pairs."""
    g = np.random.default_rng(seed)
    for _ in range(200):
        i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
        v = workloads.edge_vector(n, i, j)
        if np.min(np.diff(oracle.semi_plan(n, 2.0, v)["mu"])) > 1e-6:
            return v
    raise AssertionError("no simple edge found")


def _grad_kind(n, kind):
    g = np.random.default_rng(777 + n)
    if kind == "dense":
        return 1.0, workloads.unit_vector(g, n)
    if kind == "edge":
        return 2.0, _edge_without_double_eigenvalues(n, 31 + n)
    if kind == "loopn":
        v = np.zeros(n); v[-1] = 1.0
        return 1.5, v
    if kind == "negative":
        return -0.6, workloads.unit_vector(g, n)
    raise ValueError(kind)


@pytest.mark.parametrize("route", ["dense", "fast"])
@pytest.mark.parametrize("n,kind", [(64, "edge"), (64, "loopn"), (64, "negative"), (256, "edge"),
                                    (256, "negative"), (1024, "dense"), (1024, "edge"), (4096, "dense"),
                                    (4096, "negative")])
def test_gradient_graph_kinds_vs_oracle(route, n, kind):
    rho, v = _grad_kind(n, kind)
    batch = 1024 if n <= 256 else 256
    x = np.random.default_rng(5 + n).standard_normal((batch, n)).astype(np.float32)
    gpu, ref = _grad_case(n, rho, v, x, route)
    _check_grad(gpu, ref)


def test_gradient_workload5_full_batch():
    """The full gradient workload: n = 256, 65,536 N(0,1) signals, rho = 1, unit v.
    G's FP32 accumulation then runs 16 stages of 32 rows per split (the register
    prefetch loop); dl/dx is compared on 512 sampled signals, d rho and d v in full."""
    n = 256
    W = workloads.workload5()
    rho, v, x = W["rho"], W["v"], W["x"]
    assert x.shape == (65536, 256)
    rows = np.sort(np.random.default_rng(3).choice(x.shape[0], 512, replace=False))
    gpu, ref = _grad_case(n, rho, v, x, "auto", rows=rows)
    e = _check_grad(gpu, ref)
    print(f"workload 5 gradient: d rho rel err {e[0]:.2e}, d v rel err {e[1]:.2e}")


@pytest.mark.parametrize("n,kind", [(256, "dense"), (256, "negative"), (1024, "edge")])
def test_gradient_split_products_vs_oracle(n, kind):
    """Gradients of a split-BF16 plan (forward and dl/dx on the split product): the FP32 bars."""
    rho, v = _grad_kind(n, kind)
    batch = 1024 if n <= 256 else 256
    x = np.random.default_rng(9 + n).standard_normal((batch, n)).astype(np.float32)
    gpu, ref = _grad_case(n, rho, v, x, "dense", dtype="f32split")
    _check_grad(gpu, ref)


def test_gradient_workload5_full_batch_split():
    """The full gradient workload on a split-BF16 plan (128 x 128 tiles of the split product)."""
    n = 256
    W = workloads.workload5()
    rho, v, x = W["rho"], W["v"], W["x"]
    rows = np.sort(np.random.default_rng(4).choice(x.shape[0], 512, replace=False))
    gpu, ref = _grad_case(n, rho, v, x, "dense", rows=rows, dtype="f32split")
    e = _check_grad(gpu, ref)
    print(f"workload 5 gradient, split products: d rho rel err {e[0]:.2e}, d v rel err {e[1]:.2e}")


def test_gradient_double_eigenvalue_is_refused():
    """A mirror-symmetric edge makes secular roots coincide with deflated lambdas: the
    eigenbasis inside the double eigenvalue (and the row order) is not differentiable in
    (rho, v), so d rho / d v are refused before any device work; dl/dx (the adjoint)
    is still defined and computed."""
    torch = _torch()
    from paper_2409_08970_amd import DctPlusError, dctplus_grad, dctplus_plan_table
    n = 32
    v = workloads.edge_vector(n, 3, n - 4)
    p = make_plan(n, 2.0, v, "dense")
    assert int(dctplus_plan_table(p.handle, "ntie")[0]) > 0
    x = torch.randn(64, n, device="cuda")
    y = p.forward(x)
    gy = torch.sign(y) / y.numel()
    grho = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    gx = torch.full_like(gy, 3.0)
    with pytest.raises(DctPlusError) as ei:
        dctplus_grad(p.handle, y.data_ptr(), gy.data_ptr(), 64, gx.data_ptr(), grho.data_ptr(), 0)
    assert ei.value.status == 6                      # DCTPLUS_EDEGENERATE
    torch.cuda.synchronize()
    assert grho.item() == 7.0 and bool((gx == 3.0).all())     # nothing written
    dctplus_grad(p.handle, y.data_ptr(), gy.data_ptr(), 64, gx.data_ptr(), 0, 0)
    ref = p.adjoint(gy)
    torch.cuda.synchronize()
    assert torch.equal(gx, ref)
    p.close()


def test_gradient_n256_vs_finite_differences():
    """Workload-5 shape (n = 256, rho = 1, unit v) on 4096 signals: dl/drho and a
    directional derivative of dl/dv against FP64 central differences (h = 1e-6)
    of the oracle loss (semi-oracle forward, independent of the perturbation formula)."""
    n = 256
    W = workloads.workload5(n=n, batch=4096)
    rho, v, x = W["rho"], W["v"], W["x"]
    gpu, ref = _grad_case(n, rho, v, x, "dense")
    _check_grad(gpu, ref)
    xd = x.astype(np.float64)

    def loss(r, vv):
        return oracle.loss_l1(oracle.semi_forward(n, r, vv, xd))
    h = 1e-6
    fd_rho = (loss(rho + h, v) - loss(rho - h, v)) / (2 * h)
    d = np.random.default_rng(1).standard_normal(n)
    d /= np.linalg.norm(d)
    fd_v = (loss(rho, v + h * d) - loss(rho, v - h * d)) / (2 * h)
    # central differences in FP64 of a loss of size ~1: truncation O(h^2), rounding
    # ~ 1e-16 / h = 1e-10 relative; sign changes of y within h leave O(h) kinks
    scale = max(abs(fd_rho), np.abs(gpu["dv"]).max())
    assert abs(gpu["drho"] - fd_rho) <= 1e-6 * scale
    assert abs(gpu["dv"] @ d - fd_v) <= 1e-6 * scale


def test_autograd_function():
    """DctPlusFn under torch.autograd with a smooth loss, l = sum_i c_i mean_b y_bi^2
    (c fixed, varying over i, so that d rho and d v are not zero), against the oracle's
    perturbation gradient computed from its own y (gy = 2 c y / batch is continuous in
    y, so both sides differentiate the same function)."""
    torch = _torch()
    from paper_2409_08970_amd import dctplus
    n = 64
    W = workloads.workload5(n=n, batch=1024)
    c = np.linspace(0.5, 1.5, n)
    x = torch.from_numpy(W["x"]).cuda().requires_grad_(True)
    rho = torch.tensor(W["rho"], dtype=torch.float64, requires_grad=True)
    v = torch.tensor(W["v"], dtype=torch.float64, requires_grad=True)
    y = dctplus(x, rho, v)
    ct = torch.from_numpy(c).float().cuda()
    loss = ((y * y) * ct).sum() / y.shape[0]
    loss.backward()
    mu, X = oracle.basis(n, W["rho"], W["v"])
    yr = oracle.forward(X, W["x"].astype(np.float64))
    gy = 2.0 * c * yr / yr.shape[0]
    dx, drho, dv = oracle.grad_perturbation(mu, X, W["rho"], W["v"], yr, gy)
    assert relerr(y.detach().cpu().double().numpy(), yr) <= TOL32
    assert relerr(x.grad.cpu().double().numpy(), dx) <= TOL32
    scale = max(abs(drho), np.abs(dv).max())
    assert abs(rho.grad.item() - drho) <= TOLGRAD * scale
    assert np.abs(v.grad.numpy() - dv).max() <= TOLGRAD * scale


def _random_plan_case(g, n_max):
    n = int(2 ** g.integers(2, int(np.log2(n_max)) + 1))
    kind = g.choice(["dense", "negative", "loop0", "loopn", "edge"])
    if kind == "dense":
        rho, v = float(g.uniform(0.05, 3.0)), workloads.unit_vector(g, n)
    elif kind == "negative":
        rho, v = float(-g.uniform(0.05, 1.5)), workloads.unit_vector(g, n)
    elif kind in ("loop0", "loopn"):
        v = np.zeros(n)
        v[0 if kind == "loop0" else -1] = 1.0
        rho = float(g.uniform(0.1, 2.0))
    else:
        i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
        rho, v = 2.0 * float(g.uniform(0.2, 2.0)), workloads.edge_vector(n, i, j)
    return n, kind, rho, v


@pytest.mark.parametrize("route", ["fast", "dense", "gft", "auto"])
def test_random_plans_against_the_semi_oracle(route):
    """Seeded random plans beyond the fixed cases: n = 4 ... 2048, dense v with
    rho of either sign, self-loops at either end and added edges of random weight,
    1 to 8 signals; FP32 signals (and FP64 on the FAST route) against the secular
    semi-oracle, forward and adjoint, at the FP32 bar and the FP64 FAST bar."""
    g = np.random.default_rng({"fast": 11, "dense": 12, "gft": 13, "auto": 14}[route])
    for _ in range(40):
        n, kind, rho, v = _random_plan_case(g, 2048)
        dt = "f64" if (route == "fast" and g.random() < 0.3) else "f32"
        batch = int(g.integers(1, 9))
        x = g.standard_normal((batch, n))
        if dt == "f32":
            x = x.astype(np.float32)
        p = make_plan(n, rho, v, route, dtype=dt)
        y, xa = run(p, x), run(p, x, adjoint=True)
        p.close()
        sp = oracle.semi_plan(n, rho, v)
        xd = x.astype(np.float64)
        bar = TOL32 if dt == "f32" else TOL_FAST64
        assert relerr(y, oracle.semi_forward(n, rho, v, xd, sp)) <= bar, (n, kind, rho, dt)
        assert relerr(xa, oracle.semi_adjoint(n, rho, v, xd, sp)) <= bar, (n, kind, rho, dt)


@pytest.mark.parametrize("seed", range(6))
def test_gradient_random_cases(seed):
    """Seeded random gradient problems: n = 16 ... 256, a dense v with rho of either sign,
    a self-loop or an added edge anywhere (simple spectrum, so that the basis is
    differentiable), 64 to 1024 signals, any route; dl/dx, dl/drho and dl/dv against the
    oracle's perturbation formula at the gradient bars."""
    g = np.random.default_rng(7000 + seed)
    for _ in range(50):
        n = int(2 ** g.integers(4, 9))
        u = g.random()
        if u < 0.5:
            rho, v = float(g.choice([-1.0, 1.0]) * g.uniform(0.1, 1.5)), workloads.unit_vector(g, n)
        elif u < 0.75:
            i = int(g.integers(0, n))
            rho, v = oracle.candidate_update(n, 0, i, i, float(g.uniform(0.3, 2.0)))
        else:
            i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
            rho, v = oracle.candidate_update(n, 1, i, j, float(g.uniform(0.3, 2.0)))
        if np.diff(np.linalg.eigvalsh(oracle.laplacian(n, rho, v))).min() > 1e-6:
            break
    route = str(g.choice(["fast", "dense", "gft", "auto"]))
    batch = int(g.integers(64, 1025))
    x = g.standard_normal((batch, n)).astype(np.float32)
    gpu, ref = _grad_case(n, rho, v, x, route)
    _check_grad(gpu, ref)
