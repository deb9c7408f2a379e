"""Rank-k updates (Sec. 4.3, Cor. 4.5) on the GPU against the oracle.

The oracle diagonalises the assembled L_path + sum_j rho_j v_j v_j^T with Jacobi and
applies the chain's sign convention (``oracle.basis_rank_k``, pinned on the CPU).  The
library builds the chain of Cauchy factors in FP64 on the GPU and composes it.
Bars: FP32 signals 1e-5 per-signal relative L2 (the rank-one bar: the composite factor
is formed in FP64 and rounded once); FP64 signals max(1e-12, 100 eps ||L|| / min gap),
the first-order error of the Jacobi eigenvectors, as for rank-one plans.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def relerr(y, yref):
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    return float(np.max(np.linalg.norm(y - yref, axis=-1) / np.maximum(np.linalg.norm(yref, axis=-1), 1e-300)))


def updates(n, kind, seed):
    """(rhos, V) of a seeded rank-k case with a simple spectrum at every stage."""
    g = np.random.default_rng(seed)
    for _ in range(50):
        if kind == "edges2" or kind == "edges3":
            k = 2 if kind == "edges2" else 3
            rhos, V = [], []
            for _ in range(k):
                i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
                rho, v = oracle.candidate_update(n, 1, i, j, float(g.uniform(0.5, 2.0)))
                rhos.append(rho)
                V.append(v)
        elif kind == "loop_edge":
            r1, v1 = oracle.candidate_update(n, 0, 0, 0, float(g.uniform(0.25, 2.0)))
            i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
            r2, v2 = oracle.candidate_update(n, 1, i, j, 1.0)
            rhos, V = [r1, r2], [v1, v2]
        elif kind == "dense_mixed":
            rhos = [float(g.uniform(0.1, 2.0)), -float(g.uniform(0.05, 0.3)), float(g.uniform(0.1, 2.0))]
            V = [workloads.unit_vector(g, n) for _ in range(3)]
        else:
            raise ValueError(kind)
        ok = all(np.diff(np.linalg.eigvalsh(oracle.laplacian_rank_k(n, rhos[:j + 1], V[:j + 1]))).min() > 1e-7
                 for j in range(len(rhos)))
        if ok:
            return rhos, np.array(V)
    raise AssertionError("no case with simple spectra")


_CACHE = {}


def ref_basis(n, kind, seed):
    key = (n, kind, seed)
    if key not in _CACHE:
        rhos, V = updates(n, kind, seed)
        mu, X = oracle.basis_rank_k(n, rhos, V)
        _CACHE[key] = (rhos, V, mu, X)
    return _CACHE[key]


def make(n, rhos, V, route, dtype="f32"):
    from paper_2409_08970_amd import Plan
    if route == "dense-factored":
        return Plan(n, rhos, V, route="dense", dtype=dtype, factored=True)
    return Plan(n, rhos, V, route=route, dtype=dtype)


def run(p, arr, adjoint=False):
    torch = _torch()
    dt = torch.float64 if p.dtype == "f64" else torch.float32
    t = torch.from_numpy(np.ascontiguousarray(arr)).to("cuda", dt)
    out = p.adjoint(t) if adjoint else p.forward(t)
    torch.cuda.synchronize()
    return out.cpu().double().numpy()


CASES = [(n, kind) for n in (16, 64, 256) for kind in ("edges2", "edges3", "loop_edge", "dense_mixed")] + \
        [(1024, "edges3")]


@pytest.mark.parametrize("n,kind", CASES)
@pytest.mark.parametrize("route", ["dense", "dense-factored", "gft"])
def test_rank_k_parity(n, kind, route):
    _torch()
    rhos, V, mu, X = ref_basis(n, kind, 900 + n)
    p = make(n, rhos, V, route)
    info = p.info
    assert np.abs(info["mu"] - mu).max() <= 1e-12 * max(1.0, np.abs(mu).max())
    g = np.random.default_rng(n + 3)
    x = workloads.ar1(g, 301, n, 0.95)
    assert relerr(run(p, x), oracle.forward(X, x.astype(np.float64))) <= TOL32, (n, kind, route)
    yin = g.standard_normal((301, n)).astype(np.float32)
    assert relerr(run(p, yin, adjoint=True), oracle.adjoint(X, yin.astype(np.float64))) <= TOL32
    p.close()


@pytest.mark.parametrize("n,kind", [(64, "edges3"), (256, "dense_mixed")])
def test_rank_k_fp64(n, kind):
    _torch()
    rhos, V, mu, X = ref_basis(n, kind, 900 + n)
    p = make(n, rhos, V, "dense", dtype="f64")
    g = np.random.default_rng(n)
    x = g.standard_normal((65, n))
    L = oracle.laplacian_rank_k(n, rhos, V)
    tol = max(1e-12, 100 * np.finfo(float).eps * np.abs(np.linalg.eigvalsh(L)).max() / np.diff(mu).min())
    assert relerr(run(p, x), oracle.forward(X, x)) <= tol
    assert relerr(run(p, x, adjoint=True), oracle.adjoint(X, x)) <= tol
    p.close()


def test_rank_k_factored_split_n64_full_batch():
    """The factored split-BF16 kernel with a rank-3 composite factor at the workload-2
    batch (2^20 signals): sampled rows against the oracle, the round trip on all rows."""
    torch = _torch()
    n = 64
    rhos, V, mu, X = ref_basis(n, "edges3", 900 + n)
    p = make(n, rhos, V, "dense-factored", dtype="f32split")
    x = workloads.ar1(np.random.default_rng(5), 1 << 20, n, 0.95)
    xt = torch.from_numpy(x).cuda()
    y = p.forward(xt)
    xr = p.adjoint(y)
    torch.cuda.synchronize()
    rows = np.random.default_rng(1).choice(x.shape[0], 1024, replace=False)
    ri = torch.from_numpy(rows).cuda()
    assert relerr(y[ri].cpu().double().numpy(), oracle.forward(X, x[rows].astype(np.float64))) <= TOL32
    assert relerr(xr[ri].cpu().double().numpy(), x[rows]) <= 2 * TOL32
    p.close()


def test_rank_k_reduces_to_rank_one_and_splits():
    """k = 1 through dctplus_plan_rank_k is dctplus_plan bit for bit; an update split into
    two halves along the same v gives the same transform (the second stage is a rank-one
    update along an eigen-aligned v)."""
    torch = _torch()
    from paper_2409_08970_amd import Plan
    n = 64
    v = workloads.unit_vector(np.random.default_rng(3), n)
    x = torch.randn(200, n, device="cuda")
    p1 = Plan(n, 0.8, v, route="dense")
    pk = Plan(n, [0.8], [v], route="dense")
    assert torch.equal(p1.forward(x), pk.forward(x))
    p2 = Plan(n, [0.4, 0.4], [v, v], route="dense")
    y1, y2 = p1.forward(x), p2.forward(x)
    torch.cuda.synchronize()
    assert relerr(y2.cpu().numpy(), y1.cpu().numpy()) <= TOL32
    for p in (p1, pk, p2):
        p.close()


def test_rank_k_errors():
    _torch()
    from paper_2409_08970_amd import _binding as B
    from paper_2409_08970_amd import DctPlusError, Plan
    n = 64
    V = np.stack([workloads.unit_vector(np.random.default_rng(s), n) for s in range(2)])
    o = B.dctplus_default_opts()
    o.route = B.DCTPLUS_ROUTE_FAST
    assert B.dctplus_plan_rank_k(n, [1.0, 0.5], V, o, check=False)[0] == B.DCTPLUS_EUNSUPPORTED
    # d/drho, d/dv of a rank-k plan are refused; dl/dx is the adjoint
    torch = _torch()
    p = Plan(n, [1.0, 0.5], V, route="dense")
    y = p.forward(torch.randn(8, n, device="cuda"))
    gy = torch.sign(y)
    with pytest.raises(DctPlusError) as ei:
        p.grad(y, gy)
    assert ei.value.status == B.DCTPLUS_EUNSUPPORTED
    gx = torch.empty_like(gy)
    B.dctplus_grad(p.handle, y.data_ptr(), gy.data_ptr(), 8, gx.data_ptr(), 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(gx, p.adjoint(gy))
    p.close()


def _random_chain(g, n):
    """k = 2..4 updates, each a dense v with rho of either sign, an added edge or a
    self-loop at any vertex; the spectrum is simple at every stage."""
    for _ in range(50):
        k = int(g.integers(2, 5))
        rhos, V = [], []
        for _ in range(k):
            u = g.random()
            if u < 0.4:
                rhos.append(float(g.choice([-1.0, 1.0]) * g.uniform(0.05, 1.5)))
                V.append(workloads.unit_vector(g, n))
            elif u < 0.75:
                i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
                rho, v = oracle.candidate_update(n, 1, i, j, float(g.uniform(0.3, 2.0)))
                rhos.append(rho)
                V.append(v)
            else:
                i = int(g.integers(0, n))
                rho, v = oracle.candidate_update(n, 0, i, i, float(g.uniform(0.3, 2.0)))
                rhos.append(rho)
                V.append(v)
        if all(np.diff(np.linalg.eigvalsh(oracle.laplacian_rank_k(n, rhos[:j + 1], V[:j + 1]))).min() > 1e-7
               for j in range(k)):
            return rhos, np.array(V)
    raise AssertionError("no chain with simple spectra")


@pytest.mark.parametrize("seed", range(6))
def test_rank_k_random_chains(seed):
    """Seeded random chains of two to four updates (either sign, edges and self-loops
    anywhere) at n = 8 ... 128 on the dense, factored and GFT routes against the
    Jacobi oracle of the assembled Laplacian, forward and adjoint."""
    _torch()
    g = np.random.default_rng(5000 + seed)
    n = int(2 ** g.integers(3, 8))
    rhos, V = _random_chain(g, n)
    mu, X = oracle.basis_rank_k(n, rhos, V)
    x = g.standard_normal((37, n)).astype(np.float32)
    for route in ("dense", "dense-factored", "gft"):
        p = make(n, rhos, V, route)
        assert np.abs(p.info["mu"] - mu).max() <= 1e-12 * max(1.0, np.abs(mu).max()), (n, route)
        assert relerr(run(p, x), oracle.forward(X, x.astype(np.float64))) <= TOL32, (n, route, rhos)
        assert relerr(run(p, x, adjoint=True), oracle.adjoint(X, x.astype(np.float64))) <= TOL32, (n, route)
        p.close()
