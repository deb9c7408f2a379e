"""A rank-one update of a general base (Thm 3.1 on any symmetric base; Thm 3.2) and the
DTT+ case (the ADST graph's DST-VII as the base, Sec. 4.3) on the GPU against the oracle.

The oracle diagonalises the assembled U diag(lambda) U^T + rho v v^T with Jacobi
(``oracle.basis_general``, pinned on the CPU).  Bars as for rank-one plans: FP32 signals
1e-5 per-signal relative L2; FP64 max(1e-12, 100 eps ||L|| / min gap).
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


def base_case(n, kind, seed):
    g = np.random.default_rng(seed)
    if kind == "adst":
        lam, U = oracle.dst7_basis(n)
    else:
        U, _ = np.linalg.qr(g.standard_normal((n, n)))
        lam = np.sort(g.uniform(0.0, 4.0, n))
    return lam, U, g


def run(p, arr, adjoint=False):
    torch = _torch()
    dt = torch.float64 if p.dtype == "f64" else torch.float32
    t = torch.from_numpy(np.ascontiguousarray(arr)).to("cuda", dt)
    out = p.adjoint(t) if adjoint else p.forward(t)
    torch.cuda.synchronize()
    return out.cpu().double().numpy()


@pytest.mark.parametrize("n", [16, 64, 256, 1024])
@pytest.mark.parametrize("kind,rho", [("random", 0.8), ("random", -0.4), ("adst", 1.3)])
def test_general_base_parity(n, kind, rho):
    _torch()
    from paper_2409_08970_amd import Plan
    lam, U, g = base_case(n, kind, 77 + n)
    v = workloads.unit_vector(g, n)
    mu, X = oracle.basis_general(lam, U, rho, v)
    p = Plan(n, rho, v, base=(lam, U))
    assert np.abs(p.info["mu"] - mu).max() <= 1e-12 * max(1.0, np.abs(mu).max())
    x = workloads.ar1(g, 301, n, 0.95)
    assert relerr(run(p, x), oracle.forward(X, x.astype(np.float64))) <= TOL32
    yin = g.standard_normal((301, n)).astype(np.float32)
    assert relerr(run(p, yin, adjoint=True), oracle.adjoint(X, yin.astype(np.float64))) <= TOL32
    p.close()


def test_general_base_deflation_and_fp64():
    """v in the span of four base vectors: every other z_k is zero, those rows are the
    base vectors themselves; FP64 signals at the Jacobi bar."""
    _torch()
    from paper_2409_08970_amd import Plan
    n = 64
    lam, U, g = base_case(n, "random", 5)
    v = U[:, [3, 10, 11, 40]] @ g.standard_normal(4)
    v /= np.linalg.norm(v)
    mu, X = oracle.basis_general(lam, U, 0.6, v)
    for dtype in ("f32", "f64"):
        p = Plan(n, 0.6, v, base=(lam, U), dtype=dtype)
        assert int(p.info["counts"][0]) == n - 4
        x = g.standard_normal((100, n))
        L = (U * lam) @ U.T + 0.6 * np.outer(v, v)
        tol = TOL32 if dtype == "f32" else \
            max(1e-12, 100 * np.finfo(float).eps * np.abs(np.linalg.eigvalsh(L)).max() / np.diff(mu).min())
        xin = x.astype(np.float32) if dtype == "f32" else x
        assert relerr(run(p, xin), oracle.forward(X, xin.astype(np.float64))) <= tol
        assert relerr(run(p, xin, adjoint=True), oracle.adjoint(X, xin.astype(np.float64))) <= tol
        p.close()


@pytest.mark.parametrize("n", [64, 256])
def test_dtt_plus_base_equals_rank_two_chain(n):
    """DTT+ through the general base (DST-VII) and through the rank-two path chain
    (self-loop at vertex 0, then the update) give the same transform on the GPU."""
    torch = _torch()
    from paper_2409_08970_amd import Plan
    lam, U, g = base_case(n, "adst", 3)
    rho, v = oracle.candidate_update(n, 1, 5, n - 9, 1.0)
    e0 = np.zeros(n)
    e0[0] = 1.0
    pg = Plan(n, rho, v, base=(lam, U))
    pc = Plan(n, [1.0, rho], [e0, v], route="dense")
    x = torch.randn(257, n, device="cuda")
    yg, yc = pg.forward(x), pc.forward(x)
    torch.cuda.synchronize()
    assert relerr(yg.cpu().numpy(), yc.cpu().numpy()) <= 2 * TOL32
    pg.close()
    pc.close()
