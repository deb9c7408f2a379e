"""Launch autotuner (dctplus_tune): every configuration it may keep computes the same
transform, and its choices persist through the JSON cache into new plans."""
import json
import os

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
    return float(np.max(np.linalg.norm(y - yref, axis=-1) / np.linalg.norm(yref, axis=-1)))


@pytest.mark.parametrize("n,batch,route,kw,bitwise", [
    (64, 1 << 17, "dense", dict(dtype="f32split", factored=True), True),
    (64, 5000, "gft", dict(), True),
    (256, 8192, "dense", dict(), True),
    (1024, 256, "dense", dict(), True),
    (4096, 64, "fast", dict(), False),
    (256, 300, "fast", dict(), False),
])
def test_tuned_configurations_keep_the_transform(n, batch, route, kw, bitwise, tmp_path):
    torch = _torch()
    from paper_2409_08970_amd import Plan, dctplus_plan_table
    g = np.random.default_rng(n + batch)
    v = workloads.unit_vector(g, n)
    rho = 0.7
    p = Plan(n, rho, v, route=route, **kw)
    x = torch.from_numpy(g.standard_normal((batch, n)).astype(np.float32)).cuda()
    y0 = p.forward(x)
    r0 = p.adjoint(y0)
    cache = str(tmp_path / "tune.json")
    chosen, ms = p.tune(x, cache_path=cache)
    tab = dctplus_plan_table(p.handle, "tune").reshape(2, 64)
    b = int(np.floor(np.log2(batch)))
    assert tab[0, b] == chosen[0] and tab[1, b] == chosen[1]
    y1 = p.forward(x)
    r1 = p.adjoint(y1)
    torch.cuda.synchronize()
    if bitwise:
        assert torch.equal(y0, y1) and torch.equal(r0, r1)
    rows = np.arange(min(batch, 64))
    if n <= 256:
        _, X = oracle.basis(n, rho, v)
        yref = oracle.forward(X, x[:64].cpu().double().numpy())
    else:
        yref = oracle.semi_forward(n, rho, v, x[:64].cpu().double().numpy(), oracle.semi_plan(n, rho, v))
    assert relerr(y1[rows].cpu().double().numpy(), yref) <= TOL32
    assert relerr(r1.cpu().double().numpy(), x.cpu().double().numpy()) <= 2 * TOL32
    # the cache holds both directions of this bucket and a new plan picks them up (a route
    # with a single configuration has nothing to tune and writes nothing)
    if chosen[0] == 0:
        assert chosen == [0, 0] and not os.path.exists(cache)
    else:
        data = json.load(open(cache))
        keys = [k for k in data if k.endswith(f"|bucket={b}")]
        assert len(keys) == 2
        os.environ["DCTPLUS_TUNE_CACHE"] = cache
        try:
            q = Plan(n, rho, v, route=route, **kw)
        finally:
            del os.environ["DCTPLUS_TUNE_CACHE"]
        tq = dctplus_plan_table(q.handle, "tune").reshape(2, 64)
        assert tq[0, b] == chosen[0] and tq[1, b] == chosen[1]
        assert torch.equal(q.forward(x), y1)
        q.close()
    p.close()
