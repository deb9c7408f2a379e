"""HIP graph capture of the hot path: forward + adjoint (dense streaming route and the
FAST route with its buffer in LDS) and the persistent selection launch are captured
once and replayed several times, with eager work and synchronisations between the
replays; every replay must equal the eager result bit for bit (the kernels are
deterministic and allocate nothing per call)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("route,n,batch", [("dense", 64, 70001), ("dense", 32, 4099), ("fast", 64, 1001),
                                           ("fast", 1024, 37)])
def test_forward_adjoint_graph_replays(route, n, batch):
    torch = _torch()
    from paper_2409_08970_amd import Plan
    g = np.random.default_rng(n + batch)
    v = workloads.unit_vector(g, n)
    p = Plan(n, 0.8, v, route=route)
    x = torch.from_numpy(workloads.ar1(g, batch, n, 0.95)).cuda()
    y = torch.empty_like(x)
    r = torch.empty_like(x)
    p.forward(x, out=y)
    p.adjoint(y, out=r)
    torch.cuda.synchronize()
    y_ref, r_ref = y.clone(), r.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):           # warm-up on the capture stream
        p.forward(x, out=y)
        p.adjoint(y, out=r)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        p.forward(x, out=y)
        p.adjoint(y, out=r)
    for k in range(4):
        y.zero_()
        r.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * (k + 1)     # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref) and torch.equal(r, r_ref), (route, n, k)
        del junk
    del graph
    p.close()


def test_selection_graph_replays():
    torch = _torch()
    from paper_2409_08970_amd import SelectPlan
    W = workloads.workload4(blocks=500, sub=3)
    sel = SelectPlan(W["n"], W["cand"], S=W["signals"])
    x = torch.from_numpy(np.ascontiguousarray(W["x"], dtype=np.float32)).cuda()
    nb, K = len(W["n"]), W["cand"].shape[1]
    best = torch.empty(nb, dtype=torch.int32, device="cuda")
    cost = torch.empty(nb, K, device="cuda")
    y = torch.empty_like(x)
    from paper_2409_08970_amd import _binding as B

    def call():
        B.dctplus_select(sel._h, x.data_ptr(), 0, 0.1, best.data_ptr(), cost.data_ptr(), y.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    call()
    torch.cuda.synchronize()
    ref = best.clone(), cost.clone(), y.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for k in range(4):
        best.fill_(-1)
        cost.zero_()
        y.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(best, ref[0]) and torch.equal(cost, ref[1]) and torch.equal(y, ref[2]), k
    del graph
    sel.close()
