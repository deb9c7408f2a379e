"""Benchmark: DCT+ forward + adjoint throughput on one MI355X.

A step is one forward (y = X^T x) plus one adjoint (x = X y) pass of the
DCT+ transform over the whole batch of the shared-transform workload
(n = 64, 2^20 AR(0.95) signals, random unit v, rho ~ U[0.1, 2]; FP32),
inputs resident in HBM.  The transform is applied as Thm 3.1 factors it: a
DCT-II of every signal, then the product with the Cauchy factor
diag(a) C(mu, lambda) diag(z) (split-BF16 MFMA products, FP32-accurate).
value = batch * n / (time per step): signal-samples per second through the
round trip.  Beside it: the dense GFT (the paper's naive product y = X^T x,
the DCT folded into one matrix) on the same GPU, with our MFMA kernel and
with torch.matmul, the BF16-operand dense route, the O(n log n) route, the
large-graph workloads (256 signals at n = 1024, 4096 and 16384, a dense v
and an added edge, with the FP64-vector roofline of the O(n log n) kernels),
the FP64 self-loop workload at n = 64, the roofline of the dominant kernel (HIP events
on its launch stream), and the FP64 oracle timed on the host cores (a
baseline, not a target).

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "signal-samples/s DCT+ fwd+bwd vs dense GFT, n=64 & 4096, FP32, rel err ≤1e-5"
HBM_PEAK_GBS = 8000.0


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "factored_stream_n64_hbm_counters.md")


def sources_hash(paths):
    """sha256 over the full text of the kernel's source files, in the listed order."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what the counter reads for a plain
    device copy of known size), or None when any source file of the kernel has
    changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
        k = rec["kernels"][kernel_key]
        if sources_hash(rec["source_files"]) != rec["source_sha256"]:
            return None
        kib = k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]
        return kib * 1024.0
    except (OSError, IndexError, KeyError, ValueError):
        return None


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_pair(torch, fwd, adj, steps, warmup):
    """Times `steps` (fwd, adj) pairs back to back, each launch bracketed by HIP events
    on the current stream (the stream the library launches on).  Returns
    (ms/step, mean fwd ms, mean adj ms, median fwd ms, median adj ms)."""
    import statistics
    for _ in range(warmup):
        fwd()
        adj()
    torch.cuda.synchronize()
    t0, t1 = _events(torch)
    fe = [_events(torch) for _ in range(steps)]
    ae = [_events(torch) for _ in range(steps)]
    t0.record()
    for k in range(steps):
        fe[k][0].record()
        fwd()
        fe[k][1].record()
        adj()
        ae[k][1].record()
    t1.record()
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1) / steps
    fl = [fe[k][0].elapsed_time(fe[k][1]) for k in range(steps)]
    al = [fe[k][1].elapsed_time(ae[k][1]) for k in range(steps)]
    return total, sum(fl) / steps, sum(al) / steps, statistics.median(fl), statistics.median(al)


def fast_flops_per_signal(n, width):
    """Algorithmic flops of one FAST-route transform of one signal (Alg. 1): the DCT-II
    as a half-length complex FFT (5 (n/2) log2(n/2), FP32), the DST-I as a packed FFT of
    length n (5 n log2 n), the oversampled grid DST of length 2n (5 2n log2 2n) and the
    window gather (2 (w + 2) taps per output row); the last three in FP64."""
    import math
    fp32 = 5 * (n / 2) * math.log2(n / 2)
    fp64 = 5 * n * math.log2(n) + 5 * 2 * n * math.log2(2 * n) + 2 * (width + 2) * n
    return fp32, fp64


def cpu_baseline(W, sample, min_seconds=10.0):
    """FP64 oracle on `sample` signals of the workload, all host cores."""
    import numpy as np
    import oracle
    n = W["n"]
    _, X = oracle.basis(n, W["rho"], W["v"])
    x = W["x"][:sample].astype(np.float64)
    oracle.forward(X, x[:16])
    reps = 0
    t = time.perf_counter()
    while True:                                 # about ten seconds of CPU work
        y = oracle.forward(X, x)
        oracle.adjoint(X, y)
        reps += 1
        dt = time.perf_counter() - t
        if dt >= min_seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": reps * sample * n / dt, "unit": "signal-samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample} of the {W['x'].shape[0]} signals (n={n}), forward + adjoint, FP64 dense "
                      f"apply of the Jacobi basis, {reps} repetitions in {dt:.1f} s; setup excluded"}


def bench_selection(torch, dev, steps, warmup):
    """Progressive selection with pruning on 10,000 blocks (n in {4, ..., 64}, 64
    AR(0.9) signals each, K = 8 candidates, c_p = max(2, n/2), tau = 0.1): one
    persistent launch per pass, inputs resident in HBM."""
    import numpy as np
    import workloads
    from paper_2409_08970_amd import SelectPlan
    W = workloads.workload4()
    nb, cand, S, K = W["n"], W["cand"], W["signals"], W["K"]
    t0 = time.perf_counter()
    sel = SelectPlan(nb, cand, S=S)
    plan_ms = (time.perf_counter() - t0) * 1e3
    x = torch.from_numpy(W["x"]).to(dev)
    y = torch.empty_like(x)
    chosen, tune_ms = sel.tune(x)      # launch autotuner: persistent workgroups per CU
    for _ in range(warmup):
        sel.select(x, out=y)
    torch.cuda.synchronize()
    reps = max(5, steps)
    ev = [_events(torch) for _ in range(reps)]
    for k in range(reps):
        ev[k][0].record()
        sel.select(x, out=y)
        ev[k][1].record()
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps

    def pass_ms(tau):
        ev2 = [_events(torch) for _ in range(reps)]
        for k in range(reps):
            ev2[k][0].record()
            sel.select(x, prune_tau=tau, out=y)
            ev2[k][1].record()
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in ev2) / reps
    # Thm 3.4's saving: the same pass with no signal pruned (tau = -1) and with every
    # signal pruned (tau = 10)
    ms_none, ms_all = pass_ms(-1.0), pass_ms(10.0)
    n64 = nb.astype(np.int64)
    samples = int(np.sum(n64 * S))
    flops = float(np.sum((K + 1) * S * 2 * n64 * n64))          # K candidate products + the winner's
    bytes_ = float(samples * 4 * 2 + np.sum(K * n64 * n64 * 4) + len(nb) * (K + 1) * 4)
    xq = [W["x"][W["offsets"][b]:W["offsets"][b + 1]].reshape(S, -1).astype(np.float64) for b in range(len(nb))]
    pruned = sum(int(np.sum(np.sum(np.diff(v, axis=1) ** 2, axis=1) <= 0.1 * np.sum(v * v, axis=1))) for v in xq)
    sel.close()
    return {"workload": f"{len(nb)} blocks, n in {{4,8,16,32,64}}, {S} AR(0.9) signals, K={K}, "
                        f"c_p=max(2,n/2), tau=0.1",
            "kernel": "k_select (persistent, FP32 MFMA)", "ms_per_pass": ms, "blocks_per_s": len(nb) / (ms * 1e-3),
            "signal_samples_per_s": samples / (ms * 1e-3), "pruned_fraction": pruned / (len(nb) * S),
            "plan_ms_host": plan_ms,
            "pruning": {"ms_per_pass_tau_minus1_none_pruned": ms_none, "ms_per_pass_tau10_all_pruned": ms_all,
                        "speedup_all_pruned_vs_none": ms_none / ms_all,
                        "speedup_tau0.1_vs_none": ms_none / ms},
            "autotune": {"workgroups_per_cu": chosen, "ms_per_pass_by_candidate": tune_ms},
            "roofline": {"mfma_tflops": flops / (ms * 1e-3) / 1e12, "mfma_peak_tflops": 157.3,
                         "hbm_gbs": bytes_ / (ms * 1e-3) / 1e9, "hbm_peak_gbs": HBM_PEAK_GBS,
                         "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_}}


def bench_gradient(torch, dev, steps, warmup):
    """Gradient workload: n = 256, 65,536 N(0,1) signals, rho = 1, random unit v,
    loss = mean |y|.  A step = forward + gradient (dl/dx via the adjoint, dl/drho
    and dl/dv via the batch Gram matrix), inputs resident in HBM.  Timed for an FP32
    plan (FP32 MFMA products) and a split-BF16 plan (FP32-accurate BF16 products)."""
    import workloads
    from paper_2409_08970_amd import Plan
    W = workloads.workload5()
    n, batch = W["n"], W["x"].shape[0]
    x = torch.from_numpy(W["x"]).to(dev)
    y = torch.empty_like(x)

    def timed(pl):
        def step():
            pl.forward(x, out=y)
            gy = torch.sign(y) / y.numel()
            pl.grad(y, gy)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        a, b = _events(torch)
        reps = max(5, steps)
        a.record()
        for _ in range(reps):
            step()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        pl.close()
        return ms

    ms = timed(Plan(n, W["rho"], W["v"], route="auto"))
    ms_split = timed(Plan(n, W["rho"], W["v"], route="dense", dtype="f32split"))
    return {"workload": f"n={n}, {batch} N(0,1) signals, rho={W['rho']}, random unit v, loss mean|y|",
            "ms_per_step": ms, "signal_samples_per_s": batch * n / (ms * 1e-3),
            "step": "forward + dl/dx (adjoint) + dl/drho, dl/dv (Gram matrix G = sum gy y^T, 2 B n^2 flops)",
            "gram_tflops_if_alone": 2.0 * batch * n * n / (ms * 1e-3) / 1e12,
            "f32split": {"ms_per_step": ms_split, "signal_samples_per_s": batch * n / (ms_split * 1e-3),
                         "products": "forward and dl/dx on the split-BF16 product (FP32 accuracy)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline DCT+ route (for profiler passes): no comparators, no CPU baseline")
    ap.add_argument("--fast-n", type=int, default=0,
                    help="only the FAST route at this n on the large-graph workload (256 N(0,1) signals): "
                         "three forward + adjoint pairs, for profiler passes; prints nothing timed")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run 3 device copies of the 256 MiB input (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the transform needs no "
              f"cross-GPU exchange: each GPU would transform its own share of the signals)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_2409_08970_amd import Plan

    dev = torch.device("cuda:0")
    W = workloads.workload2(64)
    n, batch = W["n"], W["x"].shape[0]
    x = torch.from_numpy(W["x"]).to(dev)
    y = torch.empty_like(x)
    xr = torch.empty_like(x)
    print(f"workload: n={n}, batch={batch}, rho={W['rho']:.4f}", file=sys.stderr, flush=True)
    if args.fast_n:
        W3 = workloads.workload3(args.fast_n, "dense")
        x3 = torch.from_numpy(W3["x"]).to(dev)
        y3 = torch.empty_like(x3)
        r3 = torch.empty_like(x3)
        pf = Plan(args.fast_n, W3["rho"], W3["v"], route="fast")
        for _ in range(3):
            pf.forward(x3, out=y3)
            pf.adjoint(y3, out=r3)
        torch.cuda.synchronize()
        pf.close()
        print(json.dumps({"fast_n": args.fast_n, "signals": x3.shape[0], "pairs": 3}), flush=True)
        return
    if args.copy_probe:
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": batch * n * 4}), flush=True)
        return

    # DCT+ as the paper factors it (Thm 3.1): a DCT-II of every signal (radix, in registers),
    # then the product with the Cauchy factor diag(a) C(mu, lambda) diag(z) on MFMA with
    # FP32-accurate split-BF16 products; the adjoint applies the transposed factors
    # plan setup (secular roots, tables, the dense Cauchy factor), timed apart from the
    # transform: the first plan of the process also loads the library's kernels, a second
    # one of the same graph shows the steady cost
    setup_ms = []
    for _ in range(2):
        torch.cuda.synchronize()
        t_plan = time.perf_counter()
        plan = Plan(n, W["rho"], W["v"], route="dense", dtype="f32split", factored=True)
        torch.cuda.synchronize()
        setup_ms.append((time.perf_counter() - t_plan) * 1e3)
        if len(setup_ms) == 1:
            plan.close()
    # the device reaches its sustained clocks only after some time under load (on a fresh
    # device half a second was not always enough): a second and a half of the headline's
    # own launches (untimed) comes before anything is timed
    t_end = time.perf_counter() + 1.5
    while time.perf_counter() < t_end:
        for _ in range(25):
            plan.forward(x, out=y)
            plan.adjoint(y, out=xr)
        torch.cuda.synchronize()
    ms, f_ms, a_ms, f_med, a_med = time_pair(torch, lambda: plan.forward(x, out=y), lambda: plan.adjoint(y, out=xr),
                                             args.steps, args.warmup)
    route = plan.route
    value = batch * n / (ms * 1e-3)
    alg_bytes = 2 * batch * n * 4                       # read + write of the signals, per launch
    launch_ms = 0.5 * (f_ms + a_ms)                     # forward and adjoint: the same kernel, transposed
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    if args.headline_only:
        args.no_extra = args.no_cpu = True
        t0 = (float("nan"),) * 5
    else:
        # the factored form with FP32 MFMA products, for comparison
        p0 = Plan(n, W["rho"], W["v"], route="dense", dtype="f32", factored=True)
        t0 = time_pair(torch, lambda: p0.forward(x, out=y), lambda: p0.adjoint(y, out=xr), args.steps,
                       args.warmup)
        p0.close()
    result = {
        "metric": METRIC, "value": value, "unit": "signal-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (DCT-II in fp32; bf16x3 split operands, fp32 accumulate)",
        "data": "synthetic",
        "config": {"workload": f"shared-transform batch: n={n}, {batch} AR(0.95) signals, random unit v, "
                               f"rho={W['rho']:.4f}",
                   "route": "DENSE factored (DCT-II, then the Cauchy factor)", "n": n, "batch": batch},
        "plan_setup_ms_host": {"first_in_process": setup_ms[0], "steady": setup_ms[1],
                               "note": "Plan() wall time incl. device sync; excluded from value"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_factored_stream<2>"),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_factored_stream<2> (forward and adjoint launches)", "avg_launch_ms": launch_ms,
                     "median_launch_ms": 0.5 * (f_med + a_med), "launches_timed": 2 * args.steps,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "forward_ms": f_ms, "adjoint_ms": a_ms, "forward_median_ms": f_med, "adjoint_median_ms": a_med,
        "dct_plus_configs": {"factored_f32split": {"ms_per_step": ms, "value": value},
                             "factored_f32_mfma": {"ms_per_step": t0[0], "value": batch * n / (t0[0] * 1e-3),
                                                   "median_launch_ms": 0.5 * (t0[3] + t0[4])}},
    }
    print(f"dct+ factored: {ms:.3f} ms/step (fwd {f_ms:.3f}, adj {a_ms:.3f})", file=sys.stderr, flush=True)

    if not args.no_extra:
        comp = {}
        # dense GFT (the paper's naive product y = X^T x) on the same GPU: our streaming MFMA
        # kernel on X^T (split-BF16 and FP32 products), and the library GEMM
        for key, dt in (("gft_mfma_f32split", "f32split"), ("gft_mfma_f32", "f32")):
            gp = Plan(n, W["rho"], W["v"], route="gft", dtype=dt)
            g = time_pair(torch, lambda: gp.forward(x, out=y), lambda: gp.adjoint(y, out=xr), args.steps,
                          args.warmup)
            comp[key] = {"ms_per_step": g[0], "value": batch * n / (g[0] * 1e-3),
                         "median_launch_ms": 0.5 * (g[3] + g[4])}
            if dt == "f32":
                XtT = torch.empty(n, n, device=dev)
                Xt = torch.from_numpy(np.ascontiguousarray(np.eye(n, dtype=np.float32))).to(dev)
                gp.forward(Xt, out=XtT)                  # rows: X^T e_i -> X[i, :]
                Xm = XtT.contiguous()                    # X (rows = spatial index)
                XmT = Xm.t().contiguous()
            gp.close()
        l = time_pair(torch, lambda: torch.matmul(x, Xm, out=y), lambda: torch.matmul(y, XmT, out=xr),
                      args.steps, args.warmup)
        comp["gft_torch_matmul"] = {"ms_per_step": l[0], "value": batch * n / (l[0] * 1e-3)}
        bp = Plan(n, W["rho"], W["v"], route="dense", dtype="bf16")
        b_ms = time_pair(torch, lambda: bp.forward(x, out=y), lambda: bp.adjoint(y, out=xr),
                         args.steps, args.warmup)[0]
        comp["dense_bf16_operands"] = {"ms_per_step": b_ms, "value": batch * n / (b_ms * 1e-3)}
        bp.close()
        # the O(n log n) route of Alg. 1 on the same workload
        fp = Plan(n, W["rho"], W["v"], route="fast")
        f_ms2 = time_pair(torch, lambda: fp.forward(x, out=y), lambda: fp.adjoint(y, out=xr),
                          max(3, args.steps // 4), 1)[0]
        comp["fast_route"] = {"ms_per_step": f_ms2, "value": batch * n / (f_ms2 * 1e-3)}
        fp.close()
        # the same workload at n = 32 (2^20 AR(0.95) signals), both FP32-accurate configurations
        W32 = workloads.workload2(32)
        x32 = torch.from_numpy(W32["x"]).to(dev)
        y32 = torch.empty_like(x32)
        r32 = torch.empty_like(x32)
        n32 = {}
        for dt in ("f32", "f32split"):
            p32 = Plan(32, W32["rho"], W32["v"], route="auto", dtype=dt)
            t32 = time_pair(torch, lambda: p32.forward(x32, out=y32), lambda: p32.adjoint(y32, out=r32),
                            args.steps, args.warmup)[0]
            n32[dt] = {"ms_per_step": t32, "value": x32.shape[0] * 32 / (t32 * 1e-3),
                       "hbm_gbs": 2 * 2 * x32.numel() * 4 / (t32 * 1e-3) / 1e9}
            p32.close()
        comp["n32_workload"] = n32
        del x32, y32, r32
        # workload 1: FP64 signals, n = 64, unit self-loop at vertex 0 (the DST-VII), 1,024
        # N(0,1) signals; latency-bound (0.5 MiB each way), so time only, per route
        W1 = workloads.workload1()
        x1 = torch.from_numpy(W1["x"]).to(dev)
        y1 = torch.empty_like(x1)
        r1 = torch.empty_like(x1)
        fp64 = {"workload": "n=64, rho=1, v=e_0 (DST-VII), 1024 N(0,1) signals, FP64"}
        for rt in ("auto", "fast"):
            p1 = Plan(64, W1["rho"], W1["v"], route=rt, dtype="f64")
            t1 = time_pair(torch, lambda: p1.forward(x1, out=y1), lambda: p1.adjoint(y1, out=r1),
                           max(20, args.steps), 2)
            fp64[p1.route if rt == "auto" else "fast_route"] = {"ms_per_step": t1[0],
                                                                "median_launch_ms": 0.5 * (t1[3] + t1[4])}
            p1.close()
        comp["fp64_self_loop_n64"] = fp64
        del x1, y1, r1
        # a mid-size graph: n = 1024, 8,192 N(0,1) signals (the O(n log n) route against the
        # dense products in FP32 and split-BF16 arithmetic)
        W3 = workloads.workload3(1024, "dense", batch=8192)
        x3 = torch.from_numpy(W3["x"]).to(dev)
        y3 = torch.empty_like(x3)
        r3 = torch.empty_like(x3)
        mid = {}
        for name, kw in (("fast", dict(route="fast")), ("dense", dict(route="dense")),
                         ("dense_f32split", dict(route="dense", dtype="f32split"))):
            pm = Plan(1024, W3["rho"], W3["v"], **kw)
            tm = time_pair(torch, lambda: pm.forward(x3, out=y3), lambda: pm.adjoint(y3, out=r3),
                           max(20, args.steps), 2)
            mid[name] = {"ms_per_step": tm[0], "value": 8192 * 1024 / (tm[0] * 1e-3)}
            pm.close()
        A = torch.randn(1024, 1024, device=dev)
        At = A.t().contiguous()
        tm = time_pair(torch, lambda: torch.matmul(x3, A, out=y3), lambda: torch.matmul(y3, At, out=r3),
                       max(3, args.steps // 4), 2)[0]
        mid["gft_torch_matmul"] = {"ms_per_step": tm, "value": 8192 * 1024 / (tm * 1e-3)}
        comp["n1024_workload"] = mid
        del A, At, x3, y3, r3
        # large graphs: 256 N(0,1) signals, dense unit v, rho = 0.5
        for nl in (1024, 4096, 16384):
            W3 = workloads.workload3(nl, "dense")
            x3 = torch.from_numpy(W3["x"]).to(dev)
            y3 = torch.empty_like(x3)
            r3 = torch.empty_like(x3)
            large = {}
            for rt in ("dense", "gft", "fast"):
                p3 = Plan(nl, W3["rho"], W3["v"], route=rt)
                t3 = time_pair(torch, lambda: p3.forward(x3, out=y3), lambda: p3.adjoint(y3, out=r3),
                               max(20, args.steps), 2)
                large[rt] = {"ms_per_step": t3[0], "value": 256 * nl / (t3[0] * 1e-3)}
                if rt == "fast":
                    # FP64-vector roofline of the FAST kernels (Alg. 1): algorithmic flops of
                    # 256 signals per launch over the mean launch time (HIP events)
                    f32f, f64f = fast_flops_per_signal(nl, 12)
                    lm = 0.5 * (t3[1] + t3[2])
                    ach = 256 * (f32f + f64f) / (lm * 1e-3) / 1e12
                    large["fast_roofline"] = {
                        "bound": "alu", "achieved": ach, "peak": 78.6, "unit": "TFLOP/s", "frac": ach / 78.6,
                        "kernel": "k_fast_fwd / k_fast_adj", "avg_launch_ms": lm,
                        "median_launch_ms": 0.5 * (t3[3] + t3[4]),
                        "flops_per_signal": {"fp32": f32f, "fp64": f64f},
                        "flop_formula": "5 (n/2) log2(n/2) [fp32 DCT] + 5 n log2 n [DST-I] + 5 (2n) log2(2n) "
                                        "[grid DST] + 2 (w+2) n [window gather, w=12], fp64 except the DCT; "
                                        "peak = FP64 vector 78.6 TFLOP/s (FP32 counted against it too)"}
                p3.close()
            if nl <= 4096:
                # the split-BF16 dense product (FP32 accuracy; plans up to n = 4096)
                ps = Plan(nl, W3["rho"], W3["v"], route="dense", dtype="f32split")
                t3 = time_pair(torch, lambda: ps.forward(x3, out=y3), lambda: ps.adjoint(y3, out=r3),
                               max(20, args.steps), 2)
                large["dense_f32split"] = {"ms_per_step": t3[0], "value": 256 * nl / (t3[0] * 1e-3)}
                ps.close()
            # AUTO as a user gets it (at n = 1024 it runs batches below 1,024 signals on the
            # FAST route and reports the dense route it keeps for larger ones)
            torch.cuda.synchronize()
            t_plan = time.perf_counter()
            pa = Plan(nl, W3["rho"], W3["v"], route="auto")
            torch.cuda.synchronize()
            pa_ms = (time.perf_counter() - t_plan) * 1e3
            t3 = time_pair(torch, lambda: pa.forward(x3, out=y3), lambda: pa.adjoint(y3, out=r3),
                           max(20, args.steps), 2)
            large["dct_plus_auto"] = {"plan_route": pa.route, "ms_per_step": t3[0],
                                      "value": 256 * nl / (t3[0] * 1e-3), "plan_ms_host": pa_ms}
            pa.close()
            A = torch.randn(nl, nl, device=dev)
            At = A.t().contiguous()
            t3 = time_pair(torch, lambda: torch.matmul(x3, A, out=y3), lambda: torch.matmul(y3, At, out=r3),
                           max(3, args.steps // 4), 2)[0]
            large["gft_torch_matmul"] = {"ms_per_step": t3, "value": 256 * nl / (t3 * 1e-3)}
            # the same workload's second graph: one added edge of weight 1 (rho = 2,
            # v = (e_i - e_j)/sqrt(2)), through AUTO and the FAST route
            W3e = workloads.workload3(nl, "edge")
            xe = torch.from_numpy(W3e["x"]).to(dev)
            edge = {"rho": W3e["rho"], "edge": [int(t) for t in np.flatnonzero(W3e["v"])]}
            for rt in ("auto", "fast"):
                pe = Plan(nl, W3e["rho"], W3e["v"], route=rt)
                te = time_pair(torch, lambda: pe.forward(xe, out=y3), lambda: pe.adjoint(y3, out=r3),
                               max(20, args.steps), 2)
                edge["dct_plus_auto" if rt == "auto" else rt] = {"ms_per_step": te[0],
                                                                 "value": 256 * nl / (te[0] * 1e-3)}
                pe.close()
            large["added_edge"] = edge
            del xe
            comp["n1024_256_signals" if nl == 1024 else f"n{nl}_workload"] = large
            del A, At, x3, y3, r3
            torch.cuda.empty_cache()
        # rank-k updates (Cor. 4.5): three added edges (weights in [0.5, 2]) on the workload-2
        # batch; the composite Cauchy factor goes through the same factored kernel
        g3 = np.random.default_rng(4242)
        rk_rhos, rk_V = [], []
        for _ in range(3):
            i3, j3 = sorted(int(t) for t in g3.choice(n, 2, replace=False))
            r3, v3 = workloads.edge_update(n, i3, j3, float(g3.uniform(0.5, 2.0)))
            rk_rhos.append(r3)
            rk_V.append(v3)
        torch.cuda.synchronize()
        t_plan = time.perf_counter()
        pk = Plan(n, rk_rhos, rk_V, route="dense", dtype="f32split", factored=True)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t_plan) * 1e3
        tk = time_pair(torch, lambda: pk.forward(x, out=y), lambda: pk.adjoint(y, out=xr), args.steps, args.warmup)
        pk.close()
        # DTT+ (Sec. 4.3): a rank-one update of the ADST graph, the DST-VII as the base
        # (general-base plan: the dense product with X^T, split-BF16)
        lam7, U7 = workloads.adst_base(n)
        pd = Plan(n, W["rho"], W["v"], dtype="f32split", base=(lam7, U7))
        td = time_pair(torch, lambda: pd.forward(x, out=y), lambda: pd.adjoint(y, out=xr), args.steps, args.warmup)
        pd.close()
        comp["dtt_plus_adst_n64"] = {"ms_per_step": td[0], "value": batch * n / (td[0] * 1e-3),
                                     "median_launch_ms": 0.5 * (td[3] + td[4]),
                                     "base": "ADST graph (DST-VII), general-base plan, dense X^T"}
        comp["rank3_edges_n64"] = {"ms_per_step": tk[0], "value": batch * n / (tk[0] * 1e-3),
                                   "median_launch_ms": 0.5 * (tk[3] + tk[4]), "plan_ms_host": plan_ms,
                                   "updates": "3 added edges, weights U[0.5, 2]; DENSE factored split-BF16"}
        result["comparators"] = comp
        for k, v in comp.items():
            print(k, v, file=sys.stderr, flush=True)

    if not args.no_extra:
        result["selection"] = bench_selection(torch, dev, args.steps, args.warmup)
        print("selection", result["selection"], file=sys.stderr, flush=True)
        result["gradient"] = bench_gradient(torch, dev, args.steps, args.warmup)
        print("gradient", result["gradient"], file=sys.stderr, flush=True)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(W, args.cpu_sample)
    plan.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
