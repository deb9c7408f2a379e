"""Seeded synthetic inputs for the DCT+ workloads.

This module holds only random-number draws and shapes: none of the
transform's arithmetic.  Both the HIP path (tests, benchmark) and the FP64
oracle consume the arrays it returns, so the two sides see bit-identical
inputs.

Generators use numpy PCG64 with ``seed = 1000 * workload_id + sub`` and draw
in the fixed order (rho, v, vertex indices, signals).

Workloads (the sizes and distributions of the paper's experiments, Sec. 5,
scaled to a GPU):
  1  n = 64, self-loop of weight 1 at vertex 0 (v = e_0), 1024 N(0,1) signals, FP64.
  2  n in {32, 64}, v a random unit vector, rho ~ U[0.1, 2], 2**20 AR(1)
     signals with correlation 0.95 (image-row-like; the paper uses AR(0.99)
     rows for its runtime study), FP32.
  3  n in {1024, 4096, 16384}, 256 N(0,1) signals; v dense unit with rho = 0.5,
     or one added edge of weight 1: v = (e_i - e_j)/sqrt(2), rho = 2.
  4  10,000 blocks, n uniform on {4, 8, 16, 32, 64}, 64 AR(0.9) signals each,
     K = 8 candidate updates per block (self-loop at either end with weight
     w ~ U[0.25, 2], or one added edge of weight 1 between random vertices).
  5  n = 256, 65,536 N(0,1) signals, rho = 1, v a random unit vector.
"""
from __future__ import annotations

import numpy as np


def rng(workload: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * workload + sub))


def ar1(g: np.random.Generator, batch: int, n: int, r: float, dtype=np.float32) -> np.ndarray:
    """Stationary AR(1) rows: x_0 = e_0, x_t = r x_{t-1} + sqrt(1 - r^2) e_t, e ~ N(0,1)."""
    e = g.standard_normal((batch, n), dtype=np.float32 if dtype == np.float32 else np.float64)
    x = np.empty((batch, n), dtype=dtype)
    c = np.sqrt(1.0 - r * r)
    x[:, 0] = e[:, 0]
    for t in range(1, n):
        x[:, t] = r * x[:, t - 1] + c * e[:, t]
    return x


def unit_vector(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal(n)
    return v / np.linalg.norm(v)


def edge_vector(n: int, i: int, j: int) -> np.ndarray:
    v = np.zeros(n)
    v[i] = 1.0 / np.sqrt(2.0)
    v[j] = -1.0 / np.sqrt(2.0)
    return v


def edge_update(n: int, i: int, j: int, w: float):
    """(rho, v) of an added edge (i, j) of weight w: w (e_i - e_j)(e_i - e_j)^T = 2w v v^T
    with the unit v = (e_i - e_j)/sqrt(2)."""
    return 2.0 * float(w), edge_vector(n, i, j)


def adst_base(n: int):
    """The base graph of the DTT+ workloads as a (lambda, U) input: the path with a unit
    self-loop at vertex 0 (the ADST graph, Sec. 4.3), whose eigenpairs have the closed
    form lambda_k = 2 - 2 cos(pi (2k+1)/(2n+1)), U[j, k] = 2/sqrt(2n+1) sin(pi (j+1)(2k+1)/(2n+1))
    (the DST-VII), ascending in k."""
    t = np.pi * (2.0 * np.arange(n) + 1.0) / (2 * n + 1)
    lam = 2.0 - 2.0 * np.cos(t)
    U = (2.0 / np.sqrt(2 * n + 1)) * np.sin(np.outer(np.arange(1, n + 1), t))
    return lam, U


def workload1(batch: int = 1024, n: int = 64):
    g = rng(1)
    v = np.zeros(n)
    v[0] = 1.0
    x = g.standard_normal((batch, n))
    return dict(n=n, rho=1.0, v=v, x=x)


def workload2(n: int, batch: int = 1 << 20, sub: int = 0):
    g = rng(2, sub * 100 + n)
    rho = float(g.uniform(0.1, 2.0))
    v = unit_vector(g, n)
    x = ar1(g, batch, n, 0.95)
    return dict(n=n, rho=rho, v=v, x=x)


def workload3(n: int, kind: str = "dense", batch: int = 256, sub: int = 0):
    g = rng(3, sub * 100000 + n + (0 if kind == "dense" else 50000))
    if kind == "dense":
        rho = 0.5
        v = unit_vector(g, n)
        i = j = -1
    else:
        rho = 2.0
        i, j = (int(t) for t in g.choice(n, size=2, replace=False))
        v = edge_vector(n, i, j)
    x = g.standard_normal((batch, n)).astype(np.float32)
    return dict(n=n, rho=rho, v=v, x=x, edge=(i, j))


SELECT_SIZES = (4, 8, 16, 32, 64)


def workload4(blocks: int = 10000, signals: int = 64, K: int = 8, sub: int = 0):
    """Block descriptors for progressive selection.

    Returns n[b], cand[b, k] = (kind, i, j, w) with kind 0 = self-loop
    (rho = w, v = e_i) and kind 1 = added edge of weight w (rho = 2w,
    v = (e_i - e_j)/sqrt(2)), and the signals concatenated block after block
    (offset[b] = start row of block b in a [sum, n_b]-ragged float array)."""
    g = rng(4, sub)
    n = g.choice(np.array(SELECT_SIZES), size=blocks)
    kinds = g.integers(0, 3, size=(blocks, K))            # 0: loop at 0, 1: loop at n-1, 2: edge
    w = g.uniform(0.25, 2.0, size=(blocks, K))
    cand = np.zeros((blocks, K, 4), dtype=np.float64)
    for b in range(blocks):
        nb = int(n[b])
        for k in range(K):
            if kinds[b, k] == 0:
                cand[b, k] = (0, 0, 0, w[b, k])
            elif kinds[b, k] == 1:
                cand[b, k] = (0, nb - 1, nb - 1, w[b, k])
            else:
                i, j = g.choice(nb, size=2, replace=False)
                cand[b, k] = (1, min(i, j), max(i, j), 1.0)
    offs = np.zeros(blocks + 1, dtype=np.int64)
    offs[1:] = np.cumsum(n.astype(np.int64) * signals)
    x = np.empty(int(offs[-1]), dtype=np.float32)
    for nb in SELECT_SIZES:
        idx = np.nonzero(n == nb)[0]
        if len(idx) == 0:
            continue
        xs = ar1(g, len(idx) * signals, nb, 0.9).reshape(len(idx), signals * nb)
        for r, b in enumerate(idx):
            x[offs[b]:offs[b + 1]] = xs[r]
    return dict(n=n.astype(np.int32), cand=cand, x=x, offsets=offs, signals=signals, K=K)


def workload5(n: int = 256, batch: int = 65536):
    g = rng(5)
    rho = 1.0
    v = unit_vector(g, n)
    x = g.standard_normal((batch, n)).astype(np.float32)
    return dict(n=n, rho=rho, v=v, x=x)
