"""DCT+ on AMD MI355X: the graph Fourier transform of a path graph after a
rank-one Laplacian update, L = L_path + rho v v^T (arXiv 2409.08970).

The compute lives in ``libdctplus.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/dctplus.h``).  This package marshals torch tensors into it:

    plan = Plan(n, rho, v, route="auto", dtype="f32")
    y = plan.forward(x)        # x: [batch, n] device tensor
    x2 = plan.adjoint(y)
    y = dctplus(x, rho, v)     # differentiable in x, rho and v
    sel = SelectPlan(n_blocks, cand, S=64)   # progressive selection with pruning
    best, cost, y = sel.select(x)

torch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes

from . import _binding as B
from ._binding import (DctPlusError, dctplus_adjoint, dctplus_default_opts, dctplus_forward, dctplus_grad,
                       dctplus_grad_noalloc, dctplus_plan_general, dctplus_plan_rank_k, dctplus_tune,
                       dctplus_last_error, dctplus_plan, dctplus_plan_destroy, dctplus_plan_info,
                       dctplus_plan_table, dctplus_select, dctplus_select_destroy, dctplus_select_factor,
                       dctplus_select_plan, dctplus_select_size, dctplus_select_tune, dctplus_status_string)

__all__ = [
    "Plan", "DctPlusFn", "dctplus", "DctPlusError", "dctplus_plan", "dctplus_forward", "dctplus_adjoint",
    "dctplus_grad", "dctplus_grad_noalloc", "dctplus_plan_rank_k", "dctplus_plan_general", "dctplus_tune", "dctplus_plan_info", "dctplus_plan_table", "dctplus_plan_destroy", "dctplus_status_string",
    "dctplus_last_error", "dctplus_default_opts", "SelectPlan", "dctplus_select_plan", "dctplus_select",
    "dctplus_select_factor", "dctplus_select_size", "dctplus_select_destroy", "dctplus_select_tune",
]

_ROUTES = {"auto": B.DCTPLUS_ROUTE_AUTO, "fast": B.DCTPLUS_ROUTE_FAST, "dense": B.DCTPLUS_ROUTE_DENSE,
           "gft": B.DCTPLUS_ROUTE_GFT}
_DTYPES = {"f32": B.DCTPLUS_F32, "f64": B.DCTPLUS_F64, "bf16": B.DCTPLUS_BF16, "f32split": B.DCTPLUS_F32_SPLIT}
ROUTE_NAMES = {v: k for k, v in _ROUTES.items()}


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """Owns one dctplus plan (device tables built on the GPU in FP64).

    rho, v: one rank-one update (a float and n values), or k updates for a rank-k plan
    (k floats and a k x n array, row j = v_j; Cor. 4.5).  `route` is the route the plan
    was built for; an AUTO plan at n = 1024 (FP32) reports "dense" and still runs calls
    of fewer than 1,024 signals on the FAST route."""

    def __init__(self, n: int, rho, v, route: str = "auto", dtype: str = "f32",
                 nufft_width: int = 0, direct_kappa: float = 0.0, defl_tol: float = 0.0, device: int = -1,
                 stream=None, factored: bool = False, base=None):
        """base: None (the path graph, DCT-II) or (lambda, U) of a caller's base graph
        (dctplus_plan_general)."""
        import numpy as np
        import torch
        o = B.dctplus_default_opts()
        o.route = _ROUTES[route]
        o.dtype = _DTYPES[dtype]
        if nufft_width:
            o.nufft_width = nufft_width
        if direct_kappa:
            o.direct_kappa = direct_kappa
        if defl_tol:
            o.defl_tol = defl_tol
        if device < 0:
            device = torch.cuda.current_device()
        o.device = device
        o.factored = 1 if factored else 0
        self.n = int(n)
        rhos = np.atleast_1d(np.asarray(rho, dtype=np.float64))
        self.k = int(rhos.size)
        self.rho = float(rhos[0]) if self.k == 1 else rhos.copy()
        self.v = np.asarray(v, dtype=np.float64).reshape(self.k, -1).copy()
        if self.k == 1:
            self.v = self.v.reshape(-1)
        self.dtype = dtype
        self.device = device
        self._h = None
        with torch.cuda.device(device):
            if base is not None:
                lam, U = base
                _, self._h = B.dctplus_plan_general(self.n, lam, U, self.rho, self.v, o, _stream(stream))
            elif self.k == 1:
                _, self._h = B.dctplus_plan(self.n, self.rho, self.v, o, _stream(stream))
            else:
                _, self._h = B.dctplus_plan_rank_k(self.n, rhos, self.v, o, _stream(stream))
        info = B.dctplus_plan_info(self._h, self.n)
        self.route = ROUTE_NAMES[int(info["counts"][3])]
        self.info = info

    @property
    def handle(self):
        return self._h

    def _io_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32

    def _check(self, t):
        import torch
        if not (t.is_cuda and t.dtype == self._io_dtype() and t.dim() >= 1 and t.shape[-1] == self.n):
            raise ValueError(f"expected a CUDA tensor [..., {self.n}] of {self._io_dtype()}")
        return t.contiguous()

    def forward(self, x, out=None, stream=None):
        import torch
        x = self._check(x)
        y = torch.empty_like(x) if out is None else out
        B.dctplus_forward(self._h, x.data_ptr(), y.data_ptr(), x.numel() // self.n, _stream(stream))
        return y

    def adjoint(self, y, out=None, stream=None):
        import torch
        y = self._check(y)
        x = torch.empty_like(y) if out is None else out
        B.dctplus_adjoint(self._h, y.data_ptr(), x.data_ptr(), y.numel() // self.n, _stream(stream))
        return x

    def grad(self, y, gy, want_x: bool = True, stream=None):
        """(dx or None, drho [1] float64, dv [n] float64) for y = forward(x) and gy = dl/dy."""
        import torch
        y = self._check(y)
        gy = self._check(gy)
        gx = torch.empty_like(gy) if want_x else None
        grho = torch.zeros(1, dtype=torch.float64, device=y.device)
        gv = torch.zeros(self.n, dtype=torch.float64, device=y.device)
        B.dctplus_grad(self._h, y.data_ptr(), gy.data_ptr(), y.numel() // self.n,
                       gx.data_ptr() if gx is not None else 0, grho.data_ptr(), gv.data_ptr(), _stream(stream))
        return gx, grho, gv

    def tune(self, x, cache_path=None, stream=None):
        """Launch autotuner for batches the size of x ([batch, n] device tensor, left
        unchanged): returns (chosen [forward, adjoint], ms per config)."""
        import torch
        x = self._check(x)
        a, b = x.clone(), torch.empty_like(x)
        _, chosen, ms = B.dctplus_tune(self._h, a.data_ptr(), b.data_ptr(), x.numel() // self.n, _stream(stream),
                                       cache_path)
        return chosen, ms

    def close(self):
        if self._h:
            import torch
            torch.cuda.synchronize(self.device)
            B.dctplus_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SelectPlan:
    """Batched progressive selection (one dctplus selection plan).

    n_blocks: [nblocks] block sizes; cand: [nblocks, K, 4] (kind, i, j, w);
    S: signals per block.  select(x) takes the concatenated [sum_b S n_b]
    FP32 device signals and returns (best [nblocks] int32, cost [nblocks, K]
    FP32, y_best like x)."""

    def __init__(self, n_blocks, cand, S: int = 64, stream=None):
        import numpy as np
        import torch
        self.n_blocks = np.asarray(n_blocks, dtype=np.int32).reshape(-1).copy()
        cand = np.asarray(cand, dtype=np.float64)
        self.K = int(cand.shape[1]) if cand.ndim == 3 else int(cand.size // (4 * max(1, self.n_blocks.size)))
        self.S = int(S)
        self.device = torch.cuda.current_device()
        self._h = None
        _, self._h = B.dctplus_select_plan(self.n_blocks, self.K, self.S, cand, _stream(stream))
        self.size = B.dctplus_select_size(self._h)

    def select(self, x, c_p: int = 0, prune_tau: float = 0.1, out=None, stream=None):
        import torch
        nb = self.n_blocks.size
        if not (x.is_cuda and x.dtype == torch.float32 and x.numel() == self.size):
            raise ValueError(f"expected a CUDA FP32 tensor of {self.size} elements")
        x = x.contiguous()
        best = torch.empty(nb, dtype=torch.int32, device=x.device)
        cost = torch.empty(nb, self.K, dtype=torch.float32, device=x.device)
        y = torch.empty_like(x) if out is None else out
        B.dctplus_select(self._h, x.data_ptr(), c_p, prune_tau, best.data_ptr(), cost.data_ptr(), y.data_ptr(),
                         _stream(stream))
        return best, cost, y

    def tune(self, x, c_p: int = 0, prune_tau: float = 0.1, stream=None):
        """Time the persistent grid at 1..4 workgroups per CU on x, keep the fastest for
        later select() calls; returns (chosen, [ms per call of each candidate])."""
        import torch
        if not (x.is_cuda and x.dtype == torch.float32 and x.numel() == self.size):
            raise ValueError(f"expected a CUDA float32 tensor of {self.size} elements")
        x = x.contiguous()
        best = torch.empty(self.n_blocks.shape[0], dtype=torch.int32, device=x.device)
        cost = torch.empty(self.n_blocks.shape[0], self.K, dtype=torch.float32, device=x.device)
        y = torch.empty_like(x)
        _, chosen, ms = B.dctplus_select_tune(self._h, x.data_ptr(), c_p, prune_tau, best.data_ptr(), cost.data_ptr(),
                                              y.data_ptr(), _stream(stream))
        return chosen, ms

    def factor(self, block: int, r: int):
        return B.dctplus_select_factor(self._h, block, r, int(self.n_blocks[block]))

    def close(self):
        if self._h:
            B.dctplus_select_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DctPlusFn:
    """torch.autograd.Function for y = X(rho, v)^T x, differentiable in x, rho and v.

    The plan is rebuilt when (rho, v) change; gradients come from the
    library's adjoint and perturbation kernels (dctplus_grad)."""

    _impl = None

    @classmethod
    def _get(cls):
        if cls._impl is None:
            import torch

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, rho, v, route):
                    rv = float(rho.detach().cpu())
                    vv = v.detach().to("cpu", torch.float64).numpy()
                    plan = Plan(x.shape[-1], rv, vv, route=route)
                    y = plan.forward(x)
                    ctx.plan = plan
                    ctx.save_for_backward(y)
                    ctx.rho_meta = (rho.dtype, rho.device)
                    ctx.v_meta = (v.dtype, v.device)
                    return y

                @staticmethod
                def backward(ctx, gy):
                    (y,) = ctx.saved_tensors
                    gx, grho, gv = ctx.plan.grad(y, gy.contiguous(), want_x=ctx.needs_input_grad[0])
                    grho = grho.reshape(()).to(dtype=ctx.rho_meta[0], device=ctx.rho_meta[1])
                    gv = gv.to(dtype=ctx.v_meta[0], device=ctx.v_meta[1])
                    ctx.plan.close()
                    return gx, grho, gv, None

            cls._impl = _Fn
        return cls._impl

    @classmethod
    def apply(cls, x, rho, v, route: str = "auto"):
        return cls._get().apply(x, rho, v, route)


def dctplus(x, rho, v, route: str = "auto"):
    """Differentiable DCT+ forward of x [batch, n] (FP32, on the GPU)."""
    return DctPlusFn.apply(x, rho, v, route)
