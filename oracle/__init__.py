"""FP64 reference (oracle) for the DCT+ transform of arXiv 2409.08970.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code,
header, table or constant generator with the HIP library, and it imports
nothing from it.

Routes
------
* ``basis(n, rho, v)``: the plain definition.  Assemble ``L = L_path +
  rho v v^T`` (Sec. 2, Def. of rank-one updates; Prop. 2.4 for the path
  Laplacian), diagonalise it with the hand-written cyclic Jacobi solver in
  ``oracle.c``, sort eigenpairs ascending (Lemma 4.1 order) and fix signs.
* ``semi_forward / semi_adjoint``: Thm 3.1 evaluated row by row, with the
  secular roots found by bisection in offset form.  Used where Jacobi is too
  slow (n > 1024); checked against the Jacobi route by the tests.
* ``grad_perturbation``: first-order eigenvector perturbation applied to
  ``y = X^T x`` (derivation in the docstring), plus ``loss_l1``.
* ``select_block``: progressive selection with pruning (Thm 3.4, Fig. 2,
  Sec. 5 pruning experiment); each candidate's factor comes from the Jacobi
  eigenvectors or, where an update makes eigenvalues coincide, from the
  secular roots with deflation (``candidate_factor``).

Sign convention: eigenvector ``x_i`` gets ``rho * v^T x_i > 0``
(equivalently ``a_i > 0`` in ``X^T = diag(a) C(mu, lambda) diag(z) U^T``);
rows with ``v^T x_i ~ 0`` get their largest ``|U^T x_i|`` entry positive, so
``rho = 0`` gives the orthonormal DCT-II exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# Threshold on |v^T x_i| / ||v|| below which a Jacobi eigenvector is treated
# as a deflated direction for the sign rule.  Jacobi eigenvector components
# carry errors ~ eps * ||L|| / gap, far below this for the sizes used here.
SIGN_DEFL_TOL = 1e-9
# Relative tolerance below which z_k is an exact zero (deflation, Sec. 4).
DEFL_TOL = 1e-13


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _get():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_laplacian.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.orc_jacobi.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int]
        lib.orc_jacobi.restype = ctypes.c_int
        lib.orc_apply.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int64, ctypes.c_int]
        lib.orc_secular_roots.argtypes = [ctypes.c_int, ctypes.c_double, dp, ip, dp, ip]
        lib.orc_secular_roots.restype = ctypes.c_int
        lib.orc_cauchy_apply.argtypes = [ctypes.c_int, dp, ip, dp, ip, dp, dp, ctypes.c_int64,
                                         ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# --------------------------------------------------------------------------
# Plain definition: L, Jacobi, sign convention, apply.
# --------------------------------------------------------------------------
def laplacian(n: int, rho: float, v) -> np.ndarray:
    """L = L_path + rho v v^T (unit-weight path graph), dense FP64."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (n,)
    L = np.empty((n, n), dtype=np.float64)
    _get().orc_laplacian(n, float(rho), _dp(v), _dp(L))
    return L


def eigh_jacobi(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic Jacobi: returns (eigenvalues ascending, eigenvectors as columns)."""
    n = A.shape[0]
    W = np.ascontiguousarray(A, dtype=np.float64).copy()
    V = np.empty((n, n), dtype=np.float64)
    sweeps = _get().orc_jacobi(n, _dp(W), _dp(V), tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    ev = np.diag(W).copy()
    order = np.argsort(ev, kind="stable")
    return ev[order], np.ascontiguousarray(V[:, order])


def dct2_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II basis U with columns u_k: U[j, k] = c_k cos(pi k (2j+1) / 2n).

    The path-graph GFT is the DCT-II (Sec. 1, Def. of DCT+)."""
    j = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    U = np.cos(np.pi * k * (2 * j + 1) / (2.0 * n)) * np.sqrt(2.0 / n)
    U[:, 0] = np.sqrt(1.0 / n)
    return U


def fix_signs(X: np.ndarray, rho: float, v, tol: float = SIGN_DEFL_TOL, base=None) -> np.ndarray:
    """Apply the sign convention to the eigenvector columns of X (copy).  base: the
    unperturbed basis (columns) for the deflated rows' rule, the DCT-II by default."""
    n = X.shape[0]
    v = np.asarray(v, dtype=np.float64)
    X = X.copy()
    vx = v @ X
    scale = tol * max(np.linalg.norm(v), 1e-300)
    U = base
    for i in range(n):
        if rho != 0.0 and abs(vx[i]) > scale:
            if rho * vx[i] < 0:
                X[:, i] = -X[:, i]
        else:
            if U is None:
                U = dct2_matrix(n)
            c = U.T @ X[:, i]
            if c[np.argmax(np.abs(c))] < 0:
                X[:, i] = -X[:, i]
    return X


def basis(n: int, rho: float, v):
    """(mu, X): eigenvalues ascending and signed eigenvectors (columns) of L_path + rho v v^T."""
    mu, X = eigh_jacobi(laplacian(n, rho, v))
    return mu, fix_signs(X, rho, v)


# --------------------------------------------------------------------------
# A rank-one update of a general base (Thm 3.1 for any symmetric base; Thm 3.2).
# --------------------------------------------------------------------------
def basis_general(lam, U, rho: float, v):
    """(mu, X) of U diag(lam) U^T + rho v v^T: Jacobi on the assembled matrix, eigenvalues
    ascending; signs rho v^T x_i > 0, and for rows orthogonal to v the largest |U^T x_i|
    entry positive (the base's own vectors, as the DCT-II is for the path)."""
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    L = (U * lam[None, :]) @ U.T + float(rho) * np.outer(v, v)
    L = 0.5 * (L + L.T)
    mu, X = eigh_jacobi(L)
    return mu, fix_signs(X, rho, v, base=U)


def dst7_basis(n: int):
    """(lambda, U) of the ADST graph (the path with a unit self-loop at vertex 0): the
    DST-VII, lambda_k = 2 - 2 cos(pi (2k+1)/(2n+1)), U[j, k] = 2/sqrt(2n+1) sin(pi (2k+1)(j+1)/(2n+1))
    (Sec. 4.3, the DTT family; closed form of the self-loop case)."""
    k = np.arange(n)
    lam = 2.0 - 2.0 * np.cos(np.pi * (2 * k + 1) / (2 * n + 1))
    j = np.arange(n)[:, None]
    U = 2.0 / np.sqrt(2 * n + 1) * np.sin(np.pi * (2 * k[None, :] + 1) * (j + 1) / (2 * n + 1))
    return lam, U


# --------------------------------------------------------------------------
# Rank-k updates (Sec. 4.3, Cor. 4.5): L_k = L_path + sum_j rho_j v_j v_j^T.
# --------------------------------------------------------------------------
def laplacian_rank_k(n: int, rhos, vs) -> np.ndarray:
    """L_path + sum_j rho_j v_j v_j^T, dense FP64 (Cor. 4.5's L_k)."""
    L = laplacian(n, 0.0, np.zeros(n))
    for rho, v in zip(rhos, vs):
        v = np.asarray(v, dtype=np.float64)
        L += float(rho) * np.outer(v, v)
    return L


def fix_signs_rank_k(X: np.ndarray, rhos, vs, tol: float = SIGN_DEFL_TOL) -> np.ndarray:
    """Sign convention of a chain of rank-one updates (Cor. 4.5 applied one update at a
    time, each stage with the rank-one convention): column i gets rho_j v_j^T x_i > 0 for
    the last update j whose v_j is not orthogonal to x_i (an eigenvector orthogonal to
    v_j is a deflated direction of stage j and keeps the sign it had before it); columns
    orthogonal to every v_j get their largest |U^T x_i| entry positive."""
    n = X.shape[0]
    X = X.copy()
    U = None
    for i in range(n):
        for rho, v in reversed(list(zip(rhos, vs))):
            v = np.asarray(v, dtype=np.float64)
            t = float(v @ X[:, i])
            if rho != 0.0 and abs(t) > tol * max(np.linalg.norm(v), 1e-300):
                if rho * t < 0:
                    X[:, i] = -X[:, i]
                break
        else:
            if U is None:
                U = dct2_matrix(n)
            c = U.T @ X[:, i]
            if c[np.argmax(np.abs(c))] < 0:
                X[:, i] = -X[:, i]
    return X


def basis_rank_k(n: int, rhos, vs):
    """(mu, X) of L_path + sum_j rho_j v_j v_j^T: Jacobi on the assembled matrix, eigenvalues
    ascending, signs by ``fix_signs_rank_k``."""
    mu, X = eigh_jacobi(laplacian_rank_k(n, rhos, vs))
    return mu, fix_signs_rank_k(X, rhos, vs)


def forward(X: np.ndarray, x) -> np.ndarray:
    """y = X^T x for every row x of a [batch, n] array (FP64)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = X.shape[0]
    xb = x.reshape(-1, n)
    out = np.empty_like(xb)
    _get().orc_apply(n, _dp(np.ascontiguousarray(X)), _dp(xb), _dp(out), xb.shape[0], 0)
    return out.reshape(x.shape)


def adjoint(X: np.ndarray, y) -> np.ndarray:
    """x = X y for every row y of a [batch, n] array (FP64)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = X.shape[0]
    yb = y.reshape(-1, n)
    out = np.empty_like(yb)
    _get().orc_apply(n, _dp(np.ascontiguousarray(X)), _dp(yb), _dp(out), yb.shape[0], 1)
    return out.reshape(y.shape)


def path_eigenvalues(n: int) -> np.ndarray:
    """lambda_k = 2 - 2 cos(pi k / n), k = 0..n-1 (Sec. 4.2, roots of U_{n-1} shifted)."""
    return 2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n)


# --------------------------------------------------------------------------
# Semi-oracle: Thm 3.1 row by row, secular roots by bisection.
# --------------------------------------------------------------------------
def _dct2(x):
    # Library FFT primitive (orthonormal DCT-II along the last axis).
    import scipy.fft
    return scipy.fft.dct(np.asarray(x, dtype=np.float64), type=2, norm="ortho", axis=-1)


def semi_plan(n: int, rho: float, v, defl_tol: float = DEFL_TOL):
    """z = U^T v (deflated), roots in offset form: dict(z, origin, tau, kind, mu)."""
    z = _dct2(np.asarray(v, dtype=np.float64))
    z = np.where(np.abs(z) <= defl_tol * np.linalg.norm(z), 0.0, z)
    origin = np.zeros(n, dtype=np.int32)
    tau = np.zeros(n, dtype=np.float64)
    kind = np.zeros(n, dtype=np.int32)
    if rho == 0.0 or not np.any(z):
        origin[:] = np.arange(n)
        kind[:] = 1
    else:
        z = np.ascontiguousarray(z)
        rc = _get().orc_secular_roots(n, float(rho), _dp(z), _ip(origin), _dp(tau), _ip(kind))
        assert rc == 0
    mu = path_eigenvalues(n)[origin] + tau
    return dict(z=z, origin=origin, tau=tau, kind=kind, mu=mu, n=n, rho=float(rho))


def semi_apply(plan, sd, adjoint: bool = False) -> np.ndarray:
    """Apply diag(a) C(mu, lambda) diag(z) (or its transpose) in the DCT domain."""
    n = plan["n"]
    sd = np.ascontiguousarray(sd, dtype=np.float64).reshape(-1, n)
    out = np.empty_like(sd)
    _get().orc_cauchy_apply(n, _dp(plan["z"]), _ip(plan["origin"]), _dp(plan["tau"]),
                            _ip(plan["kind"]), _dp(sd), _dp(out), sd.shape[0], int(adjoint))
    return out


def semi_forward(n: int, rho: float, v, x, plan=None) -> np.ndarray:
    """y = X^T x via Thm 3.1 (DCT-II, then the Cauchy rows)."""
    plan = plan or semi_plan(n, rho, v)
    return semi_apply(plan, _dct2(np.asarray(x, dtype=np.float64).reshape(-1, n)))


def semi_adjoint(n: int, rho: float, v, y, plan=None) -> np.ndarray:
    """x = X y via the transpose of Thm 3.1 (Cauchy transpose, then DCT-III)."""
    import scipy.fft
    plan = plan or semi_plan(n, rho, v)
    sd = semi_apply(plan, np.asarray(y, dtype=np.float64).reshape(-1, n), adjoint=True)
    return scipy.fft.idct(sd, type=2, norm="ortho", axis=-1)


def semi_rows(plan, rows) -> np.ndarray:
    """Explicit rows of M = diag(a) C(mu, lambda) diag(z) (deflated rows are e_k)."""
    n = plan["n"]
    lam = path_eigenvalues(n)
    out = np.zeros((len(rows), n))
    for r, i in enumerate(rows):
        o = plan["origin"][i]
        if plan["kind"][i] == 1:
            out[r, o] = 1.0
            continue
        j = np.arange(n)
        d = 4.0 * np.sin(np.pi * (j - o) / (2.0 * n)) * np.sin(np.pi * (j + o) / (2.0 * n))
        gap = plan["tau"][i] - d
        row = np.where(plan["z"] != 0.0, plan["z"] / np.where(gap == 0, 1.0, gap), 0.0)
        out[r] = row / np.linalg.norm(row)
    del lam
    return out


# --------------------------------------------------------------------------
# Gradient of a loss of y = X^T x with respect to x, rho and v.
# --------------------------------------------------------------------------
def loss_l1(y) -> float:
    """Mean absolute value of the coefficients."""
    return float(np.mean(np.abs(y)))


def loss_l1_grad(y) -> np.ndarray:
    """d loss / d y for loss_l1, with sign(0) = 0."""
    return np.sign(y) / y.size


def grad_perturbation(mu, X, rho: float, v, y, gy):
    """(dx, drho, dv) for y = X^T x given gy = d loss / d y.

    With eigenpairs L x_i = mu_i x_i, first-order perturbation gives
    dx_i = sum_{k != i} x_k (x_k^T dL x_i) / (mu_i - mu_k), and
    dL = drho v v^T + rho (dv v^T + v dv^T) for L = L_path + rho v v^T.
    Collecting terms with G_ik = sum_b gy_bi y_bk, A_ik = G_ik / (mu_i - mu_k)
    (A_ii = 0) and w = X^T v:
        d loss / d x   = X gy
        d loss / d rho = w^T A w
        d loss / d v   = rho X (A + A^T) w
    """
    y = np.asarray(y, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    n = X.shape[0]
    dx = gy @ X.T
    G = gy.T @ y
    diff = mu[:, None] - mu[None, :]
    np.fill_diagonal(diff, 1.0)
    A = G / diff
    np.fill_diagonal(A, 0.0)
    w = X.T @ np.asarray(v, dtype=np.float64)
    drho = float(w @ A @ w)
    dv = rho * (X @ ((A + A.T) @ w))
    assert dx.shape[1] == n
    return dx, drho, dv


# --------------------------------------------------------------------------
# Progressive selection with pruning (Thm 3.4, Fig. 2, Sec. 5).
# --------------------------------------------------------------------------
def candidate_update(n: int, kind: int, i: int, j: int, w: float):
    """(rho, v) of one candidate rank-one update (Prop. 2.4 baby Laplacians).

    kind 0: self-loop of weight w at vertex i  -> rho = w, v = e_i.
    kind 1: added edge (i, j) of weight w      -> rho = 2 w, v = (e_i - e_j) / sqrt(2).
    """
    v = np.zeros(n)
    if kind == 0:
        v[i] = 1.0
        return float(w), v
    v[i] = 1.0 / np.sqrt(2.0)
    v[j] = -1.0 / np.sqrt(2.0)
    return 2.0 * float(w), v


def path_quadratic_form(x) -> np.ndarray:
    """x^T L_path x = sum_j (x_{j+1} - x_j)^2 per row."""
    x = np.asarray(x, dtype=np.float64)
    return np.sum(np.diff(x, axis=-1) ** 2, axis=-1)


def candidate_factor(n: int, kind: int, i: int, j: int, w: float, method: str = "jacobi") -> np.ndarray:
    """C~ = X^T U of one candidate: row i holds eigenvector x_i in the DCT domain (Thm 3.1).

    method "jacobi": eigenvectors of the assembled Laplacian (cyclic Jacobi,
    sign convention of fix_signs).  method "semi": the factor
    diag(a) C(mu, lambda) diag(z) from the secular roots with deflation
    (Thm 3.1, Remark 1), which fixes the basis inside a multiple eigenvalue
    the way the method does (deflated DCT vector first)."""
    rho, v = candidate_update(n, kind, i, j, w)
    if method == "jacobi":
        _, X = basis(n, rho, v)
        return X.T @ dct2_matrix(n)
    if method == "semi":
        return semi_rows(semi_plan(n, rho, v), range(n))
    raise ValueError(method)


def select_block(x, cands, c_p: int, prune_tau: float, factor: str = "jacobi"):
    """One block: returns (best index, cost per candidate, winner coefficients, pruned mask).

    x: [S, n] signals.  cands: list of (kind, i, j, w).
    Signal s is pruned iff x_s^T L_path x_s <= prune_tau * ||x_s||^2; a pruned
    signal keeps only the upper-left c_p x c_p block of
    C~_r = diag(a_r) C(mu_r, lambda) diag(z_r) = X_r^T U (Thm 3.4), others use
    the full transform.  cost_r = sum over signals of ||yhat||_1; ties go to the
    lowest r.  factor: how C~_r is formed (see candidate_factor).
    """
    x = np.asarray(x, dtype=np.float64)
    S, n = x.shape
    U = dct2_matrix(n)
    sd = x @ U                                   # DCT-II of every signal
    pruned = path_quadratic_form(x) <= prune_tau * np.sum(x * x, axis=-1)
    costs = np.zeros(len(cands))
    outs = []
    for r, (kind, i, j, w) in enumerate(cands):
        Ct = candidate_factor(n, int(kind), int(i), int(j), float(w), factor)
        yfull = sd @ Ct.T
        ypr = np.zeros_like(yfull)
        ypr[:, :c_p] = sd[:, :c_p] @ Ct[:c_p, :c_p].T
        yhat = np.where(pruned[:, None], ypr, yfull)
        costs[r] = np.sum(np.abs(yhat))
        outs.append(yhat)
    best = int(np.argmin(costs))
    return best, costs, outs[best], pruned
