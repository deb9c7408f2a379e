"""Pins for the FP64 oracle (CPU only).

Each check ties the oracle to something other than itself: closed forms the
paper fixes (rho = 0 gives the DCT-II, Sec. 1 and Def. of DCT+; the
self-loop graph gives a sine transform), the interlacing lemma (Lemma 4.1),
the secular equation whose roots are the new eigenvalues (Remark 1),
brute-force 50-digit eigenpairs at n <= 8, the eigenvector formula of
Lemma 4.2 / Thm 3.1 through the independent semi-oracle, finite differences
for the gradient, and the pruning bound of Thm 3.4.  The mutation tests at
the end plant plausible mistakes in copies of oracle functions and check that
some pin fails.
"""
import numpy as np
import pytest

import oracle
import workloads


def _rng(s):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# pin functions (take the oracle entry points as arguments so that the
# mutation tests can feed them broken variants)
# --------------------------------------------------------------------------
def explicit_dct2(n):
    """Orthonormal DCT-II written out entry by entry (pure Python loops)."""
    U = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            c = np.sqrt(1.0 / n) if k == 0 else np.sqrt(2.0 / n)
            U[j, k] = c * np.cos(np.pi * k * (2 * j + 1) / (2 * n))
    return U


def pin_rho_zero(basis_fn, n, seed=0):
    v = _rng(seed).standard_normal(n)
    mu, X = basis_fn(n, 0.0, v)
    lam = np.array([2 - 2 * np.cos(np.pi * k / n) for k in range(n)])
    return max(np.abs(X - explicit_dct2(n)).max(), np.abs(mu - lam).max())


def dst7(n, mirrored=False):
    """Eigenvectors of the path graph with a unit self-loop at an end vertex.

    L = L_path + e_0 e_0^T is tridiag(-1, 2, -1) with a 1 in the last diagonal
    entry; its eigenvectors are sin(pi (2k+1)(j+1) / (2n+1)) (a DST-VII), with
    eigenvalues 2 - 2 cos(pi (2k+1) / (2n+1)).  A loop at vertex n-1 mirrors j."""
    j = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    jj = (n - 1 - j) if mirrored else j
    X = 2.0 / np.sqrt(2 * n + 1) * np.sin(np.pi * (2 * k + 1) * (jj + 1) / (2 * n + 1))
    mu = 2 - 2 * np.cos(np.pi * (2 * np.arange(n) + 1) / (2 * n + 1))
    return mu, X


def eig_tol(mu, norm_l=4.0):
    """Attainable eigenvector accuracy of a backward-stable solver: ~ eps ||L|| / gap."""
    return 64 * np.finfo(float).eps * norm_l / np.min(np.diff(np.sort(mu)))


def pin_self_loop(basis_fn, n, mirrored=False):
    """Error of the self-loop basis against the DST-VII closed form, in units of eig_tol."""
    v = np.zeros(n)
    v[n - 1 if mirrored else 0] = 1.0
    mu, X = basis_fn(n, 1.0, v)
    mu_c, X_c = dst7(n, mirrored)
    return max(np.abs(X - X_c).max(), np.abs(mu - mu_c).max()) / eig_tol(mu_c)


def secular_newton_step(n, rho, v, mu):
    """|f(mu)/f'(mu)| for f(m) = 1 + rho sum_j z_j^2 / (lambda_j - m): distance to a root."""
    U = explicit_dct2(n)
    z = U.T @ v
    lam = np.array([2 - 2 * np.cos(np.pi * k / n) for k in range(n)])
    out = []
    for m in mu:
        f = 1.0 + rho * np.sum(z * z / (lam - m))
        fp = rho * np.sum(z * z / (lam - m) ** 2)
        out.append(abs(f / fp))
    return np.array(out)


# --------------------------------------------------------------------------
# pins against the real oracle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 5, 8, 17, 64])
def test_rho_zero_gives_dct2(n):
    assert pin_rho_zero(oracle.basis, n) < 1e-12


def test_dct2_matrix_matches_definition_and_library():
    for n in (1, 4, 7, 32):
        U = explicit_dct2(n)
        assert np.abs(oracle.dct2_matrix(n) - U).max() < 1e-14
        x = _rng(n).standard_normal((3, n))
        # the semi-oracle's DCT step is scipy's orthonormal DCT-II
        assert np.abs(oracle._dct2(x) - x @ U).max() < 1e-13


@pytest.mark.parametrize("n", [4, 16, 64, 128])
@pytest.mark.parametrize("mirrored", [False, True])
def test_self_loop_is_dst7(n, mirrored):
    assert pin_self_loop(oracle.basis, n, mirrored) < 1.0


@pytest.mark.parametrize("rho", [0.3, 2.0, -0.7])
@pytest.mark.parametrize("n", [8, 33, 64])
def test_interlacing_secular_zero_trace(n, rho):
    v = workloads.unit_vector(_rng(n), n)
    mu, X = oracle.basis(n, rho, v)
    lam = oracle.path_eigenvalues(n)
    if rho > 0:   # Lemma 4.1: lambda_1 < mu_1 < lambda_2 < ... < lambda_n < mu_n
        assert np.all(lam < mu) and np.all(mu[:-1] < lam[1:])
    else:         # reversed for rho < 0
        assert np.all(mu < lam) and np.all(lam[:-1] < mu[1:])
    assert secular_newton_step(n, rho, v, mu).max() < 1e-13
    assert abs(mu.sum() - lam.sum() - rho * (v @ v)) < 64 * n * np.finfo(float).eps * 4
    # Lemma 4.2: x_i is proportional to U (mu_i I - Lambda)^{-1} z
    U = explicit_dct2(n)
    z = U.T @ v
    for i in range(n):
        d = U @ (z / (mu[i] - lam))
        d /= np.linalg.norm(d)
        assert min(np.abs(X[:, i] - d).max(), np.abs(X[:, i] + d).max()) < 1e-10
        # sign convention: rho v^T x_i > 0
        assert rho * (v @ X[:, i]) > 0


def _mp_eigpairs(L, dps=50):
    """Brute force: characteristic polynomial roots and null vectors in 50 digits."""
    import mpmath as mp
    mp.mp.dps = dps
    n = L.shape[0]
    A = mp.matrix([[mp.mpf(float(L[i, j])) for j in range(n)] for i in range(n)])
    # Faddeev-LeVerrier: p(t) = t^n + c_{n-1} t^{n-1} + ... + c_0
    M = mp.zeros(n, n)
    I = mp.eye(n)
    coeffs = [mp.mpf(1)]
    c = mp.mpf(1)
    for k in range(1, n + 1):
        M = A * M + c * I
        AM = A * M
        c = -sum(AM[i, i] for i in range(n)) / k
        coeffs.append(c)
    roots = mp.polyroots(coeffs, maxsteps=500, extraprec=200)
    roots = sorted([mp.re(r) for r in roots])
    vecs = []
    for r in roots:
        B = A - (r + mp.mpf(10) ** (-35)) * I
        x = mp.lu_solve(B, mp.matrix([1] * n))
        nrm = mp.sqrt(sum(x[i] ** 2 for i in range(n)))
        vecs.append([float(x[i] / nrm) for i in range(n)])
    return np.array([float(r) for r in roots]), np.array(vecs).T


@pytest.mark.parametrize("n,rho,kind", [(2, 1.3, "dense"), (4, 0.4, "dense"), (5, 1.9, "dense"),
                                        (8, 0.7, "dense"), (8, 2.0, "edge"), (6, 1.5, "loop")])
def test_bruteforce_mpmath(n, rho, kind):
    g = _rng(100 + n)
    if kind == "dense":
        v = workloads.unit_vector(g, n)
    elif kind == "edge":
        v = workloads.edge_vector(n, 1, 5)
    else:
        v = np.zeros(n); v[2] = 1.0
    L = oracle.laplacian(n, rho, v)
    # the Laplacian itself, entry by entry (Prop. 2.4 with unit weights)
    Lb = rho * np.outer(v, v)
    for i in range(n - 1):
        Lb[i, i] += 1; Lb[i + 1, i + 1] += 1; Lb[i, i + 1] -= 1; Lb[i + 1, i] -= 1
    assert np.abs(L - Lb).max() < 1e-15
    mu_b, X_b = _mp_eigpairs(L)
    X_b = oracle.fix_signs(X_b, rho, v)
    mu, X = oracle.basis(n, rho, v)
    assert np.abs(mu - mu_b).max() < 1e-13
    assert np.abs(X - X_b).max() < 1e-12


def test_library_eigh_cross_check():
    n, rho = 48, 0.9
    v = workloads.unit_vector(_rng(7), n)
    mu, X = oracle.basis(n, rho, v)
    w, V = np.linalg.eigh(oracle.laplacian(n, rho, v))
    assert np.abs(mu - w).max() < 1e-13
    assert np.abs(np.abs(X.T @ V) - np.eye(n)).max() < 1e-10


@pytest.mark.parametrize("n", [16, 64, 256])
@pytest.mark.parametrize("kind", ["dense", "loop0", "loopn", "edge", "mirror_edge"])
def test_semi_oracle_matches_jacobi(n, kind):
    g = _rng(1000 + n)
    rho = 0.8
    if kind == "dense":
        v = workloads.unit_vector(g, n)
    elif kind == "loop0":
        v = np.zeros(n); v[0] = 1.0
    elif kind == "loopn":
        v = np.zeros(n); v[-1] = 1.0
    elif kind == "edge":
        v = workloads.edge_vector(n, 3, n // 2 + 1); rho = 2.0
    else:  # i + j + 1 = n: mirror-symmetric edge, half of z is exactly zero
        v = workloads.edge_vector(n, 2, n - 3); rho = 2.0
    x = g.standard_normal((6, n))
    mu, X = oracle.basis(n, rho, v)
    plan = oracle.semi_plan(n, rho, v)
    assert np.abs(plan["mu"] - mu).max() < 1e-12
    # The semi-oracle basis (rows of X^T) must be orthonormal eigenvectors of L
    # whatever the spectrum; this pins it independently of its own formula.
    Xs = oracle.semi_forward(n, rho, v, np.eye(n))            # y(e_b)_i = X[b, i]
    L = oracle.laplacian(n, rho, v)
    assert np.abs(L @ Xs - Xs * plan["mu"]).max() < 1e-12
    assert np.abs(Xs.T @ Xs - np.eye(n)).max() < 1e-12
    # Where the spectrum is simple the basis is unique up to the sign rule.
    gap = np.min(np.diff(mu))
    simple = np.ones(n, dtype=bool)
    if gap < 1e-9:
        close = np.nonzero(np.diff(mu) < 1e-9)[0]
        simple[close] = False
        simple[close + 1] = False
        assert kind in ("edge", "mirror_edge")      # only edges make double eigenvalues
    y = oracle.forward(X, x)
    ys = oracle.semi_forward(n, rho, v, x, plan)
    assert np.abs(y - ys)[:, simple].max() < 1e-9 * np.abs(y).max()
    xs = oracle.semi_adjoint(n, rho, v, ys, plan)
    assert np.abs(xs - x).max() < 1e-12
    # sum_i a_i^2 = rho^2 ||v||^2  (w = X^T v has w_i = a_i / rho)
    lam = oracle.path_eigenvalues(n)
    z = plan["z"]
    a2 = 0.0
    for i in range(n):
        if plan["kind"][i] == 0:
            nz = z != 0.0
            a2 += 1.0 / np.sum(z[nz] ** 2 / (plan["mu"][i] - lam[nz]) ** 2)
    assert abs(a2 - rho * rho * (v @ v)) < 1e-10
    if kind == "mirror_edge":
        assert int(np.sum(plan["kind"])) >= n // 2 - 1


@pytest.mark.parametrize("n", [8, 64])
def test_forward_adjoint_orthogonal(n):
    v = workloads.unit_vector(_rng(3), n)
    mu, X = oracle.basis(n, 1.1, v)
    x = _rng(4).standard_normal((5, n))
    y = oracle.forward(X, x)
    assert np.abs(np.linalg.norm(y, axis=1) - np.linalg.norm(x, axis=1)).max() < 1e-12
    assert np.abs(oracle.adjoint(X, y) - x).max() < 1e-12
    # intertwining: X^T (L s) = mu * X^T s
    L = oracle.laplacian(n, 1.1, v)
    assert np.abs(oracle.forward(X, x @ L) - mu * y).max() < 1e-11


# --------------------------------------------------------------------------
# gradient: perturbation formula vs finite differences
# --------------------------------------------------------------------------
def _loss(n, rho, v, x):
    _, X = oracle.basis(n, rho, v)
    return oracle.loss_l1(oracle.forward(X, x))


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    n, h = 16, 1e-6
    g = _rng(50 + seed)
    rho = 1.0
    v = workloads.unit_vector(g, n)
    x = g.standard_normal((8, n))
    mu, X = oracle.basis(n, rho, v)
    y = oracle.forward(X, x)
    assert np.abs(y).min() > 1e-4      # L1 is smooth within h of these points
    gy = oracle.loss_l1_grad(y)
    dx, drho, dv = oracle.grad_perturbation(mu, X, rho, v, y, gy)
    fd_rho = (_loss(n, rho + h, v, x) - _loss(n, rho - h, v, x)) / (2 * h)
    assert abs(fd_rho - drho) < 1e-7 * max(1.0, abs(drho))
    fd_v = np.array([(_loss(n, rho, v + h * e, x) - _loss(n, rho, v - h * e, x)) / (2 * h)
                     for e in np.eye(n)])
    assert np.abs(fd_v - dv).max() < 1e-7
    for (b, j) in [(0, 0), (3, 7), (7, 15)]:
        xp = x.copy(); xp[b, j] += h
        xm = x.copy(); xm[b, j] -= h
        fd = (_loss(n, rho, v, xp) - _loss(n, rho, v, xm)) / (2 * h)
        assert abs(fd - dx[b, j]) < 1e-7
    # L depends on (rho, v) only through rho v v^T: v . grad_v = 2 rho d/drho
    assert abs(v @ dv - 2 * rho * drho) < 1e-12


# --------------------------------------------------------------------------
# progressive selection with pruning (Thm 3.4)
# --------------------------------------------------------------------------
def test_pruning_bound_and_exact_limit():
    g = _rng(9)
    for n in (8, 16, 32):
        x = workloads.ar1(g, 16, n, 0.9, dtype=np.float64)
        U = oracle.dct2_matrix(n)
        s = x @ U
        for (kind, i, j, w) in [(0, 0, 0, 1.5), (0, n - 1, n - 1, 0.4), (1, 1, n - 2, 1.0)]:
            rho, v = oracle.candidate_update(n, kind, i, j, w)
            _, X = oracle.basis(n, rho, v)
            Ct = X.T @ U
            for c_p in (2, n // 2, n):
                Chat = np.zeros_like(Ct)
                Chat[:c_p, :c_p] = Ct[:c_p, :c_p]
                err = np.linalg.norm(s @ Ct.T - s @ Chat.T, axis=1)
                bound = (np.linalg.norm(s[:, c_p:], axis=1)
                         + np.linalg.norm(s[:, :c_p] @ Ct[c_p:, :c_p].T, axis=1))
                assert np.all(err <= bound + 1e-12)
                if c_p == n:
                    assert err.max() < 1e-12


def test_select_block_argmin():
    g = _rng(11)
    n = 16
    x = workloads.ar1(g, 64, n, 0.9, dtype=np.float64)
    cands = [(0, 0, 0, 0.3), (0, n - 1, n - 1, 1.7), (1, 2, 9, 1.0), (0, 0, 0, 1.9)]
    best, costs, ybest, pruned = oracle.select_block(x, cands, c_p=n // 2, prune_tau=0.1)
    assert best == int(np.argmin(costs))
    assert pruned.dtype == bool and 0 < pruned.sum() < 64
    # full transform (no pruning) reproduces the candidate's forward exactly
    best_f, costs_f, yb_f, _ = oracle.select_block(x, cands, c_p=n, prune_tau=0.1)
    rho, v = oracle.candidate_update(n, *cands[best_f])
    _, X = oracle.basis(n, rho, v)
    assert np.abs(yb_f - oracle.forward(X, x)).max() < 1e-12
    assert abs(costs_f[best_f] - np.abs(oracle.forward(X, x)).sum()) < 1e-9


def _candidates_all_kinds(n):
    """Self-loops at both ends, an interior edge, a mirror edge (i + j = n - 1:
    every even-index DCT vector is deflated and many eigenvalues are double)
    and an adjacent edge."""
    return [(0, 0, 0, 0.7), (0, n - 1, n - 1, 1.9), (1, 1, n // 2, 1.0), (1, 1, n - 2, 1.0),
            (1, n // 2 - 1, n // 2, 1.0)]


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_candidate_factor_semi_diagonalises_every_candidate(n):
    # the factor from the secular roots is orthogonal and diagonalises U^T L U
    # (Thm 3.1) for every candidate kind, including the degenerate ones
    U = oracle.dct2_matrix(n)
    for cand in _candidates_all_kinds(n):
        rho, v = oracle.candidate_update(n, *cand)
        Ct = oracle.candidate_factor(n, *cand, method="semi")
        mu = np.linalg.eigvalsh(oracle.laplacian(n, rho, v))
        assert np.abs(Ct @ Ct.T - np.eye(n)).max() < 1e-12, cand
        assert np.abs(Ct.T @ np.diag(mu) @ Ct - U.T @ oracle.laplacian(n, rho, v) @ U).max() < 1e-11, cand
        # sign convention: rho v^T x_i > 0 where v^T x_i is not ~0
        vx = (Ct @ U.T) @ v
        assert np.all((np.abs(vx) < 1e-9) | (rho * vx > 0)), cand


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_candidate_factor_semi_matches_jacobi_on_simple_spectra(n):
    for cand in [(0, 0, 0, 0.25), (0, n - 1, n - 1, 2.0), (0, 0, 0, 1.3)]:
        a = oracle.candidate_factor(n, *cand, method="semi")
        b = oracle.candidate_factor(n, *cand, method="jacobi")
        assert np.abs(a - b).max() < 1e-10, cand


def test_select_block_pruning_limits():
    g = _rng(12)
    n = 32
    x = workloads.ar1(g, 64, n, 0.9, dtype=np.float64)
    cands = _candidates_all_kinds(n)
    # quadratic form against the assembled path Laplacian (no update)
    Lp = oracle.laplacian(n, 0.0, np.zeros(n))
    q = np.einsum("si,ij,sj->s", x, Lp, x)
    assert np.allclose(oracle.path_quadratic_form(x), q, rtol=1e-12)
    _, _, _, pruned = oracle.select_block(x, cands, c_p=2, prune_tau=0.1, factor="semi")
    assert np.array_equal(pruned, q <= 0.1 * np.sum(x * x, axis=1))
    # nothing pruned: every cost is the L1 norm of the full transform, for any c_p
    _, c_none, _, pr = oracle.select_block(x, cands, c_p=2, prune_tau=-1.0, factor="semi")
    assert not pr.any()
    _, c_full, _, _ = oracle.select_block(x, cands, c_p=n, prune_tau=1e9, factor="semi")
    assert np.allclose(c_none, c_full, rtol=1e-13)
    for r, cand in enumerate(cands):
        rho, v = oracle.candidate_update(n, *cand)
        y = oracle.semi_forward(n, rho, v, x)
        assert abs(c_none[r] - np.abs(y).sum()) < 1e-9 * c_none[r]
    # everything pruned to c_p = 2: two coefficients per signal, error within the Thm 3.4 bound
    b2, c2, y2, pr2 = oracle.select_block(x, cands, c_p=2, prune_tau=1e9, factor="semi")
    assert pr2.all() and np.count_nonzero(y2[:, 2:]) == 0
    rho, v = oracle.candidate_update(n, *cands[b2])
    yf = oracle.semi_forward(n, rho, v, x)
    sd = x @ oracle.dct2_matrix(n)
    Ct = oracle.candidate_factor(n, *cands[b2], method="semi")
    bound = np.linalg.norm(sd[:, 2:], axis=1) + np.linalg.norm(sd[:, :2] @ Ct[2:, :2].T, axis=1)
    assert np.all(np.linalg.norm(yf - y2, axis=1) <= bound + 1e-12)


def graph_laplacian(n, edges=(), loops=()):
    """Generalized Laplacian D - W + V of a weighted graph (Def. of the GFT):
    W the weighted adjacency (unit path edges (j, j+1) plus the extra edges,
    whose weights add to an existing edge), D its degree matrix, V the diagonal
    self-loop matrix.  Built from the graph alone, not from a rank-one term."""
    W = np.zeros((n, n))
    for j in range(n - 1):
        W[j, j + 1] = W[j + 1, j] = 1.0
    for (i, j, w) in edges:
        W[i, j] += w
        W[j, i] += w
    V = np.zeros((n, n))
    for (i, w) in loops:
        V[i, i] += w
    return np.diag(W.sum(axis=1)) - W + V


def pin_candidate_update(update_fn, n):
    """Largest gap between L_path + rho v v^T, with (rho, v) from update_fn, and the
    generalized Laplacian of the graph the candidate describes (a self-loop of
    weight w at i, or an edge of weight w between i and j: Prop. on baby Laplacians,
    scenarios (i) and (ii))."""
    worst = 0.0
    cases = [(0, 0, 0, 0.7), (0, n - 1, n - 1, 1.9), (1, 1, n - 2, 1.0), (1, 0, 1, 0.35),
             (1, n // 2 - 1, n // 2, 2.5), (1, 2, n - 1, 0.6)]
    for (kind, i, j, w) in cases:
        rho, v = update_fn(n, kind, i, j, w)
        L = oracle.laplacian(n, rho, v)
        G = graph_laplacian(n, loops=[(i, w)]) if kind == 0 else graph_laplacian(n, edges=[(i, j, w)])
        worst = max(worst, np.abs(L - G).max())
    return worst


@pytest.mark.parametrize("n", [4, 8, 16, 64])
def test_candidate_update_is_the_graph_laplacian(n):
    assert pin_candidate_update(oracle.candidate_update, n) < 1e-14


# --------------------------------------------------------------------------
# mutation tests: plausible mistakes must trip at least one pin
# --------------------------------------------------------------------------
def _basis_with(lap=None, signs=None, order=None):
    def fn(n, rho, v):
        L = lap(n, rho, v) if lap else oracle.laplacian(n, rho, v)
        mu, X = oracle.eigh_jacobi(L)
        if order == "descending":
            mu, X = mu[::-1], X[:, ::-1]
        X = signs(X, rho, v) if signs else oracle.fix_signs(X, rho, v)
        return mu, np.ascontiguousarray(X)
    return fn


def _lap_wrong_offdiag(n, rho, v):
    L = oracle.laplacian(n, rho, v)
    off = np.diag(np.diag(L, 1), 1)
    return L - 2 * (off + off.T)                       # +1 instead of -1 off the diagonal


def _lap_dropped_end_degree(n, rho, v):
    L = oracle.laplacian(n, rho, v)
    L[0, 0] += 1.0                                     # degree 2 at the end vertex
    return L


def _lap_rho_twice(n, rho, v):
    return oracle.laplacian(n, 2 * rho, v)


def _signs_flipped(X, rho, v):
    return -oracle.fix_signs(X, rho, v)


def _update_edge_rho_w(n, kind, i, j, w):
    rho, v = oracle.candidate_update(n, kind, i, j, w)
    return (w, v) if kind == 1 else (rho, v)       # edge weight w read as rho = w


def _update_loop_unit_v_scaled(n, kind, i, j, w):
    rho, v = oracle.candidate_update(n, kind, i, j, w)
    return (rho, v / np.sqrt(2.0)) if kind == 0 else (rho, v)


@pytest.mark.parametrize("mutant", [_update_edge_rho_w, _update_loop_unit_v_scaled])
def test_candidate_update_pin_catches_mutants(mutant):
    assert pin_candidate_update(mutant, 16) > 0.1


@pytest.mark.parametrize("mutant", ["offdiag", "end_degree", "rho_twice", "signs", "order"])
def test_pins_catch_mutants(mutant):
    fn = {
        "offdiag": _basis_with(lap=_lap_wrong_offdiag),
        "end_degree": _basis_with(lap=_lap_dropped_end_degree),
        "rho_twice": _basis_with(lap=_lap_rho_twice),
        "signs": _basis_with(signs=_signs_flipped),
        "order": _basis_with(order="descending"),
    }[mutant]
    caught = (pin_rho_zero(fn, 8) > 1e-6) or (pin_self_loop(fn, 8) > 1e6) \
        or (pin_self_loop(fn, 8, True) > 1e6)
    assert caught


# --------------------------------------------------------------------------
# rank-k updates (Sec. 4.3, Cor. 4.5)
# --------------------------------------------------------------------------
def _edges_case(n, seed, count):
    """`count` seeded added edges (random i != j, weights in [0.5, 2]) as rank-one updates
    (rho = 2 w, v = (e_i - e_j)/sqrt 2) and as an edge list."""
    g = np.random.default_rng(seed)
    rhos, vs, edges = [], [], []
    for _ in range(count):
        i, j = sorted(int(t) for t in g.choice(n, 2, replace=False))
        w = float(g.uniform(0.5, 2.0))
        rho, v = oracle.candidate_update(n, 1, i, j, w)
        rhos.append(rho)
        vs.append(v)
        edges.append((i, j, w))
    return rhos, vs, edges


def _chain_basis(n, rhos, vs, z_from_base=False):
    """X_k built stage by stage as Cor. 4.5 states it, X_j = X_{j-1} diag(z_j)
    C(mu_{j-1}, mu_j) diag(a_j), with a_j > 0 in the forward orientation
    (X_j^T = diag(a_j) C(mu_j, mu_{j-1}) diag(z_j) X_{j-1}^T).  The eigenvalues mu_j of each
    stage are taken from Jacobi on the stage's assembled matrix (so this checks the
    eigenvector structure only), z_j = X_{j-1}^T v_j (or U^T v_j with z_from_base, the
    printed form of the corollary).  Directions with z_j,m = 0 (every added edge keeps the
    constant vector) are deflated: the stage keeps x_m with eigenvalue mu_{j-1,m}.  Stages
    must have simple spectra."""
    X = oracle.dct2_matrix(n)
    d = oracle.path_eigenvalues(n)
    for k in range(len(rhos)):
        v = np.asarray(vs[k], dtype=np.float64)
        z = (oracle.dct2_matrix(n).T @ v) if z_from_base else (X.T @ v)
        live = np.abs(z) > 1e-12 * np.linalg.norm(z)
        mu, _ = oracle.eigh_jacobi(oracle.laplacian_rank_k(n, rhos[:k + 1], vs[:k + 1]))
        Wt = np.zeros((n, n))
        used = set()
        for i in range(n):
            hit = [m for m in np.nonzero(~live)[0] if abs(d[m] - mu[i]) < 1e-9 and m not in used]
            if hit:
                Wt[i, hit[0]] = 1.0                            # deflated: x_m itself
                used.add(hit[0])
                continue
            w = z[live] / (mu[i] - d[live])                    # row of C(mu_j, mu_{j-1}) diag(z)
            Wt[i, live] = w / np.linalg.norm(w)                # times a_i > 0
        X = X @ Wt.T
        d = mu
    return d, X


@pytest.mark.parametrize("n", [8, 16, 64])
def test_rank_k_laplacian_is_the_graph_laplacian(n):
    rhos, vs, edges = _edges_case(n, 100 + n, 3)
    L = oracle.laplacian_rank_k(n, rhos, vs)
    assert np.abs(L - graph_laplacian(n, edges=edges)).max() < 1e-14
    # a self-loop and an edge together
    r1, v1 = oracle.candidate_update(n, 0, n - 1, n - 1, 0.8)
    r2, v2 = oracle.candidate_update(n, 1, 1, n - 2, 1.3)
    L = oracle.laplacian_rank_k(n, [r1, r2], [v1, v2])
    assert np.abs(L - graph_laplacian(n, edges=[(1, n - 2, 1.3)], loops=[(n - 1, 0.8)])).max() < 1e-14


@pytest.mark.parametrize("n", [8, 32, 64])
def test_rank_k_basis_diagonalises_and_signs(n):
    rhos, vs, _ = _edges_case(n, 200 + n, 3)
    mu, X = oracle.basis_rank_k(n, rhos, vs)
    L = oracle.laplacian_rank_k(n, rhos, vs)
    assert np.all(np.diff(mu) > 0)
    assert np.abs(X.T @ X - np.eye(n)).max() < 1e-12
    assert np.abs(X @ np.diag(mu) @ X.T - L).max() < 1e-12
    # the last update sees every eigenvector it is not orthogonal to with a positive sign
    t = rhos[-1] * (vs[-1] @ X)
    assert np.all((t > 0) | (np.abs(t) < 1e-9))


@pytest.mark.parametrize("n", [8, 64])
def test_rank_k_reduces_to_rank_one(n):
    g = np.random.default_rng(7 + n)
    v = workloads.unit_vector(g, n)
    mu1, X1 = oracle.basis(n, 0.9, v)
    muk, Xk = oracle.basis_rank_k(n, [0.9], [v])
    assert np.abs(mu1 - muk).max() < 1e-13 and np.abs(X1 - Xk).max() < 1e-12
    # one update split into two halves along the same v: the same L, the same signs
    mu2, X2 = oracle.basis_rank_k(n, [0.45, 0.45], [v, v])
    assert np.abs(mu1 - mu2).max() < 1e-12 and np.abs(X1 - X2).max() < 1e-10


@pytest.mark.parametrize("n", [16, 64])
def test_rank_k_order_of_updates(n):
    rhos, vs, _ = _edges_case(n, 300 + n, 2)
    mu_a, X_a = oracle.basis_rank_k(n, rhos, vs)
    mu_b, X_b = oracle.basis_rank_k(n, rhos[::-1], vs[::-1])
    assert np.abs(mu_a - mu_b).max() < 1e-12
    assert np.abs(np.abs(X_a) - np.abs(X_b)).max() < 1e-10


@pytest.mark.parametrize("n", [8, 16, 32])
def test_rank_k_chain_of_cauchy_factors(n):
    """Cor. 4.5 with z_k = X_{k-1}^T v_k reproduces the Jacobi basis of L_k column by
    column (values and the chain's sign convention); with z_k = U^T v_k, as printed, it
    does not (the corollary's induction needs the previous stage's basis)."""
    for seed in range(3):
        rhos, vs, _ = _edges_case(n, 400 + 10 * n + seed, 3)
        mu, X = oracle.basis_rank_k(n, rhos, vs)
        gaps = min(np.diff(oracle.eigh_jacobi(oracle.laplacian_rank_k(n, rhos[:j + 1], vs[:j + 1]))[0]).min()
                   for j in range(3))
        if gaps < 1e-6:
            continue
        d, Xc = _chain_basis(n, rhos, vs)
        assert np.abs(d - mu).max() < 1e-12
        assert np.abs(Xc - X).max() < 1e-9, np.abs(Xc - X).max()
        _, Xw = _chain_basis(n, rhos, vs, z_from_base=True)
        assert not (np.abs(np.abs(Xw) - np.abs(X)).max() <= 1e-3)     # NaN or far off


# --------------------------------------------------------------------------
# a rank-one update of a general base (Thm 3.1 / 3.2) and the DTT+ case
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 64])
def test_general_base_with_the_path_is_the_path_case(n):
    v = workloads.unit_vector(np.random.default_rng(11 + n), n)
    mu_p, X_p = oracle.basis(n, 0.7, v)
    mu_g, X_g = oracle.basis_general(oracle.path_eigenvalues(n), oracle.dct2_matrix(n), 0.7, v)
    assert np.abs(mu_p - mu_g).max() < 1e-12 and np.abs(X_p - X_g).max() < 1e-10


@pytest.mark.parametrize("n", [8, 32, 64])
def test_dst7_basis_is_the_adst_graph(n):
    lam, U = oracle.dst7_basis(n)
    e0 = np.zeros(n)
    e0[0] = 1.0
    L = oracle.laplacian(n, 1.0, e0)
    assert np.abs(U.T @ U - np.eye(n)).max() < 1e-12
    assert np.abs(L @ U - U * lam[None, :]).max() < 1e-12
    assert np.all(np.diff(lam) > 0)


@pytest.mark.parametrize("n", [8, 64])
def test_benchmark_inputs_are_the_graphs_they_name(n):
    """The benchmark's rank-k and DTT+ inputs come from the input module: an added edge
    gives the Laplacian of the edge, and the ADST base diagonalises the path with its unit
    self-loop at vertex 0 (and equals the oracle's DST-VII)."""
    for i, j, w in [(0, n - 1, 1.0), (2, n // 2, 0.6)]:
        rho, v = workloads.edge_update(n, i, j, w)
        d = np.zeros(n)
        d[i], d[j] = 1.0, -1.0
        L_edge = oracle.laplacian(n, 0.0, np.zeros(n)) + w * np.outer(d, d)
        assert np.abs(oracle.laplacian(n, rho, v) - L_edge).max() < 1e-14
    lam, U = workloads.adst_base(n)
    e0 = np.zeros(n)
    e0[0] = 1.0
    L = oracle.laplacian(n, 1.0, e0)
    assert np.abs(U.T @ U - np.eye(n)).max() < 1e-12
    assert np.abs(L @ U - U * lam[None, :]).max() < 1e-12
    lam_o, U_o = oracle.dst7_basis(n)
    assert np.abs(lam - lam_o).max() < 1e-14 and np.abs(U - U_o).max() < 1e-14


@pytest.mark.parametrize("n", [8, 32, 64])
def test_dtt_plus_equals_the_rank_two_path_chain(n):
    """DTT+: a rank-one update of the ADST graph (DST-VII base) is the path graph with
    the unit self-loop at vertex 0 and then the update, whose chain signs agree with the
    general-base convention (the DST-VII vectors have a positive first entry)."""
    g = np.random.default_rng(21 + n)
    e0 = np.zeros(n)
    e0[0] = 1.0
    for rho, v in [(0.8, workloads.unit_vector(g, n)), oracle.candidate_update(n, 1, 2, n - 5, 1.0),
                   (-0.3, workloads.unit_vector(g, n))]:
        lam, U = oracle.dst7_basis(n)
        mu_g, X_g = oracle.basis_general(lam, U, rho, v)
        mu_c, X_c = oracle.basis_rank_k(n, [1.0, rho], [e0, v])
        assert np.abs(mu_g - mu_c).max() < 1e-12
        assert np.abs(X_g - X_c).max() < 1e-9


@pytest.mark.parametrize("n", [8, 32])
def test_general_base_random(n):
    g = np.random.default_rng(31 + n)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.sort(g.uniform(-1.0, 3.0, n))
    v = workloads.unit_vector(g, n)
    mu, X = oracle.basis_general(lam, Q, 0.9, v)
    L = (Q * lam) @ Q.T + 0.9 * np.outer(v, v)
    assert np.abs(X @ np.diag(mu) @ X.T - L).max() < 1e-12
    assert np.all(lam < mu) and np.all(mu[:-1] < lam[1:])          # Lemma 4.1 interlacing
    assert np.all(0.9 * (v @ X) > 0)
    mu0, X0 = oracle.basis_general(lam, Q, 0.0, v)                   # rho = 0: the base itself
    assert np.abs(mu0 - lam).max() < 1e-12 and np.abs(X0 - Q).max() < 1e-10
