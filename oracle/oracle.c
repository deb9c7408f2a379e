/*
 * FP64 reference for the DCT+ transform (Fernandez-Menduina, Pavez, Ortega,
 * "Fast DCT+: A Family of Fast Transforms Based on Rank-One Updates of the
 * Path Graph", arXiv 2409.08970).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * What it computes is the plain definition (Sec. 2, Def. of the GFT and of
 * rank-one updates): assemble L = L_path + rho v v^T in FP64, diagonalise it
 * with a hand-written cyclic Jacobi eigensolver (textbook two-sided Jacobi
 * rotations), order the eigenpairs ascending, fix the sign of every
 * eigenvector, and apply X^T (forward) or X (adjoint) to signals.
 *
 * A second, independent large-n route ("semi-oracle") follows Thm 3.1
 * literally: roots of the secular equation by plain bisection in offset form
 * (interlacing brackets of Lemma 4.1), then row-wise Cauchy sums.  It is
 * checked against the Jacobi route at moderate n by the tests.
 *
 * Sign convention (the paper leaves eigenvector signs free): an eigenvector
 * x_i with |v^T x_i| above a threshold gets rho * v^T x_i > 0, which is the
 * same as taking a_i > 0 in X^T = diag(a) C(mu, lambda) diag(z) U^T.  A row
 * with v^T x_i ~ 0 (a deflated direction) gets its largest |U^T x_i|
 * component positive; for rho = 0 this reproduces the DCT-II exactly.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Laplacian of the unit-weight path graph plus a rank-one term.
 * Path Laplacian (Prop. 2.4 with unit edge weights): degree on the diagonal
 * (1 at both ends, 2 inside), -1 on the first off-diagonals.               */
int orc_laplacian(int n, double rho, const double *v, double *L)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) L[(size_t)i * n + j] = rho * v[i] * v[j];
    for (int i = 0; i + 1 < n; ++i) {
        /* edge (i, i+1) of weight 1 contributes (e_i - e_{i+1})(e_i - e_{i+1})^T */
        L[(size_t)i * n + i] += 1.0;
        L[(size_t)(i + 1) * n + (i + 1)] += 1.0;
        L[(size_t)i * n + (i + 1)] -= 1.0;
        L[(size_t)(i + 1) * n + i] -= 1.0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi for a symmetric matrix, parallel (round-robin) ordering.
 *
 * In each step the indices 0..m-1 (m = n rounded up to even) are split into
 * m/2 disjoint pairs; the 2x2 symmetric Schur decomposition of every pair is
 * computed from the current matrix, then all column rotations are applied,
 * then all row rotations.  Rotations on disjoint pairs never touch each
 * other's 2x2 block, so this is the same iteration as the serial cyclic
 * method with a different pair order.  m-1 steps form one sweep; sweeps stop
 * once off(A) <= tol * ||A||_F, or once off(A) <= 1e-13 ||A||_F and a
 * sweep no longer halves it (the rounding floor).
 *
 * A: n*n row-major, overwritten (diagonal -> eigenvalues).
 * V: n*n row-major, receives eigenvectors as COLUMNS (V[r*n + c] = x_c[r]).
 * Returns the number of sweeps, or -1 if max_sweeps was reached.           */
static void schur2(double app, double apq, double aqq, double *c, double *s)
{
    if (apq == 0.0) { *c = 1.0; *s = 0.0; return; }
    double tau = (aqq - app) / (2.0 * apq);
    double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
}

static double off_norm2(int n, const double *A)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) s += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    return s;
}

int orc_jacobi(int n, double *A, double *V, double tol, int max_sweeps)
{
    double fro2 = 0.0;
    for (size_t k = 0; k < (size_t)n * n; ++k) fro2 += A[k] * A[k];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (n == 1) return 0;

    int m = n + (n & 1);                 /* padded index count (dummy = n) */
    int *ring = (int *)malloc(sizeof(int) * m);
    int *pp = (int *)malloc(sizeof(int) * (m / 2));
    int *qq = (int *)malloc(sizeof(int) * (m / 2));
    double *cc = (double *)malloc(sizeof(double) * (m / 2));
    double *ss = (double *)malloc(sizeof(double) * (m / 2));
    for (int i = 0; i < m; ++i) ring[i] = i;

    int sweeps = 0;
    double prev = -1.0;
    for (;;) {
        double off2 = off_norm2(n, A);
        if (off2 <= tol * tol * fro2) break;
        /* at the rounding floor a sweep no longer halves off(A): stop there */
        if (prev >= 0.0 && off2 > 0.25 * prev && off2 <= 1e-26 * fro2) break;
        prev = off2;
        if (sweeps >= max_sweeps) { sweeps = -1; break; }
        for (int step = 0; step < m - 1; ++step) {
            /* pairs of the round-robin tournament: ring[k] vs ring[m-1-k] */
            int np = 0;
            for (int k = 0; k < m / 2; ++k) {
                int p = ring[k], q = ring[m - 1 - k];
                if (p == n || q == n) continue;
                if (p > q) { int t = p; p = q; q = t; }
                pp[np] = p; qq[np] = q;
                schur2(A[(size_t)p * n + p], A[(size_t)p * n + q], A[(size_t)q * n + q],
                       &cc[np], &ss[np]);
                ++np;
            }
            /* A <- A J (columns p, q) and V <- V J */
            #pragma omp parallel for schedule(static) if (n >= 128)
            for (int r = 0; r < n; ++r) {
                double *Ar = A + (size_t)r * n, *Vr = V + (size_t)r * n;
                for (int k = 0; k < np; ++k) {
                    int p = pp[k], q = qq[k];
                    double c = cc[k], s = ss[k];
                    double ap = Ar[p], aq = Ar[q];
                    Ar[p] = c * ap - s * aq;
                    Ar[q] = s * ap + c * aq;
                    double vp = Vr[p], vq = Vr[q];
                    Vr[p] = c * vp - s * vq;
                    Vr[q] = s * vp + c * vq;
                }
            }
            /* A <- J^T A (rows p, q) */
            #pragma omp parallel for schedule(static) if (n >= 128)
            for (int k = 0; k < np; ++k) {
                int p = pp[k], q = qq[k];
                double c = cc[k], s = ss[k];
                double *Ap = A + (size_t)p * n, *Aq = A + (size_t)q * n;
                for (int col = 0; col < n; ++col) {
                    double ap = Ap[col], aq = Aq[col];
                    Ap[col] = c * ap - s * aq;
                    Aq[col] = s * ap + c * aq;
                }
            }
            /* rotate the tournament: keep ring[0] fixed, shift the rest */
            int last = ring[m - 1];
            for (int k = m - 1; k > 1; --k) ring[k] = ring[k - 1];
            ring[1] = last;
        }
        ++sweeps;
    }
    free(ring); free(pp); free(qq); free(cc); free(ss);
    return sweeps;
}

/* ------------------------------------------------------------------------ */
/* Apply X^T (forward) or X (adjoint) to a batch of row-major signals.
 * X: n*n row-major with eigenvectors as columns.
 * forward: y[b, i] = sum_r X[r, i] x[b, r];  adjoint: x[b, r] = sum_i X[r, i] y[b, i] */
void orc_apply(int n, const double *X, const double *in, double *out, int64_t batch,
               int adjoint)
{
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; ++b) {
        const double *ib = in + b * n;
        double *ob = out + b * n;
        if (!adjoint) {
            for (int i = 0; i < n; ++i) ob[i] = 0.0;
            for (int r = 0; r < n; ++r) {
                double xr = ib[r];
                const double *Xr = X + (size_t)r * n;
                for (int i = 0; i < n; ++i) ob[i] += Xr[i] * xr;
            }
        } else {
            for (int r = 0; r < n; ++r) {
                const double *Xr = X + (size_t)r * n;
                double acc = 0.0;
                for (int i = 0; i < n; ++i) acc += Xr[i] * ib[i];
                ob[r] = acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Semi-oracle (large n): Thm 3.1 evaluated row by row.
 *
 * lambda_k = 2 - 2 cos(pi k / n) are the path-graph eigenvalues (the roots of
 * U_{n-1} in Sec. 4.2 shifted back).  Differences lambda_j - lambda_o are
 * formed from the product formula 4 sin(pi (j - o) / 2n) sin(pi (j + o) / 2n)
 * so that they keep full relative accuracy.                                  */
static double lam_diff(int n, int j, int o)
{
    return 4.0 * sin(M_PI * (double)(j - o) / (2.0 * n)) * sin(M_PI * (double)(j + o) / (2.0 * n));
}

/* secular function 1/rho + sum_j z_j^2 / (lambda_j - mu), mu = lambda_o + t */
static double secular_at(int n, const double *z2, const double *d, double rho_inv, double t)
{
    double s = rho_inv;
    for (int j = 0; j < n; ++j)
        if (z2[j] != 0.0) s += z2[j] / (d[j] - t);
    return s;
}

/* Roots of the secular equation 1 + rho * sum_j z_j^2 / (lambda_j - mu) = 0
 * by bisection, one bracket per pair of consecutive non-deflated poles
 * (Lemma 4.1), plus the outer bracket [lambda_max, lambda_max + rho ||z||^2]
 * (rho > 0) or [lambda_min - |rho| ||z||^2, lambda_min] (rho < 0).
 *
 * z: length n, exact zeros mark deflated directions (|z_k| <= defl * ||z||
 * is zeroed by the caller).  Outputs, sorted by eigenvalue:
 *   origin[i]: index o of the nearer pole (or the deflated index),
 *   tau[i]   : mu_i - lambda_o,
 *   kind[i]  : 0 = secular root, 1 = deflated direction (mu = lambda_o).
 * Returns 0, or -1 if rho == 0.                                             */
int orc_secular_roots(int n, double rho, const double *z, int *origin, double *tau, int *kind)
{
    if (rho == 0.0) return -1;
    int *J = (int *)malloc(sizeof(int) * n);
    double *z2 = (double *)malloc(sizeof(double) * n);
    int nj = 0;
    double zz = 0.0;
    for (int j = 0; j < n; ++j) {
        z2[j] = z[j] * z[j];
        zz += z2[j];
        if (z[j] != 0.0) J[nj++] = j;
    }
    /* one entry per eigenvalue: nj roots + (n - nj) deflated */
    double *mu_sort = (double *)malloc(sizeof(double) * n);
    int cnt = 0;
    double rinv = 1.0 / rho;

    #pragma omp parallel
    {
        double *d = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(dynamic, 16)
        for (int r = 0; r < nj; ++r) {
            int a, b;          /* bracket poles (b = -1: outer bracket) */
            if (rho > 0) { a = J[r]; b = (r + 1 < nj) ? J[r + 1] : -1; }
            else         { b = J[r]; a = (r > 0) ? J[r - 1] : -1; }
            int o;
            double lo, hi;     /* bracket for t = mu - lambda_o */
            if (a >= 0 && b >= 0) {
                /* choose the origin from the sign at the bracket midpoint */
                for (int j = 0; j < n; ++j) d[j] = lam_diff(n, j, a);
                double gap = d[b];
                double fm = secular_at(n, z2, d, rinv, 0.5 * gap);
                if (fm >= 0.0) { o = a; lo = 0.0; hi = 0.5 * gap; }
                else {
                    o = b;
                    for (int j = 0; j < n; ++j) d[j] = lam_diff(n, j, b);
                    lo = -0.5 * gap; hi = 0.0;
                }
            } else if (rho > 0) {
                o = a;
                for (int j = 0; j < n; ++j) d[j] = lam_diff(n, j, a);
                lo = 0.0; hi = rho * zz * (1.0 + 1e-12) + 1e-300;
            } else {
                o = b;
                for (int j = 0; j < n; ++j) d[j] = lam_diff(n, j, b);
                lo = rho * zz * (1.0 + 1e-12) - 1e-300; hi = 0.0;
            }
            /* f is increasing in t between its poles: f(lo+) < 0 < f(hi-) */
            for (int it = 0; it < 400; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double f = secular_at(n, z2, d, rinv, mid);
                if (f > 0.0) hi = mid; else lo = mid;
            }
            double t = 0.5 * (lo + hi);
            /* position of this root in the ascending order of all eigenvalues */
            #pragma omp critical
            {
                origin[cnt] = o; tau[cnt] = t; kind[cnt] = 0;
                mu_sort[cnt] = 2.0 - 2.0 * cos(M_PI * o / (double)n) + t;
                ++cnt;
            }
        }
        free(d);
    }
    for (int j = 0; j < n; ++j)
        if (z[j] == 0.0) {
            origin[cnt] = j; tau[cnt] = 0.0; kind[cnt] = 1;
            mu_sort[cnt] = 2.0 - 2.0 * cos(M_PI * j / (double)n);
            ++cnt;
        }
    /* Insertion sort by eigenvalue.  Two roots never coincide (strict
     * interlacing) and deflated eigenvalues are distinct path eigenvalues, so
     * the only possible tie is a root landing on a deflated lambda_k (it
     * happens for some added edges).  The eigenvalue is then double and the
     * basis is not unique; the deflation basis used here (u_k, plus the root's
     * eigenvector, which has no u_k component) is taken as canonical, and a
     * tie within tie_tol is ordered deflated-first.                          */
    double tie_tol = 1e-12 * (4.0 + fabs(rho) * zz);
    for (int i = 1; i < n; ++i) {
        double m0 = mu_sort[i]; int o0 = origin[i]; double t0 = tau[i]; int k0 = kind[i];
        int k = i - 1;
        while (k >= 0 && (mu_sort[k] > m0 + tie_tol ||
                          (fabs(mu_sort[k] - m0) <= tie_tol && kind[k] < k0))) {
            mu_sort[k + 1] = mu_sort[k]; origin[k + 1] = origin[k];
            tau[k + 1] = tau[k]; kind[k + 1] = kind[k];
            --k;
        }
        mu_sort[k + 1] = m0; origin[k + 1] = o0; tau[k + 1] = t0; kind[k + 1] = k0;
    }
    free(J); free(z2); free(mu_sort);
    return 0;
}

/* Row-wise Thm 3.1: y[b, i] = a_i sum_j z_j sd[b, j] / (mu_i - lambda_j) for
 * secular rows, y[b, i] = sd[b, o_i] for deflated rows, with
 * a_i = (sum_j z_j^2 / (mu_i - lambda_j)^2)^(-1/2) > 0.
 * adjoint != 0 applies the transpose: sd[b, j] = sum_i (row_i)_j y[b, i].
 * Differences mu_i - lambda_j = tau_i - (lambda_j - lambda_o) in FP64.      */
void orc_cauchy_apply(int n, const double *z, const int *origin, const double *tau,
                      const int *kind, const double *in, double *out, int64_t batch,
                      int adjoint)
{
    if (adjoint) memset(out, 0, sizeof(double) * (size_t)n * batch);
    double *row = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) {
        int o = origin[i];
        if (kind[i] == 1) {
            for (int64_t b = 0; b < batch; ++b) {
                if (!adjoint) out[b * n + i] = in[b * n + o];
                else out[b * n + o] += in[b * n + i];
            }
            continue;
        }
        double ss = 0.0;
        for (int j = 0; j < n; ++j) {
            double gap = tau[i] - lam_diff(n, j, o);      /* mu_i - lambda_j */
            row[j] = (z[j] != 0.0) ? z[j] / gap : 0.0;
            ss += row[j] * row[j];
        }
        double a = 1.0 / sqrt(ss);
        for (int j = 0; j < n; ++j) row[j] *= a;
        #pragma omp parallel for schedule(static) if (batch >= 64)
        for (int64_t b = 0; b < batch; ++b) {
            if (!adjoint) {
                double acc = 0.0;
                const double *sb = in + b * n;
                for (int j = 0; j < n; ++j) acc += row[j] * sb[j];
                out[b * n + i] = acc;
            } else {
                double yi = in[b * n + i];
                double *xb = out + b * n;
                for (int j = 0; j < n; ++j) xb[j] += row[j] * yi;
            }
        }
    }
    free(row);
}
