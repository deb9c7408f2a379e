/*
 * dctplus: the DCT+ transform on AMD Instinct MI355X (gfx950).
 *
 * DCT+ is the graph Fourier transform (GFT) of a path graph whose Laplacian
 * has received a rank-one update, L = L_path + rho v v^T (Fernandez-Menduina,
 * Pavez, Ortega, arXiv 2409.08970, Sec. 2, Def. of rank-one updates and
 * Def. of DCT+).  With L_path = U diag(lambda) U^T (U the orthonormal
 * DCT-II basis, lambda_k = 2 - 2 cos(pi k / n)) and L = X diag(mu) X^T, the
 * paper's Thm 3.1 factors the new basis as
 *
 *     X^T = diag(a) C(mu, lambda) diag(z) U^T,   z = U^T v,
 *     C(mu, lambda)_ij = 1 / (mu_i - lambda_j),  a_i = column normalisers,
 *
 * where mu are the roots of the secular equation (Remark 1) interlacing
 * lambda (Lemma 4.1).  The library applies y = X^T x (forward), x = X y
 * (adjoint = inverse, X is orthogonal), the gradient of a loss of y with
 * respect to x, rho and v, and batched progressive selection with pruning
 * (Thm 3.4).
 *
 * Conventions
 *   - Indices are 0-based.  Output row i of y corresponds to mu_i in
 *     ascending order.
 *   - Sign: every eigenvector satisfies rho * v^T x_i > 0 (a_i > 0 above).
 *     Directions with z_k = 0 after deflation (|z_k| <= defl_tol * ||z||)
 *     are the DCT vectors u_k themselves (mu = lambda_k, sign +).  When a
 *     secular root coincides with such a lambda_k (a double eigenvalue) the
 *     deflation basis is kept and the deflated row is ordered first.
 *   - rho = 0 or v = 0 gives exactly the orthonormal DCT-II.
 *   - Signals are contiguous row-major [batch, n] arrays in DEVICE memory,
 *     4-byte aligned (FP32) or 8-byte aligned (FP64); the caller owns them.
 *   - All calls taking a stream are stream-ordered and asynchronous unless
 *     stated; stream is a hipStream_t passed as void* (NULL = null stream).
 *   - Errors are reported through the return status only; nothing aborts.
 *     On any non-OK status no output has been written (argument errors are
 *     detected before any device work).  dctplus_last_error() gives a
 *     thread-local message for the last failure.
 *   - A plan is immutable after creation (its tables) and may be used
 *     concurrently from several streams.  Routes that need scratch memory
 *     (FAST with a per-signal buffer too large for LDS, the factored DENSE form
 *     above n = 64, the gradient) keep one workspace per stream handle in the
 *     plan: calls on different streams never share it, calls on one stream are
 *     ordered by the stream.  The first such call on a stream, or a larger batch
 *     than before, allocates (after waiting for that stream's earlier work):
 *     make one call per stream before capturing such a route into a graph.
 *     Selection plans have one work-queue counter: calls on one selection plan
 *     must not overlap.
 */
#ifndef DCTPLUS_H
#define DCTPLUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dctplus_plan_s *dctplus_plan_t;

typedef enum {
    DCTPLUS_OK = 0,
    DCTPLUS_EINVAL = 1,       /* invalid argument (null/misaligned pointer, bad size, non-finite input, aliasing) */
    DCTPLUS_ENOMEM = 2,       /* device or host allocation failed */
    DCTPLUS_EDEVICE = 3,      /* HIP runtime error (see dctplus_last_error) */
    DCTPLUS_EUNSUPPORTED = 4, /* valid request outside what this build implements (route, dtype, n) */
    DCTPLUS_ENOCONV = 5,      /* the secular-equation solver did not converge */
    DCTPLUS_EDEGENERATE = 6   /* the request needs simple eigenvalues and the plan has a double one */
} dctplus_status;

/* Element type of signals, and the arithmetic of the bulk of the transform. */
typedef enum {
    DCTPLUS_F32 = 0,  /* FP32 signals; FP32 DCT, FP64 Cauchy stage (fast), FP32 MFMA (dense; for
                         64 < n <= 4096 the plan keeps the factor and its transpose, 8 n^2 bytes) */
    DCTPLUS_F64 = 1,  /* FP64 signals and FP64 arithmetic throughout (dense routes: FP64 MFMA
                         product with the FP64 X^T, 8 n^2 bytes) */
    DCTPLUS_BF16 = 2, /* FP32 signals; dense routes only: BF16 MFMA operands, FP32 accumulation */
    DCTPLUS_F32_SPLIT = 3 /* FP32 signals; dense routes, 32 <= n <= 4096 (the factored form: n = 64):
                             both operands split into three BF16 pieces, the six cross products of
                             order >= 2^-16 accumulated in FP32 on MFMA (FP32-level accuracy); arrays
                             16-byte aligned.  Above n = 64 the plan keeps the three pieces of its
                             factor for each direction (12 n^2 bytes besides the FP32 factor) */
} dctplus_dtype;

/* How the product with diag(a) C(mu, lambda) diag(z) is formed. */
typedef enum {
    DCTPLUS_ROUTE_AUTO = 0,  /* FP32: the faster route measured on MI355X, DENSE for n <= 1024,
                                FAST for n >= 2048, and at n = 1024 (one update) FAST for calls
                                of fewer than 1,024 signals (chosen per call; plan_info reports
                                DENSE); other dtypes: DENSE */
    DCTPLUS_ROUTE_FAST = 1,  /* Alg. 1 / Thm 3.3: DCT-II, DST-I, sine NUFFT, O(n log n) */
    DCTPLUS_ROUTE_DENSE = 2, /* Thm 3.1: DCT-II, then an MFMA product with the n x n Cauchy factor */
    DCTPLUS_ROUTE_GFT = 3    /* dense GFT (the paper's naive product): MFMA product with X^T */
} dctplus_route;

typedef struct {
    int32_t dtype;        /* dctplus_dtype */
    int32_t route;        /* dctplus_route */
    double defl_tol;      /* deflation threshold on |z_k| / ||z||; <= 0 selects 1e-13 */
    int32_t nufft_width;  /* window taps of the sine NUFFT (FAST route), even, 4..16; 0 (the
                             default) selects 12 for FP32 signals and 16 for FP64 */
    double direct_kappa;  /* FAST route: rows whose NUFFT error amplification exceeds this are
                             summed exactly in FP64; <= 0 (the default) selects 1e5 for FP32
                             signals and 1e3 for FP64 */
    int32_t device;       /* HIP device ordinal; < 0 uses the current device */
    int32_t factored;     /* DENSE route only, F32 or BF16: 1 keeps the two factors of Thm 3.1
                             apart (a DCT-II of every signal, then the product with the Cauchy
                             factor diag(a) C(mu, lambda) diag(z)); 0 (default) folds the DCT
                             into one matrix X^T at plan time.  Same transform either way. */
} dctplus_opts;

/* Fill *opts with the defaults. */
void dctplus_default_opts(dctplus_opts *opts);

/*
 * Build a plan for L = L_path + rho v v^T on n vertices (setup, Remark 1).
 *   n       : 4 <= n <= 16384, a power of two (EUNSUPPORTED otherwise; EINVAL if n < 2).
 *   rho     : finite.  rho < 0 is supported by every route.
 *   v_host  : HOST pointer to n finite doubles (copied; need not stay valid).
 *   opts    : NULL for defaults.
 *   stream  : the plan's tables are computed on this stream (FP64 secular solve
 *             on the GPU); the call synchronises the stream once before returning.
 *   out     : receives the plan (owned by the caller, release with dctplus_plan_destroy).
 * The DENSE and GFT routes allocate an n x n matrix (4 n^2 bytes, plus 2 n^2 for BF16;
 * 8 n^2 for FP64): 1 GiB in FP32 at n = 16384.
 */
dctplus_status dctplus_plan(int64_t n, double rho, const double *v_host, const dctplus_opts *opts,
                            void *stream, dctplus_plan_t *out);

/*
 * Build a plan for k rank-one updates, L = L_path + sum_{j<k} rho_j v_j v_j^T (Sec. 4.3,
 * Cor. 4.5: rank-k updates keep the Cauchy structure, by induction over the updates).
 *   k       : 1 <= k <= 64; k = 1 is dctplus_plan.
 *   rho_host: HOST array of k finite doubles; V_host: HOST k x n doubles, row j = v_j
 *             (both copied).
 * Update j >= 2 is a rank-one update of diag(mu_{j-1}) with z_j = X_{j-1}^T v_j (the basis
 * of the updates before it; the corollary's induction needs it):
 *     X_j^T = diag(a_j) C(mu_j, mu_{j-1}) diag(z_j) X_{j-1}^T,
 * with the rank-one conventions per update (a_j > 0, deflation of z_j,m = 0 keeping row m,
 * ascending rows, a root tying a deflated eigenvalue ordered after it).  The set-up runs
 * in FP64 on the GPU and composes the updates' Cauchy factors into one n x n factor C_k
 * (X_k^T = C_k U^T), which the DENSE route applies after the DCT-II (factored) or folds
 * with it; GFT applies X_k^T.  Resulting sign convention: eigenvector x_i has
 * rho_j v_j^T x_i > 0 for the last update j with v_j^T x_i != 0.
 * Limits for k > 1: DENSE and GFT routes only (AUTO = DENSE; FAST is EUNSUPPORTED: the
 * later poles are not Chebyshev nodes), n <= 4096 (EUNSUPPORTED above).
 * Errors: as dctplus_plan, plus EDEGENERATE when an update meets two equal eigenvalues of
 * the updates before it and touches both (the stage would first need a rotation inside
 * that eigenspace).  dctplus_grad on such a plan gives dl/dx only (grho / gv requested:
 * EUNSUPPORTED).  Forward, adjoint, plan_info (the last update's tables) and destroy as
 * for rank-one plans.
 */
dctplus_status dctplus_plan_rank_k(int64_t n, int32_t k, const double *rho_host, const double *V_host,
                                   const dctplus_opts *opts, void *stream, dctplus_plan_t *out);

/*
 * Build a plan for a rank-one update of a caller's base, L = U diag(lambda) U^T + rho v v^T
 * (Thm 3.1 holds for any symmetric base: X^T = diag(a) C(mu, lambda) diag(z) U^T with
 * z = U^T v; Thm 3.2).  A DTT+ transform, for example, takes the ADST graph's DST-VII
 * basis and eigenvalues as the base.
 *   lambda_host: HOST n doubles, strictly increasing (the base eigenvalues).
 *   U_host     : HOST n x n doubles, row-major, column k = the base eigenvector of
 *                lambda_k (orthonormal columns; not checked).
 *   rho, v_host: the update (HOST, n doubles).
 * Set-up in FP64 on the GPU (secular roots with the poles lambda, the Cauchy factor, and
 * X^T = diag(a) C diag(z) U^T formed once); the transform is the dense product with X^T
 * (route AUTO, DENSE or GFT, not factored: a general U has no fast product here; FAST
 * and factored are EUNSUPPORTED).  n: a power of two in [4, 4096].
 * Conventions as for dctplus_plan with U in place of the DCT-II: rho v^T x_i > 0, and a
 * deflated row (z_k = 0) is u_k itself.
 * Errors: EINVAL (null or non-finite input, lambda not strictly increasing),
 * EUNSUPPORTED, ENOMEM, ENOCONV, EDEVICE.  dctplus_grad gives dl/dx only.
 */
dctplus_status dctplus_plan_general(int64_t n, const double *lambda_host, const double *U_host, double rho,
                                    const double *v_host, const dctplus_opts *opts, void *stream,
                                    dctplus_plan_t *out);

/* y = X^T x for `batch` signals (Thm 3.1; Alg. 1 on the FAST route).
 * x, y: device arrays [batch, n] of the plan's element type; x and y must not alias.
 * batch == 0 is a no-op; batch < 0 is EINVAL. */
dctplus_status dctplus_forward(dctplus_plan_t plan, const void *x, void *y, int64_t batch, void *stream);

/* x = X y for `batch` signals: the inverse (X is orthogonal), formed by
 * applying the transposed steps of the forward in reverse order (Sec. 3,
 * Thm 3.3: backward transform by step-wise inversion).  Same layout rules. */
dctplus_status dctplus_adjoint(dctplus_plan_t plan, const void *y, void *x, int64_t batch, void *stream);

/*
 * Gradient of a scalar loss l(y), y = X^T x, given gy = dl/dy (FP32 plans only).
 *   y, gy  : device [batch, n] FP32 (y from dctplus_forward on the same x).
 *   gx     : device [batch, n] FP32 receiving dl/dx = X gy, or NULL to skip.
 *   grho   : device pointer to one double receiving dl/drho, or NULL.
 *   gv     : device pointer to n doubles receiving dl/dv, or NULL.
 * With G = sum_b gy_b y_b^T, A_ik = G_ik / (mu_i - mu_k) (A_ii = 0) and
 * w = X^T v:  dl/drho = w^T A w,  dl/dv = rho X (A + A^T) w  (first-order
 * eigenvector perturbation of L x_i = mu_i x_i, with Lemma 4.2 for w).
 * Uses the workspace of `stream` in the plan (see the conventions above).
 * Errors (all detected before any device work, so nothing is written):
 *   EUNSUPPORTED  grho or gv requested with n > 4096;
 *   EDEGENERATE   grho or gv requested on a plan with a double eigenvalue (a secular
 *                 root on a deflated lambda_k, e.g. a mirror-symmetric added edge): the
 *                 eigenbasis, and the row order, are not differentiable in (rho, v)
 *                 there.  dl/dx alone is always available.
 */
dctplus_status dctplus_grad(dctplus_plan_t plan, const void *y, const void *gy, int64_t batch, void *gx,
                            double *grho, double *gv, void *stream);

/*
 * dctplus_grad without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as dctplus_grad; the
 * Gram partials, G and the O(n) vectors live in one fixed 16 MiB device
 * array per GPU, set up on the first call on that GPU and held until the
 * process ends.  Nothing of the array needs to start at zero (every kernel
 * writes the whole of what it later reads).  No hipMalloc, hipFree or
 * allocating library routine is called.
 * Limits (EUNSUPPORTED, before any device work):
 *   - grho or gv requested with n > 512 (the scratch holds the n x n G and G^T
 *     in FP64 plus at least one n x n FP32 partial);
 *   - gx requested on a plan whose adjoint needs a workspace: DENSE plans in the
 *     factored form with n > 64, and FAST plans whose per-signal buffer does not fit
 *     in LDS.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams, threads or plans) race and give wrong results;
 * order them (one stream, or events).
 */
dctplus_status dctplus_grad_noalloc(dctplus_plan_t plan, const void *y, const void *gy, int64_t batch, void *gx,
                                    double *grho, double *gv, void *stream);

/*
 * Launch autotuner of the transform (forward and adjoint).  For `batch` signals it times
 * every launch configuration the plan's route offers (HIP events on `stream`, one warm-up
 * and three calls each) and keeps the fastest in the plan for batches of the same size
 * bucket floor(log2 batch), per direction:
 *   streaming dense kernels (n <= 64): persistent workgroups per CU, 1..4;
 *   the dense product above n = 64: GEMM tiles 64 x 64 or 128 x 128;
 *   FAST: signals per workgroup, the built-in count, a half or a quarter of it.
 * Every configuration computes the same transform (the dense kernels give the same bits;
 * FAST may differ in rounding within its bar).
 *   x, y       : DEVICE scratch arrays [batch, n] of the plan's type; both are overwritten.
 *   cache_path : NULL, or a file that receives the choices as a JSON object keyed by device
 *                architecture, n, route, dtype, form, direction and batch bucket (merged
 *                with what the file holds).  Plans created while the environment variable
 *                DCTPLUS_TUNE_CACHE names such a file start with its matching choices.
 *   chosen     : HOST int32[2] (nullable): the configuration ids kept (0: nothing to tune).
 *   ms         : HOST float[16] (nullable): mean ms per call, [direction][config id - 1].
 * Synchronises `stream`; not for use under graph capture.  Errors: as dctplus_forward;
 * EINVAL when the cache file cannot be written (the plan keeps its choices).
 */
dctplus_status dctplus_tune(dctplus_plan_t plan, void *x, void *y, int64_t batch, void *stream,
                            const char *cache_path, int32_t *chosen, float *ms);

/*
 * Copy plan tables to HOST arrays (synchronous; for tests and tools).
 * Any pointer may be NULL.  mu, a: n doubles in row order (a_i = 1 for
 * deflated rows); z: n doubles, U^T v after deflation; kind: n int32 per row
 * (0 = NUFFT row, 1 = deflated row, 2 = row summed directly);
 * counts: 4 int32 = {deflated rows, direct rows, NUFFT window width, route used}.
 */
dctplus_status dctplus_plan_info(dctplus_plan_t plan, double *mu, double *a, double *z, int32_t *kind,
                                 int32_t *counts);

/* Copy one named plan table to HOST memory (synchronous; for tests and tools).
 * name: "z", "zraw", "mu", "a", "tau", "hz", "deconv", "rowA", "rowB", "win", "direct",
 *       "sintab" (double); "wina" (double [18 taps][n], tap-major: the window weight of
 *       bin b at grid point 2b + 1 - width/2 + tap, times the bin's row factor);
 *       "wspr" (double [10][2n]: grid point P's weight for bin blo(P) + slot, the
 *       adjoint's spreading); "origin", "kind", "ref", "m0", "rowOfBin", "rowOfK",
 *       "direct_row", "ntie" (one value: the number of secular roots tying a deflated
 *       lambda) (int32); "tune": int8 [2][64], the launch configuration dctplus_tune chose
 *       per direction (0 forward, 1 adjoint) and batch bucket floor(log2 batch), 0 = built-in.
 * *bytes: capacity of dst on input, size of the table on output; dst may be NULL to
 * query the size.  Unknown name: EINVAL. */
dctplus_status dctplus_plan_table(dctplus_plan_t plan, const char *name, void *dst, int64_t *bytes);

/* Release a plan and its device memory (NULL is a no-op).  Synchronises the device. */
void dctplus_plan_destroy(dctplus_plan_t plan);

/*
 * Batched progressive transform selection with pruning (Thm 3.1: every
 * candidate rank-one update of one path graph shares the graph's DCT-II;
 * Thm 3.4: a signal with small path-Laplacian quadratic form keeps only the
 * upper-left c_p x c_p block of the candidate's Cauchy factor; Sec. 5:
 * block-wise selection among self-loop and added-edge candidates).
 *
 * Problem: nblocks independent blocks.  Block b is a path graph of n_b
 * vertices (n_b in {4, 8, 16, 32, 64}) with S signals (1 <= S <= 64) and K
 * candidates (1 <= K <= 16).  Candidate r of block b is four doubles
 * cand[(b*K + r)*4 .. +3] = (kind, i, j, w):
 *   kind 0: self-loop of weight w at vertex i   (rho = w,  v = e_i; j ignored
 *           but must lie in [0, n_b)),
 *   kind 1: added edge (i, j), i != j, weight w (rho = 2w, v = (e_i - e_j)/sqrt 2),
 * with integer-valued i, j in [0, n_b) and finite w > 0.  Candidate r's
 * transform is the DCT+ basis of L_path + rho v v^T with the conventions
 * above (rows in ascending eigenvalue order, rho v^T x_i > 0, deflated rows =
 * DCT vectors, deflation tolerance 1e-13).
 *
 * dctplus_select_plan: n_host[nblocks] (int32) and cand_host[nblocks*K*4]
 *   are HOST arrays (copied).  Builds every candidate's factor
 *   diag(a) C(mu, lambda) diag(z) on the GPU in FP64 and keeps it in FP32
 *   (4 K sum_b n_b^2 bytes of device memory).  Synchronises `stream` once.
 *   Errors: EINVAL (bad sizes or candidates; nothing allocated), EUNSUPPORTED
 *   (a block size outside the list), ENOMEM, ENOCONV (secular solver),
 *   EDEVICE.  nblocks == 0 gives a valid empty plan.
 *
 * dctplus_select: x is the DEVICE array of all signals, block after block,
 *   each block S x n_b row-major FP32 (block b starts at float
 *   sum_{b' < b} S n_b'; dctplus_select_size() gives the total).  Signal s of
 *   block b is pruned when sum_j (x_{j+1} - x_j)^2 <= prune_tau * ||x||^2
 *   (sums in FP64 of the FP32 samples); pruned signals use the c_p x c_p block (c_p <= 0:
 *   max(2, n_b / 2); c_p > n_b: n_b).  cost[b*K + r] (DEVICE, FP32) = sum
 *   over the block's signals of the L1 norm of candidate r's coefficients;
 *   best[b] (DEVICE, int32) = argmin_r cost (ties: lowest r); y_best (DEVICE,
 *   same layout as x, 16-byte aligned, not overlapping x) = the winner's
 *   coefficients (zero outside the c_p block for pruned signals).
 *   Asynchronous on `stream`; one persistent kernel launch.  Calls on one
 *   selection plan must not overlap (they share its work-queue counter).
 *
 * dctplus_select_tune: the launch autotuner of dctplus_select.  Runs the
 *   selection with the persistent grid at 1, 2, 3 and 4 workgroups per CU
 *   (one warm-up and three timed calls each, HIP events on `stream`), keeps
 *   the fastest in the plan for later dctplus_select calls, writes it to
 *   *chosen (nullable) and the average milliseconds per call of each
 *   candidate to ms[0..3] (HOST, nullable).  Arguments and errors as for
 *   dctplus_select; the outputs hold the (grid-independent) result of the
 *   last call.  Synchronises `stream`; not for use under graph capture.
 * dctplus_select_factor: HOST copy (n_b x n_b doubles, row-major, the FP32
 *   values as stored) of candidate r's factor of block `block`; synchronous.
 * dctplus_select_size: total floats of x / y_best (-1 for a NULL plan).
 * dctplus_select_destroy: releases the plan (NULL is a no-op); synchronises the device.
 */
typedef struct dctplus_select_s *dctplus_select_t;

dctplus_status dctplus_select_plan(int64_t nblocks, int32_t K, int32_t S, const int32_t *n_host,
                                   const double *cand_host, void *stream, dctplus_select_t *out);
dctplus_status dctplus_select(dctplus_select_t plan, const float *x, int32_t c_p, double prune_tau, int32_t *best,
                              float *cost, float *y_best, void *stream);
dctplus_status dctplus_select_tune(dctplus_select_t plan, const float *x, int32_t c_p, double prune_tau,
                                   int32_t *best, float *cost, float *y_best, void *stream, int32_t *chosen,
                                   float *ms);
dctplus_status dctplus_select_factor(dctplus_select_t plan, int64_t block, int32_t r, double *dst);
int64_t dctplus_select_size(dctplus_select_t plan);
void dctplus_select_destroy(dctplus_select_t plan);

const char *dctplus_status_string(dctplus_status s);
const char *dctplus_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCTPLUS_H */
