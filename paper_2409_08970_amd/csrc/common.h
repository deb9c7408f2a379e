// Internal declarations shared by the dctplus HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "dctplus.h"

namespace dctplus {

constexpr int kMaxLogN = 14;            // n <= 16384
constexpr int kMaxDirect = 512;         // rows summed exactly on the FAST route
constexpr int kMaxWidth = 16;           // NUFFT window taps
constexpr int kTaps = kMaxWidth + 2;    // stride of the aligned window table (taps past width + 2 are 0)
constexpr int kReach = kTaps / 2 + 1;   // bins whose window reaches one grid point, at most
constexpr int kMaxRank = 64;            // rank-one updates of a rank-k plan

template <typename T>
struct cplx {
    T re, im;
};

// Row kinds of the output ordering.
enum RowKind : int32_t { ROW_NUFFT = 0, ROW_DEFLATED = 1, ROW_DIRECT = 2 };

// Device-side tables of a plan (all pointers into one device allocation).
struct PlanTables {
    int n, logn;
    double rho;
    // spectrum and rows
    double *z;          // [n]    U^T v after deflation
    double *zraw;       // [n]    U^T v before deflation
    double *mu;         // [n]    eigenvalues in row order
    double *a;          // [n]    column normalisers in row order (1 for deflated rows)
    int32_t *origin;    // [n]    nearer pole (or deflated index) per row
    double *tau;        // [n]    mu - lambda_origin per row
    int32_t *kind;      // [n]    RowKind per row
    int32_t *ref;       // [n]    bin (NUFFT), index k (deflated) or slot (direct)
    // FAST route
    double *hz;         // [n]    (-1)^(j+1) z_j / sin(pi j / n), hz_0 = 0
    double *deconv;     // [n]    1 / window transform at frequency l
    double *rowA;       // [n]    per bin: -a / (2 sin(n psi))
    double *rowB;       // [n]    per bin: a z_0 / mu
    int32_t *m0;        // [n]    per bin: first grid tap
    double *win;        // [n * width] per bin window weights (0 for empty bins)
    double *wina;       // [kTaps * n] tap-major: entry (k, b) is rowA_b times the window weight at
                        //   grid point 2b + 1 - width/2 + k (taps aligned to a closed-form origin;
                        //   0 for empty bins)
    double *wspr;       // [kReach * 2n] the transposed interpolation per grid point P: entry (k, P)
                        //   is the weight of bin blo(P) + k, blo(P) = max(0, ((P - w/2 - 3) >> 1) + 1),
                        //   with the odd-extension folds of P near 0 and 2n merged in
    double *direct;     // [ndirect * n] exact rows a_i z_j / (mu_i - lambda_j)
    float *direct32;    // [ndirect * n] the same rows rounded to FP32 (plans with FP32 signals:
                        //   half the bytes for the kernels that read them per signal)
    int32_t *direct_row;// [ndirect] output row of each direct slot
    int32_t *rowOfBin;  // [n]    output row of the NUFFT root in bin b, or -1
    int32_t *rowOfK;    // [n]    output row of deflated index k, or -1
    cplx<double> *tw64; // [4n]   exp(-2 pi i k / 4n)
    cplx<float> *tw32;  // [4n]
    double *sintab;     // [2n+1] sin(pi k / 2n)
    // DENSE / GFT routes
    float *mt32;        // [n * n] column-major M (M^T row-major) or X^T for GFT
    uint16_t *mt16;     // [n * n] BF16 copy
    double *mt64;       // [n * n] FP64 X^T (FP64 plans)
    int32_t *status;    // [4]    plan-build status words
    int ndirect, ndefl, width, nj;
    int ntie;           // secular roots tying a deflated lambda_k (double eigenvalues)
    int folded;         // dense factor holds X^T (DCT folded in) rather than M
};

}  // namespace dctplus

struct dctplus_plan_s {
    int64_t n;
    int logn;
    double rho;
    int dtype, route, device;
    double defl_tol, direct_kappa;
    int width;
    int factored;             // DENSE route keeps the DCT and the Cauchy factor apart
    int defer_dense;          // plan_build leaves the dense operands to the caller (rank-k plans)
    int rank;                 // number of rank-one updates (1 for dctplus_plan)
    int64_t auto_fast_below = 0;   // AUTO plans on the dense product: batches below this run FAST
    // launch configuration chosen by dctplus_tune, per direction (0 forward, 1 adjoint)
    // and batch bucket floor(log2 batch); 0 = the built-in choice
    int8_t tune_cfg[2][64];
    int general;              // base basis given by the caller (dctplus_plan_general)
    void *dev_mem;            // one allocation holding every table
    size_t dev_bytes;
    // workspaces (FAST-route scratch for large n, the factored route's DCT output above
    // n = 64, gradient partials): one per stream handle, grown on demand, so calls on
    // different streams never share one
    struct StreamWork {
        hipStream_t stream;
        void *ptr;
        size_t bytes;
    };
    std::mutex work_mu;
    std::vector<StreamWork> works;
    void *simg;               // LDS images of the streaming kernel's operands (forward, adjoint), n <= 64
    size_t simg_bytes;        // bytes of one image
    dctplus::PlanTables t;
};

namespace dctplus {
// thread-local error message helpers (capi.hip)
dctplus_status fail(dctplus_status s, const char *fmt, ...);
dctplus_status hip_fail(hipError_t e, const char *what);

// route launchers (fast.hip, dense.hip, grad.hip)
dctplus_status fast_apply(dctplus_plan_s *p, const void *in, void *out, int64_t batch, bool adjoint,
                          hipStream_t s);
dctplus_status dense_apply(dctplus_plan_s *p, const void *in, void *out, int64_t batch, bool adjoint,
                           hipStream_t s);
dctplus_status dense_build(dctplus_plan_s *p, hipStream_t s);
// dense operands from a given FP64 Cauchy factor (row-major n x n) instead of the plan's
// (src_is_xt: src is X^T itself, applied as the folded product)
dctplus_status dense_build_from(dctplus_plan_s *p, const double *src, hipStream_t s, bool src_is_xt = false);
// the plan's device tables, allocated and the twiddle tables filled (no spectrum)
dctplus_status plan_alloc_tables(dctplus_plan_s *p, hipStream_t s);
// L = U diag(lambda) U^T + rho v v^T for a caller's base (Thm 3.1 on a general base; rankk.hip)
dctplus_status general_build(dctplus_plan_s *p, const double *lam_host, const double *U_host, const double *v_host,
                             hipStream_t s);
// M = diag(a) C(mu, lambda) diag(z) of a rank-one plan, FP64 row-major n x n
void launch_cauchy_f64(const dctplus_plan_s *p, double *M, hipStream_t s);
// FP64 C = A B(k, j) on MFMA: B(k, j) = P[j][k] (transb) or P[k][j]; A is [batch x n]
void gemm64(const double *A, const double *P, double *C, int64_t batch, int n, bool transb, hipStream_t s);
// the chain of Cor. 4.5 for updates 2..k (rankk.hip), after plan_build of update 1
dctplus_status rank_k_build(dctplus_plan_s *p, int k, const double *rho_host, const double *V_host, hipStream_t s);
void dense_release(dctplus_plan_s *p);
dctplus_status grad_apply(dctplus_plan_s *p, const float *y, const float *gy, int64_t batch, float *gx,
                          double *grho, double *gv, hipStream_t s);
// the gradient with its scratch in a caller-given device buffer (no allocation)
constexpr int kStaticGradMaxN = 512;
dctplus_status grad_apply_static(dctplus_plan_s *p, const float *y, const float *gy, int64_t batch, float *gx,
                                 double *grho, double *gv, void *scratch, size_t scratch_bytes, hipStream_t s);
// true when the plan's forward and adjoint need neither the plan workspace nor a library call
bool route_alloc_free(const dctplus_plan_s *p);
bool fast_in_lds(const dctplus_plan_s *p);
// launch configurations the tuner may choose from for this plan and batch (ids 1..count;
// 1 when there is nothing to choose)
int dense_tune_count(const dctplus_plan_s *p, int64_t batch);
int fast_tune_count(const dctplus_plan_s *p);
inline int batch_bucket(int64_t batch) {
    int b = 0;
    while (b < 63 && (int64_t(2) << b) <= batch) ++b;
    return b;
}
// the route a call of `batch` signals takes: the plan's, except that an AUTO plan kept on
// the dense product runs small batches on the FAST route (its tables are always built)
inline bool use_fast(const dctplus_plan_s *p, int64_t batch) {
    return p->route == DCTPLUS_ROUTE_FAST || batch < p->auto_fast_below;
}
inline int tuned(const dctplus_plan_s *p, bool adjoint, int64_t batch) {
    return p->tune_cfg[adjoint ? 1 : 0][batch_bucket(batch)];
}
dctplus_status plan_build(dctplus_plan_s *p, const double *v_host, hipStream_t s);
// the workspace of stream s, at least `bytes` long (grows it: waits for s, frees, allocates)
dctplus_status stream_work(dctplus_plan_s *p, hipStream_t s, size_t bytes, void **out);
void release_works(dctplus_plan_s *p);
}  // namespace dctplus
