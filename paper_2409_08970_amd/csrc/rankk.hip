// Rank-k updates of the path graph (Sec. 4.3, Cor. 4.5):
//   L_k = L_path + sum_{j=1..k} rho_j v_j v_j^T = X_k diag(mu_k) X_k^T,
//   X_j^T = W_j^T X_{j-1}^T,  W_j^T = diag(a_j) C(mu_j, mu_{j-1}) diag(z_j),
//   z_j = X_{j-1}^T v_j  (the corollary's induction needs the previous stage's basis),
// each stage a rank-one update of the diagonal matrix diag(mu_{j-1}): its eigenvalues
// are the roots of 1 + rho_j sum_m z_m^2 / (mu_{j-1,m} - mu) = 0 (Lemma 4.1 interlacing,
// Remark 1), with the rank-one conventions (a_j > 0, deflation of z_m = 0, rows in
// ascending eigenvalue order, a root tying a deflated pole ordered after it).
//
// Setup, FP64 on the GPU: stage 1 is the rank-one plan of (rho_1, v_1) (Chebyshev poles,
// Thm 3.1), whose Cauchy factor M_1 = diag(a) C(mu_1, lambda) diag(z) is formed as a
// dense FP64 matrix; for j >= 2 the stage's poles are the previous eigenvalues and its
// factor W_j^T is formed densely and composed, C_j = W_j^T C_{j-1} (FP64 MFMA GEMM).  The
// composite C_k = W_k^T ... W_2^T M_1 is the Cauchy factor of the rank-k transform:
//   X_k^T = C_k U^T,
// so the transform is applied as for a rank-one plan (DCT-II, then one dense product
// with C_k, or C_k folded with the DCT at plan time).
//
// The same stage kernels serve a rank-one update of a caller's base L_base = U diag(lambda)
// U^T (Thm 3.1 holds for any symmetric base; Thm 3.2): z = U^T v, the secular roots with
// the poles lambda, and X^T = W^T U^T formed in FP64, applied as a dense product.
#include <vector>

#include "fft.h"

namespace dctplus {

namespace {

constexpr int kRkThreads = 1024;

// u = U^T v (orthonormal DCT-II) in FP64: one workgroup, LDS FFT.
__global__ void __launch_bounds__(kRkThreads) k_rk_dct(PlanTables t, const double *__restrict__ v,
                                                       double *__restrict__ u) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<double> *buf = reinterpret_cast<cplx<double> *>(smem);
    const int n = t.n, logn = t.logn, tid = threadIdx.x, nthr = blockDim.x;
    const int M = n / 2, logT = logn + 2;
    for (int m = tid; m < M; m += nthr) buf[fft_slot<double>(m)] = dct2_pack<double>(v, m, n);
    __syncthreads();
    const RadixPlan rp = radix_plan(logn - 1, 1, nthr);
    fft_dif(buf, 1, M, logn - 1, t.tw64, logT, rp);
    for (int k = tid; k <= M; k += nthr) {
        double Xk, XNk;
        dct2_post(buf, k, logn, rp, t.tw64, logT, Xk, XNk);
        u[k] = Xk;
        if (k > 0 && k < M) u[n - k] = XNk;
    }
}

// z = U^T v (U row-major n x n, column k = u_k), FP64; one wave per k.
__global__ void __launch_bounds__(256) k_rk_gemv_t(const double *__restrict__ U, const double *__restrict__ v,
                                                   double *__restrict__ z, int n) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= n) return;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += U[(size_t)j * n + k] * v[j];
    s = wave_sum(s);
    if (lane == 0) z[k] = s;
}

// z = C u (C row-major n x n, FP64); one wave per row.
__global__ void __launch_bounds__(256) k_rk_gemv(const double *__restrict__ C, const double *__restrict__ u,
                                                 double *__restrict__ z, int n) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;
    double s = 0.0;
    for (int m = lane; m < n; m += 64) s += C[(size_t)i * n + m] * u[m];
    s = wave_sum(s);
    if (lane == 0) z[i] = s;
}

// Deflation |z_m| <= tol ||z|| -> z_m = 0 (all of z when rho = 0), and the ascending list
// J of the remaining indices.  st[0] = nj, misc[0] = ||z||^2.  One workgroup.
__global__ void __launch_bounds__(kRkThreads) k_rk_deflate(double *__restrict__ z, int n, double rho, double tol,
                                                           int32_t *__restrict__ J, int32_t *__restrict__ st,
                                                           double *__restrict__ misc) {
    __shared__ double red[kRkThreads / 64];
    __shared__ int cnt[kRkThreads];
    __shared__ int total;
    const int tid = threadIdx.x, nthr = blockDim.x;
    double ss = 0.0;
    for (int m = tid; m < n; m += nthr) ss += z[m] * z[m];
    ss = wave_sum(ss);
    if ((tid & 63) == 0) red[tid >> 6] = ss;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < nthr / 64; ++w) s += red[w];
        red[0] = s;
        misc[0] = s;
    }
    __syncthreads();
    const double thr = tol * sqrt(red[0]);
    const int chunk = (n + nthr - 1) / nthr;
    const int k0 = tid * chunk, k1 = min(n, k0 + chunk);
    int c = 0;
    for (int m = k0; m < k1; ++m) {
        if (!(fabs(z[m]) > thr) || rho == 0.0) z[m] = 0.0;
        c += (z[m] != 0.0);
    }
    cnt[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < nthr; ++i) {
            const int x = cnt[i];
            cnt[i] = acc;
            acc += x;
        }
        total = acc;
    }
    __syncthreads();
    int pos = cnt[tid];
    for (int m = k0; m < k1; ++m)
        if (z[m] != 0.0) J[pos++] = m;
    if (tid == 0) st[0] = total;
}

struct SecSums {
    double F, Fp;   // 1/rho + sum over non-origin poles of z^2 / (d - t), and of z^2 / (d - t)^2
};

// Secular sums of one root about pole o (offset t = mu - d_o), split over the wave.
__device__ __forceinline__ SecSums sec_sums(const double *d, const double *z, const int32_t *J, int nj, int o,
                                            double tt, double rho, int lane) {
    double F = 0.0, Fp = 0.0;
    const double dO = d[o];
    for (int q = lane; q < nj; q += 64) {
        const int m = J[q];
        if (m == o) continue;
        const double zm = z[m];
        const double r = zm / ((d[m] - dO) - tt);
        F += zm * r;
        Fp += r * r;
    }
    return SecSums{1.0 / rho + wave_sum(F), wave_sum(Fp)};
}

// One wave per secular root of the stage (poles d ascending, weights z^2 on J), solved in
// offset form about the nearer pole: safeguarded Newton on g(t) = z_o^2 - t F(t) with a
// bisection bracket from the sign of the secular function, as for the rank-one plan.
// st[1] |= 1: no convergence; st[1] |= 4: two non-deflated poles coincide (the stage
// would need a rotation of that eigenspace first).
__global__ void __launch_bounds__(256) k_rk_roots(const double *__restrict__ d, const double *__restrict__ z,
                                                  const int32_t *__restrict__ J, int32_t *__restrict__ st,
                                                  const double *__restrict__ misc, double rho,
                                                  int32_t *__restrict__ r_o, double *__restrict__ r_tau,
                                                  double *__restrict__ r_a) {
    const int nj = st[0];
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nj) return;   // the whole wave leaves
    const double znorm2 = misc[0];
    int pa, pb;
    if (rho > 0) {
        pa = J[r];
        pb = (r + 1 < nj) ? J[r + 1] : -1;
    } else {
        pb = J[r];
        pa = (r > 0) ? J[r - 1] : -1;
    }
    int o;
    double lo, hi;
    if (pa >= 0 && pb >= 0) {
        const double gap = d[pb] - d[pa];
        if (!(gap > 1e-14 * (fabs(d[pa]) + fabs(d[pb]) + 1e-300))) {
            if (lane == 0) atomicOr(&st[1], 4);
            o = pa; lo = 0.0; hi = 0.0;
        } else {
            const SecSums s = sec_sums(d, z, J, nj, pa, 0.5 * gap, rho, lane);
            const double za = z[pa];
            const double f = s.F - za * za / (0.5 * gap);
            if (f >= 0.0) {
                o = pa; lo = 0.0; hi = 0.5 * gap;
            } else {
                o = pb; lo = -0.5 * gap; hi = 0.0;
            }
        }
    } else if (rho > 0) {
        o = pa; lo = 0.0; hi = rho * znorm2 * (1.0 + 1e-12);
    } else {
        o = pb; lo = rho * znorm2 * (1.0 + 1e-12); hi = 0.0;
    }
    const double zo2 = z[o] * z[o];
    double tt = 0.5 * (lo + hi);
    SecSums s{};
    bool conv = (hi == lo);
    for (int it = 0; it < 200 && !conv; ++it) {
        s = sec_sums(d, z, J, nj, o, tt, rho, lane);
        const double f = s.F - zo2 / tt;
        if (f > 0.0) hi = tt;
        else if (f < 0.0) lo = tt;
        else { conv = true; break; }
        const double g = zo2 - tt * s.F;
        const double gp = -s.F - tt * s.Fp;
        double tn = tt - g / gp;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == tt || fabs(tn - tt) <= 2.0 * 2.220446049250313e-16 * fabs(tn) || hi - lo <= 0.0) {
            tt = tn;
            conv = true;
            break;
        }
        tt = tn;
    }
    s = sec_sums(d, z, J, nj, o, tt, rho, lane);
    const double fp = s.Fp + zo2 / (tt * tt);
    if (lane == 0) {
        r_o[r] = o;
        r_tau[r] = tt;
        r_a[r] = 1.0 / sqrt(fp);
        if (!conv) atomicOr(&st[1], 1);
    }
}

// Row order of the stage (ascending eigenvalue; a root tying a deflated pole after it) and
// its tables: mu, a, kind, origin, tau per row.  st[2] = number of such ties.  One workgroup.
__global__ void __launch_bounds__(kRkThreads) k_rk_rows(const double *__restrict__ d, const double *__restrict__ z,
                                                        int n, double rho, const int32_t *__restrict__ st_in,
                                                        int32_t *__restrict__ st, const double *__restrict__ misc,
                                                        const int32_t *__restrict__ r_o,
                                                        const double *__restrict__ r_tau,
                                                        const double *__restrict__ r_a, double *__restrict__ mu,
                                                        double *__restrict__ a, int32_t *__restrict__ kind,
                                                        int32_t *__restrict__ origin, double *__restrict__ tau) {
    extern __shared__ __align__(16) unsigned char smem[];
    int *cntD = reinterpret_cast<int *>(smem);   // [n + 1]: deflated poles below each index
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nj = st_in[0];
    const double dmax = fmax(fabs(d[0]), fabs(d[n - 1]));
    const double tie = 1e-12 * (dmax + fabs(rho) * misc[0] + 1e-300);
    if (tid == 0) {
        int acc = 0;
        for (int m = 0; m < n; ++m) {
            cntD[m] = acc;
            acc += (z[m] == 0.0);
        }
        cntD[n] = acc;
    }
    for (int i = tid; i < n; i += nthr) kind[i] = -1;
    __syncthreads();
    for (int r = tid; r < nj; r += nthr) {
        const int o = r_o[r];
        const double m_r = d[o] + r_tau[r];
        int lo = -1, hi = n - 1;   // largest m with d_m <= mu + tie
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid] <= m_r + tie) lo = mid; else hi = mid - 1;
        }
        const int row = r + ((lo >= 0) ? cntD[lo + 1] : 0);
        mu[row] = m_r;
        a[row] = r_a[r];
        kind[row] = ROW_NUFFT;
        origin[row] = o;
        tau[row] = r_tau[r];
        if (lo >= 0 && z[lo] == 0.0 && fabs((d[lo] - d[o]) - r_tau[r]) <= tie) atomicAdd(&st[2], 1);
    }
    for (int m = tid; m < n; m += nthr) {
        if (z[m] != 0.0) continue;
        int lo = 0, hi = nj;   // roots with mu < d_m - tie (the complement of the test above)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const double mm = d[r_o[mid]] + r_tau[mid];
            if (!(d[m] <= mm + tie)) lo = mid + 1; else hi = mid;
        }
        const int row = cntD[m] + lo;
        mu[row] = d[m];
        a[row] = 1.0;
        kind[row] = ROW_DEFLATED;
        origin[row] = m;
        tau[row] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nthr)
        if (kind[i] < 0) atomicOr(&st[1], 2);
}

// The stage factor W^T (row-major n x n, FP64): row i = a_i z_m / (mu_i - d_m) over m, the
// gap formed as tau_i - (d_m - d_o); a deflated row is e_o.  One workgroup per row.
__global__ void __launch_bounds__(256) k_rk_factor(const double *__restrict__ d, const double *__restrict__ z,
                                                   int n, const double *__restrict__ a,
                                                   const int32_t *__restrict__ kind, const int32_t *__restrict__ origin,
                                                   const double *__restrict__ tau, double *__restrict__ W) {
    const int i = blockIdx.x;
    const int o = origin[i];
    const bool defl = kind[i] == ROW_DEFLATED;
    const double ai = a[i], ti = tau[i], dO = d[o];
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        double w;
        if (defl) w = (m == o) ? 1.0 : 0.0;
        else w = (z[m] != 0.0) ? ai * z[m] / (ti - (d[m] - dO)) : 0.0;
        W[(size_t)i * n + m] = w;
    }
}

}  // namespace

dctplus_status rank_k_build(dctplus_plan_s *p, int k, const double *rho_host, const double *V_host, hipStream_t s) {
    const int n = (int)p->n;
    PlanTables &t = p->t;
    const size_t nn = (size_t)n * n, nd = sizeof(double) * n;
    // device scratch: C, W, Cnext (n x n FP64), v, u, z, d, mu, a, tau (n), int tables, status
    char *buf = nullptr;
    const size_t mat = sizeof(double) * nn;
    const size_t bytes = 3 * mat + 9 * nd + 4 * sizeof(int32_t) * n + 64 * sizeof(int32_t) * (size_t)k + 64;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc(%zu) for the rank-k set-up failed", bytes);
    }
    double *C = (double *)buf, *W = C + nn, *Cn = W + nn;
    double *v = Cn + nn, *u = v + n, *z = u + n, *d = z + n, *mu = d + n, *a = mu + n, *tau = a + n;
    double *r_tau = tau + n, *r_a = r_tau + n;
    int32_t *J = (int32_t *)(r_a + n), *kind = J + n, *origin = kind + n, *r_o = origin + n;
    int32_t *st = r_o + n;   // per stage: [nj, flags, ties, pad]
    double *misc = (double *)(st + 4 * k + 4);
    dctplus_status ret = DCTPLUS_OK;
    auto done = [&](dctplus_status r) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        return r;
    };
    if ((e = hipMemsetAsync(st, 0, sizeof(int32_t) * (4 * k + 4), s)) != hipSuccess)
        return done(hip_fail(e, "rank-k status clear"));
    // stage 1: the rank-one plan's Cauchy factor in FP64, its eigenvalues as the next poles
    launch_cauchy_f64(p, C, s);
    if ((e = hipMemcpyAsync(d, t.mu, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return done(hip_fail(e, "rank-k poles"));
    const size_t lds_dct = sizeof(cplx<double>) * (n / 2);
    for (int j = 1; j < k; ++j) {
        const double rho = rho_host[j];
        int32_t *sj = st + 4 * j;
        if ((e = hipMemcpyAsync(v, V_host + (size_t)j * n, nd, hipMemcpyHostToDevice, s)) != hipSuccess)
            return done(hip_fail(e, "copy v_j"));
        // z_j = X_{j-1}^T v_j = C_{j-1} U^T v_j
        hipLaunchKernelGGL(k_rk_dct, dim3(1), dim3(kRkThreads), lds_dct, s, t, (const double *)v, u);
        hipLaunchKernelGGL(k_rk_gemv, dim3((n + 3) / 4), dim3(256), 0, s, (const double *)C, (const double *)u, z, n);
        hipLaunchKernelGGL(k_rk_deflate, dim3(1), dim3(kRkThreads), 0, s, z, n, rho, p->defl_tol, J, sj, misc);
        hipLaunchKernelGGL(k_rk_roots, dim3((n + 3) / 4), dim3(256), 0, s, (const double *)d, (const double *)z,
                           (const int32_t *)J, sj, (const double *)misc, rho, r_o, r_tau, r_a);
        hipLaunchKernelGGL(k_rk_rows, dim3(1), dim3(kRkThreads), sizeof(int) * (n + 1), s, (const double *)d,
                           (const double *)z, n, rho, (const int32_t *)sj, sj, (const double *)misc,
                           (const int32_t *)r_o, (const double *)r_tau, (const double *)r_a, mu, a, kind, origin,
                           tau);
        hipLaunchKernelGGL(k_rk_factor, dim3(n), dim3(256), 0, s, (const double *)d, (const double *)z, n,
                           (const double *)a, (const int32_t *)kind, (const int32_t *)origin, (const double *)tau,
                           W);
        // C_j = W_j^T C_{j-1}
        gemm64(W, C, Cn, n, n, false, s);
        double *tmp = C;
        C = Cn;
        Cn = tmp;
        if ((e = hipMemcpyAsync(d, mu, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return done(hip_fail(e, "rank-k poles"));
    }
    if ((e = hipGetLastError()) != hipSuccess) return done(hip_fail(e, "rank-k stage kernels"));
    std::vector<int32_t> sth(4 * k + 4);
    if ((e = hipMemcpyAsync(sth.data(), st, sizeof(int32_t) * (4 * k + 4), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return done(hip_fail(e, "rank-k status copy"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return done(hip_fail(e, "rank-k synchronize"));
    int ties = t.ntie;
    for (int j = 1; j < k; ++j) {
        const int32_t f = sth[4 * j + 1];
        if (f & 1) return done(fail(DCTPLUS_ENOCONV, "secular solver of update %d did not converge", j + 1));
        if (f & 4)
            return done(fail(DCTPLUS_EDEGENERATE, "update %d meets two coinciding eigenvalues of the earlier "
                                                  "updates (a double eigenvalue with both directions touched)",
                             j + 1));
        if (f & 2) return done(fail(DCTPLUS_EDEVICE, "internal error: rank-k row order is not a permutation"));
        ties += sth[4 * j + 2];
    }
    t.ntie = ties;
    if (k > 1) {
        // the plan's spectrum tables describe the last stage (plan_info)
        if ((e = hipMemcpyAsync(t.mu, mu, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(t.a, a, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(t.z, z, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(t.kind, kind, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return done(hip_fail(e, "rank-k tables"));
        int32_t nd_last = 0;
        std::vector<int32_t> kh(n);
        if ((e = hipMemcpyAsync(kh.data(), kind, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return done(hip_fail(e, "rank-k kinds"));
        for (int i = 0; i < n; ++i) nd_last += (kh[i] == ROW_DEFLATED);
        t.ndefl = nd_last;
        t.ndirect = 0;
    }
    ret = dense_build_from(p, C, s);
    return done(ret);
}

}  // namespace dctplus

namespace dctplus {

dctplus_status general_build(dctplus_plan_s *p, const double *lam_host, const double *U_host, const double *v_host,
                             hipStream_t s) {
    const int n = (int)p->n;
    dctplus_status st0 = plan_alloc_tables(p, s);
    if (st0 != DCTPLUS_OK) return st0;
    PlanTables &t = p->t;
    const size_t nn = (size_t)n * n, nd = sizeof(double) * n;
    const size_t mat = sizeof(double) * nn;
    const size_t bytes = 3 * mat + 9 * nd + 4 * sizeof(int32_t) * n + 64 * sizeof(int32_t) + 64;
    char *buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc(%zu) for the general-base set-up failed", bytes);
    }
    double *U = (double *)buf, *W = U + nn, *Xt = W + nn;
    double *v = Xt + nn, *z = v + n, *d = z + n, *mu = d + n, *a = mu + n, *tau = a + n;
    double *r_tau = tau + n, *r_a = r_tau + n, *misc = r_a + n;
    int32_t *J = (int32_t *)(misc + n), *kind = J + n, *origin = kind + n, *r_o = origin + n;
    int32_t *st = r_o + n;
    auto done = [&](dctplus_status r) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        return r;
    };
    if ((e = hipMemsetAsync(st, 0, sizeof(int32_t) * 4, s)) != hipSuccess ||
        (e = hipMemcpyAsync(U, U_host, mat, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d, lam_host, nd, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(v, v_host, nd, hipMemcpyHostToDevice, s)) != hipSuccess)
        return done(hip_fail(e, "general-base inputs"));
    const double rho = p->rho;
    hipLaunchKernelGGL(k_rk_gemv_t, dim3((n + 3) / 4), dim3(256), 0, s, (const double *)U, (const double *)v, z, n);
    if ((e = hipMemcpyAsync(t.zraw, z, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return done(hip_fail(e, "general-base z"));
    hipLaunchKernelGGL(k_rk_deflate, dim3(1), dim3(kRkThreads), 0, s, z, n, rho, p->defl_tol, J, st, misc);
    hipLaunchKernelGGL(k_rk_roots, dim3((n + 3) / 4), dim3(256), 0, s, (const double *)d, (const double *)z,
                       (const int32_t *)J, st, (const double *)misc, rho, r_o, r_tau, r_a);
    hipLaunchKernelGGL(k_rk_rows, dim3(1), dim3(kRkThreads), sizeof(int) * (n + 1), s, (const double *)d,
                       (const double *)z, n, rho, (const int32_t *)st, st, (const double *)misc, (const int32_t *)r_o,
                       (const double *)r_tau, (const double *)r_a, mu, a, kind, origin, tau);
    hipLaunchKernelGGL(k_rk_factor, dim3(n), dim3(256), 0, s, (const double *)d, (const double *)z, n,
                       (const double *)a, (const int32_t *)kind, (const int32_t *)origin, (const double *)tau, W);
    // X^T = W^T U^T:  X^T[i][j] = sum_k W^T[i][k] U[j][k]
    gemm64(W, U, Xt, n, n, true, s);
    if ((e = hipGetLastError()) != hipSuccess) return done(hip_fail(e, "general-base kernels"));
    int32_t sth[4];
    std::vector<int32_t> kh(n);
    if ((e = hipMemcpyAsync(sth, st, sizeof(sth), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(kh.data(), kind, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(hip_fail(e, "general-base status"));
    if (sth[1] & 1) return done(fail(DCTPLUS_ENOCONV, "secular solver did not converge"));
    if (sth[1] & 4)
        return done(fail(DCTPLUS_EDEGENERATE, "two base eigenvalues coincide and v touches both directions"));
    if (sth[1] & 2) return done(fail(DCTPLUS_EDEVICE, "internal error: row order is not a permutation"));
    t.nj = sth[0];
    t.ntie = sth[2];
    t.ndirect = 0;
    int ndefl = 0;
    for (int i = 0; i < n; ++i) ndefl += (kh[i] == ROW_DEFLATED);
    t.ndefl = ndefl;
    if ((e = hipMemcpyAsync(t.mu, mu, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(t.a, a, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(t.z, z, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(t.kind, kind, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(t.origin, origin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(t.tau, tau, nd, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return done(hip_fail(e, "general-base tables"));
    return done(dense_build_from(p, Xt, s, true));
}

}  // namespace dctplus
