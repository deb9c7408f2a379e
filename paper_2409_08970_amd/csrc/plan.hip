// Plan construction (setup of Remark 1), computed in FP64 on the GPU.
//
//   z = U^T v                       FP64 DCT-II of v (Makhoul, LDS FFT)
//   deflation                       |z_k| <= defl_tol ||z||  ->  z_k = 0, row = u_k
//   secular roots                   1 + rho sum_j z_j^2 / (lambda_j - mu) = 0, one root per
//                                   bracket between consecutive non-deflated poles (Lemma 4.1),
//                                   solved in offset form mu = lambda_o + tau
//   a_i                             (sum_j z_j^2 / (mu_i - lambda_j)^2)^(-1/2)  (Thm 3.1)
//   row order                       ascending eigenvalue; a root tying a deflated lambda_k is
//                                   ordered after it
//   FAST-route tables               per Chebyshev bin: window taps of the sine NUFFT, the
//                                   divide/compensate factors of Alg. 1, and the rows whose
//                                   NUFFT error amplification is too large (summed exactly)
//
// Differences lambda_j - lambda_o are always formed as 4 sin(pi (j-o)/2n) sin(pi (j+o)/2n)
// from a table of sin(pi k / 2n), so gaps keep full relative accuracy.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "fft.h"

namespace dctplus {

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kQuad = 192;  // Gauss-Legendre nodes for the window transform

__device__ __forceinline__ double lam(const double *sintab, int n, int k) {
    const double s = sintab[k];
    return 4.0 * s * s;
}

// exp(beta (sqrt(1 - (2u/w)^2) - 1)) on |u| < w/2: the "exponential of
// semicircle" window of Barnett, Magland and af Klinteberg (2019).
__device__ __forceinline__ double es_window(double u, int w, double beta) {
    const double t = 2.0 * u / w;
    const double s = 1.0 - t * t;
    return s > 0.0 ? exp(beta * (sqrt(s) - 1.0)) : 0.0;
}

__global__ void k_tables(PlanTables t) {
    const int n = t.n;
    const int T = 4 * n;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < T; k += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * k / T, &s, &c);
        t.tw64[k] = {c, -s};
        t.tw32[k] = {(float)c, (float)-s};
        if (k <= 2 * n) t.sintab[k] = sinpi((double)k / (2.0 * n));
    }
}

// z = DCT-II(v) in FP64, deflation, hz, compaction of non-deflated indices.
// One workgroup; LDS holds n/2 complex doubles.
__global__ void __launch_bounds__(kPlanThreads) k_z(PlanTables t, const double *__restrict__ v, double defl_tol,
                                                    int32_t *__restrict__ J, double *__restrict__ misc) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<double> *buf = reinterpret_cast<cplx<double> *>(smem);
    __shared__ double red[kPlanThreads / 64];
    __shared__ int scan_tot;
    const int n = t.n, logn = t.logn, tid = threadIdx.x, nthr = blockDim.x;
    const int M = n / 2, logT = logn + 2;
    for (int m = tid; m < M; m += nthr) buf[fft_slot<double>(m)] = dct2_pack<double>(v, m, n);
    __syncthreads();
    const RadixPlan rp = radix_plan(logn - 1, 1, nthr);
    fft_dif(buf, 1, M, logn - 1, t.tw64, logT, rp);
    double ss = 0.0;
    for (int k = tid; k <= M; k += nthr) {
        double Xk, XNk;
        dct2_post(buf, k, logn, rp, t.tw64, logT, Xk, XNk);
        t.z[k] = Xk;
        t.zraw[k] = Xk;
        ss += Xk * Xk;
        if (k > 0 && k < M) {
            t.z[n - k] = XNk;
            t.zraw[n - k] = XNk;
            ss += XNk * XNk;
        }
    }
    ss = wave_sum(ss);
    if ((tid & 63) == 0) red[tid >> 6] = ss;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < nthr / 64; ++w) s += red[w];
        red[0] = s;
    }
    __syncthreads();
    const double znorm2 = red[0];
    const double thr = defl_tol * sqrt(znorm2);
    __syncthreads();
    // deflate and build hz
    double hzmax = 0.0;
    for (int k = tid; k < n; k += nthr) {
        double zk = t.z[k];
        if (!(fabs(zk) > thr) || t.rho == 0.0) zk = 0.0;
        t.z[k] = zk;
        double h = 0.0;
        if (k > 0) h = ((k & 1) ? 1.0 : -1.0) * zk / sinpi((double)k / n);
        t.hz[k] = h;
        hzmax = fmax(hzmax, fabs(h));
    }
    // block max of |hz|
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hzmax = fmax(hzmax, __shfl_xor(hzmax, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = hzmax;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < nthr / 64; ++w) s = fmax(s, red[w]);
        misc[0] = znorm2;
        misc[1] = s;
    }
    __syncthreads();
    // compaction: sequential chunks per thread, then an exclusive scan of counts
    int *cnt = reinterpret_cast<int *>(smem);   // reuse LDS (FFT data no longer needed)
    const int chunk = (n + nthr - 1) / nthr;
    const int k0 = tid * chunk, k1 = min(n, k0 + chunk);
    int c = 0;
    for (int k = k0; k < k1; ++k) c += (t.z[k] != 0.0);
    cnt[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < nthr; ++i) {
            const int x = cnt[i];
            cnt[i] = acc;
            acc += x;
        }
        scan_tot = acc;
    }
    __syncthreads();
    int pos = cnt[tid];
    for (int k = k0; k < k1; ++k)
        if (t.z[k] != 0.0) J[pos++] = k;
    if (tid == 0) t.status[1] = scan_tot;   // nj
}

struct Secular {
    double F, Fp;   // sum over non-origin poles of z^2 / (d - t) and z^2 / (d - t)^2
};

// Secular sums of one root, split over the 64 lanes of a wave (poles q = lane,
// lane + 64, ...) and reduced with a butterfly, so every lane holds the same sums.
__device__ __forceinline__ Secular secular_eval_wave(const PlanTables &t, const int32_t *J, int nj, int o,
                                                     double tt, int lane) {
    double F = 0.0, Fp = 0.0;
    for (int q = lane; q < nj; q += 64) {
        const int j = J[q];
        if (j == o) continue;
        const double zj = t.z[j];
        const double den = lam_diff(t.sintab, t.n, j, o) - tt;
        const double r = zj / den;
        F += zj * r;
        Fp += r * r;
    }
    return Secular{1.0 / t.rho + wave_sum(F), wave_sum(Fp)};
}

// One wave per secular root.  Safeguarded Newton on g(t) = z_o^2 - t F(t)
// (the secular function times -t, which removes the pole at the origin), with
// a bisection bracket kept from the sign of the secular function itself.  All
// control flow is uniform across the wave (the sums are identical on every lane).
__global__ void __launch_bounds__(256) k_roots(PlanTables t, const int32_t *__restrict__ J,
                                               const double *__restrict__ misc, int32_t *__restrict__ r_o,
                                               double *__restrict__ r_tau, double *__restrict__ r_a) {
    const int nj = t.status[1];
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nj) return;   // the whole wave leaves
    const int n = t.n;
    const double rho = t.rho, znorm2 = misc[0];
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
        const double gap = lam_diff(t.sintab, n, pb, pa);
        const Secular s = secular_eval_wave(t, J, nj, pa, 0.5 * gap, lane);
        const double za = t.z[pa];
        const double f = s.F - za * za / (0.5 * gap);
        if (f >= 0.0) {
            o = pa; lo = 0.0; hi = 0.5 * gap;
        } else {
            o = pb; lo = -0.5 * gap; hi = 0.0;
        }
    } else if (rho > 0) {
        o = pa; lo = 0.0; hi = rho * znorm2 * (1.0 + 1e-12);
    } else {
        o = pb; lo = rho * znorm2 * (1.0 + 1e-12); hi = 0.0;
    }
    const double zo = t.z[o], zo2 = zo * zo;
    double tt = 0.5 * (lo + hi);
    Secular s{};
    bool conv = false;
    for (int it = 0; it < 200; ++it) {
        s = secular_eval_wave(t, J, nj, o, tt, lane);
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
    s = secular_eval_wave(t, J, nj, o, tt, lane);
    const double fp = s.Fp + zo2 / (tt * tt);
    if (lane == 0) {
        r_o[r] = o;
        r_tau[r] = tt;
        r_a[r] = 1.0 / sqrt(fp);
        if (!conv) atomicOr(&t.status[0], 1);
    }
}

// Row ordering and per-row tables.  One workgroup.
__global__ void __launch_bounds__(kPlanThreads) k_rows(PlanTables t, const int32_t *__restrict__ J,
                                                       const double *__restrict__ misc,
                                                       const int32_t *__restrict__ r_o,
                                                       const double *__restrict__ r_tau,
                                                       const double *__restrict__ r_a, double kappa_max,
                                                       int32_t *__restrict__ rowOfBin, int32_t *__restrict__ rowOfK) {
    extern __shared__ __align__(16) unsigned char smem[];
    int *cntD = reinterpret_cast<int *>(smem);   // [n + 1] inclusive-exclusive deflated counts
    int *isdir = cntD + (t.n + 1);               // [n]
    __shared__ int sdirect;
    const int n = t.n, tid = threadIdx.x, nthr = blockDim.x;
    const int nj = t.status[1];
    const double rho = t.rho;
    const double tie = 1e-12 * (4.0 + fabs(rho) * misc[0]);
    const double maxhz = misc[1];
    const int w = t.width;
    const double beta = 2.30 * w;
    const double hgrid = M_PI / (2.0 * n);

    // deflated prefix counts: cntD[k] = #deflated indices < k
    if (tid == 0) {
        int acc = 0;
        for (int k = 0; k < n; ++k) {
            cntD[k] = acc;
            acc += (t.z[k] == 0.0);
        }
        cntD[n] = acc;
        t.status[2] = acc;   // ndefl
    }
    for (int i = tid; i < n; i += nthr) {
        isdir[i] = 0;
        t.kind[i] = -1;
        rowOfBin[i] = -1;
        rowOfK[i] = -1;
        t.rowA[i] = 0.0;
        t.rowB[i] = 0.0;
        t.m0[i] = 2 * i + 1 - w / 2;
        for (int q = 0; q < w; ++q) t.win[(size_t)i * w + q] = 0.0;
        for (int k = 0; k < kTaps; ++k) t.wina[(size_t)k * n + i] = 0.0;
    }
    __syncthreads();

    // roots
    for (int r = tid; r < nj; r += nthr) {
        const int o = r_o[r];
        const double tau = r_tau[r];
        const double mu = lam(t.sintab, n, o) + tau;
        // deflated k with lambda_k <= mu + tie come first
        int lo = -1, hi = n - 1;   // largest k with lambda_k <= mu + tie
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lam(t.sintab, n, mid) <= mu + tie) lo = mid; else hi = mid - 1;
        }
        const int below = (lo >= 0) ? cntD[lo + 1] : 0;
        const int row = r + below;
        t.mu[row] = mu;
        t.a[row] = r_a[r];
        t.origin[row] = o;
        t.tau[row] = tau;
        // a root tying a deflated lambda_k (a double eigenvalue): lo is the largest k with
        // lambda_k <= mu + tie, and the gap is formed in offset form
        if (lo >= 0 && t.z[lo] == 0.0 && fabs(lam_diff(t.sintab, n, lo, o) - tau) <= tie)
            atomicAdd(&t.status[4], 1);
        bool direct = !(mu > 0.0) || !(mu < 4.0);
        if (!direct) {
            const double th = M_PI * o / n;
            double d;
            if (o == 0) {
                d = 2.0 * asin(0.5 * sqrt(tau));
            } else {
                d = 2.0 * asin(fmin(1.0, 0.5 * sqrt(mu))) - th;
                for (int k = 0; k < 4; ++k) {
                    const double F = 4.0 * sin(th + 0.5 * d) * sin(0.5 * d) - tau;
                    d -= F / (2.0 * sin(th + d));
                }
            }
            const double sn = ((o & 1) ? -1.0 : 1.0) * sin(n * d);
            const double a = r_a[r];
            const double kappa = (sn != 0.0) ? a * sqrt(2.0 * n) * maxhz / (2.0 * fabs(sn)) : INFINITY;
            const double psi = th + d;
            const double x = psi / hgrid;
            // the Chebyshev bin (theta_b, theta_b+1) the root lies in, from its angle: a
            // deflated lambda between the root and its origin puts it past the origin's bin
            const int b = (int)floor(0.5 * x);
            const int m0 = (int)ceil(x - 0.5 * w);
            // the aligned taps start at 2b + 1 - w/2: the first real tap must sit 0..2 past it
            const int sh = m0 - (2 * b + 1 - w / 2);
            direct = !(kappa <= kappa_max) || b < 0 || b > n - 2 || sh < 0 || sh > 2;
            // interlacing leaves at most one root per bin; a root on a bin boundary (rounding)
            // that finds its bin taken is summed exactly instead
            if (!direct) direct = atomicCAS(&rowOfBin[b], -1, row) != -1;
            if (!direct) {
                t.rowA[b] = -0.5 * a / sn;
                t.rowB[b] = a * t.z[0] / mu;
                t.m0[b] = m0;
                for (int q = 0; q < w; ++q) t.win[(size_t)b * w + q] = es_window(x - (m0 + q), w, beta);
                for (int k = 0; k < w + 2; ++k) {
                    const int q = k - sh;
                    t.wina[(size_t)k * n + b] =
                        (q >= 0 && q < w) ? t.rowA[b] * es_window(x - (m0 + q), w, beta) : 0.0;
                }
                t.kind[row] = ROW_NUFFT;
                t.ref[row] = b;
            }
        }
        if (direct) {
            t.kind[row] = ROW_DIRECT;
            isdir[row] = 1;
        }
    }
    // deflated directions
    for (int k = tid; k < n; k += nthr) {
        if (t.z[k] != 0.0) continue;
        const double lk = lam(t.sintab, n, k);
        int lo = 0, hi = nj;   // number of roots with mu < lambda_k - tie
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const double mum = lam(t.sintab, n, r_o[mid]) + r_tau[mid];
            if (!(lk <= mum + tie)) lo = mid + 1; else hi = mid;   // complement of the root-side test
        }
        const int row = cntD[k] + lo;
        t.mu[row] = lk;
        t.a[row] = 1.0;
        t.origin[row] = k;
        t.tau[row] = 0.0;
        t.kind[row] = ROW_DEFLATED;
        t.ref[row] = k;
        rowOfK[k] = row;
    }
    __syncthreads();
    // every row must have been assigned exactly once (the two searches are complementary)
    for (int i = tid; i < n; i += nthr)
        if (t.kind[i] < 0) t.status[0] |= 2;
    __syncthreads();
    if (tid == 0) {
        int c = 0;
        for (int i = 0; i < n; ++i)
            if (isdir[i]) {
                if (c < kMaxDirect) t.direct_row[c] = i;
                t.ref[i] = c++;
            }
        sdirect = c;
        t.status[3] = c;   // ndirect
    }
    __syncthreads();
}

// Exact rows a_i z_j / (mu_i - lambda_j), one workgroup per direct slot.
__global__ void k_direct(PlanTables t) {
    const int slot = blockIdx.x;
    const int row = t.direct_row[slot];
    const int n = t.n, o = t.origin[row];
    const double tau = t.tau[row], a = t.a[row];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double zj = t.z[j];
        t.direct[(size_t)slot * n + j] = (zj != 0.0) ? a * zj / (tau - lam_diff(t.sintab, n, j, o)) : 0.0;
    }
}

// The exact rows rounded to FP32 (for plans with FP32 signals).
__global__ void k_direct32(const double *__restrict__ d, float *__restrict__ d32, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        d32[i] = (float)d[i];
}

// Window transform 1 / phi_hat(l h), h = pi / 2n, by Gauss-Legendre quadrature
// (nodes from Newton's method on the Legendre recurrence, recomputed by every
// workgroup; each workgroup then covers its own range of frequencies l).
__global__ void k_deconv(PlanTables t) {
    __shared__ double xq[kQuad], wq[kQuad];
    const int w = t.width;
    const double beta = 2.30 * w;
    for (int k = threadIdx.x; k < kQuad; k += blockDim.x) {
        double x = cos(M_PI * (k + 0.75) / (kQuad + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int l = 2; l <= kQuad; ++l) {
                const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            dp = kQuad * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xq[k] = x;
        wq[k] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    __syncthreads();
    const int n = t.n;
    const double h = M_PI / (2.0 * n);
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n; l += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < kQuad; ++q) {
            const double u = 0.5 * w * xq[q];
            s += wq[q] * es_window(u, w, beta) * cos(l * h * u);
        }
        t.deconv[l] = 1.0 / (0.5 * w * s);
    }
}

// The adjoint's spreading in gather form, tabulated per grid point.  Grid point P
// collects the bins whose aligned window reaches it; the odd extension of the grid
// folds the points -P (for P <= w/2) and 4n - P (for P >= 2n - w/2) back onto P with
// a minus sign.  Every such bin lies in the kReach bins from blo(P) on, so one table
// row per tap slot k holds the combined weight of bin blo(P) + k (zero past the last
// bin); a fold bin outside that window would be a construction error (status bit 4).
__global__ void k_spread(PlanTables t) {
    const int n = t.n, w = t.width, hw = w / 2;
    auto blo_of = [&](int Q) {
        const int b = ((Q - hw - 3) >> 1) + 1;   // bins with 0 <= Q - (2b + 1 - hw) < w + 2
        return b < 0 ? 0 : b;
    };
    for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < 2 * n; P += gridDim.x * blockDim.x) {
        double c[kReach];
        for (int k = 0; k < kReach; ++k) c[k] = 0.0;
        const int base = blo_of(P);
        auto add = [&](int Q, double sign) {
            const int blo = blo_of(Q);
            int bhi = (Q - 1 + hw) >> 1;
            if (bhi > n - 2) bhi = n - 2;
            for (int b = blo; b <= bhi; ++b) {
                const int k = b - base;
                const int tap = Q - 2 * b - 1 + hw;
                if (k < 0 || k >= kReach || tap < 0 || tap >= kTaps) {
                    atomicOr(&t.status[0], 4);
                    continue;
                }
                c[k] += sign * t.wina[(size_t)tap * n + b];
            }
        };
        if (P > 0) {
            add(P, 1.0);
            if (P <= hw) add(-P, -1.0);
            if (P >= 2 * n - hw) add(4 * n - P, -1.0);
        }
        for (int k = 0; k < kReach; ++k) t.wspr[(size_t)k * 2 * n + P] = c[k];
    }
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Scratch of the rank-one set-up, carved from the plan's table allocation.
struct PlanScratch {
    double *v_dev, *misc, *r_tau, *r_a;
    int32_t *J, *r_o;
};

// Every table of the plan in one device allocation, the twiddle and sine tables filled.
dctplus_status plan_alloc(dctplus_plan_s *p, PlanScratch &sc, hipStream_t s) {
    const int n = (int)p->n;
    const int w = p->width;
    PlanTables &t = p->t;
    memset(&t, 0, sizeof(t));
    t.n = n;
    t.logn = p->logn;
    t.rho = p->rho;
    t.width = w;

    // one allocation for every table (sizes in bytes)
    struct Item { void **ptr; size_t bytes; };
    double *v_dev = nullptr, *misc = nullptr, *r_tau = nullptr, *r_a = nullptr;
    int32_t *J = nullptr, *r_o = nullptr, *rowOfBin = nullptr, *rowOfK = nullptr;
    const size_t nd = sizeof(double) * n, ni = sizeof(int32_t) * n;
    std::vector<Item> items = {
        {(void **)&t.z, nd}, {(void **)&t.zraw, nd}, {(void **)&t.mu, nd}, {(void **)&t.a, nd}, {(void **)&t.origin, ni},
        {(void **)&t.tau, nd}, {(void **)&t.kind, ni}, {(void **)&t.ref, ni}, {(void **)&t.hz, nd},
        {(void **)&t.deconv, nd}, {(void **)&t.rowA, nd}, {(void **)&t.rowB, nd}, {(void **)&t.m0, ni},
        {(void **)&t.win, nd * w}, {(void **)&t.wina, nd * kTaps}, {(void **)&t.wspr, nd * 2 * kReach}, {(void **)&t.direct_row, sizeof(int32_t) * kMaxDirect},
        {(void **)&t.tw64, sizeof(cplx<double>) * 4 * n}, {(void **)&t.tw32, sizeof(cplx<float>) * 4 * n},
        {(void **)&t.sintab, sizeof(double) * (2 * n + 1)}, {(void **)&t.status, sizeof(int32_t) * 8},
        {(void **)&rowOfBin, ni}, {(void **)&rowOfK, ni},
        {(void **)&v_dev, nd}, {(void **)&misc, sizeof(double) * 4}, {(void **)&J, ni},
        {(void **)&r_o, ni}, {(void **)&r_tau, nd}, {(void **)&r_a, nd},
    };
    size_t total = 0;
    for (auto &it : items) total += align_up(it.bytes);
    hipError_t e = hipMalloc(&p->dev_mem, total);
    if (e != hipSuccess) {
        p->dev_mem = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc(%zu) for plan tables failed", total);
    }
    p->dev_bytes = total;
    {
        char *base = (char *)p->dev_mem;
        for (auto &it : items) {
            *it.ptr = base;
            base += align_up(it.bytes);
        }
    }
    t.rowOfBin = rowOfBin;
    t.rowOfK = rowOfK;
    if ((e = hipMemsetAsync(t.status, 0, sizeof(int32_t) * 8, s)) != hipSuccess) return hip_fail(e, "memset");
    hipLaunchKernelGGL(k_tables, dim3((4 * n + 255) / 256), dim3(256), 0, s, t);
    sc = PlanScratch{v_dev, misc, r_tau, r_a, J, r_o};
    return DCTPLUS_OK;
}

dctplus_status plan_alloc_tables(dctplus_plan_s *p, hipStream_t s) {
    PlanScratch sc;
    return plan_alloc(p, sc, s);
}

dctplus_status plan_build(dctplus_plan_s *p, const double *v_host, hipStream_t s) {
    const int n = (int)p->n;
    PlanTables &t = p->t;
    PlanScratch sc;
    dctplus_status ast = plan_alloc(p, sc, s);
    if (ast != DCTPLUS_OK) return ast;
    double *v_dev = sc.v_dev, *misc = sc.misc, *r_tau = sc.r_tau, *r_a = sc.r_a;
    int32_t *J = sc.J, *r_o = sc.r_o, *rowOfBin = t.rowOfBin, *rowOfK = t.rowOfK;
    const size_t nd = sizeof(double) * n;
    hipError_t e;
    if ((e = hipMemcpyAsync(v_dev, v_host, nd, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "copy v");

    const size_t lds_z = sizeof(cplx<double>) * (n / 2) > sizeof(int) * kPlanThreads
                             ? sizeof(cplx<double>) * (n / 2)
                             : sizeof(int) * kPlanThreads;
    hipLaunchKernelGGL(k_z, dim3(1), dim3(kPlanThreads), lds_z, s, t, (const double *)v_dev, p->defl_tol, J, misc);
    hipLaunchKernelGGL(k_roots, dim3((n + 3) / 4), dim3(256), 0, s, t, (const int32_t *)J, (const double *)misc,
                       r_o, r_tau, r_a);
    const size_t lds_rows = sizeof(int) * (2 * n + 1);
    hipLaunchKernelGGL(k_rows, dim3(1), dim3(kPlanThreads), lds_rows, s, t, (const int32_t *)J,
                       (const double *)misc, (const int32_t *)r_o, (const double *)r_tau, (const double *)r_a,
                       p->direct_kappa, rowOfBin, rowOfK);
    hipLaunchKernelGGL(k_deconv, dim3((n + 255) / 256), dim3(256), 0, s, t);
    hipLaunchKernelGGL(k_spread, dim3((2 * n + 255) / 256), dim3(256), 0, s, t);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "plan kernels");

    int32_t st[8];
    if ((e = hipMemcpyAsync(st, t.status, sizeof(st), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "status copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "plan synchronize");
    if (st[0] & 1) return fail(DCTPLUS_ENOCONV, "secular solver did not converge");
    if (st[0] & 2) return fail(DCTPLUS_EDEVICE, "internal error: eigenvalue ordering is not a permutation");
    if (st[0] & 4) return fail(DCTPLUS_EDEVICE, "internal error: spreading table out of its window");
    t.nj = st[1];
    t.ndefl = st[2];
    t.ndirect = st[3];
    t.ntie = st[4];
    const bool need_fast = (p->route == DCTPLUS_ROUTE_FAST);
    if (need_fast && t.ndirect > kMaxDirect)
        return fail(DCTPLUS_EUNSUPPORTED, "%d ill-conditioned rows exceed the FAST route limit %d", t.ndirect,
                    kMaxDirect);
    if (t.ndirect > 0 && t.ndirect <= kMaxDirect) {
        if ((e = hipMalloc(&t.direct, sizeof(double) * (size_t)t.ndirect * n)) != hipSuccess) {
            t.direct = nullptr;
            (void)hipGetLastError();
            return fail(DCTPLUS_ENOMEM, "hipMalloc for %d direct rows failed", t.ndirect);
        }
        hipLaunchKernelGGL(k_direct, dim3(t.ndirect), dim3(256), 0, s, t);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "direct rows");
        if (p->dtype != DCTPLUS_F64) {
            const int64_t count = (int64_t)t.ndirect * n;
            if ((e = hipMalloc(&t.direct32, sizeof(float) * (size_t)count)) != hipSuccess) {
                t.direct32 = nullptr;
                (void)hipGetLastError();
                return fail(DCTPLUS_ENOMEM, "hipMalloc for %d FP32 direct rows failed", t.ndirect);
            }
            const int64_t blocks = (count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096;
            hipLaunchKernelGGL(k_direct32, dim3((unsigned)blocks), dim3(256), 0, s, t.direct, t.direct32, count);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "FP32 direct rows");
        }
    }
    if ((p->route == DCTPLUS_ROUTE_DENSE || p->route == DCTPLUS_ROUTE_GFT) && !p->defer_dense) {
        dctplus_status ds = dense_build(p, s);
        if (ds != DCTPLUS_OK) return ds;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "plan synchronize");
    return DCTPLUS_OK;
}

}  // namespace dctplus
