// Gradient of a loss l(y), y = X^T x, with respect to x, rho and v.
//
// First-order perturbation of L x_i = mu_i x_i gives
//   dx_i = sum_{k != i} x_k (x_k^T dL x_i) / (mu_i - mu_k),
//   dL   = drho v v^T + rho (dv v^T + v dv^T).
// With G = sum_b gy_b y_b^T (n x n), A_ik = G_ik / (mu_i - mu_k) (A_ii = 0)
// and w = X^T v (w_i = a_i / rho for secular rows by Lemma 4.2 and the
// secular equation; w_k = u_k^T v for deflated rows):
//   dl/dx   = X gy                       (the adjoint transform)
//   dl/drho = w^T A w
//   dl/dv   = rho X (A + A^T) w
// G is a batch reduction (K = batch) on MFMA with split-K partials summed in
// FP64 in a fixed order (deterministic); the mu gaps and the O(n^2) tail
// are FP64.
#include "fft.h"

namespace dctplus {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int GT = 128;     // output tile (i and k)
constexpr int GK = 32;      // batch rows per LDS stage
constexpr int GP = GT + 4;  // LDS row stride (floats)

// partial[split][i][k] = sum over this split's rows b of gy[b][i] * y[b][k].
// 128 x 128 tile per workgroup, 64 x 64 per wave (4 x 4 MFMA 16x16x4 tiles);
// the next stage of rows is loaded into registers while the current one is
// multiplied out of LDS.
__global__ void __launch_bounds__(256) k_gram(const float *__restrict__ gy, const float *__restrict__ y,
                                              float *__restrict__ partial, int64_t batch, int n, int64_t rows_per) {
    __shared__ float As[GK][GP];   // gy rows [b][i]
    __shared__ float Bs[GK][GP];   // y rows  [b][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int i0 = blockIdx.x * GT, k0 = blockIdx.y * GT, split = blockIdx.z;
    const int64_t b0 = (int64_t)split * rows_per;
    int64_t b1 = b0 + rows_per;
    if (b1 > batch) b1 = batch;
    const int wi = (wave >> 1) * 64, wk = (wave & 1) * 64;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    // stage loader: 32 rows x 128 columns of each operand, 16 floats per thread and operand
    // thread t owns column c = t % 128 of rows t / 128 + 2u, u = 0 .. 15
    float ra[16], rb[16];
    const int c = tid & 127, r0 = tid >> 7;
    const bool ci = i0 + c < n, ck = k0 + c < n;
    const int64_t step = 2 * (int64_t)n;
    auto fetch = [&](int64_t bb) {
        const float *pa = gy + (bb + r0) * n + i0 + c;
        const float *pb = y + (bb + r0) * n + k0 + c;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const bool rin = bb + r0 + 2 * u < b1;
            ra[u] = (rin && ci) ? pa[u * step] : 0.0f;
            rb[u] = (rin && ck) ? pb[u * step] : 0.0f;
        }
    };
    fetch(b0);
    for (int64_t bb = b0; bb < b1; bb += GK) {
        __syncthreads();                            // the previous stage is consumed
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            As[r0 + 2 * u][c] = ra[u];
            Bs[r0 + 2 * u][c] = rb[u];
        }
        __syncthreads();
        if (bb + GK < b1) fetch(bb + GK);           // in flight while this stage is multiplied
#pragma unroll
        for (int s = 0; s < GK / 4; ++s) {
            float av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[4 * s + lq][wi + 16 * a + l16];   // A[i][b] = gy[b][i]
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[4 * s + lq][wk + 16 * b + l16];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    float *out = partial + (size_t)split * n * n;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + 16 * a + 4 * lq + v, k = k0 + wk + 16 * b + l16;
                if (i < n && k < n) out[(size_t)i * n + k] = acc[a][b][v];
            }
}

// The same partials for split-BF16 plans: each 32-row stage is one K step of
// v_mfma_f32_16x16x32_bf16; both operands are split into three BF16 pieces per
// fragment (hardware round-to-nearest conversions) and the six cross products of
// order >= 2^-16 accumulate in FP32.  A lane's fragment is eight consecutive batch
// rows of one column (rows 8 g .. 8 g + 7), read as single floats; the row stride of
// 130 floats puts the four lane groups of a read on distinct banks.
typedef __bf16 gbf8 __attribute__((ext_vector_type(8)));
typedef __bf16 gbf2 __attribute__((ext_vector_type(2)));
typedef float gf2 __attribute__((ext_vector_type(2)));
constexpr int GPS = GT + 2;

__device__ __forceinline__ void split_frag(const float *col, int stride, gbf8 &h, gbf8 &m, gbf8 &l) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const gf2 x = {col[e * stride], col[(e + 1) * stride]};
        const gbf2 xh = __builtin_convertvector(x, gbf2);
        const gf2 r = x - __builtin_convertvector(xh, gf2);
        const gbf2 xm = __builtin_convertvector(r, gbf2);
        const gbf2 xl = __builtin_convertvector(r - __builtin_convertvector(xm, gf2), gbf2);
        h[e] = xh[0];
        h[e + 1] = xh[1];
        m[e] = xm[0];
        m[e + 1] = xm[1];
        l[e] = xl[0];
        l[e + 1] = xl[1];
    }
}

__global__ void __launch_bounds__(256) k_gram_split(const float *__restrict__ gy, const float *__restrict__ y,
                                                    float *__restrict__ partial, int64_t batch, int n,
                                                    int64_t rows_per) {
    __shared__ float As[GK][GPS];   // gy rows [b][i]
    __shared__ float Bs[GK][GPS];   // y rows  [b][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int i0 = blockIdx.x * GT, k0 = blockIdx.y * GT, split = blockIdx.z;
    const int64_t b0 = (int64_t)split * rows_per;
    int64_t b1 = b0 + rows_per;
    if (b1 > batch) b1 = batch;
    const int wi = (wave >> 1) * 64, wk = (wave & 1) * 64;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    // stage loader as in k_gram: thread t owns column c = t % 128 of rows t / 128 + 2u
    float ra[16], rb[16];
    const int c = tid & 127, r0 = tid >> 7;
    const bool ci = i0 + c < n, ck = k0 + c < n;
    const int64_t step = 2 * (int64_t)n;
    auto fetch = [&](int64_t bb) {
        const float *pa = gy + (bb + r0) * n + i0 + c;
        const float *pb = y + (bb + r0) * n + k0 + c;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const bool rin = bb + r0 + 2 * u < b1;
            ra[u] = (rin && ci) ? pa[u * step] : 0.0f;
            rb[u] = (rin && ck) ? pb[u * step] : 0.0f;
        }
    };
    fetch(b0);
    for (int64_t bb = b0; bb < b1; bb += GK) {
        __syncthreads();                            // the previous stage is consumed
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            As[r0 + 2 * u][c] = ra[u];
            Bs[r0 + 2 * u][c] = rb[u];
        }
        __syncthreads();
        if (bb + GK < b1) fetch(bb + GK);           // in flight while this stage is multiplied
        gbf8 ah[4], am[4], al[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) split_frag(&As[8 * g][wi + 16 * a + l16], GPS, ah[a], am[a], al[a]);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gbf8 bh, bm, bl;
            split_frag(&Bs[8 * g][wk + 16 * b + l16], GPS, bh, bm, bl);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[a], bm, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[a], bh, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bm, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh, acc[a][b], 0, 0, 0);
            }
        }
    }
    float *out = partial + (size_t)split * n * n;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + 16 * a + 4 * g + v, k = k0 + wk + 16 * b + l16;
                if (i < n && k < n) out[(size_t)i * n + k] = acc[a][b][v];
            }
}

__device__ __forceinline__ double wcoef(const PlanTables &t, int i) {
    // w_i = x_i^T v
    if (t.kind[i] == ROW_DEFLATED) return t.zraw[t.origin[i]];
    return t.a[i] / t.rho;
}

// G = sum of the split-K partials, in FP64 and in a fixed order; written as
// G (row-major) and G^T so that both are read along rows below.
__global__ void __launch_bounds__(256) k_gram_sum(const float *__restrict__ partial, int nsplit, int n,
                                                  double *__restrict__ G, double *__restrict__ GT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    if (e >= nn) return;
    double g = 0.0;
    // unrolled so that the loads of eight partials are in flight together; the additions
    // keep their order
#pragma unroll 8
    for (int sp = 0; sp < nsplit; ++sp) g += (double)partial[(size_t)sp * nn + e];
    const int i = (int)(e / n), k = (int)(e % n);
    G[e] = g;
    GT[(size_t)k * n + i] = g;
}

// r_i = sum_k (G_ik - G_ki) / (mu_i - mu_k) w_k ,  q_i = w_i sum_k G_ik w_k / (mu_i - mu_k);
// one wave per i, lanes over k.  Every eigenvalue is stored as its origin pole and offset,
// mu = lambda_o + tau, so the gap is (lambda_oi - lambda_ok) + (tau_i - tau_k) with the pole
// difference in product form: a root hugging a pole keeps the gap's relative accuracy.
__global__ void __launch_bounds__(256) k_grad_vec(PlanTables t, const double *__restrict__ G,
                                                  const double *__restrict__ GT, double *__restrict__ rvec,
                                                  double *__restrict__ qvec) {
    const int n = t.n;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;   // the whole wave leaves
    const int oi = t.origin[i];
    const double taui = t.tau[i];
    double r = 0.0, q = 0.0;
    for (int k = lane; k < n; k += 64) {
        if (k == i) continue;
        const double gik = G[(size_t)i * n + k], gki = GT[(size_t)i * n + k];
        const double inv = 1.0 / (lam_diff(t.sintab, n, oi, t.origin[k]) + (taui - t.tau[k]));
        const double wk = wcoef(t, k);
        r += (gik - gki) * inv * wk;
        q += gik * inv * wk;
    }
    r = wave_sum(r);
    q = wave_sum(q);
    if (lane == 0) {
        rvec[i] = r;
        qvec[i] = q * wcoef(t, i);
    }
}

// dl/drho = sum_i q_i ; dl/dv = rho X r  (FP64: Cauchy transpose, then DCT-III)
// s_j = sum_i M_ij r_i (M = diag(a) C(mu, lambda) diag(z), deflated rows e_o);
// one wave per j, lanes over i.
__global__ void __launch_bounds__(256) k_grad_s(PlanTables t, const double *__restrict__ rvec,
                                                double *__restrict__ svec) {
    const int n = t.n;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= n) return;   // the whole wave leaves
    const double zj = t.z[j];
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
        const int kind = t.kind[i], o = t.origin[i];
        if (kind == ROW_DEFLATED) {
            if (o == j) s += rvec[i];
        } else if (zj != 0.0) {
            const double sj = (j - o) >= 0 ? t.sintab[j - o] : -t.sintab[o - j];
            const double d = 4.0 * sj * t.sintab[j + o];
            s += t.a[i] * zj / (t.tau[i] - d) * rvec[i];
        }
    }
    s = wave_sum(s);
    if (lane == 0) svec[j] = s;
}

// dl/drho = sum_i q_i; dl/dv = rho U s (an inverse DCT of s).  One workgroup.
__global__ void __launch_bounds__(256) k_grad_final(PlanTables t, const double *__restrict__ svec,
                                                    const double *__restrict__ qvec, double *__restrict__ grho,
                                                    double *__restrict__ gv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = t.n, logn = t.logn, tid = threadIdx.x, nthr = blockDim.x;
    double *sdv = reinterpret_cast<double *>(smem);
    cplx<double> *Z = reinterpret_cast<cplx<double> *>(sdv + n);
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = tid; i < n; i += nthr) acc += qvec[i];
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    for (int j = tid; j < n; j += nthr) sdv[j] = svec[j];
    __syncthreads();
    if (tid == 0 && grho) {
        double s = 0.0;
        for (int w = 0; w < nthr / 64; ++w) s += red[w];
        *grho = s;
    }
    if (!gv) return;
    const int logT = logn + 2;
    for (int k = tid; k < n / 2; k += nthr) {
        auto get = [&](int kk) -> double { return sdv[kk]; };
        Z[fft_slot<double>(k)] = dct3_pack<double>(get, k, logn, t.tw64, logT);
    }
    __syncthreads();
    const RadixPlan rp = radix_plan(logn - 1, 1, nthr);
    fft_dif(Z, 1, n / 2, logn - 1, t.tw64, logT, rp);
    for (int j = tid; j < n; j += nthr) gv[j] = t.rho * dct3_sample(Z, j, logn, rp);
}

// Gram split count: ~512+ workgroups over the 128 x 128 output tiles, partials within
// `cap` bytes (the workspace), at least one split.
static int gram_splits(int n, size_t cap) {
    const int nt = (n + GT - 1) / GT;
    const int tiles = nt * nt;
    int nsplit = 512 / tiles;
    if (nsplit < 1) nsplit = 1;
    if (nsplit > 128) nsplit = 128;
    while (nsplit > 1 && (size_t)nsplit * n * n * sizeof(float) > cap) nsplit >>= 1;
    return nsplit;
}

static size_t grad_tail_bytes(int n) {
    return 2 * sizeof(double) * (size_t)n * n + 3 * sizeof(double) * n;   // G, G^T, r, q, s
}

// Checks shared by both gradient entry points (before any launch: no output on error).
static dctplus_status grad_check(const dctplus_plan_s *p, const double *grho, const double *gv) {
    if ((grho || gv) && p->n > 4096)
        return fail(DCTPLUS_EUNSUPPORTED, "gradient with respect to rho and v supports n <= 4096");
    // a double eigenvalue (a secular root on a deflated lambda_k) has no unique eigenbasis:
    // the basis, and the row order, are not differentiable in (rho, v) there
    if ((grho || gv) && p->t.ntie > 0)
        return fail(DCTPLUS_EDEGENERATE, "the plan has %d double eigenvalue(s): d/drho and d/dv are undefined",
                    p->t.ntie);
    return DCTPLUS_OK;
}

// dl/drho and dl/dv with the Gram partials, G, G^T and the vectors in `work`
// (gram_splits(n) * 4 n^2 + grad_tail_bytes(n) bytes, nothing needs to start at zero:
// every kernel writes its whole output).
static dctplus_status grad_launch(dctplus_plan_s *p, const float *y, const float *gy, int64_t batch, double *grho,
                                  double *gv, void *work, int nsplit, hipStream_t s) {
    const int n = (int)p->n;
    const int nt = (n + GT - 1) / GT;
    int64_t rows_per = (batch + nsplit - 1) / nsplit;
    rows_per = (rows_per + GK - 1) / GK * GK;
    if (rows_per < GK) rows_per = GK;
    const size_t pbytes = (size_t)nsplit * n * n * sizeof(float);
    float *partial = (float *)work;
    double *G = (double *)((char *)work + pbytes);
    double *GT = G + (size_t)n * n;
    double *rvec = GT + (size_t)n * n;
    double *qvec = rvec + n;
    double *svec = qvec + n;
    if (p->dtype == DCTPLUS_F32_SPLIT)
        hipLaunchKernelGGL(k_gram_split, dim3(nt, nt, nsplit), dim3(256), 0, s, gy, y, partial, batch, n, rows_per);
    else
        hipLaunchKernelGGL(k_gram, dim3(nt, nt, nsplit), dim3(256), 0, s, gy, y, partial, batch, n, rows_per);
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256), 0, s,
                       (const float *)partial, nsplit, n, G, GT);
    hipLaunchKernelGGL(k_grad_vec, dim3((n + 3) / 4), dim3(256), 0, s, p->t, (const double *)G, (const double *)GT,
                       rvec, qvec);
    const size_t lds = sizeof(double) * n + sizeof(cplx<double>) * (n / 2);
    hipLaunchKernelGGL(k_grad_s, dim3((n + 3) / 4), dim3(256), 0, s, p->t, (const double *)rvec, svec);
    hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), lds, s, p->t, (const double *)svec, (const double *)qvec,
                       grho, gv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gradient launch");
    return DCTPLUS_OK;
}

}  // namespace

dctplus_status grad_apply(dctplus_plan_s *p, const float *y, const float *gy, int64_t batch, float *gx,
                          double *grho, double *gv, hipStream_t s) {
    const int n = (int)p->n;
    dctplus_status st = grad_check(p, grho, gv);
    if (st != DCTPLUS_OK) return st;
    if (gx) {
        st = use_fast(p, batch) ? fast_apply(p, gy, gx, batch, true, s)
                                              : dense_apply(p, gy, gx, batch, true, s);
        if (st != DCTPLUS_OK) return st;
    }
    if (!grho && !gv) return DCTPLUS_OK;
    const int nsplit = gram_splits(n, (size_t)256 << 20);
    // the stream's workspace may already hold a FAST/DENSE scratch of the gx call above,
    // which uses it earlier in the same stream's order
    void *work = nullptr;
    st = stream_work(p, s, (size_t)nsplit * n * n * sizeof(float) + grad_tail_bytes(n), &work);
    if (st != DCTPLUS_OK) return st;
    return grad_launch(p, y, gy, batch, grho, gv, work, nsplit, s);
}

dctplus_status grad_apply_static(dctplus_plan_s *p, const float *y, const float *gy, int64_t batch, float *gx,
                                 double *grho, double *gv, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int n = (int)p->n;
    dctplus_status st = grad_check(p, grho, gv);
    if (st != DCTPLUS_OK) return st;
    const bool need = grho || gv;
    const size_t tail = grad_tail_bytes(n);
    if (need && tail + sizeof(float) * (size_t)n * n > scratch_bytes)
        return fail(DCTPLUS_EUNSUPPORTED,
                    "n = %d needs %zu bytes of scratch for dl/drho and dl/dv; the static scratch holds %zu "
                    "(n <= %d)", n, tail + sizeof(float) * (size_t)n * n, scratch_bytes, kStaticGradMaxN);
    if (gx && !route_alloc_free(p))
        return fail(DCTPLUS_EUNSUPPORTED, "dl/dx on this plan's route needs the plan workspace or a library "
                                          "GEMM; use dctplus_grad");
    if (gx) {
        st = use_fast(p, batch) ? fast_apply(p, gy, gx, batch, true, s)
                                              : dense_apply(p, gy, gx, batch, true, s);
        if (st != DCTPLUS_OK) return st;
    }
    if (!need) return DCTPLUS_OK;
    const int nsplit = gram_splits(n, scratch_bytes - tail);
    return grad_launch(p, y, gy, batch, grho, gv, scratch, nsplit, s);
}

}  // namespace dctplus
