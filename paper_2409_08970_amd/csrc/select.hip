// Batched progressive transform selection with pruning (Thm 3.1 shared DCT,
// Thm 3.4 pruning; the block-wise selection experiment of Sec. 5).
//
// A selection plan holds nblocks independent path-graph blocks of n_b
// vertices (n_b in {4, 8, 16, 32, 64}) with S <= 64 signals each and K <= 16
// candidate rank-one updates per block (a self-loop or an added edge).
//
// dctplus_select_plan computes the Cauchy factor
//     C~_r = diag(a_r) C(mu_r, lambda) diag(z_r)        (Thm 3.1)
// of every candidate on the GPU in FP64 (one wave per candidate: z = U^T v in
// closed form, deflation, safeguarded Newton on the secular equation in offset
// form, the same row order and tie rule as the single-transform plan) and
// stores it in FP32, for n_b >= 16 already in the lane order of the MFMA
// operand so that the selection kernel reads it with coalesced 16-byte loads.
//
// dctplus_select is one persistent launch.  Workgroups take blocks from an
// atomic work queue (largest n_b first).  Per block: the S signals go to LDS;
// each signal's path-Laplacian quadratic form decides whether it is pruned
// (x^T L_path x <= tau ||x||^2); one DCT-II of all signals (a product with the
// DCT matrix on MFMA, in LDS) is shared by every candidate (the progressive
// property); each candidate's
// coefficients C~_r s_d follow on MFMA (pruned signals keep the upper-left
// c_p x c_p block of C~_r, Thm 3.4); the L1 norm of the coefficients is the
// candidate's cost; the lowest cost wins (ties: lowest index) and the
// winner's coefficients are written out.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "dct64.h"
#include "fft.h"

struct dctplus_select_s {
    int64_t nblocks = 0;
    int32_t K = 0, S = 0, device = 0;
    int64_t total_x = 0;              // floats of x and y_best
    std::vector<int32_t> n_host;      // block sizes
    std::vector<int64_t> xoff_host, moff_host;
    int32_t *n_dev = nullptr;         // [nblocks]
    int64_t *xoff_dev = nullptr;      // [nblocks] first float of block b in x
    int64_t *moff_dev = nullptr;      // [nblocks] first float of block b's K factors
    int32_t *order_dev = nullptr;     // [nblocks] processing order
    int32_t *counter_dev = nullptr;   // work-queue head
    int32_t *status_dev = nullptr;
    float *M = nullptr;               // all factors
    float *dctm = nullptr;            // orthonormal DCT-II matrices of the five sizes (factor layout)
    dctplus::d64::GroupConst *kc = nullptr;   // lane constants of the register DCT-II (n = 64)
    int32_t wgs_per_cu = 4;           // persistent workgroups per CU (set by dctplus_select_tune)
};

namespace dctplus {

namespace {

constexpr int kSelThreads = 256;
constexpr int kSelTuneCands = 4;      // persistent grid candidates: 1..4 workgroups per CU
constexpr int kSelMaxN = 64;
constexpr int kSelMaxS = 64;
constexpr int kSelMaxK = 16;

// Position of factor entry (i, k) in the stored layout.  n < 16: row-major.
// n >= 16: float4 number l of group (c, s4) holds M[16c + l%16][16 s4 + 4 e + l/16],
// e = 0..3, i.e. lane l's A operands of four consecutive 16x16x4 MFMA steps.
__host__ __device__ __forceinline__ int64_t sel_frag_index(int n, int i, int k) {
    if (n < 16) return (int64_t)i * n + k;
    const int c = i >> 4, l16 = i & 15, s = k >> 2, g = k & 3;
    const int lane = l16 + 16 * g;
    return ((int64_t)((c * (n >> 4) + (s >> 2)) * 64 + lane) << 2) + (s & 3);
}

// start of the n x n DCT matrix of size n (matrices for n = 4, 8, ..., 64 back to back:
// 16 + 64 + ... + (n/2)^2 = (n^2 - 16) / 3 floats before it)
__host__ __device__ __forceinline__ int sel_dct_offset(int n) { return (n * n - 16) / 3; }

// ---------------------------------------------------------------------------
// Batched FP64 candidate plans: one 64-thread workgroup per candidate.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_select_plan(const int32_t *__restrict__ nb, const double *__restrict__ cand,
                                                   const int64_t *__restrict__ moff, int K, float *__restrict__ M,
                                                   int32_t *__restrict__ status) {
    __shared__ double sint[2 * kSelMaxN + 1];   // sin(pi k / 2n)
    __shared__ double z[kSelMaxN];
    __shared__ int J[kSelMaxN];
    __shared__ int r_o[kSelMaxN];
    __shared__ double r_tau[kSelMaxN], r_a[kSelMaxN];
    __shared__ int row_o[kSelMaxN], row_kind[kSelMaxN];
    __shared__ double row_tau[kSelMaxN], row_a[kSelMaxN];
    __shared__ int s_nj;
    const int64_t b = blockIdx.x / K;
    const int r = blockIdx.x % K;
    const int n = nb[b];
    const int t = threadIdx.x;
    const double *cd = cand + ((int64_t)b * K + r) * 4;
    const int kind = (int)cd[0], vi = (int)cd[1], vj = (int)cd[2];
    const double w = cd[3];
    const double rho = (kind == 0) ? w : 2.0 * w;
    for (int k = t; k <= 2 * n; k += 64) sint[k] = sinpi((double)k / (2.0 * n));
    if (t < kSelMaxN) row_kind[t] = -1;
    __syncthreads();
    auto sh = [&](int k) -> double { return k >= 0 ? sint[k] : -sint[-k]; };
    // lambda_j - lambda_o = 4 sin(pi (j - o) / 2n) sin(pi (j + o) / 2n), free of cancellation
    auto lamd = [&](int j, int o) -> double { return 4.0 * sh(j - o) * sh(j + o); };
    auto lam = [&](int k) -> double { return 4.0 * sint[k] * sint[k]; };
    // z = U^T v for v = e_i (self-loop) or (e_i - e_j) / sqrt 2 (edge): DCT-II columns in closed form
    double zz = 0.0;
    if (t < n) {
        const double ck = (t == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
        double zk = ck * cospi((double)t * (2 * vi + 1) / (2.0 * n));
        if (kind == 1) zk = (zk - ck * cospi((double)t * (2 * vj + 1) / (2.0 * n))) * 0.70710678118654752440;
        z[t] = zk;
        zz = zk * zk;
    }
    zz = wave_sum(zz);
    __syncthreads();
    if (t < n && !(fabs(z[t]) > 1e-13 * sqrt(zz))) z[t] = 0.0;    // deflation
    __syncthreads();
    if (t == 0) {
        int c = 0;
        for (int k = 0; k < n; ++k)
            if (z[k] != 0.0) J[c++] = k;
        s_nj = c;
    }
    __syncthreads();
    const int nj = s_nj;
    // F(t) = 1/rho + sum_{j != o} z_j^2 / (d_j - t) and F'(t); the secular function is F(t) - z_o^2 / t
    auto eval = [&](int o, double tt, double &F, double &Fp) {
        F = 1.0 / rho;
        Fp = 0.0;
        for (int q = 0; q < nj; ++q) {
            const int j = J[q];
            if (j == o) continue;
            const double rr = z[j] / (lamd(j, o) - tt);
            F += z[j] * rr;
            Fp += rr * rr;
        }
    };
    if (t < nj) {
        // root t lies between consecutive non-deflated poles (Lemma 4.1), above the last one
        // for rho > 0, below the first for rho < 0; its origin is the nearer pole
        int pa, pb;
        if (rho > 0) {
            pa = J[t];
            pb = (t + 1 < nj) ? J[t + 1] : -1;
        } else {
            pb = J[t];
            pa = (t > 0) ? J[t - 1] : -1;
        }
        int o;
        double lo, hi, F, Fp;
        if (pa >= 0 && pb >= 0) {
            const double gap = lamd(pb, pa);
            eval(pa, 0.5 * gap, F, Fp);
            if (F - z[pa] * z[pa] / (0.5 * gap) >= 0.0) {
                o = pa; lo = 0.0; hi = 0.5 * gap;
            } else {
                o = pb; lo = -0.5 * gap; hi = 0.0;
            }
        } else if (rho > 0) {
            o = pa; lo = 0.0; hi = rho * zz * (1.0 + 1e-12);
        } else {
            o = pb; lo = rho * zz * (1.0 + 1e-12); hi = 0.0;
        }
        const double zo2 = z[o] * z[o];
        double tt = 0.5 * (lo + hi);
        bool conv = false;
        for (int it = 0; it < 200; ++it) {
            eval(o, tt, F, Fp);
            const double f = F - zo2 / tt;
            if (f > 0.0) hi = tt;
            else if (f < 0.0) lo = tt;
            else { conv = true; break; }
            // Newton on h(t) = z_o^2 - t F(t) (no pole at the origin), kept inside the bracket
            double tn = tt - (zo2 - tt * F) / (-F - tt * Fp);
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            if (tn == tt || fabs(tn - tt) <= 4.4408920985006262e-16 * fabs(tn)) { tt = tn; conv = true; break; }
            tt = tn;
        }
        eval(o, tt, F, Fp);
        r_o[t] = o;
        r_tau[t] = tt;
        r_a[t] = 1.0 / sqrt(Fp + zo2 / (tt * tt));
        if (!conv) atomicOr(status, 1);
    }
    __syncthreads();
    // rows in ascending eigenvalue order; a root tying a deflated lambda_k goes after it
    const double tie = 1e-12 * (4.0 + fabs(rho) * zz);
    if (t < nj) {
        const double mu = lam(r_o[t]) + r_tau[t];
        int below = 0;
        for (int k = 0; k < n; ++k)
            if (z[k] == 0.0 && lam(k) <= mu + tie) ++below;
        const int row = t + below;
        row_o[row] = r_o[t];
        row_tau[row] = r_tau[t];
        row_a[row] = r_a[t];
        row_kind[row] = 0;
    }
    if (t < n && z[t] == 0.0) {
        const double lk = lam(t);
        int defl_below = 0, roots_below = 0;
        for (int k = 0; k < t; ++k) defl_below += (z[k] == 0.0);
        for (int q = 0; q < nj; ++q)
            if (!(lk <= lam(r_o[q]) + r_tau[q] + tie)) ++roots_below;
        const int row = defl_below + roots_below;
        row_o[row] = t;
        row_tau[row] = 0.0;
        row_a[row] = 1.0;
        row_kind[row] = 1;
    }
    __syncthreads();
    if (t < n && row_kind[t] < 0) atomicOr(status, 2);    // inconsistent row order: the plan is rejected
    // factor entries: a_i z_k / (mu_i - lambda_k); deflated rows are e_o
    float *Mr = M + moff[b] + (int64_t)r * n * n;
    for (int e = t; e < n * n; e += 64) {
        const int i = e / n, k = e % n;
        double val = 0.0;
        if (row_kind[i] == 1) val = (k == row_o[i]) ? 1.0 : 0.0;
        else if (row_kind[i] == 0 && z[k] != 0.0) val = row_a[i] * z[k] / (row_tau[i] - lamd(k, row_o[i]));
        Mr[sel_frag_index(n, i, k)] = (float)val;
    }
}

// DCT-II matrices A[i][j] = c_i cos(pi i (2j + 1) / 2n) (row i = frequency i, so that
// s_d = A x) for n = 4, 8, 16, 32, 64, stored like the candidate factors.
__global__ void k_select_dctm(float *dctm) {
    for (int n = 4; n <= kSelMaxN; n *= 2) {
        float *D = dctm + sel_dct_offset(n);
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
            const int i = e / n, j = e % n;
            const double ci = (i == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
            D[sel_frag_index(n, i, j)] = (float)(ci * cospi((double)i * (2 * j + 1) / (2.0 * n)));
        }
    }
}

__global__ void k_select_reset(int32_t *counter) {
    if (threadIdx.x == 0) counter[0] = 0;
}

// ---------------------------------------------------------------------------
// Persistent selection kernel
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

struct SelArgs {
    const float *x;
    const int32_t *n;
    const int64_t *xoff, *moff;
    const int32_t *order;
    int32_t *counter;
    const float *M;
    const float *dctm;
    const d64::GroupConst *kc;
    int64_t nblocks;
    int K, S, cp;
    double tau;
    int32_t *best;
    float *cost;
    float *y;
};

struct SelShared {
    float xs[kSelMaxS * (kSelMaxN + 1)];     // signals, then their DCT-II in slot order (row stride n + 1)
    float cost[kSelMaxK];
    int pruned[kSelMaxS];                    // per signal
    int slot_of[kSelMaxS];                   // slot of each signal: pruned signals first
    int sig_of[kSelMaxS];                    // signal of each slot
    int spr[kSelMaxS];                       // pruned flag per slot
    int npr;                                 // number of pruned signals (slots 0 .. npr - 1)
    int next;
    int best;
};

// DCT-II of the block's 64 rows of xs, in place, as one product with the DCT
// matrix.  n >= 16: wave w transforms the 16 signals of tile w on 16x16x4 FP32
// MFMA (each lane reads its samples before any lane of the wave writes, and the
// wave touches only its own rows).  n < 16: thread s < 64 transforms signal s.
template <int N>
__device__ __forceinline__ void sel_dct(SelShared &sh, const float *__restrict__ D, const d64::GroupConst *kc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (N == 64) {
        // radix DCT-II in registers (dct64.h): lane (l16, g) of wave w holds sixteen samples of
        // signal 16 w + l16 and ends with sixteen of its coefficients
        const int l16 = lane & 15, g = lane >> 4;
        const int sig = 16 * wave + l16;
        const float *row = sh.xs + sig * (N + 1);
        float a[16], R[16], X[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) a[m] = row[d64::in_index(g, m)];
        __syncthreads();                         // every signal is read before slots are written
        d64::rdft16(a, R);
        d64::xpose_lane_groups(R);
        const d64::GroupConst kA = kc[2 * g], kB = kc[2 * g + 1];
        d64::group_fwd(R, 0, kA, X);
        if (g < 3) d64::group_fwd(R, 2, kB, X + 8);
        else d64::special_fwd(R, X + 8);
        float *out = sh.xs + sh.slot_of[sig] * (N + 1);
#pragma unroll
        for (int q = 0; q < 16; ++q) out[d64::out_index(g, q)] = X[q];
        (void)D;
    } else if constexpr (N >= 16) {
        constexpr int CT = N / 16, KS = N / 4;
        const int l16 = lane & 15, g = lane >> 4;
        const float4 *D4 = reinterpret_cast<const float4 *>(D);
        float *row = sh.xs + (16 * wave + l16) * (N + 1);
        f4 acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s4 = 0; s4 < KS / 4; ++s4) {
            float4 q[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) q[c] = D4[(c * (KS / 4) + s4) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float bv = row[4 * (4 * s4 + e) + g];
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const float a = e == 0 ? q[c].x : e == 1 ? q[c].y : e == 2 ? q[c].z : q[c].w;
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[c], 0, 0, 0);
                }
            }
        }
        // lane holds coefficients i = 16 c + 4 g + v of its signal; written to its slot
        __syncthreads();                         // every signal is read before slots are written
        float *out = sh.xs + sh.slot_of[16 * wave + l16] * (N + 1);
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[16 * c + 4 * g + v] = acc[c][v];
    } else {
        float sd[N];
        if (threadIdx.x < 64) {
            const float *row = sh.xs + threadIdx.x * (N + 1);
            float xv[N];
#pragma unroll
            for (int j = 0; j < N; ++j) xv[j] = row[j];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int j = 0; j < N; ++j) acc += D[i * N + j] * xv[j];
                sd[i] = acc;
            }
        }
        __syncthreads();                         // every signal is read before slots are written
        if (threadIdx.x < 64) {
            float *out = sh.xs + sh.slot_of[threadIdx.x] * (N + 1);
#pragma unroll
            for (int i = 0; i < N; ++i) out[i] = sd[i];
        }
    }
}

// Cost of one candidate (n >= 16): sum over the block's 64 signal rows of
// |C~_r s_d| on 16x16x4 FP32 MFMA, one wave, the factor held in registers and
// reused for the four signal tiles (rows past the block's signals are zero, so
// all four tiles run unconditionally).  Pruned signals keep the c_p x c_p block.
// Returns this lane's share.
template <int N>
__device__ __forceinline__ float sel_cost_mfma(const SelShared &sh, const float *__restrict__ Mr, int cp) {
    constexpr int CT = N / 16, KS = N / 4;
    const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
    const float4 *M4 = reinterpret_cast<const float4 *>(Mr);
    float a[CT][KS];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int s4 = 0; s4 < KS / 4; ++s4) {
            const float4 q = M4[(c * (KS / 4) + s4) * 64 + lane];
            a[c][4 * s4 + 0] = q.x;
            a[c][4 * s4 + 1] = q.y;
            a[c][4 * s4 + 2] = q.z;
            a[c][4 * s4 + 3] = q.w;
        }
    float l1 = 0.f;
    const int npr = sh.npr;
#pragma unroll 1
    for (int tile = 0; tile < kSelMaxS / 16; ++tile) {
        const int slot = 16 * tile + l16;           // slots hold the pruned signals first
        const bool pr = sh.spr[slot] != 0;
        f4 acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        if (16 * (tile + 1) <= npr && cp == N / 2) {
            // sixteen pruned signals: only the c_p x c_p block (Thm 3.4), output tiles
            // c < c_p / 16 and contraction k < c_p, a quarter of the MFMAs
            constexpr int CTP = CT / 2 > 0 ? CT / 2 : 1;
#pragma unroll
            for (int s = 0; s < KS / 2; ++s) {
                const float bv = sh.xs[slot * (N + 1) + 4 * s + g];
#pragma unroll
                for (int c = 0; c < CTP; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c][s], bv, acc[c], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = 4 * s + g;
                float bv = sh.xs[slot * (N + 1) + k];
                if (pr && k >= cp) bv = 0.f;
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c][s], bv, acc[c], 0, 0, 0);
            }
        }
        // this lane holds outputs i = 16 c + 4 g + v of signal sig
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * c + 4 * g + v;
                l1 += (pr && i >= cp) ? 0.f : fabsf(acc[c][v]);
            }
    }
    return l1;
}

// One candidate's coefficients y_sig = C~_r s_d(sig) on 16x16x4 FP32 MFMA (n >= 16):
// wave w computes output rows 16 c .. 16 c + 15, c = w mod (n/16), for n/16 of the
// four signal tiles, so the four waves together read the factor once and hold
// only n/16 accumulators each.  Pruned signals keep the c_p x c_p block.  Returns
// this lane's share of sum |y|; writes y when yout != nullptr.
template <int N>
__device__ __forceinline__ float sel_tiles(const SelShared &sh, const float *__restrict__ Mr, int cp, int ntile,
                                           int S, float *__restrict__ yout) {
    constexpr int CT = N / 16, KS = N / 4, G = 4 / CT;   // G waves share an output tile
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int c = wave % CT, grp = wave / CT;
    const float4 *M4 = reinterpret_cast<const float4 *>(Mr);
    bool pr[CT];
    f4 acc[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        pr[j] = sh.spr[16 * (grp + j * G) + l16] != 0;
        acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int s4 = 0; s4 < KS / 4; ++s4) {
        const float4 q = M4[(c * (KS / 4) + s4) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * (4 * s4 + e) + g;
            const float a = e == 0 ? q.x : e == 1 ? q.y : e == 2 ? q.z : q.w;
#pragma unroll
            for (int j = 0; j < CT; ++j) {
                // rows past the block's signals are zero: no test needed here
                const int t = grp + j * G;
                float bv = sh.xs[(16 * t + l16) * (N + 1) + k];
                if (pr[j] && k >= cp) bv = 0.f;
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[j], 0, 0, 0);
            }
        }
    }
    float l1 = 0.f;
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        const int t = grp + j * G;
        const int sig = sh.sig_of[16 * t + l16];    // the slot's signal (rows past S are zero)
        float v4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * c + 4 * g + v;
            v4[v] = (pr[j] && i >= cp) ? 0.f : acc[j][v];
            l1 += fabsf(v4[v]);
        }
        if (yout && sig < S)
            *reinterpret_cast<float4 *>(yout + (int64_t)sig * N + 16 * c + 4 * g) =
                make_float4(v4[0], v4[1], v4[2], v4[3]);
    }
    return l1;
}

// The same for n in {4, 8} on the vector ALU: one signal per lane.
template <int N>
__device__ __forceinline__ float sel_product_valu(const SelShared &sh, const float *__restrict__ Mr, int cp, int S,
                                                  float *__restrict__ yout) {
    const int slot = threadIdx.x & 63, sig = sh.sig_of[slot];
    const bool pr = sh.spr[slot] != 0;
    float sd[N];
#pragma unroll
    for (int k = 0; k < N; ++k) sd[k] = (pr && k >= cp) ? 0.f : sh.xs[slot * (N + 1) + k];
    float l1 = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < N; ++k) acc += Mr[i * N + k] * sd[k];
        if (pr && i >= cp) acc = 0.f;
        l1 += fabsf(acc);
        if (yout && sig < S) yout[(int64_t)sig * N + i] = acc;
    }
    return l1;
}

template <int N>
__device__ __forceinline__ void sel_block(SelShared &sh, const SelArgs &A, int64_t b) {
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
    const int K = A.K, S = A.S;
    const float *xb = A.x + A.xoff[b];
    for (int e = tid; e < kSelMaxS * N; e += nthr) {
        const int s = e / N, j = e % N;
        sh.xs[s * (N + 1) + j] = (s < S) ? xb[e] : 0.f;
    }
    __syncthreads();
    if (tid < kSelMaxS) {
        // pruning test on the path-Laplacian quadratic form (Thm 3.4)
        // (FP64 sums of the FP32 samples: the decision does not depend on the summation order)
        const float *row = sh.xs + tid * (N + 1);
        double q = 0.0, e2 = (double)row[0] * row[0];
#pragma unroll
        for (int j = 1; j < N; ++j) {
            const double d = (double)row[j] - (double)row[j - 1];
            q += d * d;
            e2 += (double)row[j] * row[j];
        }
        const int pr = (q <= A.tau * e2) ? 1 : 0;
        sh.pruned[tid] = pr;
        // slots: pruned signals first, each group in signal order (wave 0 holds the 64 signals)
        const uint64_t mask = __ballot(pr);
        const int np = __popcll(mask);
        const int before = __popcll(mask & ((uint64_t(1) << tid) - 1));
        const int slot = pr ? before : np + (tid - before);
        sh.slot_of[tid] = slot;
        sh.sig_of[slot] = tid;
        sh.spr[slot] = pr;
        if (tid == 0) sh.npr = np;
    }
    __syncthreads();                            // the pruning test has read the raw rows
    sel_dct<N>(sh, A.dctm + sel_dct_offset(N), A.kc);
    __syncthreads();
    const int cp = (A.cp <= 0) ? (N / 2 > 2 ? N / 2 : 2) : (A.cp < N ? A.cp : N);
    const int ntile = (S + 15) / 16;
    const float *Mb = A.M + A.moff[b];
    for (int r = wave; r < K; r += nwave) {
        float l1;
        if constexpr (N >= 16) l1 = sel_cost_mfma<N>(sh, Mb + (int64_t)r * N * N, cp);
        else l1 = sel_product_valu<N>(sh, Mb + (int64_t)r * N * N, cp, S, nullptr);
        l1 = wave_sum(l1);
        if (lane == 0) sh.cost[r] = l1;
    }
    __syncthreads();
    if (tid == 0) {
        int bi = 0;
        for (int r = 1; r < K; ++r)
            if (sh.cost[r] < sh.cost[bi]) bi = r;
        sh.best = bi;
        A.best[b] = bi;
    }
    if (tid < K) A.cost[b * K + tid] = sh.cost[tid];
    __syncthreads();
    // the winner's coefficients, recomputed (one signal tile per wave)
    float *yb = A.y + A.xoff[b];
    const float *Mw = Mb + (int64_t)sh.best * N * N;
    if constexpr (N >= 16) (void)sel_tiles<N>(sh, Mw, cp, ntile, S, yb);
    else if (wave == 0) (void)sel_product_valu<N>(sh, Mw, cp, S, yb);
    __syncthreads();
}

__global__ void __launch_bounds__(kSelThreads) k_select(SelArgs A) {
    __shared__ SelShared sh;
    for (;;) {
        if (threadIdx.x == 0) sh.next = atomicAdd(A.counter, 1);
        __syncthreads();
        const int idx = sh.next;
        __syncthreads();
        if (idx >= A.nblocks) break;     // every workgroup leaves once the queue is drained
        const int64_t b = A.order[idx];
        switch (A.n[b]) {
            case 4: sel_block<4>(sh, A, b); break;
            case 8: sel_block<8>(sh, A, b); break;
            case 16: sel_block<16>(sh, A, b); break;
            case 32: sel_block<32>(sh, A, b); break;
            default: sel_block<64>(sh, A, b); break;
        }
    }
}

dctplus_status sel_set_device(int device) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    return DCTPLUS_OK;
}

}  // namespace

}  // namespace dctplus

using namespace dctplus;

extern "C" {

dctplus_status dctplus_select_plan(int64_t nblocks, int32_t K, int32_t S, const int32_t *n_host,
                                   const double *cand_host, void *stream, dctplus_select_t *out) {
    if (!out) return fail(DCTPLUS_EINVAL, "null output pointer");
    *out = nullptr;
    if (nblocks < 0) return fail(DCTPLUS_EINVAL, "nblocks = %lld < 0", (long long)nblocks);
    if (K < 1 || K > kSelMaxK) return fail(DCTPLUS_EINVAL, "K = %d: need 1 <= K <= %d", K, kSelMaxK);
    if (S < 1 || S > kSelMaxS) return fail(DCTPLUS_EINVAL, "S = %d: need 1 <= S <= %d", S, kSelMaxS);
    if (nblocks > 0 && (!n_host || !cand_host)) return fail(DCTPLUS_EINVAL, "null block sizes or candidates");
    if (nblocks > (int64_t)INT32_MAX / kSelMaxK) return fail(DCTPLUS_EINVAL, "too many blocks");
    for (int64_t b = 0; b < nblocks; ++b) {
        const int n = n_host[b];
        if (n != 4 && n != 8 && n != 16 && n != 32 && n != 64)
            return fail(DCTPLUS_EUNSUPPORTED, "block %lld: n = %d; supported block sizes are 4, 8, 16, 32, 64",
                        (long long)b, n);
        for (int r = 0; r < K; ++r) {
            const double *c = cand_host + ((int64_t)b * K + r) * 4;
            const bool ints = c[1] == floor(c[1]) && c[2] == floor(c[2]);
            const bool in_range = c[1] >= 0 && c[1] < n && c[2] >= 0 && c[2] < n;
            const bool ok = (c[0] == 0.0 || c[0] == 1.0) && ints && in_range && isfinite(c[3]) && c[3] > 0.0 &&
                            !(c[0] == 1.0 && c[1] == c[2]);
            if (!ok)
                return fail(DCTPLUS_EINVAL,
                            "block %lld candidate %d: need kind 0 (self-loop at i) or 1 (edge i != j), "
                            "integer vertices in [0, n), weight > 0", (long long)b, r);
        }
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    dctplus_select_s *p = new (std::nothrow) dctplus_select_s();
    if (!p) return fail(DCTPLUS_ENOMEM, "host allocation failed");
    p->nblocks = nblocks;
    p->K = K;
    p->S = S;
    p->device = dev;
    if (nblocks == 0) {
        *out = p;
        return DCTPLUS_OK;
    }
    p->n_host.assign(n_host, n_host + nblocks);
    p->xoff_host.resize(nblocks);
    p->moff_host.resize(nblocks);
    int64_t xa = 0, ma = 0;
    for (int64_t b = 0; b < nblocks; ++b) {
        p->xoff_host[b] = xa;
        p->moff_host[b] = ma;
        xa += (int64_t)S * n_host[b];
        ma += (int64_t)K * n_host[b] * n_host[b];
    }
    p->total_x = xa;
    std::vector<int32_t> order(nblocks);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t u, int32_t w) { return n_host[u] > n_host[w]; });
    hipStream_t s = (hipStream_t)stream;
    double *cand_dev = nullptr;
    auto bail = [&](dctplus_status st) {
        if (cand_dev) (void)hipFree(cand_dev);
        dctplus_select_destroy(p);
        return st;
    };
    if (hipMalloc(&p->n_dev, sizeof(int32_t) * nblocks) != hipSuccess ||
        hipMalloc(&p->xoff_dev, sizeof(int64_t) * nblocks) != hipSuccess ||
        hipMalloc(&p->moff_dev, sizeof(int64_t) * nblocks) != hipSuccess ||
        hipMalloc(&p->order_dev, sizeof(int32_t) * nblocks) != hipSuccess ||
        hipMalloc(&p->counter_dev, 256) != hipSuccess || hipMalloc(&p->status_dev, 256) != hipSuccess ||
        hipMalloc(&p->dctm, sizeof(float) * sel_dct_offset(2 * kSelMaxN)) != hipSuccess ||
        hipMalloc(&p->kc, sizeof(d64::GroupConst) * 8) != hipSuccess ||
        hipMalloc(&p->M, sizeof(float) * (size_t)ma) != hipSuccess ||
        hipMalloc(&cand_dev, sizeof(double) * 4 * (size_t)nblocks * K) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(DCTPLUS_ENOMEM, "selection plan: device allocation failed (%lld factor floats)",
                         (long long)ma));
    }
    int32_t st = 0;
    // lane constants of the register DCT-II (lane group g: frequency groups 2g + 1, 2g + 2)
    d64::GroupConst kch[8];
    for (int t = 0; t < 8; ++t) kch[t] = d64::group_const((t >> 1) * 2 + 1 + (t & 1));
    if ((e = hipMemcpyAsync(p->kc, kch, sizeof(kch), hipMemcpyHostToDevice, s)) != hipSuccess)
        return bail(hip_fail(e, "selection plan upload"));
    if ((e = hipMemcpyAsync(p->n_dev, n_host, sizeof(int32_t) * nblocks, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->xoff_dev, p->xoff_host.data(), sizeof(int64_t) * nblocks, hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->moff_dev, p->moff_host.data(), sizeof(int64_t) * nblocks, hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->order_dev, order.data(), sizeof(int32_t) * nblocks, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(cand_dev, cand_host, sizeof(double) * 4 * (size_t)nblocks * K, hipMemcpyHostToDevice,
                            s)) != hipSuccess ||
        (e = hipMemsetAsync(p->status_dev, 0, sizeof(int32_t), s)) != hipSuccess)
        return bail(hip_fail(e, "selection plan upload"));
    hipLaunchKernelGGL(k_select_dctm, dim3(16), dim3(256), 0, s, p->dctm);
    hipLaunchKernelGGL(k_select_plan, dim3((unsigned)(nblocks * K)), dim3(64), 0, s, (const int32_t *)p->n_dev,
                       (const double *)cand_dev, (const int64_t *)p->moff_dev, (int)K, p->M, p->status_dev);
    if ((e = hipGetLastError()) != hipSuccess) return bail(hip_fail(e, "selection plan launch"));
    if ((e = hipMemcpyAsync(&st, p->status_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(hip_fail(e, "selection plan"));
    (void)hipFree(cand_dev);
    cand_dev = nullptr;
    if (st & 1) return bail(fail(DCTPLUS_ENOCONV, "secular solver did not converge for a candidate"));
    if (st) return bail(fail(DCTPLUS_EDEVICE, "inconsistent eigenvalue order in a candidate plan"));
    *out = p;
    return DCTPLUS_OK;
}

dctplus_status dctplus_select(dctplus_select_t p, const float *x, int32_t c_p, double prune_tau, int32_t *best,
                              float *cost, float *y_best, void *stream) {
    if (!p) return fail(DCTPLUS_EINVAL, "null selection plan");
    if (!isfinite(prune_tau)) return fail(DCTPLUS_EINVAL, "prune_tau is not finite");
    if (p->nblocks == 0) return DCTPLUS_OK;
    if (!x || !best || !cost || !y_best) return fail(DCTPLUS_EINVAL, "null pointer");
    if (((uintptr_t)x & 3) || ((uintptr_t)y_best & 15) || ((uintptr_t)cost & 3) || ((uintptr_t)best & 3))
        return fail(DCTPLUS_EINVAL, "misaligned pointer (x, cost, best: 4 bytes; y_best: 16 bytes)");
    const size_t bytes = sizeof(float) * (size_t)p->total_x;
    const char *a = (const char *)x, *c = (const char *)y_best;
    if (a < c + bytes && c < a + bytes) return fail(DCTPLUS_EINVAL, "x and y_best overlap");
    dctplus_status ds = sel_set_device(p->device);
    if (ds != DCTPLUS_OK) return ds;
    hipStream_t s = (hipStream_t)stream;
    int ncu = 0;
    hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess || ncu <= 0) ncu = 256;
    int64_t grid = (int64_t)ncu * p->wgs_per_cu;   // persistent workgroups (at most 4 per CU fit in LDS)
    if (grid > p->nblocks) grid = p->nblocks;
    SelArgs A;
    A.x = x;
    A.n = p->n_dev;
    A.xoff = p->xoff_dev;
    A.moff = p->moff_dev;
    A.order = p->order_dev;
    A.counter = p->counter_dev;
    A.M = p->M;
    A.dctm = p->dctm;
    A.kc = p->kc;
    A.nblocks = p->nblocks;
    A.K = p->K;
    A.S = p->S;
    A.cp = c_p;
    A.tau = prune_tau;
    A.best = best;
    A.cost = cost;
    A.y = y_best;
    hipLaunchKernelGGL(k_select_reset, dim3(1), dim3(64), 0, s, p->counter_dev);
    hipLaunchKernelGGL(k_select, dim3((unsigned)grid), dim3(kSelThreads), 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "selection launch");
    return DCTPLUS_OK;
}

dctplus_status dctplus_select_tune(dctplus_select_t p, const float *x, int32_t c_p, double prune_tau, int32_t *best,
                                   float *cost, float *y_best, void *stream, int32_t *chosen, float *ms) {
    if (!p) return fail(DCTPLUS_EINVAL, "null selection plan");
    if (p->nblocks == 0) {
        if (chosen) *chosen = p->wgs_per_cu;
        return DCTPLUS_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    const int32_t keep = p->wgs_per_cu;
    float best_ms = 0.0f;
    int32_t best_c = keep;
    dctplus_status st = DCTPLUS_OK;
    for (int32_t c = 1; c <= kSelTuneCands && st == DCTPLUS_OK; ++c) {
        p->wgs_per_cu = c;
        st = dctplus_select(p, x, c_p, prune_tau, best, cost, y_best, stream);      // warm-up, validates
        if (st != DCTPLUS_OK) break;
        (void)hipEventRecord(e0, s);
        for (int it = 0; it < 3 && st == DCTPLUS_OK; ++it)
            st = dctplus_select(p, x, c_p, prune_tau, best, cost, y_best, stream);
        (void)hipEventRecord(e1, s);
        if (st != DCTPLUS_OK) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            st = hip_fail(e, "hipEventSynchronize");
            break;
        }
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        t /= 3.0f;
        if (ms) ms[c - 1] = t;
        if (c == 1 || t < best_ms) {
            best_ms = t;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->wgs_per_cu = (st == DCTPLUS_OK) ? best_c : keep;
    if (st == DCTPLUS_OK && chosen) *chosen = best_c;
    return st;
}

dctplus_status dctplus_select_factor(dctplus_select_t p, int64_t block, int32_t r, double *dst) {
    if (!p) return fail(DCTPLUS_EINVAL, "null selection plan");
    if (block < 0 || block >= p->nblocks || r < 0 || r >= p->K || !dst)
        return fail(DCTPLUS_EINVAL, "block %lld / candidate %d out of range, or null dst", (long long)block, r);
    dctplus_status ds = sel_set_device(p->device);
    if (ds != DCTPLUS_OK) return ds;
    const int n = p->n_host[block];
    std::vector<float> buf((size_t)n * n);
    hipError_t e = hipMemcpy(buf.data(), p->M + p->moff_host[block] + (int64_t)r * n * n, sizeof(float) * n * n,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy of a selection factor");
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) dst[(size_t)i * n + k] = buf[sel_frag_index(n, i, k)];
    return DCTPLUS_OK;
}

int64_t dctplus_select_size(dctplus_select_t p) { return p ? p->total_x : -1; }

void dctplus_select_destroy(dctplus_select_t p) {
    if (!p) return;
    if (p->nblocks > 0) {
        (void)sel_set_device(p->device);
        (void)hipDeviceSynchronize();
    }
    if (p->n_dev) (void)hipFree(p->n_dev);
    if (p->xoff_dev) (void)hipFree(p->xoff_dev);
    if (p->moff_dev) (void)hipFree(p->moff_dev);
    if (p->order_dev) (void)hipFree(p->order_dev);
    if (p->counter_dev) (void)hipFree(p->counter_dev);
    if (p->status_dev) (void)hipFree(p->status_dev);
    if (p->dctm) (void)hipFree(p->dctm);
    if (p->kc) (void)hipFree(p->kc);
    if (p->M) (void)hipFree(p->M);
    delete p;
}

}  // extern "C"
