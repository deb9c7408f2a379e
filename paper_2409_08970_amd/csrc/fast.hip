// FAST route: y = diag(a) C(mu, lambda) diag(z) DCT-II(x) in O(n log n)
// (Alg. 1 and the proof of Thm 3.3), and its transpose for the adjoint.
//
// Forward, per signal (0-based, s = z * s_d):
//   s_d   = DCT-II(x)                                   (element type of the plan)
//   h_j   = (-1)^(j+1) s_j / sin(pi j / n),  j >= 1      (Alg. 1 step 4; the factor
//                                                        sin / (1 - cos^2) is 1 / sin)
//   c_l   = 2 sum_j h_j sin(pi j l / n)                 (DST-I, Lemma 4.4 up to d_n)
//   t_i   = sum_l c_l sin(l psi_i)                      (sine NUFFT at the root angles,
//                                                        eq. (trigo); mu_i = 4 sin^2(psi_i / 2))
//   y_i   = a_i (-t_i / (2 sin(n psi_i)) + s_0 / mu_i)  (Alg. 1 steps 6-7 and the a-scale)
// The constant d_n of the Chebyshev identities cancels between c and the
// denominator.  Rows that cannot use the trigonometric form (the isolated top
// root of Sec. 4.2, roots outside (0, 4), and rows whose NUFFT error
// amplification is too large) use exact FP64 rows; deflated rows copy s_d.
//
// The NUFFT evaluates c on a 2x oversampled grid (one DST-I of length 2n of
// c / phi_hat) and interpolates with w window taps per root.  Interlacing
// (Lemma 4.1) puts at most one root in each Chebyshev bin (theta_b, theta_b+1),
// so every root's taps start at a fixed place near grid point 2b and the
// interpolation (and its transpose, the spreading of the adjoint) are gathers:
// no atomics, deterministic.
//
// The DCT runs in the signal's precision (FP32 for FP32 plans); everything
// from h onwards runs in FP64.  All per-signal work stays in LDS for
// n <= 4096 (FP32); larger transforms keep the FP64 buffer in global scratch
// and run each FFT as one pass in global memory followed by LDS-sized
// sub-transforms staged through a 64 KiB LDS stage (fft_dif_staged).
// The placement is a template parameter, so every access to the buffer is an
// LDS instruction or a global one and no address is ever generic: a generic
// address formed below the start of the LDS window (a negative index folded
// into the instruction's offset field) is not a legal address on the device,
// even when address plus offset is.
#include <type_traits>

#include "fft.h"

namespace dctplus {

namespace {

constexpr int kExt = 16;      // grid extension on each side (>= max window half-width)
constexpr int kMaxPair = 16;  // register staging per thread in the grid post-processing

__host__ __device__ constexpr int big_doubles(int n) {
    // per-signal FP64 buffer: 2n complex doubles, and room for the extended grid
    int d = 4 * n;
    const int need = 2 * n + 2 * kExt + 2;
    if (d < need) d = need;
    return (d + 1) & ~1;
}

// threads per workgroup and the most signals one workgroup transforms, per n = 2^logn
// (both compile-time constants of the kernels; the host may pick fewer signals)
__host__ __device__ constexpr int fast_threads(int logn) { return logn <= 8 ? 256 : 1024; }
// most exact rows summed together by the one-signal-per-workgroup kernels (forward)
constexpr int kExactRows = 8;

// the exact-row table in the kernels' internal type (FP32 plans keep an FP32 copy:
// the rows are read once per signal, and the sums stay in FP64)
template <typename TD>
__device__ __forceinline__ const TD *direct_rows(const PlanTables &t) {
    if constexpr (sizeof(TD) == 4)
        return t.direct32;
    else
        return t.direct;
}
__host__ __device__ constexpr int fast_nsig_max(int logn) {
    const int n = 1 << logn, thr = fast_threads(logn);
    int ns = n <= 256 ? 1024 / n : 4096 / n;
    if (ns < 1) ns = 1;
    // keep the register staging of the grid post-processing bounded
    while (ns > 1 && ns * n > kMaxPair * thr) ns >>= 1;
    return ns;
}
// buffer placements the kernels are built for: in LDS up to n = 4096, in global
// scratch from n = 2048 on
constexpr int kMaxLogLds = 12, kMinLogGlobal = 11;

// LDS stage of the kernels whose per-signal buffer is in global memory, in bytes:
// 64 KiB, or none where the signal's own rows in LDS leave too little room for a
// stage that pays (FP64 signals from n = 16384: a 16 KiB stage saved one pass of
// four and measured slower)
__host__ __device__ constexpr size_t stage_bytes(int logn, int tdsz) {
    return ((size_t)tdsz << logn) <= 65536 ? 65536 : 0;
}

// log2 of the complex elements of type T the stage holds (0: no stage)
template <typename T>
__host__ __device__ constexpr int stage_log_elems(size_t stage) {
    int l = 0;
    while ((sizeof(cplx<T>) << (l + 1)) <= stage) ++l;
    return stage ? l : 0;
}

// radix plan of a kernel FFT: made for the stage when the buffer is in global memory
// (logS = 0: no stage); in LDS a last pass of radix 2 is left to the FFT's reader
// (dct2_post, dst1_post, dct3_sample, through fft_out)
__host__ __device__ constexpr RadixPlan fast_plan(bool lds, int logN, int logS, int nsig, int nthreads) {
    return lds ? radix_plan_defer2(radix_plan(logN, nsig, nthreads)) : radix_plan_staged(logN, logS, nsig, nthreads);
}

// the kernels' FFTs: in LDS, or in global memory with the sub-transforms that fit
// staged through the LDS stage at smem[0] (2^logS elements; logS = 0: no stage)
template <bool kLds, typename T>
__device__ __forceinline__ void fast_fft(cplx<T> *buf, int ns, int stride, int logN, const cplx<T> *__restrict__ tw,
                                         int logT, const RadixPlan &rp, unsigned char *smem, int logS,
                                         bool zero_mid = false, bool first_done = false) {
    if constexpr (kLds)
        fft_dif(buf, ns, stride, logN, tw, logT, rp, zero_mid);
    else
        fft_dif_staged(buf, ns, stride, logN, tw, logT, rp, zero_mid, reinterpret_cast<cplx<T> *>(smem), logS,
                       first_done);
}

// whether a transform's first pass runs in global memory and can be fused into the
// stage that produces its input (fft_first_pass_from)
__host__ __device__ constexpr bool fuse_first(bool lds, const RadixPlan &rp) { return !lds && rp.nat == 1; }

struct FastCfg {
    int nsig, threads;
    bool big_in_lds;
    size_t lds, lds_max;
};

// double d of a signal's complex FP64 FFT buffer, the place where the real
// transforms write their odd extensions, under the bank swizzle of the FFT
__device__ __forceinline__ int dslot(int d) { return 2 * fft_slot<double>(d >> 1) + (d & 1); }

// grid value at any integer position from the base values G_0..G_2n (odd, period 4n)
__device__ __forceinline__ double grid_fold(const double *Gb, int p, int n) {
    const int P = 4 * n;
    int r = p % P;
    if (r < 0) r += P;
    return r <= 2 * n ? Gb[r] : -Gb[P - r];
}

template <int LOGN, typename TIO, typename TD, bool kLds>
__global__ void __launch_bounds__(fast_threads(LOGN), 4) k_fast_fwd(PlanTables t, const TIO *__restrict__ x, TIO *__restrict__ y,
                                                   int64_t batch, int nsig, double *__restrict__ gscratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int n = 1 << LOGN, logn = LOGN, nthr = fast_threads(LOGN), BD = big_doubles(n);
    // signals the radix plans are made for, and the register staging rounds
    constexpr int kPlanSig = fast_nsig_max(LOGN);
    constexpr int kRounds = (kPlanSig * n + nthr - 1) / nthr;
    static_assert(kRounds <= kMaxPair, "staging rounds");
    const int w = t.width, tid = threadIdx.x;
    const int nd = t.ndirect;
    const int64_t s0 = (int64_t)blockIdx.x * nsig;
    const int ns = (int)((batch - s0) < nsig ? (batch - s0) : nsig);
    constexpr int logT = logn + 2;
    double *big;
    if constexpr (kLds)
        big = reinterpret_cast<double *>(smem);
    else
        big = gscratch + (size_t)blockIdx.x * nsig * BD;
    constexpr size_t kStage = kLds ? 0 : stage_bytes(LOGN, sizeof(TD));   // LDS stage at smem[0]
    constexpr int kLogST = stage_log_elems<TD>(kStage), kLogSD = stage_log_elems<double>(kStage);
    size_t off = kLds ? sizeof(double) * (size_t)nsig * BD : kStage;
    TD *sd = reinterpret_cast<TD *>(smem + off);
    off += sizeof(TD) * (size_t)nsig * n;
    off = (off + 7) & ~size_t(7);
    double *dres = reinterpret_cast<double *>(smem + off);

    const cplx<TD> *twd = reinterpret_cast<const cplx<TD> *>(sizeof(TD) == 8 ? (const void *)t.tw64
                                                                             : (const void *)t.tw32);
    // 1. DCT-II of every signal (Makhoul: reorder, FFT of n/2 packed points, twiddle)
    const int strideZ = BD * (int)sizeof(double) / (int)sizeof(cplx<TD>);
    cplx<TD> *Zf = reinterpret_cast<cplx<TD> *>(big);
    bool vec4 = false;   // FP32 rows read as 16-byte chunks (coalesced), two packed points each
    if constexpr (sizeof(TIO) == 4 && sizeof(TD) == 4 && n >= 4) vec4 = (((uintptr_t)x) & 15) == 0;
    if (vec4) {
        if constexpr (sizeof(TIO) == 4 && sizeof(TD) == 4 && n >= 4) {
            for (int g = tid; g < ns * (n / 4); g += nthr) {
                const int s = g / (n / 4), tq = g % (n / 4);
                const float4 x4 = *reinterpret_cast<const float4 *>(x + (s0 + s) * n + 4 * tq);
                cplx<float> zt, zr;
                dct2_pack4(x4, zt, zr);
                Zf[(size_t)s * strideZ + fft_slot<TD>(tq)] = zt;
                Zf[(size_t)s * strideZ + fft_slot<TD>(n / 2 - 1 - tq)] = zr;
            }
        }
    } else {
        for (int g = tid; g < ns * (n / 2); g += nthr) {
            const int s = g / (n / 2), m = g % (n / 2);
            Zf[(size_t)s * strideZ + fft_slot<TD>(m)] = dct2_pack<TD>(x + (s0 + s) * n, m, n);
        }
    }
    __syncthreads();
    constexpr RadixPlan rpA = fast_plan(kLds, logn - 1, kLogST, kPlanSig, nthr);
    fast_fft<kLds>(Zf, ns, strideZ, logn - 1, twd, logT, rpA, smem, kLogST);
    // 2. the DCT's outputs X_k, X_{n-k} (thread of k), and with them the four values of
    //    the odd extension u (length 2n) of h = hz * s_d that they give: u(q) at double
    //    n + q of the signal's buffer, i.e. n complex points from double n on (under the
    //    bank swizzle).  The DCT's own FFT data (doubles [0, n)) is not overwritten.
    //    When the DST-I's first pass runs in global memory, u is never stored: the DCT's
    //    outputs go to sd (LDS) only, and that pass builds its input points from them.
    const int strideB = BD / 2;   // complex doubles per signal
    cplx<double> *Bc = reinterpret_cast<cplx<double> *>(big);
    constexpr RadixPlan rpB = fast_plan(kLds, logn, kLogSD, kPlanSig, nthr);
    constexpr bool kFuseB = fuse_first(kLds, rpB);
    for (int g = tid; g < ns * (n / 2 + 1); g += nthr) {
        const int s = g / (n / 2 + 1), k = g % (n / 2 + 1);
        TD Xk, XNk;
        dct2_post(Zf + (size_t)s * strideZ, k, logn, rpA, twd, logT, Xk, XNk);
        sd[(size_t)s * n + k] = Xk;
        if constexpr (kFuseB) {
            if (k > 0 && k < n / 2) sd[(size_t)s * n + n - k] = XNk;
            continue;
        }
        double *ub = big + (size_t)s * BD + n;
        if (k == 0) {
            ub[dslot(0)] = 0.0;
            ub[dslot(n)] = 0.0;
        } else {
            const double uk = t.hz[k] * (double)Xk;
            ub[dslot(k)] = uk;
            ub[dslot(2 * n - k)] = -uk;
            if (k < n / 2) {
                sd[(size_t)s * n + n - k] = XNk;
                const double unk = t.hz[n - k] * (double)XNk;
                ub[dslot(n - k)] = unk;
                ub[dslot(n + k)] = -unk;
            }
        }
    }
    __syncthreads();
    if constexpr (kFuseB) {
        // u(q), 0 <= q < 2n, from sd: the same products as above
        auto u = [&](int s, int q) -> double {
            const TD *sds = sd + (size_t)s * n;
            if (q < n) return q == 0 ? 0.0 : t.hz[q] * (double)sds[q];
            return q == n ? 0.0 : -(t.hz[2 * n - q] * (double)sds[2 * n - q]);
        };
        fft_first_pass_from<rpB.lr(0), double, false>(
            Bc + n / 2, ns, strideB, logn, t.tw64, logT,
            [&](int s, int e) { return cplx<double>{u(s, 2 * e), u(s, 2 * e + 1)}; });
        __syncthreads();
    }
    fast_fft<kLds>(Bc + n / 2, ns, strideB, logn, t.tw64, logT, rpB, smem, kLogSD, false, kFuseB);

    // 3. c = DST-I(h), times the window deconvolution; written as the odd
    //    extension q (length 4n, zero for n <= l <= 3n) in doubles [0, n) and (3n, 4n)
    // The grid FFT's input is zero on its middle half (doubles [n, 3n]): when its first
    // pass has radix >= 4 that pass leaves those points out, and only double 3n, which
    // shares a complex point with the last c, is written here; otherwise the middle is
    // cleared.
    constexpr RadixPlan rpC = fast_plan(kLds, logn + 1, kLogSD, kPlanSig, nthr);
    constexpr bool kPruned = rpC.lr(0) >= 2;
    for (int g = tid; g < ns * n; g += nthr) {
        const int s = g / n, l = g % n;
        double *q = big + (size_t)s * BD;
        if (l == 0) {
            q[0] = 0.0;
            if (kPruned) q[dslot(3 * n)] = 0.0;
            continue;
        }
        const double c = dst1_post(Bc + (size_t)s * strideB + n / 2, l, logn, rpB, t.tw64, logT) * t.deconv[l];
        q[dslot(l)] = c;
        q[dslot(4 * n - l)] = -c;
    }
    __syncthreads();
    if (!kPruned) {
        for (int g = tid; g < ns * (2 * n + 1); g += nthr) {
            const int s = g / (2 * n + 1), p = g % (2 * n + 1);
            big[(size_t)s * BD + dslot(n + p)] = 0.0;
        }
        __syncthreads();
    }

    // 4. grid G_m = sum_l chat_l sin(pi l m / 2n), m = 0..2n (DST-I of length 2n)
    fast_fft<kLds>(Bc, ns, strideB, logn + 1, t.tw64, logT, rpC, smem, kLogSD, kPruned);
    // pairs (m, 2n - m), m = 1..n, staged in registers (the output overwrites the FFT data)
    double gv[2 * kRounds];
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int g = tid + it * nthr;
        if (g < ns * n) {
            const int s = g / n, m = g % n + 1;
            const cplx<double> *Zs = Bc + (size_t)s * strideB;
            gv[2 * it] = 0.5 * dst1_post(Zs, m, logn + 1, rpC, t.tw64, logT);
            gv[2 * it + 1] = (m < n) ? 0.5 * dst1_post(Zs, 2 * n - m, logn + 1, rpC, t.tw64, logT) : 0.0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int g = tid + it * nthr;
        if (g < ns * n) {
            const int s = g / n, m = g % n + 1;
            double *Ge = big + (size_t)s * BD + kExt;
            Ge[m] = gv[2 * it];
            if (m < n) Ge[2 * n - m] = gv[2 * it + 1];
            if (m == 1) {
                Ge[0] = 0.0;
                Ge[2 * n] = 0.0;
            }
        }
    }
    __syncthreads();
    for (int g = tid; g < ns * 2 * kExt; g += nthr) {
        const int s = g / (2 * kExt), e = g % (2 * kExt);
        double *Gs = big + (size_t)s * BD;          // grid value G_p lives at Gs[kExt + p]
        // gi = kExt + p for p = -1..-kExt and p = 2n+1..2n+kExt; kept opaque so that
        // the compiler cannot split a negative part off into the offset field
        int gi = e < kExt ? kExt - 1 - e : 2 * n + 1 + e;
        asm volatile("" : "+v"(gi));
        Gs[gi] = grid_fold(Gs + kExt, gi - kExt, n);
    }

    // 5. exact rows (isolated top root, ill-conditioned rows): each (signal, row) pair
    //    is split over wpp waves when there are fewer pairs than waves; the partial
    //    sums are added in a fixed order
    const int wave = tid >> 6, lane = tid & 63, nwave = nthr >> 6;
    if (kPlanSig == 1) {
        // one signal per workgroup (large n): every thread takes its share of the j
        // for KR rows at once, so that many independent loads are in flight (one wave
        // per row was a long chain of dependent loads); the waves' partial sums,
        // [KR][nwave] after dres, are added in a fixed order
        auto exact_rows = [&](auto kr) {
            constexpr int KR = decltype(kr)::value;
            double *part = dres + nd;
            for (int r0 = 0; r0 < nd; r0 += KR) {
                const int nr = nd - r0 < KR ? nd - r0 : KR;
                // rows past the last are clamped to it (read, never stored): no branch
                // around the loads, which keeps them all in flight together
                const TD *Dq[KR];
#pragma unroll
                for (int q = 0; q < KR; ++q) Dq[q] = direct_rows<TD>(t) + (size_t)(q < nr ? r0 + q : nd - 1) * n;
                double acc[KR];
#pragma unroll
                for (int q = 0; q < KR; ++q) acc[q] = 0.0;
#pragma unroll 4
                for (int j = tid; j < n; j += nthr) {
                    const double xj = (double)sd[j];
#pragma unroll
                    for (int q = 0; q < KR; ++q) acc[q] += (double)Dq[q][j] * xj;
                }
#pragma unroll
                for (int q = 0; q < KR; ++q) {
                    const double a = wave_sum(acc[q]);
                    if (lane == 0 && q < nr) part[q * nwave + wave] = a;
                }
                __syncthreads();
                if (tid < nr) {
                    double sum = 0.0;
                    for (int v = 0; v < nwave; ++v) sum += part[tid * nwave + v];
                    dres[r0 + tid] = sum;
                }
                __syncthreads();
            }
        };
        if (nd <= 2)
            exact_rows(std::integral_constant<int, 2>{});
        else if (nd <= 4)
            exact_rows(std::integral_constant<int, 4>{});
        else
            exact_rows(std::integral_constant<int, kExactRows>{});
    } else {
        const int pairs = ns * nd;
        const int wpp = (pairs > 0 && pairs < nwave) ? nwave / pairs : 1;
        double *part = dres + (size_t)nsig * nd;   // [pairs * wpp <= nwave] partial sums
        for (int it = wave; it < pairs * wpp; it += nwave) {
            const int pr = it / wpp, c = it % wpp;
            const int s = pr / nd, r = pr % nd;
            const TD *D = direct_rows<TD>(t) + (size_t)r * n;
            const TD *sds = sd + (size_t)s * n;
            double acc = 0.0;
            for (int j = c * 64 + lane; j < n; j += wpp * 64) acc += (double)D[j] * (double)sds[j];
            acc = wave_sum(acc);
            if (lane == 0) {
                if (wpp == 1)
                    dres[pr] = acc;
                else
                    part[it] = acc;
            }
        }
        if (wpp > 1) {
            __syncthreads();
            for (int pr = tid; pr < pairs; pr += nthr) {
                double acc = 0.0;
                for (int c = 0; c < wpp; ++c) acc += part[pr * wpp + c];
                dres[pr] = acc;
            }
        }
    }
    __syncthreads();

    // 6. outputs.  NUFFT rows in bin order.  A thread takes one bin for a group of the
    //    workgroup's signals (every kGroups-th one), so a bin's weights are read once per
    //    group rather than once per signal, and the tap-major table makes those reads
    //    coalesced across a wave's bins.  Then the deflated rows and the exact rows.
    const int hw = w / 2;
    constexpr int kGroups = nthr / n > 1 ? nthr / n : 1;
    // NT taps per bin (fixed count: every load in flight); taps past w + 2 are zero, so
    // the default FP32 width 12 reads 14 and every other width all kTaps
    auto interpolate = [&](auto nt) {
        constexpr int NT = decltype(nt)::value;
        for (int g = tid; g < kGroups * (n - 1); g += nthr) {
            const int sg = g / (n - 1), b = g % (n - 1);
            const int row = t.rowOfBin[b];
            if (row < 0) continue;   // empty bin
            double W[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) W[k] = t.wina[(size_t)k * n + b];
            const double rb = t.rowB[b];
            // aligned taps start at grid point 2b + 1 - hw (closed form: no table lookup in
            // the address); the row factor rowA is folded into the weights
            int gi = kExt + 2 * b + 1 - hw;                // index >= kExt + 1 - hw > 0
            asm volatile("" : "+v"(gi));
            for (int s = sg; s < ns; s += kGroups) {
                const double *Gt = big + (size_t)s * BD + gi;
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < NT; ++k) acc += W[k] * Gt[k];
                y[(s0 + s) * n + row] = (TIO)(acc + rb * (double)sd[(size_t)s * n]);
            }
        }
    };
    if (w == 12)
        interpolate(std::integral_constant<int, 14>{});
    else
        interpolate(std::integral_constant<int, kTaps>{});
    for (int g = tid; g < ns * n; g += nthr) {
        const int s = g / n, k = g % n;
        const int row = t.rowOfK[k];
        if (row >= 0) y[(s0 + s) * n + row] = (TIO)(double)sd[(size_t)s * n + k];
    }
    for (int g = tid; g < ns * nd; g += nthr) {
        const int s = g / nd, r = g % nd;
        y[(s0 + s) * n + t.direct_row[r]] = (TIO)dres[g];
    }
}

template <int LOGN, typename TIO, typename TD, bool kLds>
__global__ void __launch_bounds__(fast_threads(LOGN), 4) k_fast_adj(PlanTables t, const TIO *__restrict__ y, TIO *__restrict__ x,
                                                   int64_t batch, int nsig, double *__restrict__ gscratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int n = 1 << LOGN, logn = LOGN, nthr = fast_threads(LOGN), BD = big_doubles(n);
    // signals the radix plans are made for, and the register staging rounds
    constexpr int kPlanSig = fast_nsig_max(LOGN);
    constexpr int kRounds = (kPlanSig * n + nthr - 1) / nthr;
    static_assert(kRounds <= kMaxPair, "staging rounds");
    const int w = t.width, tid = threadIdx.x;
    const int nd = t.ndirect;
    const int64_t s0 = (int64_t)blockIdx.x * nsig;
    const int ns = (int)((batch - s0) < nsig ? (batch - s0) : nsig);
    constexpr int logT = logn + 2;
    double *big;
    if constexpr (kLds)
        big = reinterpret_cast<double *>(smem);
    else
        big = gscratch + (size_t)blockIdx.x * nsig * BD;
    constexpr size_t kStage = kLds ? 0 : stage_bytes(LOGN, sizeof(TD));   // LDS stage at smem[0]
    constexpr int kLogST = stage_log_elems<TD>(kStage), kLogSD = stage_log_elems<double>(kStage);
    size_t off = kLds ? sizeof(double) * (size_t)nsig * BD : kStage;
    TD *yb = reinterpret_cast<TD *>(smem + off);   // input rows in bin order (0 for empty bins)
    off += sizeof(TD) * (size_t)nsig * n;
    off = (off + 7) & ~size_t(7);
    double *sd0 = reinterpret_cast<double *>(smem + off);
    const cplx<TD> *twd = reinterpret_cast<const cplx<TD> *>(sizeof(TD) == 8 ? (const void *)t.tw64
                                                                             : (const void *)t.tw32);
    // the NUFFT rows of the input, gathered once into bin order: every later read of
    // them is then a plain LDS read with no table lookup in its address
    for (int g = tid; g < ns * n; g += nthr) {
        const int s = g / n, b = g % n;
        const int r = (b < n - 1) ? t.rowOfBin[b] : -1;
        yb[g] = (r >= 0) ? (TD)y[(s0 + s) * n + r] : (TD)0;
    }
    double *ydir = sd0 + nsig;   // [ns * nd] input values of the exact rows
    for (int g = tid; g < ns * nd; g += nthr) {
        const int s = g / nd, r = g % nd;
        ydir[g] = (double)(TD)y[(s0 + s) * n + t.direct_row[r]];
    }
    __syncthreads();

    // transpose of the s_0 / mu compensation: sd0 = sum_b rowB_b y_row(b); each signal's
    // sum is split over wps waves, the partial sums added in a fixed order
    const int wave = tid >> 6, lane = tid & 63, nwave = nthr >> 6;
    const int wps = ns < nwave ? nwave / ns : 1;
    double *part = ydir + (size_t)nsig * nd;   // [ns * wps <= nwave] partial sums
    for (int it = wave; it < ns * wps; it += nwave) {
        const int s = it / wps, c = it % wps;
        double acc = 0.0;
        for (int b = c * 64 + lane; b < n - 1; b += wps * 64) acc += t.rowB[b] * (double)yb[(size_t)s * n + b];
        acc = wave_sum(acc);
        if (lane == 0) {
            if (wps == 1)
                sd0[s] = acc;
            else
                part[it] = acc;
        }
    }

    // transpose of the interpolation: spread u_b = rowA_b y_row(b) onto the grid in
    // gather form, folded back onto G'_1..G'_{2n-1}, then written as the odd extension
    // of length 4n for the grid DST-I.  Bin b reaches grid points 2b + 1 - hw + k,
    // k < w + 2; grid point p is reached by the kReach bins from blo(p) on, whose
    // weights (rowA and the folds G(-p), G(4n - p) near the two ends included) the
    // plan tabulates per grid point.  A thread takes one grid point for a group of the
    // signals (every kGroups-th one) and reads its weights once for all of them.
    const int hw = w / 2;
    constexpr int kGroups = nthr / (2 * n) > 1 ? nthr / (2 * n) : 1;
    // NR bins per grid point: the table is zero past the w / 2 + 2 that reach one at
    // width w, so the default FP32 width 12 reads 8 and every other width all kReach
    auto spread = [&](auto nr) {
        constexpr int NR = decltype(nr)::value;
        for (int g = tid; g < kGroups * 2 * n; g += nthr) {
            const int sg = g / (2 * n), p = g % (2 * n);
            int blo = ((p - hw - 3) >> 1) + 1;     // first bin reaching p
            blo = blo < 0 ? 0 : blo;
            asm volatile("" : "+v"(blo));          // keep the first bin whole (no negative part in the base)
            double c[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) c[k] = t.wspr[(size_t)k * 2 * n + p];
            for (int s = sg; s < ns; s += kGroups) {
                const TD *ys = yb + (size_t)s * n;
                double G = 0.0;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const int b = blo + k < n - 1 ? blo + k : n - 1;   // row n - 1 is zero
                    G += c[k] * (double)ys[b];
                }
                double *q = big + (size_t)s * BD;
                if (p == 0) {
                    q[0] = 0.0;
                    q[dslot(2 * n)] = 0.0;
                } else {
                    q[dslot(p)] = G;
                    q[dslot(4 * n - p)] = -G;
                }
            }
        }
    };
    if (w == 12)
        spread(std::integral_constant<int, 8>{});
    else
        spread(std::integral_constant<int, kReach>{});
    if (wps > 1) {
        __syncthreads();
        for (int s = tid; s < ns; s += nthr) {
            double acc = 0.0;
            for (int c = 0; c < wps; ++c) acc += part[s * wps + c];
            sd0[s] = acc;
        }
    }
    __syncthreads();
    // (the grid DST's first pass is not fused into the spread as the forward's DST-I is
    // into its producer: each grid value would be computed for both of its places in the
    // odd extension, and that cost what the saved pass gained)
    cplx<double> *Bc = reinterpret_cast<cplx<double> *>(big);
    const int strideB = BD / 2;
    constexpr RadixPlan rpC = fast_plan(kLds, logn + 1, kLogSD, kPlanSig, nthr);
    fast_fft<kLds>(Bc, ns, strideB, logn + 1, t.tw64, logT, rpC, smem, kLogSD);

    // r_l = sum_m G'_m sin(pi l m / 2n) for l < n, times the deconvolution;
    // staged in registers, then written as the odd extension (length 2n) for DST-I
    double cv[kRounds];
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int g = tid + it * nthr;
        if (g < ns * n) {
            const int s = g / n, l = g % n;
            cv[it] = (l == 0) ? 0.0
                              : 0.5 * dst1_post(Bc + (size_t)s * strideB, l, logn + 1, rpC, t.tw64, logT) *
                                    t.deconv[l];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int g = tid + it * nthr;
        if (g < ns * n) {
            const int s = g / n, l = g % n;
            double *q = big + (size_t)s * BD;
            if (l == 0) {
                q[0] = 0.0;
                q[dslot(n)] = 0.0;
            } else {
                q[dslot(l)] = cv[it];
                q[dslot(2 * n - l)] = -cv[it];
            }
        }
    }
    __syncthreads();
    constexpr RadixPlan rpB = fast_plan(kLds, logn, kLogSD, kPlanSig, nthr);
    fast_fft<kLds>(Bc, ns, strideB, logn, t.tw64, logT, rpB, smem, kLogSD);

    // s_d' = hz * DST-I(c') + deflated rows + exact rows + the compensation, in doubles [2n, 3n)
    for (int g = tid; g < ns * n; g += nthr) {
        const int s = g / n, j = g % n;
        double v = (j == 0) ? sd0[s] : t.hz[j] * dst1_post(Bc + (size_t)s * strideB, j, logn, rpB, t.tw64, logT);
        const TIO *ys = y + (s0 + s) * n;   // deflated rows come straight from the input
        const int rk = t.rowOfK[j];
        if (rk >= 0) v += (double)(TD)ys[rk];
        for (int r = 0; r < nd; ++r) v += (double)direct_rows<TD>(t)[(size_t)r * n + j] * ydir[(size_t)s * nd + r];
        big[(size_t)s * BD + 2 * n + j] = v;
    }
    __syncthreads();

    // DCT-III (inverse orthonormal DCT-II) in the signal precision
    const int strideZ = BD * (int)sizeof(double) / (int)sizeof(cplx<TD>);
    cplx<TD> *Zf = reinterpret_cast<cplx<TD> *>(big);
    for (int g = tid; g < ns * (n / 2); g += nthr) {
        const int s = g / (n / 2), k = g % (n / 2);
        const double *sds = big + (size_t)s * BD + 2 * n;
        auto get = [&](int kk) -> TD { return (TD)sds[kk]; };
        Zf[(size_t)s * strideZ + fft_slot<TD>(k)] = dct3_pack<TD>(get, k, logn, twd, logT);
    }
    __syncthreads();
    constexpr RadixPlan rpA = fast_plan(kLds, logn - 1, kLogST, kPlanSig, nthr);
    fast_fft<kLds>(Zf, ns, strideZ, logn - 1, twd, logT, rpA, smem, kLogST);
    for (int g = tid; g < ns * n; g += nthr) {
        const int s = g / n, j = g % n;
        x[(s0 + s) * n + j] = (TIO)dct3_sample(Zf + (size_t)s * strideZ, j, logn, rpA);
    }
}

// cfg (the tuner's choice): 0 or 1 = the built-in signals per workgroup, 2 = half, 3 = a quarter.
// The built-in choice takes fewer signals per workgroup while a batch of `batch` signals
// would leave CUs without a workgroup and the smaller workgroups still run in one round
// (batch 0: no such adjustment).
FastCfg fast_config(const dctplus_plan_s *p, int cfg = 0, int64_t batch = 0) {
    const int n = (int)p->n;
    const int nd = p->t.ndirect;
    const size_t tdsz = (p->dtype == DCTPLUS_F64) ? 8 : 4;
    FastCfg c;
    c.threads = fast_threads(p->logn);
    const size_t per_big = sizeof(double) * big_doubles(n);
    const size_t per_small = tdsz * n + sizeof(double) * (nd + 1);
    int lds_max = 0;   // per device (a host-side query)
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess ||
        lds_max <= 0)
        lds_max = 64 * 1024;
    size_t budget = (size_t)lds_max - 4096;
    if (budget > 150 * 1024) budget = 150 * 1024;
    c.big_in_lds = (per_big + per_small) <= budget;
    const size_t stage = c.big_in_lds ? 0 : stage_bytes(p->logn, (int)tdsz);
    int ns = fast_nsig_max(p->logn);
    while (ns > 1 && stage + (size_t)ns * ((c.big_in_lds ? per_big : 0) + per_small) > budget) ns >>= 1;
    if (cfg >= 2) {
        ns = ns >> (cfg - 1) > 0 ? ns >> (cfg - 1) : 1;
    } else if (batch > 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || ncu <= 0)
            ncu = 256;
        // halve while the halved grid still fits one workgroup per CU (one round)
        while (ns > 1 && (batch + ns / 2 - 1) / (ns / 2) <= ncu) ns >>= 1;
    }
    c.nsig = ns;
    // + exact-row partials: [kExactRows][16 waves] in the one-signal kernels, else 16
    const size_t partials = 8 * (fast_nsig_max(p->logn) == 1 ? kExactRows * 16 : 16);
    c.lds = stage + (size_t)ns * ((c.big_in_lds ? per_big : 0) + per_small) + 64 + partials;
    c.lds_max = (size_t)lds_max;
    return c;
}

// the kernel built for the plan's n (one instantiation per n and buffer placement)
template <typename TIO, typename TD, bool kLds, int LOGN = 1>
dctplus_status launch_fast(dctplus_plan_s *p, const FastCfg &c, dim3 grid, const void *in, void *out,
                           int64_t batch, bool adjoint, double *scratch, hipStream_t s) {
    if constexpr (LOGN > kMaxLogN) {
        return fail(DCTPLUS_EUNSUPPORTED, "no FAST kernel for n = %lld", (long long)p->n);
    } else {
        if (p->logn != LOGN)
            return launch_fast<TIO, TD, kLds, LOGN + 1>(p, c, grid, in, out, batch, adjoint, scratch, s);
        constexpr bool built = kLds ? LOGN <= kMaxLogLds : LOGN >= kMinLogGlobal;
        if constexpr (!built) {
            return fail(DCTPLUS_EUNSUPPORTED, "no FAST kernel for n = %lld with the buffer %s", (long long)p->n,
                        kLds ? "in LDS" : "in global memory");
        } else {
            if (c.threads != fast_threads(LOGN) || c.nsig > fast_nsig_max(LOGN))
                return fail(DCTPLUS_EINVAL, "FAST launch shape does not match the kernel");
            const dim3 block(fast_threads(LOGN));
            if (!adjoint)
                hipLaunchKernelGGL((k_fast_fwd<LOGN, TIO, TD, kLds>), grid, block, c.lds, s, p->t, (const TIO *)in,
                                   (TIO *)out, batch, c.nsig, scratch);
            else
                hipLaunchKernelGGL((k_fast_adj<LOGN, TIO, TD, kLds>), grid, block, c.lds, s, p->t, (const TIO *)in,
                                   (TIO *)out, batch, c.nsig, scratch);
            return DCTPLUS_OK;
        }
    }
}

}  // namespace

bool fast_in_lds(const dctplus_plan_s *p) { return fast_config(p).big_in_lds; }

int fast_tune_count(const dctplus_plan_s *p) {
    const int ns = fast_config(p, 0).nsig;
    return ns >= 4 ? 3 : (ns >= 2 ? 2 : 1);
}

dctplus_status fast_apply(dctplus_plan_s *p, const void *in, void *out, int64_t batch, bool adjoint,
                          hipStream_t s) {
    const FastCfg c = fast_config(p, tuned(p, adjoint, batch), batch);
    const int n = (int)p->n;
    if ((size_t)c.nsig * n > (size_t)kMaxPair * c.threads)
        return fail(DCTPLUS_EUNSUPPORTED, "n = %d too large for the FAST route", n);
    if (c.lds > c.lds_max)
        return fail(DCTPLUS_EUNSUPPORTED, "FAST route at n = %d needs %zu bytes of LDS (%d exact rows)", n, c.lds,
                    p->t.ndirect);
    const int64_t blocks = (batch + c.nsig - 1) / c.nsig;
    double *scratch = nullptr;
    if (!c.big_in_lds) {
        const size_t bytes = sizeof(double) * big_doubles(n) * (size_t)c.nsig * blocks;
        dctplus_status st = stream_work(p, s, bytes, (void **)&scratch);
        if (st != DCTPLUS_OK) return st;
    }
    if (blocks > 0x7fffffff) return fail(DCTPLUS_EINVAL, "batch too large");
    const dim3 grid((unsigned)blocks);
    if (p->t.ndirect > 0 && (p->dtype == DCTPLUS_F64 ? p->t.direct == nullptr : p->t.direct32 == nullptr))
        return fail(DCTPLUS_EINVAL, "plan has %d exact rows but no table for them", p->t.ndirect);
    dctplus_status st;
    if (p->dtype == DCTPLUS_F64)
        st = c.big_in_lds ? launch_fast<double, double, true>(p, c, grid, in, out, batch, adjoint, scratch, s)
                          : launch_fast<double, double, false>(p, c, grid, in, out, batch, adjoint, scratch, s);
    else
        st = c.big_in_lds ? launch_fast<float, float, true>(p, c, grid, in, out, batch, adjoint, scratch, s)
                          : launch_fast<float, float, false>(p, c, grid, in, out, batch, adjoint, scratch, s);
    if (st != DCTPLUS_OK) return st;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fast route launch");
    return DCTPLUS_OK;
}

}  // namespace dctplus
