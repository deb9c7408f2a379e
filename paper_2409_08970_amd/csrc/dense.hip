// DENSE and GFT routes on MFMA.
//
// DENSE (Thm 3.1 as a progressive factorisation): s_d = DCT-II(x) in LDS,
// then y = P s_d with P = M = diag(a) C(mu, lambda) diag(z) (deflated rows
// are unit rows).  GFT (the paper's naive matrix-vector product, the
// comparator): y = P x with P = X^T.  Both build P once per plan in FP64 and
// store it rounded to FP32 (and BF16).  The adjoints multiply by P^T (then a
// DCT-III for DENSE).
//
// Products run on v_mfma_f32_16x16x4_f32 (FP32) or v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation) with signals along the MFMA M dimension:
// 64-signal chunks are loaded coalesced into LDS, transformed there, and each
// wave multiplies 16 of them by P, whose B fragments stay in VGPRs for the
// whole persistent loop.  For n >= 128 a tiled GEMM with P staged through LDS
// is used, with the DCT as a separate pass.
#include <new>

#include "dct64.h"
#include "fft.h"

namespace dctplus {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ __bf16 bits2bf(uint16_t b) {
    __bf16 r;
    __builtin_memcpy(&r, &b, 2);
    return r;
}

// P rows in FP64 -> optional DCT-III along the row (GFT) -> FP32 / BF16 / FP64.
// One workgroup per row.  Row entries a z_j / (mu - lambda_j) (deflated rows:
// e_o) are computed where they are needed; LDS holds only the n/2 complex
// doubles of the FFT (gft) or the n doubles of the row (M itself).
// With `src` (row-major n x n FP64) the row entries are read from it instead (a
// composite Cauchy factor of a rank-k plan).
__global__ void __launch_bounds__(256) k_dense_rows(PlanTables t, int gft, float *__restrict__ P32,
                                                    uint16_t *__restrict__ P16, double *__restrict__ P64,
                                                    const double *__restrict__ src) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = t.n, logn = t.logn, i = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int kind = t.kind[i];
    const int o = t.origin[i];
    const double tau = t.tau[i], a = t.a[i];
    auto entry = [&](int j) -> double {
        if (src) return src[(size_t)i * n + j];
        if (kind == ROW_DEFLATED) return (j == o) ? 1.0 : 0.0;
        const double zj = t.z[j];
        if (zj == 0.0) return 0.0;
        const double sj = (j - o) >= 0 ? t.sintab[j - o] : -t.sintab[o - j];
        const double d = 4.0 * sj * t.sintab[j + o];   // lambda_j - lambda_o
        return a * zj / (tau - d);
    };
    auto put = [&](int j, double v) {
        if (P32) P32[(size_t)i * n + j] = (float)v;
        if (P16) P16[(size_t)i * n + j] = f2bf((float)v);
        if (P64) P64[(size_t)i * n + j] = v;
    };
    if (gft) {
        // row i of X^T = (U m_i)^T: inverse orthonormal DCT of the row of M
        cplx<double> *Z = reinterpret_cast<cplx<double> *>(smem);
        const int logT = logn + 2;
        for (int k = tid; k < n / 2; k += nthr) Z[fft_slot<double>(k)] = dct3_pack<double>(entry, k, logn, t.tw64, logT);
        __syncthreads();
        const RadixPlan rp = radix_plan(logn - 1, 1, nthr);
        fft_dif(Z, 1, n / 2, logn - 1, t.tw64, logT, rp);
        for (int j = tid; j < n; j += nthr) put(j, dct3_sample(Z, j, logn, rp));
    } else {
        for (int j = tid; j < n; j += nthr) put(j, entry(j));
    }
}

size_t dense_rows_lds(int n, bool gft) { return gft ? sizeof(cplx<double>) * (n / 2) : 0; }

// ---------------------------------------------------------------------------
// Small n (16 <= N <= 64): persistent chunks of 64 signals.
// ---------------------------------------------------------------------------
constexpr int kChunk = 64;

template <int N>
struct SmallLds {
    static constexpr int kPad = N + 1;              // row stride of the signal tile (floats)
    static constexpr int kTile = kChunk * kPad;     // floats
    static constexpr int kFft = kChunk * (N / 2);   // complex floats for the DCT
    static constexpr size_t bytes = sizeof(float) * kTile + sizeof(cplx<float>) * kFft;
};

// DCT-II (dir = 0) or DCT-III (dir = 1) of the 64 rows of the LDS tile, in place.
template <int N>
__device__ __forceinline__ void tile_dct(float *xs, cplx<float> *Z, const cplx<float> *__restrict__ tw, int dir) {
    constexpr int M = N / 2;
    constexpr int logN = (N == 16) ? 4 : (N == 32) ? 5 : 6;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int logT = logN + 2;
    const RadixPlan rp = radix_plan(logN - 1, kChunk, nthr);
    if (dir == 0) {
        for (int g = tid; g < kChunk * M; g += nthr) {
            const int s = g / M, m = g % M;
            Z[s * M + fft_slot<float>(m)] = dct2_pack<float>(xs + s * SmallLds<N>::kPad, m, N);
        }
        __syncthreads();
        fft_dif(Z, kChunk, M, logN - 1, tw, logT, rp);
        for (int g = tid; g < kChunk * (M + 1); g += nthr) {
            const int s = g / (M + 1), k = g % (M + 1);
            float Xk, XNk;
            dct2_post(Z + s * M, k, logN, rp, tw, logT, Xk, XNk);
            xs[s * SmallLds<N>::kPad + k] = Xk;
            if (k > 0 && k < M) xs[s * SmallLds<N>::kPad + N - k] = XNk;
        }
    } else {
        for (int g = tid; g < kChunk * M; g += nthr) {
            const int s = g / M, k = g % M;
            const float *row = xs + s * SmallLds<N>::kPad;
            auto get = [&](int kk) -> float { return row[kk]; };
            Z[s * M + fft_slot<float>(k)] = dct3_pack<float>(get, k, logN, tw, logT);
        }
        __syncthreads();
        fft_dif(Z, kChunk, M, logN - 1, tw, logT, rp);
        for (int g = tid; g < kChunk * N; g += nthr) {
            const int s = g / N, j = g % N;
            xs[s * SmallLds<N>::kPad + j] = dct3_sample(Z + s * M, j, logN, rp);
        }
    }
    __syncthreads();
}

// Forward (adj = 0): y = P s with s = DCT(x) (pre_dct) or x.
// Adjoint (adj = 1): x = DCT-III(P^T y) (pre_dct) or P^T y.
template <int N, bool BF16>
__global__ void __launch_bounds__(256) k_dense_small(const float *__restrict__ in, float *__restrict__ out,
                                                     int64_t batch, const float *__restrict__ P32,
                                                     const uint16_t *__restrict__ P16,
                                                     const cplx<float> *__restrict__ tw, int adj, int pre_dct) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);
    cplx<float> *Z = reinterpret_cast<cplx<float> *>(xs + SmallLds<N>::kTile);
    constexpr int kPad = SmallLds<N>::kPad;
    constexpr int NT = N / 16;                       // output column tiles
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int64_t nchunks = (batch + kChunk - 1) / kChunk;

    // B fragments of B = P^T (forward: B[k][j] = P[j][k]) or B = P (adjoint)
    constexpr int KS = BF16 ? N / 32 : N / 4;        // k-steps
    constexpr int KSr = KS > 0 ? KS : 1;
    float bf32[BF16 ? 1 : KSr * NT];
    bf8 bfb[BF16 ? KSr * NT : 1];
    if constexpr (!BF16) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int k = 4 * s + lq, j = 16 * t + l16;
                bf32[s * NT + t] = adj ? P32[(size_t)k * N + j] : P32[(size_t)j * N + k];
            }
    } else {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                bf8 v;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * s + 8 * lq + e, j = 16 * t + l16;
                    v[e] = bits2bf(adj ? P16[(size_t)k * N + j] : P16[(size_t)j * N + k]);
                }
                bfb[s * NT + t] = v;
            }
    }

    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t sig0 = c * kChunk;
        const int nvalid = (int)((batch - sig0) < kChunk ? (batch - sig0) : kChunk);
        // coalesced load of the chunk (rows beyond the batch are zero)
        for (int g = tid; g < kChunk * N; g += blockDim.x) {
            const int s = g / N, j = g % N;
            xs[s * kPad + j] = (s < nvalid) ? in[(sig0 + s) * N + j] : 0.0f;
        }
        __syncthreads();
        if (pre_dct && !adj) tile_dct<N>(xs, Z, tw, 0);

        // this wave's 16 signals times B
        f4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        const float *arow = xs + (16 * wave + l16) * kPad;
        if constexpr (!BF16) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const float av = arow[4 * s + lq];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf32[s * NT + t], acc[t], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                bf8 av;
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = bits2bf(f2bf(arow[32 * s + 8 * lq + e]));
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bfb[s * NT + t], acc[t], 0, 0, 0);
            }
        }
        if (adj && pre_dct) {
            // stage P^T y in the tile (this wave's own rows), then DCT-III
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) xs[(16 * wave + 4 * lq + v) * kPad + 16 * t + l16] = acc[t][v];
            __syncthreads();
            tile_dct<N>(xs, Z, tw, 1);
            for (int g = tid; g < kChunk * N; g += blockDim.x) {
                const int s = g / N, j = g % N;
                if (s < nvalid) out[(sig0 + s) * N + j] = xs[s * kPad + j];
            }
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = 16 * wave + 4 * lq + v;
                    if (s < nvalid) out[(sig0 + s) * N + 16 * t + l16] = acc[t][v];
                }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Streaming kernel for 16 <= N <= 64: each wave owns tiles of 16 signals and
// computes Y^T = A X^T with v_mfma_f32_16x16x4_f32 (or 16x16x32 BF16), with
// A = P (forward) or P^T (adjoint).  The A operands are built once per
// workgroup into LDS in lane order (one conflict-free 16-byte read per lane and
// MFMA step), which keeps the VGPR budget small enough for several waves per
// SIMD; each wave keeps kDepth tiles of signals in flight in registers (a ring
// of loads issued kDepth tiles ahead).  The contraction index k is ordered so
// that a lane's B fragment is N/16 float4 chunks of one signal, interleaved
// with the three other lanes of that signal (64 contiguous bytes per signal and
// load instruction), and its D fragment four consecutive outputs of one signal
// (float4 stores).  Workgroups are persistent: the grid is the resident capacity and
// tiles are taken in grid-stride order.
// ---------------------------------------------------------------------------
// Three-piece BF16 split of an FP32 value: x = h + m + l to within 2^-24 |x|.
__device__ __forceinline__ void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    h = f2bf(x);
    const float r1 = x - __uint_as_float((uint32_t)h << 16);
    m = f2bf(r1);
    const float r2 = r1 - __uint_as_float((uint32_t)m << 16);
    l = f2bf(r2);
}

template <int N>
struct StreamCfg {
    static constexpr int KQ = N / 4;                 // samples per lane and tile
    static constexpr int CT = N / 16;                // output tiles of 16
    static constexpr int V4 = KQ / 4;                // float4 per lane and tile
    static constexpr int kDepth = (N == 64) ? 3 : 4; // tiles in flight per wave
};

// LDS bytes of the A operands: MODE 0: CT * KQ fragments of 64 floats;
// MODE 1: CT * KQ/8 fragments of 64 x 8 BF16; MODE 2: three such sets.
template <int N, int MODE>
constexpr int stream_lds_bytes() {
    return MODE == 0 ? StreamCfg<N>::CT * StreamCfg<N>::KQ * 64 * 4
                     : (MODE == 1 ? 1 : 3) * StreamCfg<N>::CT * (StreamCfg<N>::KQ / 8) * 64 * 16;
}

// The LDS image of the streaming kernel's A operands (A = P forward, P^T adjoint), built
// once per plan and direction and copied into LDS by every workgroup.  Lane (l16, g)
// holds sample sigma(q, g) = 16 (q / 4) + 4 g + q % 4 of its signal as its q-th B value.
//   MODE 0: float  [CT][KQ/4][64 lanes][4]
//   MODE 1: bf16   [NS][64 lanes][8]
//   MODE 2: bf16   [3 pieces][NS][64 lanes][8]   (h, m, l of the three-piece split)
template <int N, int MODE>
__global__ void __launch_bounds__(256) k_stream_image(const float *__restrict__ P32, const uint16_t *__restrict__ P16,
                                                     int adj, unsigned char *__restrict__ img) {
    using C = StreamCfg<N>;
    constexpr int KQ = C::KQ, CT = C::CT;
    constexpr int NS = CT * (KQ / 8);
    auto sigma = [](int q, int gg) -> int { return 16 * (q >> 2) + 4 * gg + (q & 3); };
    auto aval = [&](int row, int col) -> float {
        return adj ? P32[(size_t)col * N + row] : P32[(size_t)row * N + col];
    };
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nthr = gridDim.x * blockDim.x;
    if constexpr (MODE == 0) {
        float *af = reinterpret_cast<float *>(img);
        for (int e = tid; e < CT * KQ * 64; e += nthr) {
            const int q4 = e & 3, ln = (e >> 2) & 63, rest = e >> 8;   // rest = c * (KQ/4) + qq
            const int c = rest / (KQ / 4), qq = rest % (KQ / 4);
            af[e] = aval(16 * c + (ln & 15), sigma(4 * qq + q4, ln >> 4));
        }
    } else {
        uint16_t *af = reinterpret_cast<uint16_t *>(img);
        for (int e = tid; e < NS * 64 * 8; e += nthr) {
            const int el = e & 7, ln = (e >> 3) & 63, f = e >> 9;      // f = c * (KQ/8) + st
            const int c = f / (KQ / 8), st = f % (KQ / 8);
            const int row = 16 * c + (ln & 15), col = sigma(8 * st + el, ln >> 4);
            if constexpr (MODE == 1) {
                af[e] = adj ? P16[(size_t)col * N + row] : P16[(size_t)row * N + col];
            } else {
                uint16_t h, m, l;
                split3(aval(row, col), h, m, l);
                af[e] = h;
                af[NS * 512 + e] = m;
                af[2 * NS * 512 + e] = l;
            }
        }
    }
}

// One tile's product on MFMA: acc[c] (output tile c, rows 16 c + 4 g + v of signal l16)
// = sum over the lane's KQ contraction values b[q] against the A image in LDS.  `la` is
// the lane index passed through an opaque copy by the caller (kept inside the tile loop).
template <int N, int MODE, bool FENCED = false>
__device__ __forceinline__ void stream_product(const float *b, const unsigned char *sa, int la, f4 *acc) {
    using C = StreamCfg<N>;
    constexpr int KQ = C::KQ, CT = C::CT;
    constexpr int NS = CT * (KQ / 8);
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 0) {
        const float4 *af = reinterpret_cast<const float4 *>(sa);
#pragma unroll
        for (int qq = 0; qq < KQ / 4; ++qq)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const float4 a4 = af[(c * (KQ / 4) + qq) * 64 + la];
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b[4 * qq + 0], acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b[4 * qq + 1], acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b[4 * qq + 2], acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b[4 * qq + 3], acc[c], 0, 0, 0);
            }
    } else {
        const bf8 *af = reinterpret_cast<const bf8 *>(sa);
#pragma unroll
        for (int st = 0; st < KQ / 8; ++st) {
            // FP32 -> BF16 with the hardware conversion (round to nearest even, two values per
            // v_cvt_pk_bf16_f32): the same bits as split3 / f2bf for finite values
            bf8 bh, bm, bl;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const f2v x = {b[8 * st + e], b[8 * st + e + 1]};
                const bf2v h = __builtin_convertvector(x, bf2v);
                bh[e] = h[0];
                bh[e + 1] = h[1];
                if constexpr (MODE == 2) {
                    const f2v r = x - __builtin_convertvector(h, f2v);
                    const bf2v m = __builtin_convertvector(r, bf2v);
                    const bf2v l = __builtin_convertvector(r - __builtin_convertvector(m, f2v), bf2v);
                    bm[e] = m[0];
                    bm[e + 1] = m[1];
                    bl[e] = l[0];
                    bl[e + 1] = l[1];
                }
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int f = c * (KQ / 8) + st;
                const bf8 ah = af[f * 64 + la];
                if constexpr (MODE == 2) {
                    const bf8 am = af[(NS + f) * 64 + la];
                    const bf8 al = af[(2 * NS + f) * 64 + la];
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc[c], 0, 0, 0);
                }
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[c], 0, 0, 0);
                // FENCED: keep the operand reads of later output tiles from being hoisted
                // (all of them in flight at once would hold 96 VGPRs)
                if constexpr (FENCED) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// MODE 0: FP32 MFMA.  MODE 1: BF16 operands.  MODE 2: FP32-accurate products from
// three-piece BF16 splits of both operands, keeping the six cross products of
// order >= 2^-16 (hh, hm, mh, mm, hl, lh) with FP32 accumulation.
template <int N, int MODE>
__global__ void __launch_bounds__(256, 4) k_dense_stream(const float *__restrict__ in, float *__restrict__ out,
                                                      int64_t batch, const unsigned char *__restrict__ img) {
    using C = StreamCfg<N>;
    constexpr int CT = C::CT, V4 = C::V4, D = C::kDepth;
    __shared__ __align__(16) unsigned char sa[stream_lds_bytes<N, MODE>()];
    // per-wave staging of one tile (16 rows of N/4 float4 chunks): tiles move between
    // HBM and registers as contiguous 1 KiB pieces and are re-laid out here
    constexpr int CH = N / 4;                        // float4 chunks per row
    __shared__ f4 stage[4][16 * CH];
    const int tid = threadIdx.x, lane = tid & 63;
    const int l16 = lane & 15, g = lane >> 4;
    f4 *st = stage[tid >> 6];
    // chunk `ch` of row `r` sits at r * CH + (ch ^ (r mod CH)): conflict-free both for a
    // row-contiguous sweep and for sixteen rows read at one chunk position
    auto spos = [](int r, int ch) -> int { return r * CH + (ch ^ (r & (CH - 1))); };
    // Full tiles (16 valid signals) run branch-free: prefetch addresses are
    // clamped to the last full tile, so every load is issued unconditionally and
    // the wait counts stay exact (a guarded load makes the compiler wait for all
    // outstanding loads).  A ragged last tile is handled once at the end.
    const int64_t nfull = batch / 16;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // a full tile is 16 N contiguous floats: lane l reads chunks 64 u + l (coalesced)
    auto loadc = [&](int64_t tile, f4 *b) {
        const int64_t t = tile < nfull ? tile : nfull - 1;
        const f4 *src = reinterpret_cast<const f4 *>(in + t * 16 * N);
#pragma unroll
        for (int u = 0; u < V4; ++u) b[u] = __builtin_nontemporal_load(src + 64 * u + lane);
    };
    // coalesced chunks -> staging -> this lane's operand chunks 4 v + g of row l16
    auto relayout_in = [&](f4 *b) {
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int L = 64 * u + lane;
            st[spos(L / CH, L % CH)] = b[u];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int v = 0; v < V4; ++v) b[v] = st[spos(l16, 4 * v + g)];
        __builtin_amdgcn_wave_barrier();
    };
    // the first kDepth tiles are requested before the A operands are built
    f4 ring[D][V4];
    if (nfull > 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) loadc(wave0 + d * nwaves, ring[d]);
    }
    // A operands: copy the plan's LDS image (built by k_stream_image)
    {
        const f4 *src = reinterpret_cast<const f4 *>(img);
        f4 *dstl = reinterpret_cast<f4 *>(sa);
        for (int e = tid; e < stream_lds_bytes<N, MODE>() / 16; e += blockDim.x) dstl[e] = src[e];
    }
    __syncthreads();

    auto compute_store = [&](int64_t tile, const f4 *bt, bool guarded) {
        // an opaque copy of the lane index keeps the LDS operand reads inside the
        // tile loop (hoisted, they would pin all of A in VGPRs)
        int la = lane;
        asm volatile("" : "+v"(la));
        f4 acc[CT];
        stream_product<N, MODE>(reinterpret_cast<const float *>(bt), sa, la, acc);
        if (guarded) {
            const int64_t sig = tile * 16 + l16;
            if (sig < batch) {
                f4 *dst = reinterpret_cast<f4 *>(out + sig * N + 4 * g);
#pragma unroll
                for (int c = 0; c < CT; ++c) __builtin_nontemporal_store(acc[c], dst + 4 * c);
            }
        } else {
            // outputs 16 c + 4 g .. + 3 of row l16 are chunk 4 c + g: stage, then store
            // the tile as contiguous 1 KiB pieces
#pragma unroll
            for (int c = 0; c < CT; ++c) st[spos(l16, 4 * c + g)] = acc[c];
            __builtin_amdgcn_wave_barrier();
            f4 *dst = reinterpret_cast<f4 *>(out + tile * 16 * N);
#pragma unroll
            for (int u = 0; u < V4; ++u) {
                const int L = 64 * u + lane;
                __builtin_nontemporal_store(st[spos(L / CH, L % CH)], dst + L);
            }
            __builtin_amdgcn_wave_barrier();
        }
    };
    if (nfull > 0) {
        int64_t base = wave0;
        for (; base + (D - 1) * nwaves < nfull; base += D * nwaves) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                relayout_in(ring[d]);
                compute_store(base + d * nwaves, ring[d], false);
                loadc(base + (d + D) * nwaves, ring[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < D - 1; ++d)
            if (base + d * nwaves < nfull) {
                relayout_in(ring[d]);
                compute_store(base + d * nwaves, ring[d], false);
            }
    }
    if (nfull * 16 < batch && wave0 == nfull % nwaves) {
        // the ragged last tile: guarded loads (zeros past the batch) and stores
        const int64_t sig = nfull * 16 + l16;
        f4 b[V4];
        const f4 *src = reinterpret_cast<const f4 *>(in + sig * N);
#pragma unroll
        for (int v = 0; v < V4; ++v) b[v] = (sig < batch) ? src[4 * v + g] : f4{0.f, 0.f, 0.f, 0.f};
        compute_store(nfull, b, true);
    }
}

// ---------------------------------------------------------------------------
// Factored streaming kernel, n = 64: Thm 3.1 applied as the product of its
// factors, y = M s_d with M = diag(a) C(mu, lambda) diag(z) and s_d = DCT-II(x)
// (forward), x = DCT-III(M^T y) (adjoint).  The DCT runs in registers on the
// four lanes holding a signal (dct64.h: a real 16-point DFT per lane, a 4 x 4
// block transposition across the lane groups with v_permlane32_swap /
// v_permlane16_swap, a radix-4 butterfly and rotation per frequency pair), the
// product with M on MFMA.  Tiles, the ring of loads in flight, the staging of
// tiles through LDS and the persistent grid are those of k_dense_stream.  The
// MFMA contraction index follows the DCT's output slots (forward) and the
// adjoint product's output rows are the inverse DCT's input slots, so the
// factors meet without a further exchange.
// ---------------------------------------------------------------------------
// Operand image of the factored kernel, laid out as k_stream_image's.
//   forward: A = M; contraction slot q of lane group g is DCT coefficient d64::out_index(g, q).
//   adjoint: A = M^T; output row 4 g + v of tile c is coefficient d64::out_index(g, 4 c + v),
//            contraction slot q of lane group g is sample 16 (q / 4) + 4 g + q % 4 of y.
// Lane constants of the DCT's frequency groups, [lane group g][group A, B] (k1 = 2 g + 1, 2 g + 2;
// the second of lane group 3 is unused: its group is the real pair k1 = 0, 8).
__global__ void k_factored_consts(d64::GroupConst *__restrict__ kc) {
    const int t = threadIdx.x;
    if (t < 8) kc[t] = d64::group_const((t >> 1) * 2 + 1 + (t & 1));
}

template <int MODE>
__global__ void __launch_bounds__(256) k_factored_image(const float *__restrict__ M, int adj,
                                                        unsigned char *__restrict__ img) {
    constexpr int N = 64;
    using C = StreamCfg<N>;
    constexpr int KQ = C::KQ, CT = C::CT;
    constexpr int NS = CT * (KQ / 8);
    // element (row m of output tile c, contraction slot q of lane group g)
    auto aval = [&](int c, int m, int q, int g) -> float {
        if (!adj) return M[(size_t)(16 * c + m) * N + d64::out_index(g, q)];
        const int k = d64::out_index(m >> 2, 4 * c + (m & 3));
        const int j = 16 * (q >> 2) + 4 * g + (q & 3);
        return M[(size_t)j * N + k];
    };
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nthr = gridDim.x * blockDim.x;
    if constexpr (MODE == 0) {
        float *af = reinterpret_cast<float *>(img);
        for (int e = tid; e < CT * KQ * 64; e += nthr) {
            const int q4 = e & 3, ln = (e >> 2) & 63, rest = e >> 8;
            const int c = rest / (KQ / 4), qq = rest % (KQ / 4);
            af[e] = aval(c, ln & 15, 4 * qq + q4, ln >> 4);
        }
    } else {
        uint16_t *af = reinterpret_cast<uint16_t *>(img);
        for (int e = tid; e < NS * 64 * 8; e += nthr) {
            const int el = e & 7, ln = (e >> 3) & 63, f = e >> 9;
            const int c = f / (KQ / 8), st = f % (KQ / 8);
            uint16_t h, m, l;
            split3(aval(c, ln & 15, 8 * st + el, ln >> 4), h, m, l);
            af[e] = h;
            af[NS * 512 + e] = m;
            af[2 * NS * 512 + e] = l;
        }
    }
}

constexpr int kFactoredDepth = 2;   // tiles in flight per wave
// The streaming kernels read each input tile and write each output tile exactly once:
// their global loads and stores carry the non-temporal hint (108 -> 100 us per launch
// at n = 64, 2^20 signals, against 97 us for a plain device copy of the same bytes).

template <int MODE, bool ADJ>
__global__ void __launch_bounds__(256, 4) k_factored_stream(const float *__restrict__ in, float *__restrict__ out,
                                                         int64_t batch, const unsigned char *__restrict__ img,
                                                         const d64::GroupConst *__restrict__ kc) {
    constexpr int N = 64;
    using C = StreamCfg<N>;
    constexpr int CT = C::CT, V4 = C::V4, D = kFactoredDepth;
    __shared__ __align__(16) unsigned char sa[stream_lds_bytes<N, MODE>()];
    constexpr int CH = N / 4;
    // per-wave staging tile, rows padded to 68 floats (272 B): chunk ch of row r at float
    // 68 r + 4 ch, so the DCT's sample gather and scatter take immediate offsets from two
    // lane bases
    constexpr int RS = N + 4;
    __shared__ __align__(16) float stage[4][16 * RS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int l16 = lane & 15, g = lane >> 4;
    float *stf = stage[tid >> 6];
    f4 *st = reinterpret_cast<f4 *>(stf);
    auto spos = [](int r, int ch) -> int { return r * (RS / 4) + ch; };
    const int64_t nfull = batch / 16;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    auto loadc = [&](int64_t tile, f4 *b) {
        const int64_t t = tile < nfull ? tile : nfull - 1;
        const f4 *src = reinterpret_cast<const f4 *>(in + t * 16 * N);
#pragma unroll
        for (int u = 0; u < V4; ++u) b[u] = __builtin_nontemporal_load(src + 64 * u + lane);
    };
    f4 ring[D][V4];
    if (nfull > 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) loadc(wave0 + d * nwaves, ring[d]);
    }
    {
        const f4 *src = reinterpret_cast<const f4 *>(img);
        f4 *dstl = reinterpret_cast<f4 *>(sa);
        for (int e = tid; e < stream_lds_bytes<N, MODE>() / 16; e += blockDim.x) dstl[e] = src[e];
    }
    __syncthreads();
    // constants of this lane group's two frequency groups (k1 = 2 g + 1, 2 g + 2)
    // the frequency groups' constants stay in LDS and are read per tile through an opaque
    // index (held across the loop they would take 28 VGPRs)
    __shared__ d64::GroupConst skc[8];
    if (tid < 8) skc[tid] = kc[tid];
    __syncthreads();

    // one tile: b = its 16 x 64 samples as coalesced chunks (row r of the tile = signal);
    // rows from `nvalid` on are not stored
    auto tile_op = [&](int64_t tile, const f4 *b, int nvalid) {
        int la = lane;
        asm volatile("" : "+v"(la));
        const d64::GroupConst kA = skc[2 * (la >> 4)], kB = skc[2 * (la >> 4) + 1];
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int L = 64 * u + lane;
            st[spos(L / CH, L % CH)] = b[u];
        }
        __builtin_amdgcn_wave_barrier();
        float R[16];
        f4 acc[CT];
        if constexpr (!ADJ) {
            // DCT-II of signal l16: the lane's sixteen Makhoul-ordered samples
            // samples 2 g + 8 m (m < 8) and 63 - 2 g - 8 (m - 8) (m >= 8) of row l16
            float a[16];
            const float *lo = stf + RS * l16 + 2 * g, *hi = stf + RS * l16 + 63 - 2 * g;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                a[m] = lo[8 * m];
                a[m + 8] = hi[-8 * m];
            }
            __builtin_amdgcn_wave_barrier();
            d64::rdft16(a, R);
            d64::xpose_lane_groups(R);
            float X[16];
            d64::group_fwd(R, 0, kA, X);
            if (g < 3) d64::group_fwd(R, 2, kB, X + 8);
            else d64::special_fwd(R, X + 8);
            stream_product<N, MODE, true>(X, sa, la, acc);
            // outputs 16 c + 4 g .. + 3 of row l16 are chunk 4 c + g
#pragma unroll
            for (int c = 0; c < CT; ++c) st[spos(l16, 4 * c + g)] = acc[c];
        } else {
            // M^T y: the lane's y samples 16 (q / 4) + 4 g + q % 4 are chunks 4 v + g
            f4 bv[V4];
#pragma unroll
            for (int v = 0; v < V4; ++v) bv[v] = st[spos(l16, 4 * v + g)];
            __builtin_amdgcn_wave_barrier();
            stream_product<N, MODE, true>(reinterpret_cast<const float *>(bv), sa, la, acc);
            float X[16];
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) X[4 * c + v] = acc[c][v];
            d64::group_adj(X, kA, R, 0);
            if (g < 3) d64::group_adj(X + 8, kB, R, 2);
            else d64::special_adj(X + 8, R);
            d64::xpose_lane_groups(R);
            float a[16];
            d64::rdft16_t(R, a);
            float *lo = stf + RS * l16 + 2 * g, *hi = stf + RS * l16 + 63 - 2 * g;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                lo[8 * m] = a[m];
                hi[-8 * m] = a[m + 8];
            }
        }
        __builtin_amdgcn_wave_barrier();
        f4 *dst = reinterpret_cast<f4 *>(out + tile * 16 * N);
        if (nvalid == 16) {
#pragma unroll
            for (int u = 0; u < V4; ++u) {
                const int L = 64 * u + lane;
                __builtin_nontemporal_store(st[spos(L / CH, L % CH)], dst + L);
            }
        } else {
#pragma unroll
            for (int u = 0; u < V4; ++u) {
                const int L = 64 * u + lane;
                if (L / CH < nvalid) __builtin_nontemporal_store(st[spos(L / CH, L % CH)], dst + L);
            }
        }
        __builtin_amdgcn_wave_barrier();
    };
    if (nfull > 0) {
        int64_t base = wave0;
        for (; base + (D - 1) * nwaves < nfull; base += D * nwaves) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                tile_op(base + d * nwaves, ring[d], 16);
                loadc(base + (d + D) * nwaves, ring[d]);
            }
        }
#pragma unroll
        for (int d = 0; d < D - 1; ++d)
            if (base + d * nwaves < nfull) tile_op(base + d * nwaves, ring[d], 16);
    }
    if (nfull * 16 < batch && wave0 == nfull % nwaves) {
        // the ragged last tile: rows past the batch read as zeros and are not stored
        const int nvalid = (int)(batch - nfull * 16);
        const f4 *src = reinterpret_cast<const f4 *>(in + nfull * 16 * N);
        f4 b[V4];
#pragma unroll
        for (int u = 0; u < V4; ++u) {
            const int L = 64 * u + lane;
            b[u] = (L / CH < nvalid) ? src[L] : f4{0.f, 0.f, 0.f, 0.f};
        }
        tile_op(nfull, b, nvalid);
    }
}

template <int N>
__global__ void __launch_bounds__(256) k_dense_tiny(const float *__restrict__ in, float *__restrict__ out, int64_t batch,
                             const float *__restrict__ P32, const cplx<float> *__restrict__ tw, int adj,
                             int pre_dct) {
    __shared__ float Ps[N * N], Us[N * N];
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        Ps[e] = P32[e];
        const int j = e / N, k = e % N;   // U[j][k] = c_k cos(pi k (2j+1) / 2N) = Re tw4N^(k(2j+1))
        const float ck = (k == 0) ? sqrtf(1.0f / N) : sqrtf(2.0f / N);
        Us[e] = ck * tw[(k * (2 * j + 1)) % (4 * N)].re;
    }
    __syncthreads();
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < batch; b += (int64_t)gridDim.x * blockDim.x) {
        float v[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = in[b * N + j];
        if (!adj) {
            if (pre_dct) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    float a = 0.f;
#pragma unroll
                    for (int j = 0; j < N; ++j) a += Us[j * N + k] * v[j];
                    w[k] = a;
                }
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] = w[k];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float a = 0.f;
#pragma unroll
                for (int k = 0; k < N; ++k) a += Ps[i * N + k] * v[k];
                w[i] = a;
            }
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                float a = 0.f;
#pragma unroll
                for (int i = 0; i < N; ++i) a += Ps[i * N + k] * v[i];
                w[k] = a;
            }
            if (pre_dct) {
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    float a = 0.f;
#pragma unroll
                    for (int k = 0; k < N; ++k) a += Us[j * N + k] * w[k];
                    v[j] = a;
                }
#pragma unroll
                for (int j = 0; j < N; ++j) w[j] = v[j];
            }
        }
#pragma unroll
        for (int j = 0; j < N; ++j) out[b * N + j] = w[j];
    }
}

// ---------------------------------------------------------------------------
// Large n: batched DCT pass + tiled MFMA GEMM  C[b][j] = sum_k A[b][k] B[k][j],
// with B = P^T (forward) or P (adjoint).  Tile 64 signals x 64 outputs, K step 16.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dct_rows(PlanTables t, const float *__restrict__ in, float *__restrict__ out,
                                                  int64_t batch, int dir, int nsig) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = t.n, logn = t.logn, tid = threadIdx.x, nthr = blockDim.x;
    const int logT = logn + 2, M = n / 2;
    cplx<float> *Z = reinterpret_cast<cplx<float> *>(smem);
    const int64_t s0 = (int64_t)blockIdx.x * nsig;
    const int ns = (int)((batch - s0) < nsig ? (batch - s0) : nsig);
    const RadixPlan rp = radix_plan(logn - 1, ns, nthr);
    if (dir == 0) {
        if ((((uintptr_t)in) & 15) == 0) {
            // 16-byte chunks of the rows (coalesced), two packed points each
            for (int g = tid; g < ns * (M / 2); g += nthr) {
                const int s = g / (M / 2), tq = g % (M / 2);
                const float4 x4 = *reinterpret_cast<const float4 *>(in + (s0 + s) * n + 4 * tq);
                cplx<float> zt, zr;
                dct2_pack4(x4, zt, zr);
                Z[(size_t)s * M + fft_slot<float>(tq)] = zt;
                Z[(size_t)s * M + fft_slot<float>(M - 1 - tq)] = zr;
            }
        } else {
            for (int g = tid; g < ns * M; g += nthr) {
                const int s = g / M, m = g % M;
                Z[(size_t)s * M + fft_slot<float>(m)] = dct2_pack<float>(in + (s0 + s) * n, m, n);
            }
        }
        __syncthreads();
        fft_dif(Z, ns, M, logn - 1, t.tw32, logT, rp);
        for (int g = tid; g < ns * (M + 1); g += nthr) {
            const int s = g / (M + 1), k = g % (M + 1);
            float Xk, XNk;
            dct2_post(Z + (size_t)s * M, k, logn, rp, t.tw32, logT, Xk, XNk);
            out[(s0 + s) * n + k] = Xk;
            if (k > 0 && k < M) out[(s0 + s) * n + n - k] = XNk;
        }
    } else {
        for (int g = tid; g < ns * M; g += nthr) {
            const int s = g / M, k = g % M;
            const float *row = in + (s0 + s) * n;
            auto get = [&](int kk) -> float { return row[kk]; };
            Z[(size_t)s * M + fft_slot<float>(k)] = dct3_pack<float>(get, k, logn, t.tw32, logT);
        }
        __syncthreads();
        fft_dif(Z, ns, M, logn - 1, t.tw32, logT, rp);
        for (int g = tid; g < ns * n; g += nthr) {
            const int s = g / n, j = g % n;
            out[(s0 + s) * n + j] = dct3_sample(Z + (size_t)s * M, j, logn, rp);
        }
    }
}

constexpr int TBM = 64, TBN = 64, TBK = 16;

// FP64 product for FP64 plans, any n >= 4: C[b][j] = sum_k A[b][k] B[k][j] with
// B[k][j] = P[j][k] (transB, forward y = P x) or P[k][j] (adjoint x = P^T y).
// 64 x 64 output tiles, 2 x 2 waves of 32 x 32 on 16x16x4 FP64 MFMA, k-steps of
// 16 through LDS; every load and store is bounds-checked, so n need not be a
// multiple of the tile.
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm64(const double *__restrict__ A, const double *__restrict__ P,
                                                double *__restrict__ C, int64_t batch, int n, int transB) {
    __shared__ double As[TBM][TBK + 1];
    __shared__ double Bs[TBK][TBN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * TBM;
    const int n0 = blockIdx.x * TBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += TBK) {
        for (int e = tid; e < TBM * TBK; e += 256) {
            const int r = e / TBK, k = e % TBK;
            const int64_t row = m0 + r;
            As[r][k] = (row < batch && k0 + k < n) ? A[row * n + k0 + k] : 0.0;
        }
        for (int e = tid; e < TBK * TBN; e += 256) {
            int k, j;
            if (transB) { j = e / TBK; k = e % TBK; }
            else { k = e / TBN; j = e % TBN; }
            const bool in = (k0 + k < n) && (n0 + j < n);
            Bs[k][j] = !in ? 0.0 : transB ? P[(size_t)(n0 + j) * n + k0 + k] : P[(size_t)(k0 + k) * n + n0 + j];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < TBK / 4; ++s) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double av = As[wm + 16 * a + l16][4 * s + lq];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double bv = Bs[4 * s + lq][wn + 16 * b + l16];
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // the FP64 16x16x4 product leaves element v of lane l at row 4 v + l / 16
                const int64_t row = m0 + wm + 16 * a + 4 * v + lq;
                const int col = n0 + wn + 16 * b + l16;
                if (row < batch && col < n) C[row * n + col] = acc[a][b][v];
            }
}

// FP32 dense product for n > 64 (Thm 3.1's product with the n x n factor P):
//   C[m][j] = sum_k A[m][k] B(k, j),  B(k, j) = P[j][k] (TRANSB: forward, y = P s)
//                                     or       P[k][j] (adjoint, x = P^T y),
// A = the [M x K] signals (row-major), C = [M x N] (row-major), K = N = n.
// BM x BN output tiles per workgroup (2 x 2 waves), k-steps of 32 through LDS with
// the next step's operands loaded into registers while the current one is
// multiplied; FP32 MFMA 16x16x4.  The contraction index is permuted inside each
// half-step of 16 (lane group g supplies k = 4 g + s to the s-th of four MFMAs), so a
// lane reads its four operand values of a row with one 16-byte LDS read; rows are
// padded to 36 floats, which makes those reads conflict-free.  The adjoint keeps P's
// rows as loaded (k-major) and reads each operand value on its own.  n must be a
// multiple of 64 (or of BN); rows of
// A and C past M are not read or written.
constexpr int GKS = 32;      // k per step (two halves of 16, each read as one float4 per lane and row)
constexpr int GPAD = 36;     // LDS row stride (floats)

template <int BM, int BN, bool TRANSB>
__global__ void __launch_bounds__(256) k_gemm32(const float *__restrict__ A, const float *__restrict__ P,
                                                float *__restrict__ C, int64_t M, int n) {
    constexpr int WM = BM / 2, WN = BN / 2;          // per-wave tile
    constexpr int TM = WM / 16, TN = WN / 16;        // MFMA tiles per wave
    constexpr int AV = BM * GKS / 4 / 256;           // float4 of A per thread and step
    constexpr int BV = BN * GKS / 4 / 256;           // float4 of B per thread and step
    static_assert(AV >= 1 && BV >= 1, "tile too small for 256 threads");
    __shared__ __align__(16) float As[BM * GPAD];
    // B in LDS: TRANSB as [output][k] rows (the layout of A); otherwise as loaded, [k][output]
    // rows of BN + 4 floats, each MFMA operand value then one 4-byte read (lane (l16, g) of a
    // read lands on bank l16 + 16 g: conflict-free), instead of a transposing store
    constexpr int LDB = BN + 4;
    __shared__ __align__(16) float Bs[TRANSB ? BN * GPAD : GKS * LDB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * BM;
    const int j0 = blockIdx.x * BN;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    // operand registers of the next k-step
    f4 ra[AV], rb[BV];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AV; ++u) {
            const int q = tid + 256 * u, r = q / (GKS / 4), c = q % (GKS / 4);   // row r, float4 c
            const int64_t row = m0 + r;
            ra[u] = row < M ? *reinterpret_cast<const f4 *>(A + row * n + k0 + 4 * c) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < BV; ++u) {
            const int q = tid + 256 * u;
            if constexpr (TRANSB) {
                const int r = q / (GKS / 4), c = q % (GKS / 4);      // output j0 + r, k0 + 4c ..
                rb[u] = *reinterpret_cast<const f4 *>(P + (size_t)(j0 + r) * n + k0 + 4 * c);
            } else {
                const int kk = q / (BN / 4), c = q % (BN / 4);       // row k0 + kk, outputs j0 + 4c ..
                rb[u] = *reinterpret_cast<const f4 *>(P + (size_t)(k0 + kk) * n + j0 + 4 * c);
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < AV; ++u) {
            const int q = tid + 256 * u, r = q / (GKS / 4), c = q % (GKS / 4);
            *reinterpret_cast<f4 *>(As + r * GPAD + 4 * c) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < BV; ++u) {
            const int q = tid + 256 * u;
            if constexpr (TRANSB) {
                const int r = q / (GKS / 4), c = q % (GKS / 4);
                *reinterpret_cast<f4 *>(Bs + r * GPAD + 4 * c) = rb[u];
            } else {
                const int kk = q / (BN / 4), c = q % (BN / 4);
                *reinterpret_cast<f4 *>(Bs + kk * LDB + 4 * c) = rb[u];
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += GKS) {
        __syncthreads();                       // the previous step's operands are consumed
        stash();
        __syncthreads();
        if (k0 + GKS < n) fetch(k0 + GKS);     // in flight while this step is multiplied
#pragma unroll
        for (int h = 0; h < GKS / 16; ++h) {
            f4 av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a)
                av[a] = *reinterpret_cast<const f4 *>(As + (wm + 16 * a + l16) * GPAD + 16 * h + 4 * g);
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                if constexpr (TRANSB) {
                    bv[b] = *reinterpret_cast<const f4 *>(Bs + (wn + 16 * b + l16) * GPAD + 16 * h + 4 * g);
                } else {
                    const float *col = Bs + (16 * h + 4 * g) * LDB + wn + 16 * b + l16;
                    bv[b] = f4{col[0], col[LDB], col[2 * LDB], col[3 * LDB]};
                }
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][s4], bv[b][s4], acc[a][b], 0, 0, 0);
        }
    }
    // element v of lane (l16, g) is row 4 g + v (signal), column l16 (output)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + wm + 16 * a + 4 * g + v;
                if (row < M) C[row * n + j0 + wn + 16 * b + l16] = acc[a][b][v];
            }
}

// ---------------------------------------------------------------------------
// The split-BF16 dense product for n > 64 (FP32 accuracy from BF16 MFMA): C = A B
// with B(k, j) = S[j][k], S given as the three pieces (h, m, l) of the plan's
// three-piece split, each an n x n BF16 matrix with the contraction index
// contiguous.  A (the signals, FP32) is staged through LDS and split on the fly,
// per MFMA fragment; the six cross products of order >= 2^-16 (hl, lh, mm, mh,
// hm, hh, smallest first) accumulate in FP32.  BM x BN tiles, a K step of 32 (one
// v_mfma_f32_16x16x32_bf16), four waves in a 2 x 2 grid; the next step's operands
// are fetched into registers while the current one is multiplied.
// ---------------------------------------------------------------------------
constexpr int SKB = 32;          // contraction step
constexpr int SPA = SKB + 4;     // A row stride in LDS (floats)
constexpr int SPB = SKB + 8;     // B row stride in LDS (bf16)

template <int BM, int BN>
__global__ void __launch_bounds__(256) k_gemm_split(const float *__restrict__ A, const uint16_t *__restrict__ S,
                                                    float *__restrict__ C, int64_t M, int n) {
    constexpr int WM = BM / 2, WN = BN / 2;          // per-wave tile
    constexpr int TM = WM / 16, TN = WN / 16;        // MFMA tiles per wave
    constexpr int AV = BM * SKB / 4 / 256;           // float4 of A per thread and step
    constexpr int BV = BN * SKB / 8 / 256;           // 8-BF16 chunks of one piece per thread and step
    static_assert(AV >= 1 && BV >= 1, "tile too small for 256 threads");
    __shared__ __align__(16) float As[BM * SPA];
    __shared__ __align__(16) uint16_t Bs[3 * BN * SPB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * BM;
    const int j0 = blockIdx.x * BN;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
    const size_t nn = (size_t)n * n;
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    f4 ra[AV];
    u4v rh[BV], rm[BV], rl[BV];   // the three pieces of the B step
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < AV; ++u) {
            const int q = tid + 256 * u, r = q / (SKB / 4), c = q % (SKB / 4);
            const int64_t row = m0 + r;
            ra[u] = row < M ? *reinterpret_cast<const f4 *>(A + row * n + k0 + 4 * c) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < BV; ++u) {
            const int q = tid + 256 * u, r = q / (SKB / 8), c = q % (SKB / 8);
            const uint16_t *src = S + (size_t)(j0 + r) * n + k0 + 8 * c;
            rh[u] = *reinterpret_cast<const u4v *>(src);
            rm[u] = *reinterpret_cast<const u4v *>(src + nn);
            rl[u] = *reinterpret_cast<const u4v *>(src + 2 * nn);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < AV; ++u) {
            const int q = tid + 256 * u, r = q / (SKB / 4), c = q % (SKB / 4);
            *reinterpret_cast<f4 *>(As + r * SPA + 4 * c) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < BV; ++u) {
            const int q = tid + 256 * u, r = q / (SKB / 8), c = q % (SKB / 8);
            *reinterpret_cast<u4v *>(Bs + (0 * BN + r) * SPB + 8 * c) = rh[u];
            *reinterpret_cast<u4v *>(Bs + (1 * BN + r) * SPB + 8 * c) = rm[u];
            *reinterpret_cast<u4v *>(Bs + (2 * BN + r) * SPB + 8 * c) = rl[u];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < n; k0 += SKB) {
        __syncthreads();                       // the previous step's operands are consumed
        stash();
        __syncthreads();
        if (k0 + SKB < n) fetch(k0 + SKB);     // in flight while this step is multiplied
        // A fragments of this wave (lane: row l16 of the tile, contraction 8 g .. 8 g + 7),
        // split into three BF16 pieces with the hardware conversion (round to nearest even)
        bf8 ah[TM], am[TM], al[TM];
#pragma unroll
        for (int a = 0; a < TM; ++a) {
            const float *src = As + (wm + 16 * a + l16) * SPA + 8 * g;
            const f4 x0 = *reinterpret_cast<const f4 *>(src), x1 = *reinterpret_cast<const f4 *>(src + 4);
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const f4 &xs = e < 4 ? x0 : x1;
                const f2v x = (e & 2) ? f2v{xs.z, xs.w} : f2v{xs.x, xs.y};
                const bf2v h = __builtin_convertvector(x, bf2v);
                const f2v r = x - __builtin_convertvector(h, f2v);
                const bf2v m = __builtin_convertvector(r, bf2v);
                const bf2v l = __builtin_convertvector(r - __builtin_convertvector(m, f2v), bf2v);
                ah[a][e] = h[0];
                ah[a][e + 1] = h[1];
                am[a][e] = m[0];
                am[a][e + 1] = m[1];
                al[a][e] = l[0];
                al[a][e + 1] = l[1];
            }
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int rowb = wn + 16 * b + l16;
            const bf8 bh = *reinterpret_cast<const bf8 *>(Bs + (0 * BN + rowb) * SPB + 8 * g);
            const bf8 bm = *reinterpret_cast<const bf8 *>(Bs + (1 * BN + rowb) * SPB + 8 * g);
            const bf8 bl = *reinterpret_cast<const bf8 *>(Bs + (2 * BN + rowb) * SPB + 8 * g);
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[a], bm, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[a], bh, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bm, acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh, acc[a][b], 0, 0, 0);
            }
        }
    }
    // element v of lane (l16, g) is row 4 g + v (signal), column l16 (output)
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + wm + 16 * a + 4 * g + v;
                if (row < M) C[row * n + j0 + wn + 16 * b + l16] = acc[a][b][v];
            }
}

// P^T of an FP32 plan with 64 < n <= 4096, so that the forward product reads its operand
// tiles k-major like the adjoint (the faster load and LDS pattern of k_gemm32).
__global__ void k_transpose32(const float *__restrict__ P, int n, float *__restrict__ PT) {
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / n), k = (int)(e % n);
        PT[e] = P[(size_t)k * n + j];
    }
}

// The split images of a folded plan with n > 64: direction d (0 forward, 1 adjoint)
// holds S_d[j][k] = P[j][k] (forward, y = P x) or P[k][j] (adjoint, x = P^T y) as three
// BF16 pieces, [d][piece][n][n].
__global__ void k_split_image(const float *__restrict__ P, int n, uint16_t *__restrict__ img) {
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * nn; e += (size_t)gridDim.x * blockDim.x) {
        const int d = (int)(e / nn);
        const size_t f = e - (size_t)d * nn;
        const int j = (int)(f / n), k = (int)(f % n);
        const float v = d == 0 ? P[(size_t)j * n + k] : P[(size_t)k * n + j];
        uint16_t h, m, l;
        split3(v, h, m, l);
        uint16_t *base = img + (size_t)d * 3 * nn;
        base[f] = h;
        base[nn + f] = m;
        base[2 * nn + f] = l;
    }
}

int num_cus() {
    // initialised once, thread-safely (a local static), from the device current at the first call
    static const int ncu = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            return v;
        return 256;
    }();
    return ncu;
}

int persistent_blocks(int64_t nchunks) {
    const int64_t cap = (int64_t)num_cus() * 4;
    return (int)(nchunks < cap ? nchunks : cap);
}

// Grid of the streaming kernels: persistent workgroups, at most the resident capacity (or
// `wpc` per CU when the tuner chose it), never more than one per four tiles.
// resident 256-thread workgroups of `kernel` per CU (2 when the runtime cannot tell)
template <typename K>
int resident_per_cu(K kernel) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || per <= 0) {
        (void)hipGetLastError();
        per = 2;
    }
    return per;
}

int persistent_grid(int per, int64_t ntiles, int wpc) {
    const int64_t cap = (int64_t)((wpc > 0 && wpc < per) ? wpc : per) * num_cus();
    const int64_t want = (ntiles + 3) / 4;
    return (int)(want < cap ? want : cap);
}

// (each kernel's occupancy is queried once, in a thread-safe local static)
template <int N, int MODE>
int stream_blocks(int64_t ntiles, int wpc) {
    static const int per = resident_per_cu(k_dense_stream<N, MODE>);
    return persistent_grid(per, ntiles, wpc);
}

template <int MODE, bool ADJ>
int factored_blocks(int64_t ntiles, int wpc) {
    static const int per = resident_per_cu(k_factored_stream<MODE, ADJ>);
    return persistent_grid(per, ntiles, wpc);
}

// The FP32 dense product for n > 64: 128 x 128 tiles from n = 512 on when they give
// at least two workgroups per CU, 64 x 64 otherwise (small batches, and n <= 256,
// where the short contraction leaves the larger tile's register cost unpaid: 104 vs
// 118 us at n = 256 on 65,536 signals); cfg 1 / 2 force 64 / 128.
void launch_gemm32(const float *A, const float *P, float *C, int64_t M, int n, bool transb, int cfg, hipStream_t s) {
    const int64_t big = ((M + 127) / 128) * (n / 128);
    const bool t128 = n % 128 == 0 && (cfg == 2 || (cfg == 0 && n >= 512 && big >= 2 * num_cus()));
    if (t128) {
        const dim3 grid((unsigned)(n / 128), (unsigned)((M + 127) / 128));
        if (transb) hipLaunchKernelGGL((k_gemm32<128, 128, true>), grid, dim3(256), 0, s, A, P, C, M, n);
        else hipLaunchKernelGGL((k_gemm32<128, 128, false>), grid, dim3(256), 0, s, A, P, C, M, n);
    } else {
        const dim3 grid((unsigned)(n / 64), (unsigned)((M + 63) / 64));
        if (transb) hipLaunchKernelGGL((k_gemm32<64, 64, true>), grid, dim3(256), 0, s, A, P, C, M, n);
        else hipLaunchKernelGGL((k_gemm32<64, 64, false>), grid, dim3(256), 0, s, A, P, C, M, n);
    }
}

// The split-BF16 product for n > 64: tiles as launch_gemm32 (cfg 1 / 2 force 64 / 128).
void launch_gemm_split(const float *A, const uint16_t *S, float *C, int64_t M, int n, int cfg, hipStream_t s) {
    const int64_t big = ((M + 127) / 128) * (n / 128);
    const bool t128 = n % 128 == 0 && (cfg == 2 || (cfg == 0 && big >= 2 * num_cus()));
    if (t128) {
        const dim3 grid((unsigned)(n / 128), (unsigned)((M + 127) / 128));
        hipLaunchKernelGGL((k_gemm_split<128, 128>), grid, dim3(256), 0, s, A, S, C, M, n);
    } else {
        const dim3 grid((unsigned)(n / 64), (unsigned)((M + 63) / 64));
        hipLaunchKernelGGL((k_gemm_split<64, 64>), grid, dim3(256), 0, s, A, S, C, M, n);
    }
}

template <int N, bool BF>
void launch_small(const dctplus_plan_s *p, const float *in, float *out, int64_t batch, int adj, int pre,
                  hipStream_t s) {
    const int64_t nchunks = (batch + kChunk - 1) / kChunk;
    const int blocks = persistent_blocks(nchunks);
    hipLaunchKernelGGL((k_dense_small<N, BF>), dim3(blocks), dim3(256), SmallLds<N>::bytes, s, in, out, batch,
                       (const float *)p->t.mt32, (const uint16_t *)p->t.mt16, (const cplx<float> *)p->t.tw32, adj,
                       pre);
}

}  // namespace

// Streaming-kernel operand images (forward and adjoint) for folded plans with n <= 64.
template <int N, int MODE>
dctplus_status build_stream_image(dctplus_plan_s *p, hipStream_t s) {
    constexpr size_t bytes = stream_lds_bytes<N, MODE>();
    hipError_t e = hipMalloc(&p->simg, 2 * bytes);
    if (e != hipSuccess) {
        p->simg = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc for the streaming operand images failed");
    }
    p->simg_bytes = bytes;
    unsigned char *img = (unsigned char *)p->simg;
    for (int adj = 0; adj < 2; ++adj)
        hipLaunchKernelGGL((k_stream_image<N, MODE>), dim3(16), dim3(256), 0, s, (const float *)p->t.mt32,
                           (const uint16_t *)p->t.mt16, adj, img + adj * bytes);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "streaming operand images");
    return DCTPLUS_OK;
}

// Factored-kernel operand images (forward: M, adjoint: M^T) for factored plans with n = 64.
template <int MODE>
dctplus_status build_factored_image(dctplus_plan_s *p, hipStream_t s) {
    constexpr size_t bytes = stream_lds_bytes<64, MODE>();
    hipError_t e = hipMalloc(&p->simg, 2 * bytes + 8 * sizeof(d64::GroupConst));
    if (e != hipSuccess) {
        p->simg = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc for the factored operand images failed");
    }
    p->simg_bytes = bytes;
    unsigned char *img = (unsigned char *)p->simg;
    for (int adj = 0; adj < 2; ++adj)
        hipLaunchKernelGGL((k_factored_image<MODE>), dim3(16), dim3(256), 0, s, (const float *)p->t.mt32, adj,
                           img + adj * bytes);
    hipLaunchKernelGGL(k_factored_consts, dim3(1), dim3(64), 0, s, (d64::GroupConst *)(img + 2 * bytes));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "factored operand images");
    return DCTPLUS_OK;
}

dctplus_status build_split_images(dctplus_plan_s *p, hipStream_t s) {
    const int n = (int)p->n;
    const size_t bytes = sizeof(uint16_t) * 3 * (size_t)n * n;   // one direction
    hipError_t e = hipMalloc(&p->simg, 2 * bytes);
    if (e != hipSuccess) {
        p->simg = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc for the split-BF16 operand images failed");
    }
    p->simg_bytes = bytes;
    const size_t total = 2 * (size_t)n * n;
    const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_split_image, dim3(blocks), dim3(256), 0, s, (const float *)p->t.mt32, n,
                       (uint16_t *)p->simg);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "split-BF16 operand images");
    return DCTPLUS_OK;
}

dctplus_status build_transposed(dctplus_plan_s *p, hipStream_t s) {
    const int n = (int)p->n;
    const size_t bytes = sizeof(float) * (size_t)n * n;
    hipError_t e = hipMalloc(&p->simg, bytes);
    if (e != hipSuccess) {
        p->simg = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc for the transposed dense factor failed");
    }
    p->simg_bytes = bytes;
    const size_t total = (size_t)n * n;
    const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_transpose32, dim3(blocks), dim3(256), 0, s, (const float *)p->t.mt32, n, (float *)p->simg);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transposed dense factor");
    return DCTPLUS_OK;
}

dctplus_status stream_images(dctplus_plan_s *p, hipStream_t s) {
    const int n = (int)p->n;
    if (p->t.folded && n > 64 && p->dtype == DCTPLUS_F32_SPLIT) return build_split_images(p, s);
    if (n > 64 && n <= 4096 && p->dtype == DCTPLUS_F32) return build_transposed(p, s);
    if (!p->t.folded && n == 64) {
        if (p->dtype == DCTPLUS_F32_SPLIT) return build_factored_image<2>(p, s);
        if (p->dtype == DCTPLUS_F32) return build_factored_image<0>(p, s);
        return DCTPLUS_OK;
    }
    if (!p->t.folded || n < 16 || n > 64) return DCTPLUS_OK;
    if (p->dtype == DCTPLUS_F32_SPLIT) return n == 32 ? build_stream_image<32, 2>(p, s) : build_stream_image<64, 2>(p, s);
    if (p->dtype == DCTPLUS_BF16) return n == 32 ? build_stream_image<32, 1>(p, s) : build_stream_image<64, 1>(p, s);
    if (p->dtype == DCTPLUS_F32) {
        if (n == 16) return build_stream_image<16, 0>(p, s);
        return n == 32 ? build_stream_image<32, 0>(p, s) : build_stream_image<64, 0>(p, s);
    }
    return DCTPLUS_OK;
}

void dense_release(dctplus_plan_s *p) {
    if (p->simg) (void)hipFree(p->simg);
    p->simg = nullptr;
}

dctplus_status dense_build_from(dctplus_plan_s *p, const double *src, hipStream_t s, bool src_is_xt) {
    const int n = (int)p->n;
    const size_t elems = (size_t)n * n;
    hipError_t e;
    if (p->dtype == DCTPLUS_F64) {
        // FP64 plans keep only the FP64 X^T (the DCT is always folded in)
        e = hipMalloc(&p->t.mt64, sizeof(double) * elems);
        if (e != hipSuccess) {
            p->t.mt64 = nullptr;
            (void)hipGetLastError();
            return fail(DCTPLUS_ENOMEM, "hipMalloc for the %d x %d FP64 dense factor failed", n, n);
        }
        p->t.folded = 1;
        const int gft64 = src_is_xt ? 0 : 1;
        const size_t lds = dense_rows_lds(n, gft64 != 0);
        if (lds > 65536 && (e = hipFuncSetAttribute((const void *)k_dense_rows,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return hip_fail(e, "dense factor build (LDS size)");
        hipLaunchKernelGGL(k_dense_rows, dim3(n), dim3(256), lds, s, p->t, gft64, (float *)nullptr,
                           (uint16_t *)nullptr, p->t.mt64, src);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "dense factor build");
        return DCTPLUS_OK;
    }
    e = hipMalloc(&p->t.mt32, sizeof(float) * elems);
    if (e != hipSuccess) {
        p->t.mt32 = nullptr;
        (void)hipGetLastError();
        return fail(DCTPLUS_ENOMEM, "hipMalloc for the %d x %d dense factor failed", n, n);
    }
    if (p->dtype == DCTPLUS_BF16) {
        e = hipMalloc(&p->t.mt16, sizeof(uint16_t) * elems);
        if (e != hipSuccess) {
            p->t.mt16 = nullptr;
            (void)hipGetLastError();
            return fail(DCTPLUS_ENOMEM, "hipMalloc for the BF16 dense factor failed");
        }
    }
    // The DCT is folded into the factor (P = M U^T = X^T, Thm 3.1) unless the
    // factored progressive form is requested; both give the same transform.
    p->t.folded = (p->route == DCTPLUS_ROUTE_GFT) || !p->factored || src_is_xt;
    const int gft = (p->t.folded && !src_is_xt) ? 1 : 0;
    const size_t lds = dense_rows_lds(n, gft != 0);
    if (lds > 65536 && (e = hipFuncSetAttribute((const void *)k_dense_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)lds)) != hipSuccess)
        return hip_fail(e, "dense factor build (LDS size)");
    hipLaunchKernelGGL(k_dense_rows, dim3(n), dim3(256), lds, s, p->t, gft, p->t.mt32, p->t.mt16,
                       (double *)nullptr, src);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "dense factor build");
    return stream_images(p, s);
}

dctplus_status dense_build(dctplus_plan_s *p, hipStream_t s) { return dense_build_from(p, nullptr, s, false); }

int dense_tune_count(const dctplus_plan_s *p, int64_t batch) {
    const int n = (int)p->n;
    if (p->dtype == DCTPLUS_F64 || n <= 8) return 1;
    if (n <= 64) return (p->simg != nullptr) ? 4 : 1;   // streaming kernels: 1..4 workgroups per CU
    (void)batch;
    return (n % 128 == 0) ? 2 : 1;                       // GEMM tiles 64 x 64 or 128 x 128
}

void launch_cauchy_f64(const dctplus_plan_s *p, double *M, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_rows, dim3((unsigned)p->n), dim3(256), 0, s, p->t, 0, (float *)nullptr,
                       (uint16_t *)nullptr, M, (const double *)nullptr);
}

void gemm64(const double *A, const double *P, double *C, int64_t batch, int n, bool transb, hipStream_t s) {
    const dim3 grid((unsigned)((n + TBN - 1) / TBN), (unsigned)((batch + TBM - 1) / TBM));
    hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, s, A, P, C, batch, n, transb ? 1 : 0);
}

dctplus_status dense_apply(dctplus_plan_s *p, const void *inv, void *outv, int64_t batch, bool adjoint,
                           hipStream_t s) {
    const int n = (int)p->n;
    const float *in = (const float *)inv;
    float *out = (float *)outv;
    const int pre = p->t.folded ? 0 : 1;
    const int adj = adjoint ? 1 : 0;
    const bool bf = (p->dtype == DCTPLUS_BF16);
    const bool split = (p->dtype == DCTPLUS_F32_SPLIT);
    const int cfg = tuned(p, adjoint, batch);   // 0: built-in launch choice
    if (p->dtype == DCTPLUS_F64) {
        // y = X^T x (or x = X y) as one FP64 product with the folded factor
        if (batch > (int64_t)65535 * TBM) return fail(DCTPLUS_EINVAL, "batch too large for the FP64 dense route");
        const dim3 grid((unsigned)((n + TBN - 1) / TBN), (unsigned)((batch + TBM - 1) / TBM));
        hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, s, (const double *)inv, (const double *)p->t.mt64,
                           (double *)outv, batch, n, adjoint ? 0 : 1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "FP64 dense route launch");
        return DCTPLUS_OK;
    }
    if (n <= 8) {
        const int64_t blocks64 = (batch + 255) / 256;
        const int blocks = (int)(blocks64 < 4096 ? blocks64 : 4096);
        if (n == 4)
            hipLaunchKernelGGL((k_dense_tiny<4>), dim3(blocks), dim3(256), 0, s, in, out, batch, p->t.mt32,
                               p->t.tw32, adj, pre);
        else
            hipLaunchKernelGGL((k_dense_tiny<8>), dim3(blocks), dim3(256), 0, s, in, out, batch, p->t.mt32,
                               p->t.tw32, adj, pre);
    } else if (n <= 64) {
        if (bf && n == 16) return fail(DCTPLUS_EUNSUPPORTED, "BF16 dense route needs n >= 32");
        // the streaming kernel moves float4s: it needs 16-byte aligned signal arrays
        const bool vec_ok = ((((uintptr_t)in) | ((uintptr_t)out)) & 15) == 0;
        if (split && (!vec_ok || n < 32 || (!p->t.folded && n != 64)))
            return fail(DCTPLUS_EUNSUPPORTED, "the split-BF16 mode needs n in {32, 64} (factored: n = 64) and "
                                              "16-byte aligned arrays");
        if (!p->t.folded && n == 64 && vec_ok && !bf) {
            // the factored form: DCT in registers, then the Cauchy factor on MFMA
            const int64_t ntiles = (batch + 15) / 16;
            if (!p->simg) return fail(DCTPLUS_EDEVICE, "no factored operand image on this plan");
            const unsigned char *img = (const unsigned char *)p->simg + (adj ? p->simg_bytes : 0);
            const d64::GroupConst *kc = (const d64::GroupConst *)((const unsigned char *)p->simg + 2 * p->simg_bytes);
#define DCTPLUS_FACTORED(MM, AA)                                                                        \
    hipLaunchKernelGGL((k_factored_stream<MM, AA>), dim3(factored_blocks<MM, AA>(ntiles, cfg)), dim3(256), 0, s, in, \
                       out, batch, img, kc)
            if (split) {
                if (adj) DCTPLUS_FACTORED(2, true);
                else DCTPLUS_FACTORED(2, false);
            } else {
                if (adj) DCTPLUS_FACTORED(0, true);
                else DCTPLUS_FACTORED(0, false);
            }
#undef DCTPLUS_FACTORED
        } else if (!p->t.folded || !vec_ok) {
            if (!bf) {
                if (n == 16) launch_small<16, false>(p, in, out, batch, adj, pre, s);
                else if (n == 32) launch_small<32, false>(p, in, out, batch, adj, pre, s);
                else launch_small<64, false>(p, in, out, batch, adj, pre, s);
            } else {
                if (n == 32) launch_small<32, true>(p, in, out, batch, adj, pre, s);
                else launch_small<64, true>(p, in, out, batch, adj, pre, s);
            }
        } else {
            const int64_t ntiles = (batch + 15) / 16;
            if (!p->simg) return fail(DCTPLUS_EDEVICE, "no streaming operand image on this plan");
            const unsigned char *img = (const unsigned char *)p->simg + (adj ? p->simg_bytes : 0);
#define DCTPLUS_STREAM(NN, MM)                                                                             \
    hipLaunchKernelGGL((k_dense_stream<NN, MM>), dim3(stream_blocks<NN, MM>(ntiles, cfg)), dim3(256), 0, s, in, out, \
                       batch, img)
            if (split) {
                if (n == 32) DCTPLUS_STREAM(32, 2);
                else DCTPLUS_STREAM(64, 2);
            } else if (!bf) {
                if (n == 16) DCTPLUS_STREAM(16, 0);
                else if (n == 32) DCTPLUS_STREAM(32, 0);
                else DCTPLUS_STREAM(64, 0);
            } else {
                if (n == 32) DCTPLUS_STREAM(32, 1);
                else DCTPLUS_STREAM(64, 1);
            }
#undef DCTPLUS_STREAM
        }
    } else {
        if (bf) return fail(DCTPLUS_EUNSUPPORTED, "BF16 dense route supports n <= 64");
        if (batch > (int64_t)65535 * 64) return fail(DCTPLUS_EINVAL, "batch too large for the dense product");
        float *tmp = nullptr;
        if (pre) {
            dctplus_status st = stream_work(p, s, sizeof(float) * (size_t)batch * n, (void **)&tmp);
            if (st != DCTPLUS_OK) return st;
        }
        const int nsig = n >= 4096 ? 1 : 4096 / n;
        const size_t lds = sizeof(cplx<float>) * (size_t)nsig * (n / 2);
        const dim3 dgrid((unsigned)((batch + nsig - 1) / nsig));
        if (split) {
            // folded plans only (the factored split form is n = 64); float4 loads of the signals
            if (pre || !p->simg) return fail(DCTPLUS_EDEVICE, "no split-BF16 operand images on this plan");
            if (((uintptr_t)in & 15) != 0)
                return fail(DCTPLUS_EUNSUPPORTED, "the split-BF16 mode needs 16-byte aligned arrays");
            const uint16_t *S = (const uint16_t *)((const unsigned char *)p->simg + (adj ? p->simg_bytes : 0));
            launch_gemm_split(in, S, out, batch, n, cfg, s);    // y_b = P x_b, or x_b = P^T y_b
        } else if (!adjoint) {
            const float *A = in;
            if (pre) {
                hipLaunchKernelGGL(k_dct_rows, dgrid, dim3(256), lds, s, p->t, in, tmp, batch, 0, nsig);
                A = tmp;
            }
            // y_b = P x_b: with P^T kept (n <= 4096), the adjoint's k-major operand path
            if (p->simg) launch_gemm32(A, (const float *)p->simg, out, batch, n, false, cfg, s);
            else launch_gemm32(A, p->t.mt32, out, batch, n, true, cfg, s);
        } else {
            float *C = pre ? tmp : out;
            launch_gemm32(in, p->t.mt32, C, batch, n, false, cfg, s);      // x_b = P^T y_b
            if (pre) hipLaunchKernelGGL(k_dct_rows, dgrid, dim3(256), lds, s, p->t, tmp, out, batch, 1, nsig);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "dense route launch");
    return DCTPLUS_OK;
}

}  // namespace dctplus
