// Workgroup-cooperative complex FFT for gfx950, plus the complex helpers the
// real transforms (DCT-II/III, DST-I) are built from.
//
// The FFT is an in-place decimation-in-frequency transform made of radix-2^r
// passes (r <= 4).  Each pass gives every thread whole R-point butterflies
// held in registers; passes are separated by workgroup barriers.  The output
// is left in digit-reversed order; dif_pos() maps a frequency index to its
// position, and the consumers of an FFT read through it (fft_out) instead of
// paying for a reordering pass; a last pass of radix 2 may be left to them as
// well.  Positions are stored bank-swizzled (fft_slot): the input is written,
// and the output read, through fft_slot.  Several independent signals (nsig,
// `stride` complex elements apart) are transformed by one call.  The buffer
// may live in LDS or in global scratch (fft_dif_staged: one pass in global
// memory, then LDS-sized sub-transforms staged through LDS and stored back in
// natural order; that first pass may instead run inside the stage that makes the
// input, fft_first_pass_from); callers pass pointers whose address space the
// compiler can see through the inlining (LDS or global), never a generic one.
#pragma once

#include "common.h"

namespace dctplus {

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
// a / (2i) = (a.im / 2, -a.re / 2)
template <typename T>
__device__ __forceinline__ cplx<T> cdiv2i(cplx<T> a) { return {a.im * T(0.5), -a.re * T(0.5)}; }

// exp(-2 pi i q / 16), q = 0..7 (the only in-register twiddles a radix-16
// butterfly needs).
__device__ constexpr double kW16re[8] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                                         0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674};
__device__ constexpr double kW16im[8] = {0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                                         -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};

template <int LR>
__device__ __forceinline__ constexpr int bitrev(int k) {
    int r = 0;
    for (int i = 0; i < LR; ++i) r |= ((k >> i) & 1) << (LR - 1 - i);
    return r;
}

// R-point DFT (R = 2^LR <= 16) in registers, natural order in and out.
template <int LR, typename T>
__device__ __forceinline__ void dft_reg(cplx<T> *x) {
    constexpr int R = 1 << LR;
#pragma unroll
    for (int s = 0; s < LR; ++s) {
        const int half = R >> (s + 1);
#pragma unroll
        for (int blk = 0; blk < R; blk += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                cplx<T> a = x[blk + j], b = x[blk + j + half];
                x[blk + j] = cadd(a, b);
                cplx<T> d = csub(a, b);
                const int q = j * (16 / (2 * half));     // twiddle exp(-2 pi i j / 2half) in 1/16 units
                if (q == 0) {
                    x[blk + j + half] = d;
                } else if (q == 4) {                        // multiply by -i
                    x[blk + j + half] = {d.im, -d.re};
                } else {
                    cplx<T> w = {T(kW16re[q]), T(kW16im[q])};
                    x[blk + j + half] = cmul(d, w);
                }
            }
        }
    }
    cplx<T> y[R];
#pragma unroll
    for (int k = 0; k < R; ++k) y[k] = x[bitrev<LR>(k)];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = y[k];
}

// Sequence of pass radices for an N = 2^logN transform of nsig signals on
// nthreads threads: radix 16 while at least two waves' worth of butterflies
// remain (a pass costs a barrier and a round of memory latency, so fewer,
// wider passes win once the transform is small), smaller radices otherwise.
// Must be computed identically by the FFT and by whoever reads its output.
// Any plan computes the same transform; nsig and nthreads only steer the
// choice of radices, so a plan made for more signals than a call transforms
// is still correct.  Evaluated at compile time where its arguments are
// constants, which turns every digit-reversal and pass loop into fixed shifts.
struct RadixPlan {
    int np;          // number of passes
    uint32_t code;   // 2 bits per pass: log2(radix) - 1
    // first pass whose sub-transforms are stored in natural order (a staged
    // transform, fft_dif_staged); passes before it leave their digits reversed
    int nat = 32;
    // the last pass (radix 2) is left to the readers (fft_out): it only adds and subtracts
    // neighbouring positions, which a reader can do while reading them
    bool defer2 = false;
    __host__ __device__ constexpr int lr(int i) const { return (int)((code >> (2 * i)) & 3u) + 1; }
};

// the plan with its last pass left to the readers when that pass has radix 2
__host__ __device__ constexpr RadixPlan radix_plan_defer2(RadixPlan rp) {
    if (rp.np > 1 && rp.lr(rp.np - 1) == 1 && rp.nat >= rp.np) rp.defer2 = true;
    return rp;
}

__host__ __device__ constexpr RadixPlan radix_plan(int logN, int nsig, int nthreads) {
    RadixPlan rp{0, 0u};
    int rem = logN;
    while (rem > 0) {
        int lr = rem < 4 ? rem : 4;
        while (lr > 1 && (nsig << (logN - lr)) < (nthreads < 128 ? nthreads : 128)) --lr;
        rp.code |= (uint32_t)(lr - 1) << (2 * rp.np);
        ++rp.np;
        rem -= lr;
    }
    return rp;
}

// Plan of a transform staged through an LDS stage of 2^logS elements (logS > 0):
// one pass in global memory over the logN - logS bits that do not fit (at most 4),
// then the stage's passes, whose sub-transforms are stored back in natural order.
// The output then sits at position (k mod 2^g) 2^(logN-g) + (k >> g), g = logN - logS:
// a wave reading consecutive frequencies reads 2^g runs of consecutive elements.
__host__ __device__ constexpr RadixPlan radix_plan_staged(int logN, int logS, int nsig, int nthreads) {
    if (logS <= 0 || logN - logS > 4) return radix_plan(logN, nsig, nthreads);
    RadixPlan rp{0, 0u};
    int rem = logN;
    if (logN > logS) {
        rp.code = (uint32_t)(logN - logS - 1);
        rp.np = 1;
        rem = logS;
    }
    rp.nat = rp.np;
    const RadixPlan tail = radix_plan(rem, 1, nthreads);
    for (int i = 0; i < tail.np; ++i) {
        rp.code |= (uint32_t)(tail.lr(i) - 1) << (2 * rp.np);
        ++rp.np;
    }
    return rp;
}

// Position of frequency k in the output (kept in slot fft_slot of that position):
// digit-reversed, except that the digits of the passes from rp.nat on stay in
// natural order.
__device__ __forceinline__ int dif_pos(int k, const RadixPlan &rp, int logN) {
    int p = 0, logL = logN;
    uint32_t code = rp.code;
    for (int i = 0; i < rp.np; ++i) {
        if (i == rp.nat) return p + k;     // the remaining digits, in natural order
        const int lr = (int)(code & 3u) + 1;
        code >>= 2;
        const int k2 = k & ((1 << lr) - 1);
        k >>= lr;
        logL -= lr;
        p += k2 << logL;
    }
    return p;
}

template <typename T>
__device__ __forceinline__ int fft_slot(int e);

// Frequency k of a transform's output (positions from dif_pos, kept in slots fft_slot),
// with the last radix-2 butterfly applied here when the plan defers it: the pair at
// positions 2m, 2m + 1 holds (a, b) and the frequencies there are a + b and a - b.
template <typename T>
__device__ __forceinline__ cplx<T> fft_out(const cplx<T> *Z, int k, const RadixPlan &rp, int logN) {
    const int q = dif_pos(k, rp, logN);
    if (!rp.defer2) return Z[fft_slot<T>(q)];
    const cplx<T> a = Z[fft_slot<T>(q & ~1)], b = Z[fft_slot<T>(q | 1)];
    return (q & 1) ? csub(a, b) : cadd(a, b);
}

// Bank swizzle of the FFT buffers.  Element e of a signal's buffer is kept in
// slot fft_slot(e) = e ^ fold(e >> B), where 2^B elements fill one 256-byte row
// of LDS banks and fold XORs all B-bit groups of its argument together.  A pass
// with a small butterfly span, and a consumer reading in digit-reversed order,
// step through the buffer in power-of-two strides; unswizzled, the lanes of a
// wave would then pile onto a few banks.  fold sends each index bit above B to
// bit (b mod B), so lanes whose indices differ in any B consecutive bits land in
// distinct bank slots.  The map is linear over XOR and permutes every aligned
// block of 2^B elements, so a buffer whose length is a power of two keeps its
// extent.  Whatever fills an FFT's input or reads its output goes through it.
template <typename T>
__device__ __forceinline__ int fft_slot(int e) {
    constexpr int B = sizeof(cplx<T>) >= 16 ? 4 : 5;
    int h = e >> B;
    h ^= h >> B;
    h ^= h >> (2 * B);
    return e ^ (h & ((1 << B) - 1));
}

// Element e of an FFT buffer in global memory: a uniform base plus a 32-bit byte
// offset, so that an address costs one register (the base stays scalar).  The
// buffer must be under 4 GiB.
template <typename T>
__device__ __forceinline__ cplx<T> buf_ld(const cplx<T> *buf, int e) {
    return *reinterpret_cast<const cplx<T> *>(reinterpret_cast<const char *>(buf) +
                                              (uint64_t)((uint32_t)e * (uint32_t)sizeof(cplx<T>)));
}
template <typename T>
__device__ __forceinline__ void buf_st(cplx<T> *buf, int e, cplx<T> a) {
    *reinterpret_cast<cplx<T> *>(reinterpret_cast<char *>(buf) + (uint64_t)((uint32_t)e * (uint32_t)sizeof(cplx<T>))) = a;
}

// Twiddles of a DIF butterfly of radix R = 2^LR at offset j in a sub-transform of
// length L = 2^logL (j > 0 possible only when L > R): x[r] *= w^r, w = exp(-2 pi i j / L).
// w, w^4 and w^8 come from the table and the rest from at most three products
// (w^r = w^(r mod 4) w^(r - r mod 4)), so a radix-16 butterfly reads 3 table entries
// instead of 15 (the table reads, shared by every workgroup through L2, bounded the
// passes at large n).
template <int LR, typename T>
__device__ __forceinline__ void dif_twiddle(cplx<T> *x, int j, int logL, const cplx<T> *tw, int logNtw) {
    constexpr int R = 1 << LR;
    const int sh = logNtw - logL;
    const cplx<T> w1 = tw[j << sh];
    if constexpr (R == 2) {
        x[1] = cmul(x[1], w1);
    } else {
        const cplx<T> w2 = cmul(w1, w1);
        const cplx<T> lo[4] = {cplx<T>{T(1), T(0)}, w1, w2, cmul(w2, w1)};
        if constexpr (R == 4) {
#pragma unroll
            for (int r = 1; r < 4; ++r) x[r] = cmul(x[r], lo[r]);
        } else {
            const cplx<T> w4 = tw[(4 * j) << sh];
            cplx<T> hi[4] = {cplx<T>{T(1), T(0)}, w4, w4, w4};
            if constexpr (R == 16) {
                const cplx<T> w8 = tw[(8 * j) << sh];
                hi[2] = w8;
                hi[3] = cmul(w8, w4);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> wr = (r >> 2) == 0 ? lo[r & 3]
                                   : ((r & 3) == 0 ? hi[r >> 2] : cmul(lo[r & 3], hi[r >> 2]));
                x[r] = cmul(x[r], wr);
            }
        }
    }
}

// ZMID: the first pass of a transform whose input is zero on its middle half
// (points [N/4, 3N/4)); with radix R >= 4 those are the butterfly inputs
// r in [R/4, 3R/4), which are taken as zero instead of read.
// STREAM: the buffer is in global memory (buf_ld / buf_st); otherwise in LDS.
template <int LR, typename T, bool ZMID = false, bool STREAM = false>
__device__ __forceinline__ void fft_pass(cplx<T> *buf, int nsig, int stride, int logN, int logL,
                                         const cplx<T> *__restrict__ tw, int logNtw, int tid, int nthr) {
    constexpr int R = 1 << LR;
    const int logm = logL - LR;
    const int m = 1 << logm;
    const int lg = logN - LR;                 // log2(groups per signal)
    const int total = nsig << lg;
    // slot offsets of the R inputs (fft_slot is linear and the butterfly's first
    // index has no bits in common with r << logm)
    int roff[R];
#pragma unroll
    for (int r = 0; r < R; ++r) roff[r] = fft_slot<T>(r << logm);
    for (int g = tid; g < total; g += nthr) {
        const int s = g >> lg;
        const int rem = g & ((1 << lg) - 1);
        const int sub = rem >> logm;
        const int j = rem & (m - 1);
        const int a = fft_slot<T>((sub << logL) + j);
        const int sb = s * stride;
        cplx<T> *sig = buf + (size_t)s * stride;
        cplx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ZMID && R >= 4 && r >= R / 4 && r < 3 * R / 4)
                x[r] = cplx<T>{T(0), T(0)};
            else if constexpr (STREAM)
                x[r] = buf_ld(buf, sb + (a ^ roff[r]));
            else
                x[r] = sig[a ^ roff[r]];
        }
        dft_reg<LR>(x);
        if (logm > 0) {
            // twiddles w^r, w = exp(-2 pi i j / L), as in dif_twiddle (written out here:
            // through the helper, the kernels built on these passes spilled)
            const int sh = logNtw - logL;
            const cplx<T> w1 = tw[j << sh];
            if constexpr (R == 2) {
                x[1] = cmul(x[1], w1);
            } else {
                const cplx<T> w2 = cmul(w1, w1);
                const cplx<T> lo[4] = {cplx<T>{T(1), T(0)}, w1, w2, cmul(w2, w1)};
                if constexpr (R == 4) {
#pragma unroll
                    for (int r = 1; r < 4; ++r) x[r] = cmul(x[r], lo[r]);
                } else {
                    const cplx<T> w4 = tw[(4 * j) << sh];
                    cplx<T> hi[4] = {cplx<T>{T(1), T(0)}, w4, w4, w4};
                    if constexpr (R == 16) {
                        const cplx<T> w8 = tw[(8 * j) << sh];
                        hi[2] = w8;
                        hi[3] = cmul(w8, w4);
                    }
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        const cplx<T> wr = (r >> 2) == 0 ? lo[r & 3]
                                           : ((r & 3) == 0 ? hi[r >> 2] : cmul(lo[r & 3], hi[r >> 2]));
                        x[r] = cmul(x[r], wr);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (STREAM)
                buf_st(buf, sb + (a ^ roff[r]), x[r]);
            else
                sig[a ^ roff[r]] = x[r];
        }
    }
}

// The first pass of a transform in global memory, fused into the stage that makes
// its input: in(s, e) returns input point e of signal s (natural order), and the
// pass's outputs go where fft_pass<LR, T, ZMID, true> would have left them, so the
// input itself is never stored.  With ZMID, in() is not called for the zero middle.
// fft_dif_staged(..., first_done = true) then runs the remaining passes.  in() must
// not read the buffer's other positions' (partly overwritten) contents; the caller
// barriers after.
template <int LR, typename T, bool ZMID, typename In>
__device__ __forceinline__ void fft_first_pass_from(cplx<T> *buf, int nsig, int stride, int logN,
                                                    const cplx<T> *__restrict__ tw, int logNtw, In in) {
    constexpr int R = 1 << LR;
    const int logm = logN - LR, m = 1 << logm;
    const int tid = threadIdx.x, nthr = blockDim.x;
    int roff[R];
#pragma unroll
    for (int r = 0; r < R; ++r) roff[r] = fft_slot<T>(r << logm);
    for (int g = tid; g < (nsig << logm); g += nthr) {
        const int s = g >> logm, j = g & (m - 1);
        const int a = fft_slot<T>(j), sb = s * stride;
        cplx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ZMID && R >= 4 && r >= R / 4 && r < 3 * R / 4)
                x[r] = cplx<T>{T(0), T(0)};
            else
                x[r] = in(s, j + (r << logm));
        }
        dft_reg<LR>(x);
        if (logm > 0) dif_twiddle<LR>(x, j, logN, tw, logNtw);
#pragma unroll
        for (int r = 0; r < R; ++r) buf_st(buf, sb + (a ^ roff[r]), x[r]);
    }
}

// In-place forward FFT (exp(-2 pi i j k / N)).  The caller must barrier
// before (input written) and may read the output right after return.
// zero_mid: the input is zero on points [N/4, 3N/4) and the plan's first radix is at
// least 4; the first pass then reads only the other half (the caller need not clear it).
template <typename T>
__device__ __forceinline__ void fft_dif(cplx<T> *buf, int nsig, int stride, int logN, const cplx<T> *__restrict__ tw,
                        int logNtw, const RadixPlan &rp, bool zero_mid = false) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    int logL = logN;
    const int np = rp.defer2 ? rp.np - 1 : rp.np;
    for (int i = 0; i < np; ++i) {
        const int lr = rp.lr(i);
        if (i == 0 && zero_mid) {
            switch (lr) {
                case 2: fft_pass<2, T, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 3: fft_pass<3, T, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                default: fft_pass<4, T, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
            }
        } else {
            switch (lr) {
                case 1: fft_pass<1, T>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 2: fft_pass<2, T>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 3: fft_pass<3, T>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                default: fft_pass<4, T>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
            }
        }
        logL -= lr;
        __syncthreads();
    }
}

// The same transform of a buffer in global memory, with an LDS stage of 2^logS
// complex elements.  The passes run in global memory only while the sub-transforms
// are longer than the stage; DIF leaves sub-transform q of length L = 2^logL on the
// contiguous positions [qL, (q+1)L), so from there on the remaining passes run on
// whole sub-transforms staged through LDS (as many per fill as the stage holds):
// one read and one write of the buffer instead of one per remaining pass.  The
// passes and their order are those of rp, so the output is the same as fft_dif's
// (consumers read it through dif_pos and fft_slot as usual).  A position's slot
// splits as fft_slot(qL + e) = fft_slot(qL) ^ fft_slot(e) (fft_slot is linear and
// the two have no bits in common), so a staged sub-transform keeps the bank
// swizzle of a transform of length L.  zero_mid as for fft_dif (the staged copy
// of an unwritten middle is never read).  first_done: the first pass has run
// already (fft_first_pass_from; only for a plan with a pass in global memory).
template <typename T>
__device__ __forceinline__ void fft_dif_staged(cplx<T> *buf, int nsig, int stride, int logN,
                                               const cplx<T> *__restrict__ tw, int logNtw, const RadixPlan &rp,
                                               bool zero_mid, cplx<T> *stage, int logS, bool first_done = false) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    int logL = logN, i = 0;
    if (first_done) {   // the first pass ran fused into the input's producer (fft_first_pass_from)
        logL -= rp.lr(0);
        i = 1;
    }
    for (; i < rp.np && logL > logS; ++i) {
        const int lr = rp.lr(i);
        if (i == 0 && zero_mid) {
            switch (lr) {
                case 2: fft_pass<2, T, true, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 3: fft_pass<3, T, true, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                default: fft_pass<4, T, true, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
            }
        } else {
            switch (lr) {
                case 1: fft_pass<1, T, false, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 2: fft_pass<2, T, false, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                case 3: fft_pass<3, T, false, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
                default: fft_pass<4, T, false, true>(buf, nsig, stride, logN, logL, tw, logNtw, tid, nthr); break;
            }
        }
        logL -= lr;
        __syncthreads();
    }
    if (i == rp.np) return;
    const int logB = logL, lgq = logN - logL;       // sub-transform length, log2 of their count per signal
    const int per = 1 << (logS - logB), nsub = nsig << lgq;
    for (int q0 = 0; q0 < nsub; q0 += per) {
        const int cnt = nsub - q0 < per ? nsub - q0 : per;
        for (int e = tid; e < (cnt << logB); e += nthr) {
            const int q = q0 + (e >> logB);
            stage[e] = buf_ld(buf, (q >> lgq) * stride + (fft_slot<T>((q & ((1 << lgq) - 1)) << logB) ^
                                                            (e & ((1 << logB) - 1))));
        }
        __syncthreads();
        int l2 = logB;
        for (int k = i; k < rp.np; ++k) {
            const int lr = rp.lr(k);
            if (k == 0 && zero_mid) {
                switch (lr) {
                    case 2: fft_pass<2, T, true>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                    case 3: fft_pass<3, T, true>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                    default: fft_pass<4, T, true>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                }
            } else {
                switch (lr) {
                    case 1: fft_pass<1, T>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                    case 2: fft_pass<2, T>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                    case 3: fft_pass<3, T>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                    default: fft_pass<4, T>(stage, cnt, 1 << logB, logB, l2, tw, logNtw, tid, nthr); break;
                }
            }
            l2 -= lr;
            __syncthreads();
        }
        for (int e = tid; e < (cnt << logB); e += nthr) {
            const int q = q0 + (e >> logB), el = e & ((1 << logB) - 1);
            int ls = fft_slot<T>(el);        // stage slot of the element stored at local position el
            if (rp.nat == i) {
                // natural order: position el holds local frequency el, which the staged
                // passes left at the digit-reversed local position
                int pos = 0, lL = logB, kk = el;
                for (int k = i; k < rp.np; ++k) {
                    const int lr = rp.lr(k);
                    lL -= lr;
                    pos += (kk & ((1 << lr) - 1)) << lL;
                    kk >>= lr;
                }
                ls = fft_slot<T>(pos);
            }
            buf_st(buf, (q >> lgq) * stride + (fft_slot<T>((q & ((1 << lgq) - 1)) << logB) ^ fft_slot<T>(el)),
                   stage[(e & ~((1 << logB) - 1)) + ls]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Real transforms on top of the complex FFT (per signal, N = 2^logN real
// points).  Twiddle tables hold exp(-2 pi i k / Ntw) with Ntw >= 4N.
// ---------------------------------------------------------------------------

// Makhoul reordering for the DCT-II: v_q = x_{2q} (q < N/2), v_{N-1-q} = x_{2q+1};
// packed complex input Z_m = v_{2m} + i v_{2m+1}, m < N/2.  Returns Z_m, to be
// stored in slot fft_slot(m).
template <typename T, typename Src>
__device__ __forceinline__ cplx<T> dct2_pack(const Src *x, int m, int N) {
    auto vq = [&](int q) -> T { return q < N / 2 ? T(x[2 * q]) : T(x[2 * (N - 1 - q) + 1]); };
    return {vq(2 * m), vq(2 * m + 1)};
}

// The same packing from four consecutive samples x[4t .. 4t+3] (one 16-byte load),
// 0 <= t < N/4: Z_t = x[4t] + i x[4t+2] and Z_{N/2-1-t} = x[4t+3] + i x[4t+1]
// (v_{2t} = x[4t], v_{2t+1} = x[4t+2]; v_{N-2-2t} = x[4t+3], v_{N-1-2t} = x[4t+1]).
__device__ __forceinline__ void dct2_pack4(const float4 x4, cplx<float> &zt, cplx<float> &zr) {
    zt = {x4.x, x4.z};
    zr = {x4.w, x4.y};
}

// Orthonormal DCT-II outputs X_k and X_{N-k} (0 <= k <= N/2) from the FFT of
// the packed sequence (M = N/2 points, digit-reversed per rp).  For k = 0 the
// second output is meaningless; for k = N/2 both are X_{N/2}.
template <typename T>
__device__ __forceinline__ void dct2_post(const cplx<T> *Zh, int k, int logN, const RadixPlan &rp,
                                          const cplx<T> *__restrict__ tw, int logNtw, T &Xk, T &XNk) {
    const int N = 1 << logN, M = N >> 1, logM = logN - 1;
    const cplx<T> a = fft_out(Zh, k & (M - 1), rp, logM);
    const cplx<T> b = cconj(fft_out(Zh, (M - k) & (M - 1), rp, logM));
    const cplx<T> E = cscale(cadd(a, b), T(0.5));
    const cplx<T> O = cdiv2i(csub(a, b));
    const cplx<T> wN = tw[(k << (logNtw - logN)) & ((1 << logNtw) - 1)];
    const cplx<T> V = cadd(E, cmul(wN, O));
    const cplx<T> w4 = tw[k << (logNtw - logN - 2)];
    const cplx<T> P = cmul(w4, V);
    const T c0 = T(1) / sqrt(T(N)), c1 = sqrt(T(2) / T(N));
    Xk = P.re * (k == 0 ? c0 : c1);
    XNk = -P.im * c1;
}

// Inverse of the above: for 0 <= k < M = N/2, the FFT input Zh_k (slot fft_slot(k),
// conjugated so that a forward FFT performs the inverse) built from the
// orthonormal coefficients X (X_k read through get(k)).
template <typename T, typename Get>
__device__ __forceinline__ cplx<T> dct3_pack(Get get, int k, int logN, const cplx<T> *__restrict__ tw,
                                             int logNtw) {
    const int N = 1 << logN, M = N >> 1;
    const T c0 = sqrt(T(N)), c1 = sqrt(T(N) / T(2));   // 1 / c_k
    auto V = [&](int kk) -> cplx<T> {
        // V_kk = exp(+i pi kk / 2N) (X'_kk - i X'_{N-kk}),  X' = X / c
        const T xr = get(kk) * (kk == 0 ? c0 : c1);
        const T xi = kk == 0 ? T(0) : get(N - kk) * c1;
        const cplx<T> w = cconj(tw[kk << (logNtw - logN - 2)]);
        return cmul(w, cplx<T>{xr, -xi});
    };
    const cplx<T> Vk = V(k);
    const cplx<T> Vm = cconj(V(M - k));
    const cplx<T> E = cscale(cadd(Vk, Vm), T(0.5));
    const cplx<T> winv = cconj(tw[(k << (logNtw - logN)) & ((1 << logNtw) - 1)]);
    const cplx<T> O = cmul(cscale(csub(Vk, Vm), T(0.5)), winv);
    const cplx<T> Z = {E.re - O.im, E.im + O.re};     // E + i O
    return cconj(Z);
}

// Output sample q of the inverse DCT: x_{2q} = v_q (q < N/2), x_{2(N-1-q)+1} = v_q,
// where v_{2m} + i v_{2m+1} = conj(FFT(conj Zh))_m / M.  Returns x_j.
template <typename T>
__device__ __forceinline__ T dct3_sample(const cplx<T> *Zf, int j, int logN, const RadixPlan &rp) {
    const int N = 1 << logN, M = N >> 1, logM = logN - 1;
    const int q = (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1);
    const cplx<T> z = fft_out(Zf, q >> 1, rp, logM);
    // conj(z) / M: real part for even q, imaginary part (of the conjugate) for odd q
    return (q & 1) ? (-z.im / T(M)) : (z.re / T(M));
}

// DST-I of length Nn-1 (c_l = 2 sum_{j=1}^{Nn-1} h_j sin(pi j l / Nn)) through
// the FFT of the odd extension u (length 2 Nn) packed into Nn complex points.
// Output c_l for 1 <= l < Nn from the digit-reversed FFT Zh.
template <typename T>
__device__ __forceinline__ T dst1_post(const cplx<T> *Zh, int l, int logNn, const RadixPlan &rp,
                                       const cplx<T> *__restrict__ tw, int logNtw) {
    const int Nn = 1 << logNn;
    const cplx<T> a = fft_out(Zh, l, rp, logNn);
    const cplx<T> b = cconj(fft_out(Zh, Nn - l, rp, logNn));
    const cplx<T> E = cscale(cadd(a, b), T(0.5));
    const cplx<T> O = cdiv2i(csub(a, b));
    const cplx<T> w = tw[l << (logNtw - logNn - 1)];   // exp(-2 pi i l / 2Nn)
    const cplx<T> D = cadd(E, cmul(w, O));
    return -D.im;
}

// ---------------------------------------------------------------------------
// Eigenvalue gaps of the path graph in product form
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sin_half(const double *sintab, int n, int k) {
    // sin(pi k / 2n) for -2n <= k <= 2n, from the table sintab[k] = sin(pi k / 2n), k = 0..2n
    return k >= 0 ? sintab[k] : -sintab[-k];
}

// lambda_j - lambda_o = 4 sin(pi (j - o) / 2n) sin(pi (j + o) / 2n): no cancellation, so
// small gaps keep full relative accuracy
__device__ __forceinline__ double lam_diff(const double *sintab, int n, int j, int o) {
    return 4.0 * sin_half(sintab, n, j - o) * sin_half(sintab, n, j + o);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace dctplus
