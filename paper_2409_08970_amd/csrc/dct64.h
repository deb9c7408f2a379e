// Orthonormal DCT-II (and its transpose, the DCT-III) of length 64 on the
// four lanes that hold one signal in the streaming kernels (lane groups
// g = lane / 16, sixteen values per lane), for the factored dense route of
// Thm 3.1: y = diag(a) C(mu, lambda) diag(z) DCT-II(x).
//
// Method (Makhoul's DCT via one complex FFT of the even/odd reordered signal,
// Cooley-Tukey split 64 = 4 x 16):
//   v[m] = x[2m] (m < 32),  v[m] = x[127 - 2m] (m >= 32);
//   V = FFT_64(v);  X[k] = c_k Re(e^{-i pi k / 128} V[k]).
//   Lane group g holds v[g + 4 m1], m1 = 0..15, and forms the real 16-point
//   DFT F_g of it in registers (stage 1).  V[k1 + 16 k2] =
//   sum_g W64^{g k1} (-i)^{g k2} F_g[k1]: the four values F_0..3[k1] meet in one
//   lane after a 4 x 4 block transposition across the lane groups (stage 2, two
//   rounds of lane-half swaps), where a radix-4 butterfly with twiddles and the
//   final rotation give eight outputs per frequency pair (stage 3).
//   Lane group q handles k1 in {2q + 1, 2q + 2} (q < 3) and {7} plus the two
//   real frequencies k1 = 0, 8 (q = 3): sixteen outputs per lane.
// Every function has a transpose (suffix _t) used by the adjoint, so the
// adjoint is exactly the transposed forward.
#pragma once

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#endif

namespace dctplus {
namespace d64 {

// Sample index of slot m1 of lane group g (the Makhoul reordering).
__host__ __device__ constexpr int in_index(int g, int m1) {
    return (g + 4 * m1) < 32 ? 2 * (g + 4 * m1) : 127 - 2 * (g + 4 * m1);
}

// DCT coefficient index of output slot s of lane group q.  Slots 0..7 belong to
// k1 = 2q + 1, slots 8..15 to k1 = 2q + 2 (q < 3) or to k1 in {0, 8} (q = 3):
// slot 2j -> k1 + 16 j, slot 2j + 1 -> 64 - k1 - 16 j.
__host__ __device__ constexpr int out_index(int q, int s) {
    return (q == 3 && s >= 8) ? (s == 8 ? 0 : s == 9 ? 32 : s == 10 ? 16 : s == 11 ? 48 : s == 12 ? 8
                                 : s == 13 ? 56 : s == 14 ? 24 : 40)
                              : ((s & 1) == 0 ? (2 * q + 1 + (s >> 3)) + 16 * ((s & 7) >> 1)
                                              : 64 - (2 * q + 1 + (s >> 3)) - 16 * ((s & 7) >> 1));
}

struct c2 {
    float r, i;
};
__host__ __device__ inline c2 cadd(c2 a, c2 b) { return {a.r + b.r, a.i + b.i}; }
__host__ __device__ inline c2 csub(c2 a, c2 b) { return {a.r - b.r, a.i - b.i}; }
__host__ __device__ inline c2 cmul(c2 a, c2 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__host__ __device__ inline c2 cmulc(c2 a, c2 b) { return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i}; }  // a conj(b)
__host__ __device__ inline c2 cconj(c2 a) { return {a.r, -a.i}; }
__host__ __device__ inline c2 mul_mi(c2 a) { return {a.i, -a.r}; }   // -i a
__host__ __device__ inline c2 mul_pi(c2 a) { return {-a.i, a.r}; }   // +i a

constexpr float kH = 0.70710678118654752f;   // cos(pi/4)

// In-place complex FFT of length 8, sign -1 (forward) or +1 (unnormalised inverse).
template <int SIGN>
__host__ __device__ inline void fft8(c2 z[8]) {
    // radix-2 decimation in frequency, natural input order, bit-reversed output reordered at the end
    c2 t[8];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        t[p] = cadd(z[p], z[p + 4]);
        t[p + 4] = csub(z[p], z[p + 4]);
    }
    // twiddles e^{SIGN 2 pi i p / 8} on the difference half
    t[5] = {kH * (t[5].r - SIGN * t[5].i), kH * (t[5].i + SIGN * t[5].r)};
    t[6] = (SIGN < 0) ? mul_mi(t[6]) : mul_pi(t[6]);
    t[7] = {-kH * (t[7].r + SIGN * t[7].i), kH * (SIGN * t[7].r - t[7].i)};
    c2 u[8];
#pragma unroll
    for (int h = 0; h < 8; h += 4) {
        u[h] = cadd(t[h], t[h + 2]);
        u[h + 1] = cadd(t[h + 1], t[h + 3]);
        u[h + 2] = csub(t[h], t[h + 2]);
        u[h + 3] = csub(t[h + 1], t[h + 3]);
        u[h + 3] = (SIGN < 0) ? mul_mi(u[h + 3]) : mul_pi(u[h + 3]);
    }
    // last radix-2 stage; outputs in bit-reversed order
    const c2 y0 = cadd(u[0], u[1]), y4 = csub(u[0], u[1]);
    const c2 y2 = cadd(u[2], u[3]), y6 = csub(u[2], u[3]);
    const c2 y1 = cadd(u[4], u[5]), y5 = csub(u[4], u[5]);
    const c2 y3 = cadd(u[6], u[7]), y7 = csub(u[6], u[7]);
    z[0] = y0; z[1] = y1; z[2] = y2; z[3] = y3; z[4] = y4; z[5] = y5; z[6] = y6; z[7] = y7;
}

// e^{-2 pi i k / 16}, k = 0..8
__host__ __device__ inline c2 w16(int k) {
    const float c[9] = {1.0f, 0.92387953251128674f, kH, 0.38268343236508977f, 0.0f,
                        -0.38268343236508977f, -kH, -0.92387953251128674f, -1.0f};
    return {c[k], -c[k <= 4 ? 4 - k : k - 4] * (k <= 4 ? 1.0f : 1.0f) * ((k == 0 || k == 8) ? 0.0f : 1.0f)};
}

// Stage 1: R = packed real DFT-16 of a (F[k] = sum_m a[m] e^{-2 pi i m k / 16}) in the
// block order of the transposition: R[4b .. 4b+3] goes to lane group b:
//   b = 0: 2F1 2F2, b = 1: 2F3 2F4, b = 2: 2F5 2F6 (re, im each), b = 3: 2F7 (re, im), F0, F8.
// The complex frequencies carry a factor 2 (the 1/2 of the half-length split is folded
// into the rotation constants of stage 3).
__host__ __device__ inline void rdft16(const float a[16], float R[16]) {
    c2 z[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) z[p] = {a[2 * p], a[2 * p + 1]};
    fft8<-1>(z);
    R[14] = z[0].r + z[0].i;   // F0
    R[15] = z[0].r - z[0].i;   // F8
    // k and 8 - k share s = z_k + conj z_{8-k} and d = z_k - conj z_{8-k}:
    // 2 F_k = s + w16(k) (-i d),  2 F_{8-k} = conj s + w16(8-k) (-i conj(-d))
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        const float sr = z[k].r + z[8 - k].r, si = z[k].i - z[8 - k].i;
        const float dr = z[k].r - z[8 - k].r, di = z[k].i + z[8 - k].i;
        const c2 w = w16(k), wc = w16(8 - k);
        R[2 * k - 2] = sr + w.r * di + w.i * dr;
        R[2 * k - 1] = si + w.i * di - w.r * dr;
        // for 8 - k: s' = (sr, -si), d' = (-dr, di)
        R[2 * (8 - k) - 2] = sr + wc.r * di - wc.i * dr;
        R[2 * (8 - k) - 1] = -si + wc.i * di + wc.r * dr;
    }
    R[6] = 2.0f * z[4].r;      // 2 F4
    R[7] = -2.0f * z[4].i;
}

// Transpose of rdft16.
__host__ __device__ inline void rdft16_t(const float R[16], float a[16]) {
    // H[k] (k = 1..7) = the transposed coefficients of 2 F_k; H[0] = F0, H[8] = F8
    c2 H[9];
    H[0] = {R[14], 0.0f};
    H[8] = {R[15], 0.0f};
#pragma unroll
    for (int k = 1; k < 8; ++k) H[k] = {R[2 * k - 2], R[2 * k - 1]};
    c2 z[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const c2 hk8 = (k == 0) ? H[8] : cconj(H[8 - k]);   // H[k + 8]
        const c2 s = cadd(H[k], hk8), d = csub(H[k], hk8);
        z[k] = cadd(s, mul_pi(cmulc(d, w16(k))));          // + i e^{+2 pi i k / 16} d
    }
    fft8<1>(z);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        a[2 * p] = z[p].r;
        a[2 * p + 1] = z[p].i;
    }
}

// Lane constants of one general frequency group k1: T_g = W64^{g k1} (g = 1..3) and
// R_j = (c / 2) e^{-i pi (k1 + 16 j) / 128} (j = 0..3), c = sqrt(2/64).
struct GroupConst {
    c2 t1, t2, t3, r0, r1, r2, r3;
};

// Constants of frequency group k1 (computed in FP64, rounded once).
__host__ __device__ inline GroupConst group_const(int k1) {
    // c = sqrt(2/64) / 2: the general groups' inputs carry the factor 2 of stage 1
    const double pi = 3.14159265358979323846, c = 0.5 * 0.17677669529663688;
    auto w = [&](double turns, double scale) -> c2 {
        return {(float)(scale * ::cos(2.0 * pi * turns)), (float)(-scale * ::sin(2.0 * pi * turns))};
    };
    GroupConst k;
    k.t1 = w(k1 / 64.0, 1.0);
    k.t2 = w(2.0 * k1 / 64.0, 1.0);
    k.t3 = w(3.0 * k1 / 64.0, 1.0);
    k.r0 = w(k1 / 256.0, c);
    k.r1 = w((k1 + 16) / 256.0, c);
    k.r2 = w((k1 + 32) / 256.0, c);
    k.r3 = w((k1 + 48) / 256.0, c);
    return k;
}

// General group: F_g (g = 0..3, complex, at T[4g + off], T[4g + off + 1]) -> 8 outputs.
__host__ __device__ inline void group_fwd(const float T[16], int off, const GroupConst &k, float out[8]) {
    const c2 g0 = {T[off], T[off + 1]};
    const c2 g1 = cmul(k.t1, {T[4 + off], T[5 + off]});
    const c2 g2 = cmul(k.t2, {T[8 + off], T[9 + off]});
    const c2 g3 = cmul(k.t3, {T[12 + off], T[13 + off]});
    const c2 s02 = cadd(g0, g2), d02 = csub(g0, g2), s13 = cadd(g1, g3), d13 = csub(g1, g3);
    const c2 y0 = cmul(k.r0, cadd(s02, s13));
    const c2 y1 = cmul(k.r1, cadd(d02, mul_mi(d13)));
    const c2 y2 = cmul(k.r2, csub(s02, s13));
    const c2 y3 = cmul(k.r3, cadd(d02, mul_pi(d13)));
    out[0] = y0.r; out[1] = -y0.i; out[2] = y1.r; out[3] = -y1.i;
    out[4] = y2.r; out[5] = -y2.i; out[6] = y3.r; out[7] = -y3.i;
}

__host__ __device__ inline void group_adj(const float in[8], const GroupConst &k, float T[16], int off) {
    const c2 v0 = cmulc({in[0], -in[1]}, k.r0);
    const c2 v1 = cmulc({in[2], -in[3]}, k.r1);
    const c2 v2 = cmulc({in[4], -in[5]}, k.r2);
    const c2 v3 = cmulc({in[6], -in[7]}, k.r3);
    const c2 s02 = cadd(v0, v2), d02 = csub(v0, v2), s13 = cadd(v1, v3), d13 = csub(v1, v3);
    const c2 g0 = cadd(s02, s13);
    const c2 g1 = cmulc(cadd(d02, mul_pi(d13)), k.t1);
    const c2 g2 = cmulc(csub(s02, s13), k.t2);
    const c2 g3 = cmulc(cadd(d02, mul_mi(d13)), k.t3);
    T[off] = g0.r; T[off + 1] = g0.i;
    T[4 + off] = g1.r; T[5 + off] = g1.i;
    T[8 + off] = g2.r; T[9 + off] = g2.i;
    T[12 + off] = g3.r; T[13 + off] = g3.i;
}

// The real frequencies k1 = 0 and 8 (lane group 3): f0_g = T[4g + 2], f8_g = T[4g + 3].
// Outputs in slot order X0, X32, X16, X48, X8, X56, X24, X40.
constexpr float kC0 = 0.125f;                         // sqrt(1/64)
constexpr float kC = 0.17677669529663688f;            // sqrt(2/64)
constexpr c2 kR16 = {0.92387953251128674f * kC, -0.38268343236508977f * kC};   // c e^{-i pi 16/128}
constexpr c2 kR8 = {0.98078528040323043f * kC, -0.19509032201612825f * kC};   // c e^{-i pi 8/128}
constexpr c2 kR24 = {0.83146961230254524f * kC, -0.55557023301960218f * kC};   // c e^{-i pi 24/128}

__host__ __device__ inline void special_fwd(const float T[16], float out[8]) {
    const float a0 = T[2], a1 = T[6], a2 = T[10], a3 = T[14];
    const float b0 = T[3], b1 = T[7], b2 = T[11], b3 = T[15];
    const c2 v16 = {a0 - a2, a3 - a1};
    const c2 v8 = {b0 + kH * (b1 - b3), -kH * (b1 + b3) - b2};
    const c2 v24 = {b0 - kH * (b1 - b3), -kH * (b1 + b3) + b2};
    const c2 y16 = cmul(kR16, v16), y8 = cmul(kR8, v8), y24 = cmul(kR24, v24);
    out[0] = kC0 * ((a0 + a2) + (a1 + a3));
    out[1] = kC * kH * ((a0 + a2) - (a1 + a3));
    out[2] = y16.r; out[3] = -y16.i;
    out[4] = y8.r; out[5] = -y8.i;
    out[6] = y24.r; out[7] = -y24.i;
}

__host__ __device__ inline void special_adj(const float in[8], float T[16]) {
    const float s = kC0 * in[0], d = kC * kH * in[1];
    const c2 v16 = cmulc({in[2], -in[3]}, kR16);
    const c2 v8 = cmulc({in[4], -in[5]}, kR8);
    const c2 v24 = cmulc({in[6], -in[7]}, kR24);
    T[2] = s + d + v16.r;
    T[6] = s - d - v16.i;
    T[10] = s + d - v16.r;
    T[14] = s - d + v16.i;
    const float pr = v8.r + v24.r, mr = v8.r - v24.r, pi = v8.i + v24.i, mi = v8.i - v24.i;
    T[3] = pr;
    T[7] = kH * (mr - pi);
    T[11] = -mi;
    T[15] = -kH * (mr + pi);
}

#ifdef __HIPCC__
// Stage 2: the 4 x 4 block transposition across the lane groups of a wave.
__device__ __forceinline__ void xpose_lane_groups(float R[16]) {
    // block b (R[4b .. 4b+3]) of lane group g goes to lane group b, where it lands in
    // block g: two rounds of lane-half swaps (lanes 0-31 <-> 32-63, then rows of 16)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(R[4 * b + e]),
                                                            __float_as_uint(R[4 * (b + 2) + e]), false, false);
            R[4 * b + e] = __uint_as_float(r[0]);
            R[4 * (b + 2) + e] = __uint_as_float(r[1]);
        }
#pragma unroll
    for (int b = 0; b < 4; b += 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(R[4 * b + e]),
                                                            __float_as_uint(R[4 * (b + 1) + e]), false, false);
            R[4 * b + e] = __uint_as_float(r[0]);
            R[4 * (b + 1) + e] = __uint_as_float(r[1]);
        }
}
#endif

}  // namespace d64
}  // namespace dctplus
