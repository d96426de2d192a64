// fft_small.h -- in-register complex float32 DFTs of size 2, 4, 8 and 16 for
// the FFT passes of the overlap-save filter (eq. (4): forward exp(-j 2 pi k n / N),
// inverse exp(+j 2 pi k n / N); the inverse's 1/N is applied elsewhere).
// Host and device: the host build lets the CPU tests check these butterflies
// against a float64 DFT.
#pragma once

#include <hip/hip_runtime.h>

#define VBW_HD __host__ __device__ __forceinline__

namespace vbw {
namespace fft {

VBW_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
VBW_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
VBW_HD float2 cmul(float2 a, float2 w) { return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x); }
VBW_HD float2 cmulc(float2 a, float2 w) {  // a * conj(w)
    return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
template <bool INV> VBW_HD float2 tmul(float2 a, float2 w) { return INV ? cmulc(a, w) : cmul(a, w); }
// a * (-j) forward, a * (+j) inverse
template <bool INV> VBW_HD float2 rotj(float2 a) { return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }
// t + h p, t - h p (component-wise, one multiply-add each)
VBW_HD float2 cfma(float h, float2 p, float2 t) { return make_float2(fmaf(h, p.x, t.x), fmaf(h, p.y, t.y)); }
VBW_HD float2 cfms(float h, float2 p, float2 t) { return make_float2(fmaf(-h, p.x, t.x), fmaf(-h, p.y, t.y)); }

// cos and sin of 2 pi e / 16, e < 16 (float32 nearest of the exact values).
VBW_HD constexpr float c16(int e) {
    constexpr float c[16] = {
        1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
        0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
        -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f,
        0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f};
    return c[e & 15];
}
VBW_HD constexpr float s16(int e) { return c16(e + 12); }  // sin x = cos(x - pi/2)

constexpr float kH = 0.707106781186547524f;   // cos(pi/4)
constexpr float kC1 = 0.923879532511286756f;  // cos(pi/8)
constexpr float kT1 = 0.414213562373095049f;  // tan(pi/8)

// For e = 2 or 6 (angles of +-45 degrees, odd multiples of pi/4) the product
// a w16^e is kH times the returned value: two additions, no multiply.
template <bool INV, int E> VBW_HD float2 w16_diag(float2 a) {
    constexpr int e = E & 15;
    static_assert((e & 3) == 2, "odd multiple of pi/4");
    constexpr float c = c16(e) > 0 ? 1.f : -1.f;
    constexpr float s = (INV ? s16(e) : -s16(e)) > 0 ? 1.f : -1.f;
    // (x + j y)(c + j s) with c, s = +-1
    return make_float2(c * a.x - s * a.y, s * a.x + c * a.y);
}

// a * w16^E with w16 = exp(-j 2 pi / 16) (forward) or its conjugate (inverse).
template <bool INV, int E> VBW_HD float2 w16mul(float2 a) {
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return rotj<INV>(a);
    } else if constexpr (e == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (e == 12) {
        return rotj<!INV>(a);
    } else if constexpr ((e & 1) == 0) {
        const float2 p = w16_diag<INV, e>(a);
        return make_float2(kH * p.x, kH * p.y);
    } else {
        constexpr float c = c16(e);
        constexpr float s = INV ? s16(e) : -s16(e);
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// ------------------------------------------------------------- small DFTs
// In place, natural order in and out: a[s] <- sum_r a[r] w_R^{r s}.
template <bool INV> VBW_HD void dft2(float2 &a0, float2 &a1) {
    const float2 t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <bool INV> VBW_HD void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const float2 t2 = cadd(a1, a3), t3 = rotj<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// Final radix-4 combination out = {t0 + g u, t1 + g v, t0 - g u, t1 - g v}
// (u = b1 + b3 and v = -j(b1 - b3) forward, already divided by g).
VBW_HD void fin4(float2 &a0, float2 &a1, float2 &a2, float2 &a3, float2 t0, float2 t1, float g, float2 u,
                 float2 v) {
    a0 = cfma(g, u, t0);
    a2 = cfms(g, u, t0);
    a1 = cfma(g, v, t1);
    a3 = cfms(g, v, t1);
}

// 16 = 4 x 4: r = 4 r1 + r2, s = s1 + 4 s2.  The inner twiddles w16^{r2 s1}
// are folded into the second radix-4 stage: a product by cos(pi/4), cos(pi/8)
// or -cos(pi/8) is pulled out of each butterfly's sum and difference and
// applied by the final multiply-adds, and the remaining tangent factors are
// tan(pi/8) (a multiply by w16^e = C (1 + j S/C) = S (C/S + j); whichever of
// |C|, |S| is larger is pulled out).  This saves 16 of the 160 operations of
// the plain twiddle-then-butterfly form.
template <bool INV> VBW_HD void dft16(float2 (&a)[16]) {
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) dft4<INV>(a[r2], a[4 + r2], a[8 + r2], a[12 + r2]);
    // slot r2 + 4 s1 now holds the inner DFT over r1 at s1
    constexpr float sg = INV ? 1.f : -1.f;   // sign of the sine in w16^e
    constexpr float tau = sg * kT1;
    // s1 = 0: no twiddles
    dft4<INV>(a[0], a[1], a[2], a[3]);
    // s1 = 1: b0 = a4, b1 = a5 w, b2 = a6 w^2, b3 = a7 w^3
    {
        const float2 p2 = w16_diag<INV, 2>(a[6]);                 // a6 w^2 = kH p2
        const float2 t0 = cfma(kH, p2, a[4]), t1 = cfms(kH, p2, a[4]);
        // a5 w^1 = kC1 z1, z1 = a5 (1 + j tau)
        const float2 z1 = make_float2(fmaf(-a[5].y, tau, a[5].x), fmaf(a[5].x, tau, a[5].y));
        // a7 w^3 = sg kC1 z3, z3 = a7 (tau' + j) with tau' = cos/sin = sg tan(pi/8)
        const float2 z3 = make_float2(fmaf(a[7].x, tau, -a[7].y), fmaf(a[7].y, tau, a[7].x));
        // b1 + b3 = kC1 (z1 + sg z3), b1 - b3 = kC1 (z1 - sg z3)
        const float2 u = INV ? cadd(z1, z3) : csub(z1, z3);
        const float2 d = INV ? csub(z1, z3) : cadd(z1, z3);
        fin4(a[4], a[5], a[6], a[7], t0, t1, kC1, u, rotj<INV>(d));
    }
    // s1 = 2: b0 = a8, b1 = a9 w^2, b2 = a10 w^4 = a10 (-+j), b3 = a11 w^6 = (a11 w^4) w^2
    {
        const float2 b2 = rotj<INV>(a[10]);
        const float2 t0 = cadd(a[8], b2), t1 = csub(a[8], b2);
        const float2 r3 = rotj<INV>(a[11]);
        // b1 +- b3 = (a9 +- r3) w^2 = kH diag(a9 +- r3)
        const float2 u = w16_diag<INV, 2>(cadd(a[9], r3));
        const float2 d = w16_diag<INV, 2>(csub(a[9], r3));
        fin4(a[8], a[9], a[10], a[11], t0, t1, kH, u, rotj<INV>(d));
    }
    // s1 = 3: b0 = a12, b1 = a13 w^3, b2 = a14 w^6, b3 = a15 w^9
    {
        const float2 p2 = w16_diag<INV, 6>(a[14]);                // a14 w^6 = kH p2
        const float2 t0 = cfma(kH, p2, a[12]), t1 = cfms(kH, p2, a[12]);
        // a13 w^3 = sg kC1 z1, z1 = a13 (tau' + j)
        const float2 z1 = make_float2(fmaf(a[13].x, tau, -a[13].y), fmaf(a[13].y, tau, a[13].x));
        // a15 w^9 = -kC1 z3, z3 = a15 (1 + j tau) (w^9 = -w^1)
        const float2 z3 = make_float2(fmaf(-a[15].y, tau, a[15].x), fmaf(a[15].x, tau, a[15].y));
        // b1 + b3 = kC1 (sg z1 - z3), b1 - b3 = kC1 (sg z1 + z3)
        const float2 u = INV ? csub(z1, z3) : make_float2(-z1.x - z3.x, -z1.y - z3.y);
        const float2 d = INV ? cadd(z1, z3) : csub(z3, z1);
        fin4(a[12], a[13], a[14], a[15], t0, t1, kC1, u, rotj<INV>(d));
    }
    // slot 4 s1 + s2 holds Y(s1 + 4 s2): transpose the 4 x 4 register grid
    float2 b[16];
#pragma unroll
    for (int s1 = 0; s1 < 4; ++s1)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) b[s1 + 4 * s2] = a[4 * s1 + s2];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = b[i];
}

// 8 = 4 x 2: r = 2 r1 + r2, s = s1 + 4 s2.
template <bool INV> VBW_HD void dft8(float2 (&a)[8]) {
    dft4<INV>(a[0], a[2], a[4], a[6]);
    dft4<INV>(a[1], a[3], a[5], a[7]);
    a[3] = w16mul<INV, 2>(a[3]);
    a[5] = w16mul<INV, 4>(a[5]);
    a[7] = w16mul<INV, 6>(a[7]);
#pragma unroll
    for (int s1 = 0; s1 < 4; ++s1) dft2<INV>(a[2 * s1], a[2 * s1 + 1]);
    float2 b[8];
#pragma unroll
    for (int s1 = 0; s1 < 4; ++s1) {
        b[s1] = a[2 * s1];
        b[s1 + 4] = a[2 * s1 + 1];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = b[i];
}

template <int R, bool INV> VBW_HD void dft_small(float2 (&a)[R]) {
    if constexpr (R == 2) {
        dft2<INV>(a[0], a[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        dft8<INV>(a);
    } else {
        dft16<INV>(a);
    }
}

}  // namespace fft
}  // namespace vbw
