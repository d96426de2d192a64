// ols_fft.hip -- gfx950 kernels for overlap-save variable-bandwidth filtering
// with HFSO coefficients (Moryakova & Johansson, arXiv 2406.14116).
//
// One workgroup (256 threads, 4 waves) owns one 4096-value tile: 4096/N
// consecutive OLS blocks of one channel.  Each block is handled by a team of
// N/16 threads and every thread holds 16 complex float32 values in registers.
// Per block (Sec. II, steps 1-4):
//   1. gather: thread t loads segment samples t + (N/16) v, v < 16 (coalesced
//      across the team; zero outside [0, len));
//   2. forward DFT as Stockham autosort passes: radix-16 passes, then one pass
//      of radix 2/4/8 when log2 N is not a multiple of 4; passes exchange data
//      through the padded LDS tile; the last pass leaves X(t + (N/16) v) in
//      registers;
//   3. multiply by H_R (Sec. III-B, eq. (6)): only the bin index decides
//      between 1 (passband), V(r) (transition) and 0 (stopband); the 1/N of the
//      inverse (eq. (4)) is folded in here;
//   4. inverse DFT as the adjoint of step 2 (same index maps and twiddles,
//      conjugated, in reverse order), ending with z0(t + (N/16) v) in registers;
//   5. the linear phase exp(-j 2 pi k D / N) of eq. (5) is a circular delay by
//      D = (N - M)/2, so the kept output samples N-M+j of the phased inverse are
//      samples D + j of z0: thread t stores v where 0 <= t + (N/16) v - D < M.
// Twiddles come from one float32 table w_4096^r (generated in float64 on the
// host, rounded to nearest).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "vbw_internal.h"

namespace vbw {
namespace {

typedef float f2v __attribute__((ext_vector_type(2)));
// Channel buffers are plain device allocations: address them as global memory
// (address space 1) so loads and stores use the global, not the flat, path.
#define VBW_GLOBAL __attribute__((address_space(1)))
typedef VBW_GLOBAL f2v gf2v;
typedef VBW_GLOBAL uint32_t gu32;

// ---------------------------------------------------------------- complex ops
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 w) {  // a * conj(w)
    return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
template <bool INV> __device__ __forceinline__ float2 tmul(float2 a, float2 w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}
// a * (-j) forward, a * (+j) inverse
template <bool INV> __device__ __forceinline__ float2 rotj(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos and sin of 2 pi e / 16, e < 16 (float32 nearest of the exact values).
__host__ __device__ constexpr float c16(int e) {
    constexpr float c[16] = {
        1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
        0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
        -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f,
        0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f};
    return c[e & 15];
}
__host__ __device__ constexpr float s16(int e) { return c16(e + 12); }  // sin x = cos(x - pi/2)

// a * w16^E with w16 = exp(-j 2 pi / 16) (forward) or its conjugate (inverse).
template <bool INV, int E> __device__ __forceinline__ float2 w16mul(float2 a) {
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
        // +-sqrt(1/2) (+-1 +- j): two adds and two multiplies
        constexpr float h = 0.707106781186547524f;
        constexpr float c = c16(e);
        constexpr float s = INV ? s16(e) : -s16(e);
        // (x + j y)(c + j s) with |c| = |s| = h
        const float p = (c > 0 ? a.x : -a.x) - (s > 0 ? a.y : -a.y);
        const float q = (s > 0 ? a.x : -a.x) + (c > 0 ? a.y : -a.y);
        return make_float2(h * p, h * q);
    } else {
        constexpr float c = c16(e);
        constexpr float s = INV ? s16(e) : -s16(e);
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// ------------------------------------------------------------- small DFTs
// In place, natural order in and out: a[s] <- sum_r a[r] w_R^{r s}.
template <bool INV> __device__ __forceinline__ void dft2(float2 &a0, float2 &a1) {
    const float2 t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <bool INV> __device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const float2 t2 = cadd(a1, a3), t3 = rotj<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV, int R2, int S1> __device__ __forceinline__ void tw16_step(float2 (&a)[16]) {
    a[R2 + 4 * S1] = w16mul<INV, R2 * S1>(a[R2 + 4 * S1]);
}

// 16 = 4 x 4: r = 4 r1 + r2, s = s1 + 4 s2.
template <bool INV> __device__ __forceinline__ void dft16(float2 (&a)[16]) {
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2) dft4<INV>(a[r2], a[4 + r2], a[8 + r2], a[12 + r2]);
    // slot r2 + 4 s1 now holds the inner DFT over r1 at s1; twiddle w16^{r2 s1}
    tw16_step<INV, 1, 1>(a); tw16_step<INV, 1, 2>(a); tw16_step<INV, 1, 3>(a);
    tw16_step<INV, 2, 1>(a); tw16_step<INV, 2, 2>(a); tw16_step<INV, 2, 3>(a);
    tw16_step<INV, 3, 1>(a); tw16_step<INV, 3, 2>(a); tw16_step<INV, 3, 3>(a);
#pragma unroll
    for (int s1 = 0; s1 < 4; ++s1) dft4<INV>(a[4 * s1], a[4 * s1 + 1], a[4 * s1 + 2], a[4 * s1 + 3]);
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
template <bool INV> __device__ __forceinline__ void dft8(float2 (&a)[8]) {
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

template <int R, bool INV> __device__ __forceinline__ void dft_small(float2 (&a)[R]) {
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

// ------------------------------------------------------------ storage
template <Storage S> struct Io;

template <> struct Io<Storage::C64> {
    __device__ static float2 ld(const void *base, int64_t i) {
        const f2v v = __builtin_nontemporal_load((const gf2v *)base + i);
        return make_float2(v.x, v.y);
    }
};

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <> struct Io<Storage::F16> {
    __device__ static float2 ld(const void *base, int64_t i) {
        const uint32_t u = __builtin_nontemporal_load((const gu32 *)base + i);
        const __half2 h = __builtin_bit_cast(__half2, u);
        return __half22float2(h);
    }
};

template <> struct Io<Storage::BF16> {
    __device__ static float2 ld(const void *base, int64_t i) {
        const uint32_t u = __builtin_nontemporal_load((const gu32 *)base + i);
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    }
};

template <Storage S, bool F32OUT> __device__ __forceinline__ void st(void *base, int64_t i, float2 v) {
    if constexpr (S == Storage::C64 || F32OUT) {
        __builtin_nontemporal_store(f2v{v.x, v.y}, (gf2v *)base + i);
    } else if constexpr (S == Storage::F16) {
        const __half2 h = __float22half2_rn(v);
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, h), (gu32 *)base + i);
    } else {
        const uint32_t u = f32_to_bf16_rne(v.x) | (f32_to_bf16_rne(v.y) << 16);
        __builtin_nontemporal_store(u, (gu32 *)base + i);
    }
}

// ------------------------------------------------------------ tile sync
// A team of <= 64 threads lives in one wave: LDS accesses of one wave are
// performed in program order, so ordering the compiler is enough.  Larger
// teams span waves and need the workgroup barrier.
template <bool WAVE_LOCAL> __device__ __forceinline__ void tile_sync() {
    if constexpr (WAVE_LOCAL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// ------------------------------------------------------------ passes
template <int LOG2N> struct Shape {
    static constexpr int N = 1 << LOG2N;
    static constexpr int T = N / 16;                 // threads per block
    static constexpr int N16 = LOG2N / 4;            // radix-16 passes
    static constexpr int REM = LOG2N % 4;
    static constexpr int NP = N16 + (REM ? 1 : 0);   // passes
    static constexpr int RLAST = REM ? (1 << REM) : 16;
    static constexpr bool WAVE_LOCAL = T <= 64;
    static constexpr int TWS = kTwiddleN / N;        // table stride of w_N
};

__device__ __forceinline__ float2 twiddle(const float2 *__restrict__ tw, int idx) { return tw[idx]; }

// Middle radix-16 pass Q (2 <= Q, not the last): Ns = 16^(Q-1).
// Forward: gather t + T r, twiddle w_{16 Ns}^{j r} (j = t mod Ns), DFT,
// scatter to (t/Ns) 16 Ns + j + Ns s.
template <int LOG2N, int Q, bool INV>
__device__ __forceinline__ void mid_pass(float2 (&a)[16], float2 *L, int t, const float2 *__restrict__ tw) {
    using Sh = Shape<LOG2N>;
    constexpr int NS = 1 << (4 * (Q - 1));
    constexpr int STRIDE = kTwiddleN / (16 * NS);
    const int j = t & (NS - 1);
    const int sbase = (t / NS) * NS * 16 + j;
    if constexpr (!INV) {
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = L[lds_pad(t + Sh::T * r)];
#pragma unroll
        for (int r = 1; r < 16; ++r) a[r] = cmul(a[r], twiddle(tw, STRIDE * j * r));
        dft16<false>(a);
        tile_sync<Sh::WAVE_LOCAL>();
#pragma unroll
        for (int s = 0; s < 16; ++s) L[lds_pad(sbase + NS * s)] = a[s];
        tile_sync<Sh::WAVE_LOCAL>();
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) a[s] = L[lds_pad(sbase + NS * s)];
        dft16<true>(a);
#pragma unroll
        for (int r = 1; r < 16; ++r) a[r] = cmulc(a[r], twiddle(tw, STRIDE * j * r));
        tile_sync<Sh::WAVE_LOCAL>();
#pragma unroll
        for (int r = 0; r < 16; ++r) L[lds_pad(t + Sh::T * r)] = a[r];
        tile_sync<Sh::WAVE_LOCAL>();
    }
}

template <int LOG2N, int Q, bool INV>
__device__ __forceinline__ void mid_passes(float2 (&a)[16], float2 *L, int t, const float2 *__restrict__ tw) {
    using Sh = Shape<LOG2N>;
    constexpr int LASTMID = Sh::NP - 1;   // passes 2 .. NP-1 are middle passes
    if constexpr (Q <= LASTMID) {
        if constexpr (!INV) {
            mid_pass<LOG2N, Q, false>(a, L, t, tw);
            mid_passes<LOG2N, Q + 1, false>(a, L, t, tw);
        } else {
            mid_passes<LOG2N, Q + 1, true>(a, L, t, tw);
            mid_pass<LOG2N, Q, true>(a, L, t, tw);
        }
    }
}

// Last pass, entirely in registers: butterfly b = t + T u (u < 16/R) has its R
// inputs in slots u + (16/R) r, twiddle w_N^{b r} (Ns = N/R, j = b), outputs
// X(b + (N/R) s) in slots u + (16/R) s.  For N = 16 this is the only pass and
// has no twiddle.
template <int LOG2N, bool INV>
__device__ __forceinline__ void last_pass(float2 (&a)[16], int t, const float2 *__restrict__ tw) {
    using Sh = Shape<LOG2N>;
    constexpr int R = Sh::RLAST;
    constexpr int U = 16 / R;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = t + Sh::T * u;
        float2 c[R];
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = a[u + U * r];
        if constexpr (!INV && Sh::NP > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) c[r] = cmul(c[r], twiddle(tw, Sh::TWS * b * r));
        }
        dft_small<R, INV>(c);
        if constexpr (INV && Sh::NP > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) c[r] = cmulc(c[r], twiddle(tw, Sh::TWS * b * r));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a[u + U * r] = c[r];
    }
}

// H_R of eq. (6) with the mirror H_R(N-k) = H_R(k), times 1/N.
// Slot v holds bin k = t + T v.
template <int LOG2N>
__device__ __forceinline__ void hfso_multiply(float2 (&a)[16], int t, int k1, int lv,
                                              const float *__restrict__ vv) {
    using Sh = Shape<LOG2N>;
    constexpr float inv_n = 1.0f / float(Sh::N);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int k = t + Sh::T * v;
        const int kk = (k <= Sh::N / 2) ? k : Sh::N - k;
        const int jj = kk - k1;
        float f = (jj < 0) ? inv_n : 0.0f;
        if (jj >= 0 && jj < lv) f = vv[jj] * inv_n;
        a[v].x *= f;
        a[v].y *= f;
    }
}

template <int LOG2N, Storage S, bool F32OUT>
__device__ __forceinline__ void process_item(const LaunchArgs &A, const WorkItem &it, float2 *lds) {
    using Sh = Shape<LOG2N>;
    constexpr int N = Sh::N, T = Sh::T;
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid - team * T;
    float2 *L = lds + team * lds_pad(N);

    const ChannelDev cd = A.ch[it.channel];
    const int64_t m = int64_t(it.first_block) + team;
    const bool active = team < it.n_blocks;
    const int hop = cd.hop;
    const int d = (N - hop) >> 1;

    // k1 in force for block m: last schedule entry with from_block <= m
    int k1 = A.sched[cd.sched_begin].k1;
    for (int e = 1; e < cd.sched_count; ++e) {
        const SchedDev sd = A.sched[cd.sched_begin + e];
        if (sd.from_block <= m) k1 = sd.k1;
    }

    // step 1: gather the segment [m hop - (N - hop), m hop + hop)
    float2 a[16];
    const int64_t base = m * hop - (N - hop);
    const void *x = A.x[it.channel];
    if (active && base >= 0 && base + N <= cd.len) {
#pragma unroll
        for (int v = 0; v < 16; ++v) a[v] = Io<S>::ld(x, base + t + T * v);
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t i = base + t + T * v;
            a[v] = (active && i >= 0 && i < cd.len) ? Io<S>::ld(x, i) : make_float2(0.f, 0.f);
        }
    }

    // step 2: forward DFT
    if constexpr (Sh::NP == 1) {
        last_pass<LOG2N, false>(a, t, A.tw);
    } else {
        dft16<false>(a);                                  // pass 1, Ns = 1
#pragma unroll
        for (int s = 0; s < 16; ++s) L[lds_pad(16 * t + s)] = a[s];
        tile_sync<Sh::WAVE_LOCAL>();
        mid_passes<LOG2N, 2, false>(a, L, t, A.tw);
#pragma unroll
        for (int v = 0; v < 16; ++v) a[v] = L[lds_pad(t + T * v)];
        last_pass<LOG2N, false>(a, t, A.tw);
    }

    // step 3: H_R and 1/N
    hfso_multiply<LOG2N>(a, t, k1, cd.lv, A.v + cd.v_offset);

    // step 4: inverse DFT (adjoint passes)
    last_pass<LOG2N, true>(a, t, A.tw);
    if constexpr (Sh::NP > 1) {
#pragma unroll
        for (int v = 0; v < 16; ++v) L[lds_pad(t + T * v)] = a[v];
        tile_sync<Sh::WAVE_LOCAL>();
        mid_passes<LOG2N, 2, true>(a, L, t, A.tw);
#pragma unroll
        for (int s = 0; s < 16; ++s) a[s] = L[lds_pad(16 * t + s)];
        dft16<true>(a);
    }

    // step 5: keep z0(D + j), j < hop, within len
    if (active) {
        void *y = A.y[it.channel];
        const int64_t obase = m * hop;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = t + T * v - d;
            if (unsigned(j) < unsigned(hop) && obase + j < cd.len) st<S, F32OUT>(y, obase + j, a[v]);
        }
    }
}

__device__ __forceinline__ int item_index(const LaunchArgs &A) {
    int wg = blockIdx.x;
    if (A.xcd_remap) {
        // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
        // contiguous run of items so neighbouring blocks share its L2.
        const int nwg = gridDim.x, q = nwg >> 3, r = nwg & 7;
        const int xcd = wg & 7, idx = wg >> 3;
        wg = xcd * q + min(xcd, r) + idx;
    }
    return wg;
}

template <int LOG2N, Storage S, bool F32OUT>
__global__ __launch_bounds__(kThreads) void ols_fft_kernel(const LaunchArgs A) {
    __shared__ float2 lds[kLdsValues];
    const WorkItem it = A.items[item_index(A)];
    if constexpr (LOG2N != 0) {
        process_item<LOG2N, S, F32OUT>(A, it, lds);
    } else {
        switch (it.log2n) {
            case 4: process_item<4, S, F32OUT>(A, it, lds); break;
            case 5: process_item<5, S, F32OUT>(A, it, lds); break;
            case 6: process_item<6, S, F32OUT>(A, it, lds); break;
            case 7: process_item<7, S, F32OUT>(A, it, lds); break;
            case 8: process_item<8, S, F32OUT>(A, it, lds); break;
            case 9: process_item<9, S, F32OUT>(A, it, lds); break;
            case 10: process_item<10, S, F32OUT>(A, it, lds); break;
            case 11: process_item<11, S, F32OUT>(A, it, lds); break;
            case 12: process_item<12, S, F32OUT>(A, it, lds); break;
            default: break;
        }
    }
}

template <Storage S, bool F32OUT>
hipError_t launch_typed(const LaunchArgs &A, int log2n, hipStream_t stream) {
    const dim3 grid(A.n_items), block(kThreads);
    switch (log2n) {
        case 0: hipLaunchKernelGGL((ols_fft_kernel<0, S, F32OUT>), grid, block, 0, stream, A); break;
        case 4: hipLaunchKernelGGL((ols_fft_kernel<4, S, F32OUT>), grid, block, 0, stream, A); break;
        case 5: hipLaunchKernelGGL((ols_fft_kernel<5, S, F32OUT>), grid, block, 0, stream, A); break;
        case 6: hipLaunchKernelGGL((ols_fft_kernel<6, S, F32OUT>), grid, block, 0, stream, A); break;
        case 7: hipLaunchKernelGGL((ols_fft_kernel<7, S, F32OUT>), grid, block, 0, stream, A); break;
        case 8: hipLaunchKernelGGL((ols_fft_kernel<8, S, F32OUT>), grid, block, 0, stream, A); break;
        case 9: hipLaunchKernelGGL((ols_fft_kernel<9, S, F32OUT>), grid, block, 0, stream, A); break;
        case 10: hipLaunchKernelGGL((ols_fft_kernel<10, S, F32OUT>), grid, block, 0, stream, A); break;
        case 11: hipLaunchKernelGGL((ols_fft_kernel<11, S, F32OUT>), grid, block, 0, stream, A); break;
        case 12: hipLaunchKernelGGL((ols_fft_kernel<12, S, F32OUT>), grid, block, 0, stream, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ols_fft(const LaunchArgs &A, int log2n_fixed, Storage in, bool f32_out,
                          hipStream_t stream) {
    if (A.n_items <= 0) return hipSuccess;
    switch (in) {
        case Storage::C64: return launch_typed<Storage::C64, false>(A, log2n_fixed, stream);
        case Storage::F16:
            return f32_out ? launch_typed<Storage::F16, true>(A, log2n_fixed, stream)
                           : launch_typed<Storage::F16, false>(A, log2n_fixed, stream);
        case Storage::BF16:
            return f32_out ? launch_typed<Storage::BF16, true>(A, log2n_fixed, stream)
                           : launch_typed<Storage::BF16, false>(A, log2n_fixed, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace vbw
