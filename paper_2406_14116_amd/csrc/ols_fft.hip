// ols_fft.hip -- gfx950 kernels for overlap-save variable-bandwidth filtering
// with HFSO coefficients (Moryakova & Johansson, arXiv 2406.14116).
//
// A persistent workgroup (256 threads, 4 waves) holds 4096/N teams of N/16
// threads; every thread holds 16 complex float32 values in registers and each
// team filters one OLS block at a time.  The workgroup works through spans
// (runs of consecutive blocks of one channel); every team takes a contiguous
// part of the span, so when hop = 3N/4 the N/4 input samples one block shares
// with the next are carried over instead of read again.
// Per block (Sec. II, steps 1-5):
//   1. gather: thread t loads segment samples t + (N/16) v, v < 16 (coalesced
//      across the team); samples past len read 0, samples before 0 read 0 or,
//      on a streaming plan, the previous call's last N - M input samples;
//   2. forward DFT as Stockham autosort passes: radix-16 passes, then one pass
//      of radix 2/4/8 when log2 N is not a multiple of 4; passes exchange data
//      through the padded LDS tile; the last pass leaves X(t + (N/16) v) in
//      registers and computes only the two outer sub-bands when the band ends
//      below N/R (the others are stopband);
//   3. multiply by H_R (Sec. III-B, eq. (6)): only the bin index decides
//      between 1 (passband), V(r) (transition) and 0 (stopband); the 1/N of the
//      inverse (eq. (4)) is folded in here;
//   4. inverse DFT as the adjoint of step 2 (same index maps and twiddles,
//      conjugated, in reverse order), ending with z0(t + (N/16) v) in registers;
//   5. the linear phase exp(-j 2 pi k D / N) of eq. (5) is a circular delay by
//      D = (N - M)/2, so the kept output samples N-M+j of the phased inverse are
//      samples D + j of z0: thread t stores v where 0 <= t + (N/16) v - D < M.
// Real input (R32 storage) runs two consecutive blocks through one complex
// block, as its real and imaginary parts (the impulse response is real).
// Twiddles come from one float32 table w_4096^r (generated in float64 on the
// host, rounded to nearest).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <utility>

#include "fft_small.h"
#include "vbw_internal.h"

#ifndef VBW_WAVES_PER_EU
#define VBW_WAVES_PER_EU 3
#endif

namespace vbw {
namespace {

using namespace fft;

typedef float f2v __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ storage
// Channel data is read and written through buffer resources: 32-bit byte
// offsets from a per-span base, and the hardware range check (offset >=
// num_records reads 0 and drops stores) provides the zero fill past the end
// of the input and the truncation of the last output block.
constexpr int kBufFlags = 0x00020000;   // raw buffer, 32-bit dword format
#ifndef VBW_LOAD_POLICY
#define VBW_LOAD_POLICY 2
#endif
#ifndef VBW_STORE_POLICY
#define VBW_STORE_POLICY 2
#endif
constexpr int kLoadPolicy = VBW_LOAD_POLICY;    // cache policy bits of channel-data loads
constexpr int kStorePolicy = VBW_STORE_POLICY;  // and stores (2: non-temporal, streamed once)
typedef unsigned u2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int64_t bytes) {
    const int64_t cap = 0x7ffff000;     // every offset used stays far below
    const int n = int(bytes <= 0 ? 0 : (bytes < cap ? bytes : cap));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, n, kBufFlags);
}

template <Storage S> struct Io;

template <> struct Io<Storage::C64> {
    static constexpr int kBytes = 8;
    __device__ static float2 ld(__amdgpu_buffer_rsrc_t r, int off) {
        const u2v u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kLoadPolicy);
        return make_float2(__uint_as_float(u.x), __uint_as_float(u.y));
    }
};

// Two float32 to packed 16-bit, round to nearest even (one v_cvt_pk_* each).
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16_rne(float2 v) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{v.x, v.y}, bf2v));
}
__device__ __forceinline__ uint32_t pack_f16_rne(float2 v) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{v.x, v.y}, h2v));
}

template <> struct Io<Storage::F16> {
    static constexpr int kBytes = 4;
    __device__ static float2 ld(__amdgpu_buffer_rsrc_t r, int off) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadPolicy);
        return __half22float2(__builtin_bit_cast(__half2, u));
    }
};

template <> struct Io<Storage::BF16> {
    static constexpr int kBytes = 4;
    __device__ static float2 ld(__amdgpu_buffer_rsrc_t r, int off) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadPolicy);
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    }
};

// Real float32 samples (real input, real output).
template <> struct Io<Storage::R32> {
    static constexpr int kBytes = 4;
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, int off) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadPolicy));
    }
    __device__ static void st(__amdgpu_buffer_rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, kStorePolicy);
    }
};

template <Storage S, bool F32OUT> struct Out {
    static constexpr int kBytes = (S == Storage::C64 || F32OUT) ? 8 : 4;
    __device__ static void st(__amdgpu_buffer_rsrc_t r, int off, float2 v) {
        if constexpr (kBytes == 8) {
            __builtin_amdgcn_raw_buffer_store_b64(u2v{__float_as_uint(v.x), __float_as_uint(v.y)}, r, off, 0, kStorePolicy);
        } else if constexpr (S == Storage::F16) {
            __builtin_amdgcn_raw_buffer_store_b32(pack_f16_rne(v), r, off, 0, kStorePolicy);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(pack_bf16_rne(v), r, off, 0, kStorePolicy);
        }
    }
};

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

// Twiddle table w_4096^r through a buffer resource: 32-bit byte offsets.
struct Tw {
    __amdgpu_buffer_rsrc_t r;
    __device__ float2 operator()(unsigned idx) const {
        const u2v u = __builtin_amdgcn_raw_buffer_load_b64(r, int(idx * 8u), 0, 0);
        return make_float2(__uint_as_float(u.x), __uint_as_float(u.y));
    }
};

// The twiddles one thread applies depend only on its index t within the team
// and on N, so a workgroup loads them once into registers and reuses them for
// every block it filters, forward (as is) and inverse (conjugated).
//   mid:  middle pass (Ns = 16, only when N >= 512): w_256^{(t mod 16) r}, r = 1..15
//   last: last pass, butterfly b = t + T u: w_N^{b r}, r = 1..R-1
template <int LOG2N> struct TwReg {
    using Sh = Shape<LOG2N>;
    static constexpr int R = Sh::RLAST;
    static constexpr int U = 16 / R;
    static constexpr bool kMid = Sh::NP == 3;
    static constexpr bool kLast = Sh::NP > 1;
    float2 mid[kMid ? 15 : 1];
    float2 last[kLast ? U * (R - 1) : 1];

    __device__ void load(const Tw &tw, int t) {
        static_assert(Sh::NP <= 3, "N <= 4096");
        if constexpr (kMid) {
            const unsigned j = unsigned(t) & 15u;
#pragma unroll
            for (int r = 1; r < 16; ++r) mid[r - 1] = tw(16u * j * unsigned(r));
        }
        if constexpr (kLast) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned b = unsigned(t + Sh::T * u);
#pragma unroll
                for (int r = 1; r < R; ++r) last[u * (R - 1) + r - 1] = tw(Sh::TWS * b * unsigned(r));
            }
        }
    }
};

// LDS slot of stride-layout value t + T r (T a multiple of 16 splits the pad).
template <int T> __device__ __forceinline__ int lds_stride_pos(int t, int r) {
    if constexpr (T % 16 == 0) return lds_pad(t) + r * (T + T / 16);
    else return lds_pad(t + T * r);
}

// Middle radix-16 pass (pass 2 of 3, Ns = 16).
// Forward: gather t + T r, twiddle w_256^{j r} (j = t mod 16), DFT, scatter
// to (t/16) 256 + j + 16 s.  Inverse: the adjoint, in reverse order.
template <int LOG2N, bool INV>
__device__ __forceinline__ void mid_pass(float2 (&a)[16], float2 *L, int t, const TwReg<LOG2N> &tw) {
    using Sh = Shape<LOG2N>;
    constexpr int NS = 16;
    const int sbase = (t / NS) * NS * 16 + (t & (NS - 1));
    const int sb = lds_pad(sbase);           // (sbase + 16 s) pads to sb + 17 s
    constexpr int SSTEP = NS + NS / 16;
    if constexpr (!INV) {
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = L[lds_stride_pos<Sh::T>(t, r)];
#pragma unroll
        for (int r = 1; r < 16; ++r) a[r] = cmul(a[r], tw.mid[r - 1]);
        dft16<false>(a);
        tile_sync<Sh::WAVE_LOCAL>();
#pragma unroll
        for (int s = 0; s < 16; ++s) L[sb + SSTEP * s] = a[s];
        tile_sync<Sh::WAVE_LOCAL>();
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) a[s] = L[sb + SSTEP * s];
        dft16<true>(a);
#pragma unroll
        for (int r = 1; r < 16; ++r) a[r] = cmulc(a[r], tw.mid[r - 1]);
        tile_sync<Sh::WAVE_LOCAL>();
#pragma unroll
        for (int r = 0; r < 16; ++r) L[lds_stride_pos<Sh::T>(t, r)] = a[r];
        tile_sync<Sh::WAVE_LOCAL>();
    }
}

// Last pass, entirely in registers: butterfly b = t + T u (u < 16/R) has its R
// inputs in slots u + (16/R) r, twiddle w_N^{b r} (Ns = N/R, j = b), outputs
// X(b + (N/R) s) in slots u + (16/R) s.  For N = 16 this is the only pass and
// has no twiddle.
template <int LOG2N, bool INV>
__device__ __forceinline__ void last_pass(float2 (&a)[16], const TwReg<LOG2N> &tw) {
    using Sh = Shape<LOG2N>;
    constexpr int R = Sh::RLAST;
    constexpr int U = 16 / R;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float2 c[R];
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = a[u + U * r];
        if constexpr (!INV && Sh::NP > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) c[r] = cmul(c[r], tw.last[u * (R - 1) + r - 1]);
        }
        dft_small<R, INV>(c);
        if constexpr (INV && Sh::NP > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) c[r] = cmulc(c[r], tw.last[u * (R - 1) + r - 1]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a[u + U * r] = c[r];
    }
}

// Stopband-pruned last pass.  Its butterfly b produces bins b + (N/R) s; when
// the passband and transition band end below N/R (k2 < N/R), every bin with
// 0 < s < R-1 is stopband, so only s = 0 and s = R-1 can be nonzero
// (eq. (6): H_R = 0 on k_s).  Forward: compute just those two outputs and zero
// the rest.  Inverse: the first pass reads just those two inputs.
template <int R, int S_, bool INV>
__device__ __forceinline__ float2 wr_mul(float2 a) {   // a * w_R^{S_} (conjugate for INV)
    return w16mul<INV, ((16 / R) * S_) & 15>(a);
}

template <int LOG2N, bool INV>
__device__ __forceinline__ void last_pass_pruned(float2 (&a)[16], const TwReg<LOG2N> &tw) {
    using Sh = Shape<LOG2N>;
    constexpr int R = Sh::RLAST;
    constexpr int U = 16 / R;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        float2 c[R];
        if constexpr (!INV) {
#pragma unroll
            for (int r = 0; r < R; ++r) c[r] = a[u + U * r];
            if constexpr (Sh::NP > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) c[r] = cmul(c[r], tw.last[u * (R - 1) + r - 1]);
            }
            // out_0 = sum_r c_r, out_{R-1} = sum_r c_r w_R^{-r}
            float2 s0 = c[0], s1 = c[0];
            [&]<int... r>(std::integer_sequence<int, r...>) {
                ((s0 = cadd(s0, c[r + 1]), s1 = cadd(s1, wr_mul<R, R - (r + 1), false>(c[r + 1]))), ...);
            }(std::make_integer_sequence<int, R - 1>{});
#pragma unroll
            for (int r = 0; r < R; ++r) a[u + U * r] = make_float2(0.f, 0.f);
            a[u] = s0;
            a[u + U * (R - 1)] = s1;
        } else {
            // c_r = Y_0 + Y_{R-1} w_R^{r}  (inverse DFT of the two nonzero inputs)
            const float2 y0 = a[u], y1 = a[u + U * (R - 1)];
            c[0] = cadd(y0, y1);
            [&]<int... r>(std::integer_sequence<int, r...>) {
                ((c[r + 1] = cadd(y0, wr_mul<R, r + 1, false>(y1))), ...);
            }(std::make_integer_sequence<int, R - 1>{});
            if constexpr (Sh::NP > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) c[r] = cmulc(c[r], tw.last[u * (R - 1) + r - 1]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) a[u + U * r] = c[r];
        }
    }
}

// Step 3: Y(k) = H_R(k) X(k) / N (eq. (6), mirror H_R(N-k) = H_R(k)).  Slot v
// holds bin k = t + T v; its mirrored index kk = min(k, N-k) is t + T v for
// v < 8 and N - T v - t for v >= 8.  When every lane of the wave uses the same
// k1, whole slots that are pure passband or pure stopband are decided by a
// scalar test; only slots that meet the transition band read V.
template <int LOG2N>
__device__ __forceinline__ void hfso_multiply(float2 (&a)[16], int t, int k1, int lv, const float *vl) {
    using Sh = Shape<LOG2N>;
    constexpr int N = Sh::N, T = Sh::T;
    constexpr float inv_n = 1.0f / float(N);
    const int k1u = __builtin_amdgcn_readfirstlane(k1);
    if (__all(k1 == k1u)) {
        const int k2u = k1u + lv - 1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int lo = (v < 8) ? T * v : N - T * v - (T - 1);
            const int hi = (v < 8) ? T * v + (T - 1) : N - T * v;
            if (hi < k1u) {
                a[v].x *= inv_n;
                a[v].y *= inv_n;
            } else if (lo > k2u) {
                a[v] = make_float2(0.f, 0.f);
            } else {
                const int kk = (v < 8) ? t + T * v : N - T * v - t;
                float f = (kk < k1u) ? inv_n : 0.0f;
                if (lo <= k2u && hi >= k1u) {
                    const int jj = kk - k1u;
                    if (jj >= 0 && jj < lv) f = vl[jj] * inv_n;
                }
                a[v].x *= f;
                a[v].y *= f;
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int kk = (v < 8) ? t + T * v : N - T * v - t;
            const int jj = kk - k1;
            float f = (jj < 0) ? inv_n : 0.0f;
            if (jj >= 0 && jj < lv) f = vl[jj] * inv_n;
            a[v].x *= f;
            a[v].y *= f;
        }
    }
}

// Work items and channel descriptors are workgroup-uniform: index them with
// values the compiler knows to be uniform so they come in by scalar loads and
// never wait behind the vector-memory queue of in-flight channel data.
// The tables are read-only for the whole launch, so they are read through the
// constant address space.
template <typename T> __device__ __forceinline__ T ld_uniform(const T *p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) T cT;
    return ((cT *)p)[__builtin_amdgcn_readfirstlane(i)];
#else
    return p[i];   // host pass: never executed
#endif
}
__device__ __forceinline__ WorkItem load_item(const LaunchArgs &A, int i) { return ld_uniform(A.items, i); }
__device__ __forceinline__ ChannelDev load_channel(const LaunchArgs &A, int c) { return ld_uniform(A.ch, c); }

// Samples before 0 (the zero history of a channel's first blocks) get an
// offset past the resource's end and read as 0, like samples past len.
constexpr int kOutOfRange = int(0x80000000u);

constexpr int kVCap = 2048;  // transition values staged in LDS (L_V <= N/2 <= 2048)

// Band schedule of one channel (Sec. III-B: an integer edge k1 per block),
// walked forward: a binary search finds the entry in force at a team's first
// block, then each later block only checks whether it has reached the next
// entry.  Entries are sorted by from_block, the first has from_block 0.  With
// one entry (no band change) nothing is read per block.
struct SchedCursor {
    int e = 0;                 // entry in force
    int k1 = 0;
    int64_t next = INT64_MAX;  // from_block of entry e + 1

    __device__ __forceinline__ void seek(const LaunchArgs &A, const ChannelDev &cd, int64_t m) {
        k1 = ld_uniform(A.sched, cd.sched_begin).k1;
        e = 0;
        next = INT64_MAX;
        const int n = cd.sched_count;
        if (n == 1) return;
        int lo = 0, hi = n;                        // sched[lo].from_block <= m < sched[hi].from_block
        for (int w = n - 1; w > 0; w >>= 1) {      // ceil(log2 n) steps, the same in every lane
            const int mid = (lo + hi) >> 1;
            if (mid > lo && A.sched[cd.sched_begin + mid].from_block <= m) lo = mid;
            else if (mid > lo) hi = mid;
        }
        e = lo;
        k1 = A.sched[cd.sched_begin + e].k1;
        next = e + 1 < n ? A.sched[cd.sched_begin + e + 1].from_block : INT64_MAX;
    }
    // k1 of block m; m never decreases between calls
    __device__ __forceinline__ int at(const LaunchArgs &A, const ChannelDev &cd, int64_t m) {
        while (m >= next) {
            ++e;
            k1 = A.sched[cd.sched_begin + e].k1;
            next = e + 1 < cd.sched_count ? A.sched[cd.sched_begin + e + 1].from_block : INT64_MAX;
        }
        return k1;
    }
};

struct WgState {
    int v_offset = -1;   // V set currently staged in LDS
    int lv = -1;
};

// Steps 2-5 for one block per team, its segment already gathered into a:
// forward DFT, HFSO multiply, inverse DFT, keep z0(D + j), j < hop.
template <int LOG2N, Storage S, bool F32OUT, bool CARRY>
__device__ __forceinline__ void filter_block(float2 (&a)[16], const LaunchArgs &A, const ChannelDev &cd, int k1,
                                             int keep, __amdgpu_buffer_rsrc_t yr, int o0,
                                             const TwReg<LOG2N> &tw, float2 *L, const float *vlds, int t) {
    using Sh = Shape<LOG2N>;
    constexpr int N = Sh::N, T = Sh::T;
    constexpr int EO = Out<S, F32OUT>::kBytes;
    const int hop = cd.hop;
    const int d = (N - hop) >> 1;

    // step 2: forward DFT
    if constexpr (Sh::NP > 1) {
        dft16<false>(a);                                  // pass 1, Ns = 1
#pragma unroll
        for (int s = 0; s < 16; ++s) L[17 * t + s] = a[s];
        tile_sync<Sh::WAVE_LOCAL>();
        if constexpr (Sh::NP == 3) mid_pass<LOG2N, false>(a, L, t, tw);
#pragma unroll
        for (int v = 0; v < 16; ++v) a[v] = L[lds_stride_pos<T>(t, v)];
    }
    // every team of the wave must meet the pruning condition (wave-uniform)
    constexpr int R = Sh::RLAST;
    const bool prune = (R > 2) && A.prune && __all(k1 + cd.lv - 1 < N / R);
    if (prune) last_pass_pruned<LOG2N, false>(a, tw);
    else last_pass<LOG2N, false>(a, tw);

    // step 3: H_R and 1/N
    hfso_multiply<LOG2N>(a, t, k1, cd.lv, vlds);

    // step 4: inverse DFT (adjoint passes); the first one reads only the
    // bins that can be nonzero when pruned
    if (prune) last_pass_pruned<LOG2N, true>(a, tw);
    else last_pass<LOG2N, true>(a, tw);
    if constexpr (Sh::NP > 1) {
#pragma unroll
        for (int v = 0; v < 16; ++v) L[lds_stride_pos<T>(t, v)] = a[v];
        tile_sync<Sh::WAVE_LOCAL>();
        if constexpr (Sh::NP == 3) mid_pass<LOG2N, true>(a, L, t, tw);
#pragma unroll
        for (int s = 0; s < 16; ++s) a[s] = L[17 * t + s];
        dft16<true>(a);
    }

    // step 5: keep z0(D + j), j < hop; o0 is the output index of slot 0
    // (may be < 0); stores past len are dropped by the buffer range check.
    // keep: bit 0 stores the block (real parts: the pair's first block),
    // bit 1 the imaginary parts as the pair's second block (real input)
    if constexpr (S == Storage::R32) {
        if (keep) {
            const bool kx = keep & 1, ky = keep & 2;
            if constexpr (CARRY) {
#pragma unroll
                for (int v = 2; v < 14; ++v) {
                    if (kx) Io<S>::st(yr, (o0 + T * v) * 4, a[v].x);
                    if (ky) Io<S>::st(yr, (o0 + hop + T * v) * 4, a[v].y);
                }
            } else {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const bool in = unsigned(t + T * v - d) < unsigned(hop);
                    Io<S>::st(yr, in && kx ? (o0 + T * v) * 4 : kOutOfRange, a[v].x);
                    Io<S>::st(yr, in && ky ? (o0 + hop + T * v) * 4 : kOutOfRange, a[v].y);
                }
            }
        }
    } else if (keep & 1) {
        if constexpr (CARRY) {
            // hop = 12 T, D = 2 T: the kept samples are exactly slots 2..13
#pragma unroll
            for (int v = 2; v < 14; ++v) Out<S, F32OUT>::st(yr, (o0 + T * v) * EO, a[v]);
        } else {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = t + T * v - d;        // index within the block's kept samples
                Out<S, F32OUT>::st(yr, unsigned(j) < unsigned(hop) ? (o0 + T * v) * EO : kOutOfRange, a[v]);
            }
        }
    }
}

// One span: blocks [first, first + n) of one channel, filtered by the
// workgroup's G = 4096/N teams.  Team g takes the contiguous sub-run
// [first + g n / G, first + (g+1) n / G) and the teams step through their
// sub-runs together.  Consecutive blocks of a team share N - hop input
// samples; when hop = 3N/4 (CARRY) they are exactly register slots 12..15 of
// one block and 0..3 of the next, so only the 12 new slots are read from
// memory and the 4 shared ones wait in LDS (cl: 4 values per thread; each
// thread reads back only what it wrote, so no barrier is needed).
template <int LOG2N, Storage S, bool F32OUT, bool CARRY>
__device__ __forceinline__ void run_span(const LaunchArgs &A, const WorkItem &sp, const ChannelDev &cd,
                                         const TwReg<LOG2N> &tw, float2 *lds, const float *vlds, float2 *cl) {
    using Sh = Shape<LOG2N>;
    constexpr int N = Sh::N, T = Sh::T;
    constexpr int G = kThreads / T;
    constexpr int EI = Io<S>::kBytes;
    constexpr int EO = Out<S, F32OUT>::kBytes;
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid - team * T;
    float2 *L = lds + team * lds_pad(N);
    const int hop = cd.hop;
    const int n = sp.n_blocks;
    const int lo = int((int64_t(team) * n) / G);
    const int cnt = int((int64_t(team + 1) * n) / G) - lo;
    const int steps = (n + G - 1) / G;

    // input resource from the span's first segment start (clipped at 0)
    const int64_t s0 = int64_t(sp.first_block) * hop - (N - hop);
    const int64_t clip = s0 > 0 ? s0 : 0;
    const auto xr = make_rsrc(static_cast<const char *>(ld_uniform(A.x, sp.channel)) + clip * EI,
                              (cd.len - clip) * EI);
    const int64_t ob = int64_t(sp.first_block) * hop;
    const auto yr = make_rsrc(static_cast<char *>(ld_uniform(A.y, sp.channel)) + ob * EO, (cd.len - ob) * EO);
    const int jb = int(s0 - clip) + lo * hop + t;     // sample of slot 0 of the team's first block, rel. to xr
    // The N - hop samples before sample 0: zeros, or the stream's history
    // (the previous call's last N - hop input samples) on a streaming plan.
    const int hl = N - hop;
    const auto hr = A.hist ? make_rsrc(static_cast<const char *>(A.hist) + cd.hist_off * EI, int64_t(hl) * EI)
                           : make_rsrc(A.tw, 0);
    const int64_t mb = A.block0 ? ld_uniform(A.block0, sp.channel) : 0;   // stream block of the call's block 0

    // step 1: all 16 slots of the block whose slot 0 is sample j0 (rel. to xr);
    // samples before 0 read 0, and on a streaming plan are then replaced by
    // the history (only for segments that start before sample 0)
    float2 a[16];
    auto gather = [&](int j0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = j0 + T * v;
            a[v] = Io<S>::ld(xr, j >= 0 ? j * EI : kOutOfRange);
        }
        if (A.hist != nullptr && j0 - t < 0) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = j0 + T * v;
                if (j < 0) a[v] = Io<S>::ld(hr, (j + hl) * EI);
            }
        }
    };
    gather(jb);
    SchedCursor sc;
    sc.seek(A, cd, mb + int64_t(sp.first_block) + lo);
    for (int s = 0; s < steps; ++s) {
        const int b = lo + s;                              // block within the span
        const bool active = s < cnt;
        const int k1 = sc.at(A, cd, mb + int64_t(sp.first_block) + b);
        const bool more = s + 1 < steps;                   // workgroup-uniform
        // For hop = 3N/4 every sample of slots 4..15 of a block after the
        // channel's block 0 lies at index >= 0, so no history test.
        const int jn = jb + (s + 1) * hop;                 // slot 0 of the next block
        if constexpr (CARRY) {
#pragma unroll
            for (int v = 0; v < 4; ++v) cl[v * kThreads + tid] = a[12 + v];
        }
        // a team that is exactly one wave skips the blocks past its run; smaller
        // teams share a wave and larger ones share barriers, so they compute
        // (and do not store) an idle block
        if (T != 64 || active)
            filter_block<LOG2N, S, F32OUT, CARRY>(a, A, cd, k1, active ? 1 : 0, yr, b * hop + t - ((N - hop) >> 1), tw,
                                                  L, vlds, t);
        if (more) {
            // the next block's loads go out at raised wave priority, ahead of
            // the arithmetic of the CU's other waves (3-4% on long spans)
            __builtin_amdgcn_s_setprio(1);
            if constexpr (CARRY) {
#pragma unroll
                for (int v = 0; v < 4; ++v) a[v] = cl[v * kThreads + tid];
#pragma unroll
                for (int v = 4; v < 16; ++v) a[v] = Io<S>::ld(xr, (jn + T * v) * EI);
            } else {
                gather(jn);
            }
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

// Real input (R32 storage).  The impulse response is real (eq. (8)), so two
// real blocks filtered as the real and the imaginary parts of one complex
// block come out as the real and imaginary parts of the result.  A team takes
// pairs of consecutive blocks (2p, 2p+1), the first in the real parts, the
// second in the imaginary parts, and walks through a contiguous run of pairs
// (spans start at even blocks).  When hop = 3N/4 slots 0..3 of block 2p+2 are
// slots 12..15 of block 2p+1 (carried in LDS) and slots 0..3 of block 2p+3
// are slots 12..15 of block 2p+2 (already in registers): 24 new samples per
// thread and pair.  A pair whose blocks fall under different band-schedule
// entries is filtered twice, once per block.
template <int LOG2N, bool F32OUT, bool CARRY>
__device__ __forceinline__ void run_span_real(const LaunchArgs &A, const WorkItem &sp, const ChannelDev &cd,
                                              const TwReg<LOG2N> &tw, float2 *lds, const float *vlds, float2 *cl) {
    using Sh = Shape<LOG2N>;
    using IoR = Io<Storage::R32>;
    constexpr int N = Sh::N, T = Sh::T;
    constexpr int G = kThreads / T;
    constexpr int E = IoR::kBytes;
    const int tid = threadIdx.x;
    const int team = tid / T;
    const int t = tid - team * T;
    float2 *L = lds + team * lds_pad(N);
    const int hop = cd.hop;
    const int np = (sp.n_blocks + 1) >> 1;
    const int lo = int((int64_t(team) * np) / G);
    const int cnt = int((int64_t(team + 1) * np) / G) - lo;
    const int steps = (np + G - 1) / G;

    const int64_t s0 = int64_t(sp.first_block) * hop - (N - hop);
    const int64_t clip = s0 > 0 ? s0 : 0;
    const auto xr = make_rsrc(static_cast<const char *>(ld_uniform(A.x, sp.channel)) + clip * E,
                              (cd.len - clip) * E);
    const int64_t ob = int64_t(sp.first_block) * hop;
    const auto yr = make_rsrc(static_cast<char *>(ld_uniform(A.y, sp.channel)) + ob * E, (cd.len - ob) * E);
    const int hl = N - hop;
    const auto hr = A.hist ? make_rsrc(static_cast<const char *>(A.hist) + cd.hist_off * E, int64_t(hl) * E)
                           : make_rsrc(A.tw, 0);
    const int64_t mb = A.block0 ? ld_uniform(A.block0, sp.channel) : 0;
    const int jb = int(s0 - clip) + 2 * lo * hop + t;  // slot 0 of the first block of the team's first pair

    float2 a[16];
    // both blocks of the pair whose first block has slot 0 at sample j0 (rel. to xr)
    auto gather_pair = [&](int j0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int jx = j0 + T * v, jy = jx + hop;
            a[v].x = IoR::ld(xr, jx >= 0 ? jx * E : kOutOfRange);
            a[v].y = IoR::ld(xr, jy >= 0 ? jy * E : kOutOfRange);
        }
        if (A.hist != nullptr && j0 - t < 0) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int jx = j0 + T * v, jy = jx + hop;
                if (jx < 0) a[v].x = IoR::ld(hr, (jx + hl) * E);
                if (jy < 0) a[v].y = IoR::ld(hr, (jy + hl) * E);
            }
        }
    };
    SchedCursor sc;
    sc.seek(A, cd, mb + int64_t(sp.first_block) + 2 * lo);
    gather_pair(jb);
    // one filter per iteration: a pair whose blocks need different k1 takes
    // two iterations (pass 1 filters the re-gathered pair for its second block)
    int s = 0, pass = 0;
    int k1a = 0, k1b = 0;                                   // edges of the pair's two blocks
    while (s < steps) {
        const int q = lo + s;                               // pair within the span
        const bool active = s < cnt;
        if (pass == 0) {                                    // the cursor only moves forward
            const int64_t ma = mb + int64_t(sp.first_block) + 2 * q;
            k1a = sc.at(A, cd, ma);
            k1b = sc.at(A, cd, ma + 1);
        }
        const bool same = k1a == k1b;
        // the second pass is taken by the whole wave (team <= one wave) or the
        // whole workgroup (teams with workgroup barriers)
        bool split;
        if constexpr (Sh::WAVE_LOCAL) split = __any(!same);
        else split = __syncthreads_or(!same);
        if (CARRY && pass == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) cl[v * kThreads + tid] = make_float2(a[12 + v].y, 0.f);
        }
        const int o0 = 2 * q * hop + t - (hl >> 1);
        const int keep = !active ? 0 : pass ? (same ? 0 : 2) : (same ? 3 : 1);
        if (T != 64 || active)
            filter_block<LOG2N, Storage::R32, F32OUT, CARRY>(a, A, cd, pass ? k1b : k1a, keep, yr, o0, tw, L, vlds,
                                                             t);
        if (split && pass == 0) {
            gather_pair(jb + 2 * s * hop);                  // the pair again, for its second block
            pass = 1;
            continue;
        }
        pass = 0;
        ++s;
        if (s < steps) {
            const int jn = jb + 2 * s * hop;                // slot 0 of the next pair's first block
            if constexpr (CARRY) {
#pragma unroll
                for (int v = 0; v < 4; ++v) a[v].x = cl[v * kThreads + tid].x;
#pragma unroll
                for (int v = 4; v < 16; ++v) a[v].x = IoR::ld(xr, (jn + T * v) * E);
#pragma unroll
                for (int v = 0; v < 4; ++v) a[v].y = a[12 + v].x;
#pragma unroll
                for (int v = 4; v < 16; ++v) a[v].y = IoR::ld(xr, (jn + hop + T * v) * E);
            } else {
                gather_pair(jn);
            }
        }
    }
}

// Consecutive spans [i, end) of size N: twiddles loaded once.  Returns the
// first span index not done.  Inlined into every kernel, so that the kernel
// that dispatches on N has no calls (a call costs spills and a stack frame).
template <int LOG2N, Storage S, bool F32OUT>
__device__ __forceinline__ int run_spans(const LaunchArgs &A, int i, int end, float2 *lds, float *vlds, float2 *cl, WgState &ws) {
    using Sh = Shape<LOG2N>;
    const int t = threadIdx.x % Sh::T;
    TwReg<LOG2N> tw;
    tw.load(Tw{make_rsrc(A.tw, int64_t(kTwiddleN) * 8)}, t);
    for (; i < end; ++i) {
        const WorkItem sp = load_item(A, i);
        if (sp.log2n != LOG2N) break;
        const ChannelDev cd = load_channel(A, sp.channel);
        // stage this channel's V in LDS (workgroup-uniform decision)
        if (cd.v_offset != ws.v_offset || cd.lv != ws.lv) {
            __syncthreads();
            for (int q = threadIdx.x; q < cd.lv; q += kThreads) vlds[q] = A.v[cd.v_offset + q];
            __syncthreads();
            ws.v_offset = cd.v_offset;
            ws.lv = cd.lv;
        }
        if constexpr (S == Storage::R32) {
            if (4 * cd.hop == 3 * Sh::N) run_span_real<LOG2N, F32OUT, true>(A, sp, cd, tw, lds, vlds, cl);
            else run_span_real<LOG2N, F32OUT, false>(A, sp, cd, tw, lds, vlds, cl);
        } else {
            if (4 * cd.hop == 3 * Sh::N) run_span<LOG2N, S, F32OUT, true>(A, sp, cd, tw, lds, vlds, cl);
            else run_span<LOG2N, S, F32OUT, false>(A, sp, cd, tw, lds, vlds, cl);
        }
    }
    return i;
}

// Persistent launch: workgroup w filters spans [wg_begin[w], wg_begin[w+1]),
// contiguous block ranges of equal estimated cost (consecutive blocks of a
// channel stay on one CU).  In the launch that covers every N (LOG2N = 0)
// each workgroup's range holds one N: the workgroup takes that N's path once.
template <int LOG2N, Storage S, bool F32OUT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(VBW_WAVES_PER_EU, 8)))
void ols_fft_kernel(const LaunchArgs A) {
    __shared__ float2 lds[kLdsValues];
    __shared__ float vlds[kVCap];
    __shared__ float2 clds[4 * kThreads];
    WgState ws;
    const int w = blockIdx.x;
    const int i = ld_uniform(A.wg_begin, w);
    const int end = ld_uniform(A.wg_begin, w + 1);
    if (i >= end) return;
    if constexpr (LOG2N != 0) {
        run_spans<LOG2N, S, F32OUT>(A, i, end, lds, vlds, clds, ws);
    } else {
        switch (load_item(A, i).log2n) {
            case 4: run_spans<4, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 5: run_spans<5, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 6: run_spans<6, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 7: run_spans<7, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 8: run_spans<8, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 9: run_spans<9, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 10: run_spans<10, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 11: run_spans<11, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            case 12: run_spans<12, S, F32OUT>(A, i, end, lds, vlds, clds, ws); break;
            default: break;
        }
    }
}

// One dispatch; with events, through hipExtLaunchKernel, which records the
// kernel's own start and end time in them.
template <typename K>
void dispatch(K kernel, dim3 grid, dim3 block, hipStream_t stream, hipEvent_t t0, hipEvent_t t1, const LaunchArgs &A) {
    if (t0 || t1) hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, t0, t1, 0, A);
    else hipLaunchKernelGGL(kernel, grid, block, 0, stream, A);
}

template <Storage S, bool F32OUT>
hipError_t launch_typed(const LaunchArgs &A, int log2n, hipStream_t stream, hipEvent_t t0, hipEvent_t t1) {
    const dim3 grid(A.n_wg), block(kThreads);
    switch (log2n) {
        case 0: dispatch(ols_fft_kernel<0, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 4: dispatch(ols_fft_kernel<4, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 5: dispatch(ols_fft_kernel<5, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 6: dispatch(ols_fft_kernel<6, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 7: dispatch(ols_fft_kernel<7, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 8: dispatch(ols_fft_kernel<8, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 9: dispatch(ols_fft_kernel<9, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 10: dispatch(ols_fft_kernel<10, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 11: dispatch(ols_fft_kernel<11, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        case 12: dispatch(ols_fft_kernel<12, S, F32OUT>, grid, block, stream, t0, t1, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <Storage S, bool F32OUT> int occupancy_typed(int log2n) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (log2n) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<0, S, F32OUT>, kThreads, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<4, S, F32OUT>, kThreads, 0); break;
        case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<5, S, F32OUT>, kThreads, 0); break;
        case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<6, S, F32OUT>, kThreads, 0); break;
        case 7: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<7, S, F32OUT>, kThreads, 0); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<8, S, F32OUT>, kThreads, 0); break;
        case 9: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<9, S, F32OUT>, kThreads, 0); break;
        case 10: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<10, S, F32OUT>, kThreads, 0); break;
        case 11: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<11, S, F32OUT>, kThreads, 0); break;
        case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_fft_kernel<12, S, F32OUT>, kThreads, 0); break;
        default: break;
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

int ols_fft_wg_per_cu(int log2n_fixed, Storage in, bool f32_out) {
    switch (in) {
        case Storage::C64: return occupancy_typed<Storage::C64, false>(log2n_fixed);
        case Storage::R32: return occupancy_typed<Storage::R32, false>(log2n_fixed);
        case Storage::F16:
            return f32_out ? occupancy_typed<Storage::F16, true>(log2n_fixed)
                           : occupancy_typed<Storage::F16, false>(log2n_fixed);
        case Storage::BF16:
            return f32_out ? occupancy_typed<Storage::BF16, true>(log2n_fixed)
                           : occupancy_typed<Storage::BF16, false>(log2n_fixed);
    }
    return 1;
}

hipError_t launch_ols_fft(const LaunchArgs &A, int log2n_fixed, Storage in, bool f32_out,
                          hipStream_t stream, hipEvent_t t0, hipEvent_t t1) {
    if (A.n_items <= 0) return hipSuccess;
    switch (in) {
        case Storage::C64: return launch_typed<Storage::C64, false>(A, log2n_fixed, stream, t0, t1);
        case Storage::R32: return launch_typed<Storage::R32, false>(A, log2n_fixed, stream, t0, t1);
        case Storage::F16:
            return f32_out ? launch_typed<Storage::F16, true>(A, log2n_fixed, stream, t0, t1)
                           : launch_typed<Storage::F16, false>(A, log2n_fixed, stream, t0, t1);
        case Storage::BF16:
            return f32_out ? launch_typed<Storage::BF16, true>(A, log2n_fixed, stream, t0, t1)
                           : launch_typed<Storage::BF16, false>(A, log2n_fixed, stream, t0, t1);
    }
    return hipErrorInvalidValue;
}

}  // namespace vbw
