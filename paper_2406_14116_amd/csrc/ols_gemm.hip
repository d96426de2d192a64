// ols_gemm.hip -- overlap-save variable-bandwidth filtering with the small DFTs
// run as dense matrix products on the gfx950 matrix cores (FP16 inputs, FP32
// accumulation), for 16-bit channel storage and N = 256.
//
// Paper: Moryakova & Johansson, arXiv 2406.14116.  Same operation as the FFT
// engine: Sec. II steps 1-5 with the HFSO coefficients of eqs. (5)-(6).
//
// The 256-point DFT is split as 16 x 16 (n = 16 n1 + n2, k = k1 + 16 k2):
//   S1  A1[n2][k1]  = sum_n1 x[n1][n2] W[n1][k1]          (W[a][b] = w16^{ab})
//       A1[n2][k1] *= w256^{n2 k1}
//   S2  X[k2][k1]   = sum_n2 W[k2][n2] A1[n2][k1]          (bin k1 + 16 k2)
//       Y = H_R X / N
//   S3  B[k1][n2]   = sum_k2 Y[k2][k1] conj W[k2][n2]
//       B[k1][n2]  *= conj w256^{n2 k1}
//   S4  z[n1][n2]   = sum_k1 conj W[n1][k1] B[k1][n2]
// Each stage is a complex 16x16x16 product done with 16x16x32 MFMAs whose K
// dimension carries (real part, imaginary part): one MFMA per real output.
// The accumulator layout of one MFMA (lane = 16 g + c holds rows 4g..4g+3 of
// column c) is exactly the B operand (K = those rows) or the transposed A
// operand of the next one, so a block never leaves the registers of its wave.
// Precision: the DFT matrix and the FP32 intermediates enter the matrix cores
// as hi + lo FP16 pairs (hi = RN(v), lo = RN(v - hi)); each real product is
// hi*hi + lo*hi + hi*lo with FP32 accumulation (the lo*lo term, ~2^-22
// relative, is dropped).  The 16-bit input samples are exact in FP16 (BF16
// samples are rounded to FP16 first; exact for normal-range values).  The
// intermediates grow to about 16 times the input's magnitude, so inputs must
// stay below about 2^11 in magnitude for the FP16 operands not to overflow.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <algorithm>

#include "vbw_internal.h"

namespace vbw {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

constexpr int kGemmN = 256;
constexpr int kGemmHop4 = 4;        // blocks per wave per item step
constexpr int kBufFlags = 0x00020000;
constexpr int kNT = 2;
constexpr int kOutOfRange = int(0x80000000u);
constexpr int kVCapG = 2048;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int64_t bytes) {
    const int64_t cap = 0x7ffff000;
    const int n = int(bytes <= 0 ? 0 : (bytes < cap ? bytes : cap));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, n, kBufFlags);
}

template <typename T> __device__ __forceinline__ T ld_uniform(const T *p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) T cT;
    return ((cT *)p)[__builtin_amdgcn_readfirstlane(i)];
#else
    return p[i];
#endif
}

typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// D += A B with A 16x32, B 32x16 (FP16), D 16x16 (FP32).  Lane 16 g + c holds
// K entries 8g .. 8g+7 of row c of A and of column c of B, and rows 4g .. 4g+3
// of column c of D.  Only the pairing of K entries between A and B matters, so
// a lane's eight K entries are used as (four rows of a real part, the same
// four rows of an imaginary part): a complex product needs one MFMA per real
// output, and the accumulator of one stage is already the next stage's operand.
__device__ __forceinline__ f4 mfma(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }

__device__ __forceinline__ h8 cat(h4 p, h4 q) { return h8{p[0], p[1], p[2], p[3], q[0], q[1], q[2], q[3]}; }

// hi + lo split of eight FP32 values
struct Split {
    h8 hi, lo;
};
__device__ __forceinline__ Split split(f4 a, f4 b) {
    Split s;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float v = i < 4 ? a[i] : b[i - 4];
        const _Float16 h = (_Float16)v;
        s.hi[i] = h;
        s.lo[i] = (_Float16)(v - (float)h);
    }
    return s;
}

// Real product of split operands: P*Q ~ Phi*Qhi + Plo*Qhi + Phi*Qlo.
__device__ __forceinline__ f4 mm3(const Split &p, const Split &q) {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    return mfma(p.hi, q.lo, mfma(p.lo, q.hi, mfma(p.hi, q.hi, z)));
}
// Exact-data product (P exact in FP16): P*Qhi + P*Qlo.
__device__ __forceinline__ f4 mm2(h8 p, const Split &q) {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    return mfma(p, q.lo, mfma(p, q.hi, z));
}

// Constants of one lane (lane = 16 g + c): the DFT matrix entries it feeds,
// W[4g + j][c] = w16^{(4g + j) c} (the same in A and B layouts since W is
// symmetric), packed as the four K-concatenations the stages use, and the four
// inter-stage twiddles w256^{(4g + r) c}.
struct GemmConst {
    Split r_ni;   // [Re W | -Im W]
    Split i_r;    // [Im W | Re W]
    Split r_i;    // [Re W | Im W]
    Split ni_r;   // [-Im W | Re W]
    float2 tw[4];
};

__device__ __forceinline__ void load_consts(GemmConst &k, const float2 *__restrict__ tw4096, int lane) {
    const int g = lane >> 4, c = lane & 15;
    f4 wr, wi;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = ((4 * g + j) * c) & 15;               // w16^e = w4096^{256 e}
        const float2 w = tw4096[256 * e];
        wr[j] = w.x;
        wi[j] = w.y;
    }
    k.r_ni = split(wr, -wi);
    k.i_r = split(wi, wr);
    k.r_i = split(wr, wi);
    k.ni_r = split(-wi, wr);
#pragma unroll
    for (int r = 0; r < 4; ++r) k.tw[r] = tw4096[(16 * (((4 * g + r) * c) & 255)) & 4095];
}

struct CF4 {
    f4 re, im;
};

template <Storage S> struct GIo;
template <> struct GIo<Storage::F16> {
    // (re, im) FP16 pair of one sample -> exact FP16 halves
    __device__ static void unpack(uint32_t u, _Float16 &re, _Float16 &im) {
        re = __builtin_bit_cast(_Float16, uint16_t(u & 0xffffu));
        im = __builtin_bit_cast(_Float16, uint16_t(u >> 16));
    }
};
template <> struct GIo<Storage::BF16> {
    __device__ static void unpack(uint32_t u, _Float16 &re, _Float16 &im) {
        re = (_Float16)__uint_as_float(u << 16);
        im = (_Float16)__uint_as_float(u & 0xffff0000u);
    }
};

// Two float32 to packed 16-bit, round to nearest even (one v_cvt_pk_* each).
typedef float gf2v __attribute__((ext_vector_type(2)));
typedef __bf16 gbf2v __attribute__((ext_vector_type(2)));
typedef _Float16 gh2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16_rne(float re, float im) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(gf2v{re, im}, gbf2v));
}
__device__ __forceinline__ uint32_t pack_f16_rne(float re, float im) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(gf2v{re, im}, gh2v));
}

template <Storage S, bool F32OUT> __device__ __forceinline__ void gstore(__amdgpu_buffer_rsrc_t r, int off, float re,
                                                                        float im) {
    if constexpr (F32OUT) {
        __builtin_amdgcn_raw_buffer_store_b64(u2v{__float_as_uint(re), __float_as_uint(im)}, r, off, 0, kNT);
    } else if constexpr (S == Storage::F16) {
        __builtin_amdgcn_raw_buffer_store_b32(pack_f16_rne(re, im), r, off, 0, kNT);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(pack_bf16_rne(re, im), r, off, 0, kNT);
    }
}

// The samples of one block: base = sample index of the segment start relative
// to the input resource (may be negative: zero history); lane (g, c) reads
// x[n1 = 4g + j][n2 = c], j < 4.  valid = false reads past the resource's end
// (zeros, no memory access).
__device__ __forceinline__ void gemm_load(__amdgpu_buffer_rsrc_t xr, int base, int lane, bool valid,
                                          uint32_t (&u)[4]) {
    const int g = lane >> 4, c = lane & 15;
    __builtin_amdgcn_s_setprio(1);   // loads out ahead of other waves' arithmetic
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = base + 16 * (4 * g + j) + c;
        u[j] = __builtin_amdgcn_raw_buffer_load_b32(xr, valid && i >= 0 ? i * 4 : kOutOfRange, 0, kNT);
    }
    __builtin_amdgcn_s_setprio(0);
}

// One OLS block of N = 256 by one wave, its samples already loaded into u.
template <Storage S, bool F32OUT>
__device__ __forceinline__ void gemm_block(const GemmConst &K, const uint32_t (&u)[4],
                                           __amdgpu_buffer_rsrc_t yr, int obase, int hop, int k1, int lv,
                                           const float *vl, int lane) {
    const int g = lane >> 4, c = lane & 15;
    // S1 operand A = x^T: lane (g, n2 = c) holds x[n1 = 4g + j][n2], j < 4
    h4 ar, ai;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        _Float16 re, im;
        GIo<S>::unpack(u[j], re, im);
        ar[j] = re;
        ai[j] = im;
    }
    // S1: D1[n2][k1] = sum_n1 x^T[n2][n1] W[n1][k1]
    CF4 d;
    {
        const h8 xa = cat(ar, ai);
        d.re = mm2(xa, K.r_ni);      // xr Wr - xi Wi
        d.im = mm2(xa, K.i_r);       // xr Wi + xi Wr
    }
    // twiddle w256^{n2 k1}: lane (g, k1 = c) holds rows n2 = 4g + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float2 w = K.tw[r];
        const float x = d.re[r], y = d.im[r];
        d.re[r] = x * w.x - y * w.y;
        d.im[r] = x * w.y + y * w.x;
    }
    // S2: D2[k2][k1] = sum_n2 W[k2][n2] D1[n2][k1]  (A = W, B = D1)
    {
        const Split b1 = split(d.re, d.im);
        CF4 e;
        e.re = mm3(K.r_ni, b1);      // Wr D1r - Wi D1i
        e.im = mm3(K.i_r, b1);       // Wi D1r + Wr D1i
        d = e;
    }
    // multiply: lane (g, k1 = c) holds bins k = c + 16 (4g + r).  The 1/N of
    // the inverse is applied as 1/16 here and 1/16 at the store, which keeps
    // every intermediate near the input's scale (FP16 operands must neither
    // overflow nor fall into the subnormal range)
    {
        constexpr float inv_n = 1.0f / 16.0f;
        const int k2 = k1 + lv - 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = c + 16 * (4 * g + r);
            const int kk = k <= kGemmN / 2 ? k : kGemmN - k;
            float f = kk < k1 ? inv_n : 0.0f;
            if (kk >= k1 && kk <= k2) f = vl[kk - k1] * inv_n;
            d.re[r] *= f;
            d.im[r] *= f;
        }
    }
    // S3: D3[k1][n2] = sum_k2 Y^T[k1][k2] conj W[k2][n2]  (A = D2^T, B = conj W)
    {
        const Split a2 = split(d.re, d.im);
        CF4 e;
        e.re = mm3(a2, K.r_i);       // Yr Wr + Yi Wi
        e.im = mm3(a2, K.ni_r);      // -Yr Wi + Yi Wr
        d = e;
    }
    // conjugate twiddle: lane (g, n2 = c) holds rows k1 = 4g + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float2 w = K.tw[r];
        const float x = d.re[r], y = d.im[r];
        d.re[r] = x * w.x + y * w.y;
        d.im[r] = y * w.x - x * w.y;
    }
    // S4: z[n1][n2] = sum_k1 conj W[n1][k1] D3[k1][n2]  (A = conj W, B = D3)
    {
        const Split b3 = split(d.re, d.im);
        CF4 e;
        e.re = mm3(K.r_i, b3);       // Wr Br + Wi Bi
        e.im = mm3(K.ni_r, b3);      // -Wi Br + Wr Bi
        d = e;
    }
    // keep z0(D + j), j < hop: lane (g, n2 = c) holds z[n1 = 4g + r][n2]
    constexpr int EO = F32OUT ? 8 : 4;
    const int dly = (kGemmN - hop) >> 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = 16 * (4 * g + r) + c - dly;
        gstore<S, F32OUT>(yr, unsigned(j) < unsigned(hop) ? (obase + j) * EO : kOutOfRange, d.re[r] * (1.0f / 16.0f),
                          d.im[r] * (1.0f / 16.0f));
    }
}

// Persistent launch over the same work items as the FFT engine (items of up
// to 16 blocks of N = 256); wave w of the workgroup filters blocks 4w..4w+3 of
// each item in turn.
template <Storage S, bool F32OUT>
__global__ __launch_bounds__(kThreads) void ols_gemm_kernel(const LaunchArgs A) {
    __shared__ float vlds[kVCapG];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    GemmConst K;
    load_consts(K, A.tw, lane);
    int v_offset = -1, lv_staged = -1;
    const int w = blockIdx.x;
    const int end = ld_uniform(A.wg_begin, w + 1);
    for (int i = ld_uniform(A.wg_begin, w); i < end; ++i) {
        const WorkItem it = ld_uniform(A.items, i);
        const ChannelDev cd = ld_uniform(A.ch, it.channel);
        if (cd.v_offset != v_offset || cd.lv != lv_staged) {
            __syncthreads();
            for (int q = threadIdx.x; q < cd.lv; q += kThreads) vlds[q] = A.v[cd.v_offset + q];
            __syncthreads();
            v_offset = cd.v_offset;
            lv_staged = cd.lv;
        }
        const int hop = cd.hop;
        const int64_t seg0 = int64_t(it.first_block) * hop - (kGemmN - hop);
        const int64_t clip = seg0 > 0 ? seg0 : 0;
        const char *xc = static_cast<const char *>(ld_uniform(A.x, it.channel));
        const auto xr = make_rsrc(xc + clip * 4, (cd.len - clip) * 4);
        constexpr int EO = F32OUT ? 8 : 4;
        const int64_t ob = int64_t(it.first_block) * hop;
        const auto yr = make_rsrc(static_cast<char *>(ld_uniform(A.y, it.channel)) + ob * EO, (cd.len - ob) * EO);
        // the next block's samples are loaded while this one is filtered; the
        // load is issued on every step (past the end after the last block) so
        // that the wait before the products has a fixed count
        const int first = kGemmHop4 * wave;                  // this wave's first block of the item
        const int nb = std::min(kGemmHop4, it.n_blocks - first);
        const int base0 = int(seg0 - clip);
        uint32_t u[4], un[4];
        if (nb > 0) gemm_load(xr, base0 + first * hop, lane, true, u);
        for (int q = 0; q < nb; ++q) {
            const int b = first + q;                         // block within the item
            gemm_load(xr, base0 + (b + 1) * hop, lane, q + 1 < nb, un);
            const int64_t m = int64_t(it.first_block) + b;
            int k1 = ld_uniform(A.sched, cd.sched_begin).k1;
            for (int e = 1; e < cd.sched_count; ++e) {
                const SchedDev sd = ld_uniform(A.sched, cd.sched_begin + e);
                if (sd.from_block <= m) k1 = sd.k1;
            }
            gemm_block<S, F32OUT>(K, u, yr, b * hop, hop, k1, cd.lv, vlds, lane);
#pragma unroll
            for (int j = 0; j < 4; ++j) u[j] = un[j];
        }
    }
}

template <Storage S, bool F32OUT> hipError_t launch_g(const LaunchArgs &A, hipStream_t s) {
    hipLaunchKernelGGL((ols_gemm_kernel<S, F32OUT>), dim3(A.n_wg), dim3(kThreads), 0, s, A);
    return hipGetLastError();
}

template <Storage S, bool F32OUT> int occ_g() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ols_gemm_kernel<S, F32OUT>, kThreads, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

int ols_gemm_wg_per_cu(Storage in, bool f32_out) {
    if (in == Storage::F16) return f32_out ? occ_g<Storage::F16, true>() : occ_g<Storage::F16, false>();
    if (in == Storage::BF16) return f32_out ? occ_g<Storage::BF16, true>() : occ_g<Storage::BF16, false>();
    return 1;
}

hipError_t launch_ols_gemm(const LaunchArgs &A, Storage in, bool f32_out, hipStream_t stream) {
    if (A.n_items <= 0 || A.n_wg <= 0) return hipSuccess;
    if (in == Storage::F16) return f32_out ? launch_g<Storage::F16, true>(A, stream) : launch_g<Storage::F16, false>(A, stream);
    if (in == Storage::BF16)
        return f32_out ? launch_g<Storage::BF16, true>(A, stream) : launch_g<Storage::BF16, false>(A, stream);
    return hipErrorInvalidValue;
}

}  // namespace vbw
