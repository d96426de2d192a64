// ols_gemm.hip -- overlap-save variable-bandwidth filtering with the small DFTs
// run as dense matrix products on the gfx950 matrix cores (FP16 operands, FP32
// accumulation), for 16-bit channel storage and N = 256.
//
// Paper: Moryakova & Johansson, arXiv 2406.14116.  Same operation as the FFT
// engine: Sec. II steps 1-5 with the HFSO coefficients of eqs. (5)-(6).
//
// The 256-point DFT is split as 16 x 16 (n = 16 n1 + n2, k = k1 + 16 k2) into
// four complex 16x16x16 products per block (S1, S2 forward; S3, S4 inverse),
// with the twiddles w256^{n2 k1} between them; gemm_layout.h gives the lane
// layout.  Each complex product is a set of 16x16x32 MFMAs whose contraction
// dimension carries (real parts, imaginary parts): one MFMA per real output.
//
// Precision.  The DFT matrix and the FP32 intermediates enter the matrix
// cores as hi + lo FP16 pairs (hi = RN(v), lo = RN(v - hi)); each real
// product is hi*hi + lo*hi + hi*lo with FP32 accumulation (the lo*lo term,
// about 2^-22 relative, is dropped).
// Range.  Linear filtering is scale-free (Sec. II), so every block is scaled
// by a power of two 2^s, exactly, before its first product and by 2^-s at the
// store: s puts the block's largest |re|, |im| in [2^t, 2^(t+1)) with t = 6
// (less when some |V(r)| exceeds 1).  The intermediates grow by at most 16 per
// product and by the 1/16 applied with H_R, so every FP16 operand stays below
// 2^15, and the operands of a block's large values stay in the normal range.
// Blocks of any finite 16-bit input (FP16 subnormals to 65504, BF16 over its
// whole range) are therefore filtered with the same relative accuracy; only
// values below 2^-20 of their block's largest contribute with absolute error
// (about 2^-31 of that largest).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "gemm_layout.h"
#include "vbw_internal.h"

namespace vbw {
namespace {

using namespace gemm;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

constexpr int kGemmN = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kBufFlags = 0x00020000;
constexpr int kNT = 2;
constexpr int kOutOfRange = int(0x80000000u);   // as an unsigned offset: past every resource's end
constexpr int kVCapG = kGemmN / 2;
constexpr int kTarget = 6;                       // block maximum scaled into [2^6, 2^7)

constexpr int64_t kMaxRecords = 0x7ffff000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int64_t bytes) {
    const int n = int(bytes <= 0 ? 0 : (bytes < kMaxRecords ? bytes : kMaxRecords));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, n, kBufFlags);
}

// Bytes from block q's first sample to the channel end, min(b0 - q step,
// kMaxRecords), in 32-bit scalar arithmetic (the scalar unit has no 64-bit
// ordered compare): the first `sat` blocks have more than kMaxRecords left,
// and below it the low 32 bits of b0 - q step are exact.  Valid for blocks
// that have samples left.
struct BytesLeft {
    uint32_t b0, step;
    int sat;
    __device__ __forceinline__ BytesLeft(int64_t bytes0, uint32_t step_) : b0(uint32_t(bytes0)), step(step_), sat(0) {
        if (bytes0 > kMaxRecords) sat = int((bytes0 - kMaxRecords + step - 1) / step);
    }
    __device__ __forceinline__ int at(int q) const {
        return q < sat ? int(kMaxRecords) : int(b0 - uint32_t(q) * step);
    }
};

template <typename T> __device__ __forceinline__ T ld_uniform(const T *p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) T cT;
    return ((cT *)p)[__builtin_amdgcn_readfirstlane(i)];
#else
    return p[i];
#endif
}

__device__ __forceinline__ f4 mfma(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }

// ------------------------------------------------------------ hi/lo split
struct Split {
    h8 hi, lo;
};

__device__ __forceinline__ uint32_t pack_f16(float a, float b) {   // RN, one v_cvt_pk_f16_f32
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, h2v));
}
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {  // RN, one v_cvt_pk_bf16_f32
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2v));
}
// FP16 pair RN(v0 - hi0), RN(v1 - hi1) for h = (hi0, hi1): one mixed-precision
// multiply-add per value reads the FP16 half and rounds straight to FP16.
// Its operands are always results of ordinary vector instructions, never a
// matrix-core result read directly: the compiler inserts the wait states such
// a read needs before its own instructions, not before inline assembly.
__device__ __forceinline__ uint32_t residual_pair(uint32_t h, float v0, float v1) {
    uint32_t l;
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=&v"(l) : "v"(h), "v"(v0));
    asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(l) : "v"(h), "v"(v1));
    return l;
}
// After the residuals of an operand: two wait states before any instruction
// reads them.  A matrix-core read of a register a vector instruction has just
// written needs them; the compiler counts them for its own instructions only,
// and this statement, which takes the four registers as inputs and outputs,
// comes after every residual and before every use.
__device__ __forceinline__ void residuals_settle(u4v &lo) {
    asm volatile("s_nop 1" : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]));
}
// operand (re[0..3] | im[0..3]) as hi + lo
__device__ __forceinline__ Split split(f4 re, f4 im) {
    u4v hi, lo;
    hi[0] = pack_f16(re[0], re[1]);
    hi[1] = pack_f16(re[2], re[3]);
    hi[2] = pack_f16(im[0], im[1]);
    hi[3] = pack_f16(im[2], im[3]);
    lo[0] = residual_pair(hi[0], re[0], re[1]);
    lo[1] = residual_pair(hi[1], re[2], re[3]);
    lo[2] = residual_pair(hi[2], im[0], im[1]);
    lo[3] = residual_pair(hi[3], im[2], im[3]);
    residuals_settle(lo);
    return {__builtin_bit_cast(h8, hi), __builtin_bit_cast(h8, lo)};
}
// operand (a0, b0, a1, b1, ..., a3, b3) as hi + lo: S1's DFT-matrix operand,
// whose contraction entries pair with the samples as stored, (re, im) each
__device__ __forceinline__ Split split_interleaved(f4 a, f4 b) {
    u4v hi, lo;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        hi[j] = pack_f16(a[j], b[j]);
        lo[j] = residual_pair(hi[j], a[j], b[j]);
    }
    residuals_settle(lo);
    return {__builtin_bit_cast(h8, hi), __builtin_bit_cast(h8, lo)};
}
// Real product of split operands: P*Q ~ Phi*Qhi + Plo*Qhi + Phi*Qlo.
__device__ __forceinline__ f4 mm3(const Split &p, const Split &q) {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    return mfma(p.hi, q.lo, mfma(p.lo, q.hi, mfma(p.hi, q.hi, z)));
}
// P exact in FP16: P*Qhi + P*Qlo.
__device__ __forceinline__ f4 mm2(h8 p, const Split &q) {
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    return mfma(p, q.lo, mfma(p, q.hi, z));
}

// ------------------------------------------------------------ constants
// The DFT-matrix operands each lane feeds to the four products (exponents
// from gemm_layout.h), as the two real operands of a complex product, and
// the four twiddles of its accumulator slots.
// S3's DFT-matrix entries are S2's (W is symmetric and S3's B layout is
// S2's A layout), so S3 runs as the conjugate of a forward product:
// sum Y conj W = conj(sum conj(Y) W), with the signs folded into the
// neighbouring multiplies.
struct GemmConst {
    Split s1r, s1i;   // S1 (B = W):      (Re W, -Im W), (Im W, Re W) interleaved
    Split s2r, s2i;   // S2 (A = W) and S3 (B = W, conjugated data)
    Split s4r, s4i;   // S4 (A = conj W): [Re W |  Im W], [-Im W | Re W]
    float2 tw[4];
};

template <int (*E)(int, int, int)>
__device__ __forceinline__ void w_entries(const float2 *tw4096, int g, int c, f4 &wr, f4 &wi) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float2 w = tw4096[256 * E(g, c, j)];   // w16^e = w4096^{256 e}
        wr[j] = w.x;
        wi[j] = w.y;
    }
}

__device__ __forceinline__ void load_consts(GemmConst &k, const float2 *__restrict__ tw4096, int lane) {
    const int g = lane >> 4, c = lane & 15;
    f4 wr, wi;
    w_entries<s1_w>(tw4096, g, c, wr, wi);
    k.s1r = split_interleaved(wr, -wi);
    k.s1i = split_interleaved(wi, wr);
    w_entries<s2_w>(tw4096, g, c, wr, wi);
    k.s2r = split(wr, -wi);
    k.s2i = split(wi, wr);
    w_entries<s4_w>(tw4096, g, c, wr, wi);
    k.s4r = split(wr, wi);
    k.s4i = split(-wi, wr);
#pragma unroll
    for (int r = 0; r < 4; ++r) k.tw[r] = tw4096[16 * tw_e(g, c, r)];
}

// ------------------------------------------------------------ block scale
// Largest of a wave's unsigned values, as a wave-uniform value: row DPP
// shifts leave each row's maximum in its lane 15, the two row broadcasts
// carry it on to lane 63.
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xf, 0xf, true)));   // row_shr:1
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xf, 0xf, true)));   // row_shr:2
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xf, 0xf, true)));   // row_shr:4
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xf, 0xf, true)));   // row_shr:8
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xa, 0xf, false)));  // row_bcast:15, rows 1, 3
    x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xc, 0xf, false)));  // row_bcast:31, rows 2, 3
    return __builtin_amdgcn_readlane(x, 63);
}

// Largest |re|, |im| of the block's 16-bit samples as a bit pattern with the
// sign cleared (for sign-magnitude formats integer order is value order).
__device__ __forceinline__ uint32_t block_max_bits(const uint32_t (&u)[4]) {
    us2 m = __builtin_bit_cast(us2, u[0] & 0x7fff7fffu);
#pragma unroll
    for (int j = 1; j < 4; ++j) m = __builtin_elementwise_max(m, __builtin_bit_cast(us2, u[j] & 0x7fff7fffu));
    return wave_max(max(uint32_t(m[0]), uint32_t(m[1])));
}

// e with 2^e <= value < 2^(e+1) for a nonzero 16-bit magnitude pattern m.
template <Storage S> __device__ __forceinline__ int exponent_of(uint32_t m) {
    constexpr int MB = S == Storage::F16 ? 10 : 7;          // mantissa bits
    constexpr int BIAS = S == Storage::F16 ? 15 : 127;
    const int eb = int(m >> MB);
    return eb ? eb - BIAS : (31 - __builtin_clz(m)) - (BIAS + MB - 1);   // subnormal: m 2^(1-BIAS-MB)
}

// ------------------------------------------------------------ one block
template <bool F32OUT, Storage S> __device__ __forceinline__ void gstore(__amdgpu_buffer_rsrc_t r, int off, float re,
                                                                        float im) {
    if constexpr (F32OUT) {
        __builtin_amdgcn_raw_buffer_store_b64(u2v{__float_as_uint(re), __float_as_uint(im)}, r, off, 0, kNT);
    } else if constexpr (S == Storage::F16) {
        __builtin_amdgcn_raw_buffer_store_b32(pack_f16(re, im), r, off, 0, kNT);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(pack_bf16(re, im), r, off, 0, kNT);
    }
}

struct CF4 {
    f4 re, im;
};

// Twiddles w256^{n2 k1} times the block scale 2^sh (FP16 input takes its
// scale there), recomputed only when sh changes from one block to the next.
struct ScaledTw {
    float2 w[4];
    int sh = INT32_MIN;
};

// One OLS block of N = 256 by one wave.  u[j]: the (re, im) 16-bit pair of
// sample 16 in_row(g, j) + c; hf[r]: H_R / 16 of the bin in slot r; tgt: the
// exponent the block maximum is scaled to; yr: the output from the block's
// first kept sample on, oofs[r]: byte offset of slot r's sample in it
// (kOutOfRange: not kept).
template <Storage S, bool F32OUT>
__device__ __forceinline__ void gemm_block(const GemmConst &K, const uint32_t (&u)[4], const float (&hf)[4], int tgt,
                                           __amdgpu_buffer_rsrc_t yr, const int (&oofs)[4], ScaledTw &tws) {
    const uint32_t mb = block_max_bits(u);                  // wave-uniform
    const int e = mb ? exponent_of<S>(mb) : tgt;
    const int sh = tgt - e;            // block scale 2^sh
    const int dsc = e - tgt - 4;       // at the store: 2^-sh and the other 1/16 of 1/N

    // S1 operand: the samples as stored, (re, im) interleaved (FP16 as is;
    // BF16 scaled, then rounded to FP16)
    u4v xa;
    if constexpr (S == Storage::F16) {
#pragma unroll
        for (int j = 0; j < 4; ++j) xa[j] = u[j];
        if (sh != tws.sh) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                tws.w[r] = make_float2(__builtin_ldexpf(K.tw[r].x, sh), __builtin_ldexpf(K.tw[r].y, sh));
            tws.sh = sh;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            xa[j] = pack_f16(__builtin_ldexpf(__uint_as_float(u[j] << 16), sh),
                             __builtin_ldexpf(__uint_as_float(u[j] & 0xffff0000u), sh));
    }
    const h8 x = __builtin_bit_cast(h8, xa);
    CF4 d;
    d.re = mm2(x, K.s1r);
    d.im = mm2(x, K.s1i);
    // twiddle w256^{n2 k1}
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float2 w = S == Storage::F16 ? tws.w[r] : K.tw[r];
        const float a = d.re[r], b = d.im[r];
        d.re[r] = a * w.x - b * w.y;
        d.im[r] = a * w.y + b * w.x;
    }
    // S2: bins k = c + 16 (4g + r)
    CF4 q;
    {
        const Split b1 = split(d.re, d.im);
        q.re = mm3(K.s2r, b1);
        q.im = mm3(K.s2i, b1);
    }
    // conj(H_R Y) / 16 (the other 1/16 of the inverse's 1/N is applied at
    // the store)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        q.re[r] *= hf[r];
        q.im[r] *= -hf[r];
    }
    // S3 as conj(sum conj(Y) W): d = -conj of the product below
    {
        const Split a2 = split(q.re, q.im);
        d.re = mm3(a2, K.s2r);
        d.im = mm3(a2, K.s2i);
    }
    // conjugate twiddle of conj(d): (a - j b) conj(w)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float2 w = K.tw[r];
        const float a = d.re[r], b = d.im[r];
        d.re[r] = a * w.x - b * w.y;
        d.im[r] = -(b * w.x) - a * w.y;
    }
    // S4: slot r of lane (g, c) holds z[out_row(g, r)][c]
    {
        const Split b3 = split(d.re, d.im);
        q.re = mm3(K.s4r, b3);
        q.im = mm3(K.s4i, b3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        gstore<F32OUT, S>(yr, oofs[r], __builtin_ldexpf(q.re[r], dsc), __builtin_ldexpf(q.im[r], dsc));
}

// H_R / 16 of this lane's four bins k = c + 16 (4 g + r) for the edge k1
// (eq. (6) with the mirror H_R(N - k) = H_R(k)); vl: V staged in LDS.
__device__ __forceinline__ void h_factors(float (&hf)[4], int lane, int k1, int lv, const float *vl) {
    const int g = lane >> 4, c = lane & 15;
    const int k2 = k1 + lv - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = c + 16 * (4 * g + r);
        const int kk = k <= kGemmN / 2 ? k : kGemmN - k;
        float f = kk < k1 ? 1.0f / 16.0f : 0.0f;
        if (kk >= k1 && kk <= k2) f = vl[kk - k1] * (1.0f / 16.0f);
        hf[r] = f;
    }
}

// ------------------------------------------------------------ kernel
// Persistent launch over spans (runs of consecutive blocks of one channel):
// wave w of the workgroup filters the contiguous quarter [w n / 4,
// (w+1) n / 4) of each span's n blocks.  With M = 192 (CARRY) a block's
// slot 0 is the previous block's slot 3, so each later block loads 3 of its
// 4 slots; the next block's loads are in flight during the current block.
// Every block gets buffer resources that start at its own first input
// sample and first output sample (scalar arithmetic), so the lanes' offsets
// stay fixed from block to block.
template <Storage S, bool F32OUT, bool CARRY>
__device__ __forceinline__ void run_span(const LaunchArgs &A, const WorkItem &sp, const ChannelDev &cd,
                                         const GemmConst &K, const float *vl, int tgt, int lane, int wave) {
    constexpr int EO = F32OUT ? 8 : 4;
    const int g = lane >> 4, c = lane & 15;
    const int hop = cd.hop;
    const int n = sp.n_blocks;
    const int lo = (wave * n) / kWaves;
    const int cnt = ((wave + 1) * n) / kWaves - lo;
    if (cnt <= 0) return;
    tgt = __builtin_amdgcn_readfirstlane(tgt);                 // wave-uniform: scalar block scales
    const char *const xb = static_cast<const char *>(ld_uniform(A.x, sp.channel));
    char *const yb = static_cast<char *>(ld_uniform(A.y, sp.channel));
    const int64_t len = cd.len;
    const int64_t m0 = int64_t(sp.first_block) + lo;         // the wave's first block
    const int64_t seg0 = m0 * hop - (kGemmN - hop);          // its first input sample (may be < 0)
    // per-lane byte offsets: input slot j from the block's first input sample,
    // output slot r from its first kept output sample (kOutOfRange: not kept)
    const int dly = (kGemmN - hop) >> 1;
    int iofs[4], oofs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) iofs[j] = 4 * (16 * in_row(g, j) + c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int jj = 16 * out_row(g, r) + c - dly;
        oofs[r] = unsigned(jj) < unsigned(hop) ? EO * jj : kOutOfRange;
    }
    // band schedule: entry in force at the wave's first block (binary search),
    // then one step forward whenever a block reaches the next entry (nq: that
    // entry's block, relative to m0)
    int ea = 0, eb = cd.sched_count;                 // sched[ea].from_block <= m0 < sched[eb].from_block
    while (eb - ea > 1) {
        const int mid = (ea + eb) >> 1;
        if (ld_uniform(A.sched, cd.sched_begin + mid).from_block <= m0) ea = mid;
        else eb = mid;
    }
    auto next_rel = [&](int e) {
        if (e + 1 >= cd.sched_count) return INT32_MAX;
        const int64_t d = ld_uniform(A.sched, cd.sched_begin + e + 1).from_block - m0;
        return d < INT32_MAX ? int(d) : INT32_MAX;
    };
    int k1 = ld_uniform(A.sched, cd.sched_begin + ea).k1;
    int nq = next_rel(ea);
    int k1c = -1;
    float hf[4];
    ScaledTw tws;

    // Loads of block q's slots J0..3 (q == cnt: none are needed; they read 0
    // from an empty resource, so that every step issues the same loads).  The
    // blocks before qpos start before sample 0: they read from the channel
    // start at a negative offset, past the resource's end as an unsigned
    // offset, which gives 0, the zero history.
    const int qpos = seg0 >= 0 ? 0 : int((-seg0 + hop - 1) / hop);
    const BytesLeft in_left(4 * (len - seg0), 4u * uint32_t(hop));
    auto issue = [&](uint32_t(&dst)[4], int q, int j0) {
        __builtin_amdgcn_s_setprio(1);
        if (q < cnt && q >= qpos) {
            const auto r = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char *>(xb + 4 * (seg0 + int64_t(q) * hop)), 0, in_left.at(q), kBufFlags);
#pragma unroll
            for (int j = j0; j < 4; ++j) dst[j] = __builtin_amdgcn_raw_buffer_load_b32(r, iofs[j], 0, kNT);
        } else {
            const auto r = make_rsrc(xb, q < cnt ? 4 * len : 0);
            const int b = q < cnt ? 4 * int(seg0 + int64_t(q) * hop) : 0;
#pragma unroll
            for (int j = j0; j < 4; ++j) dst[j] = __builtin_amdgcn_raw_buffer_load_b32(r, b + iofs[j], 0, kNT);
        }
        __builtin_amdgcn_s_setprio(0);
    };
    const BytesLeft out_left(int64_t(EO) * (len - m0 * hop), uint32_t(EO * hop));
    auto block = [&](const uint32_t(&u)[4], int q) {
        if (q >= nq) {
            ++ea;
            k1 = ld_uniform(A.sched, cd.sched_begin + ea).k1;
            nq = next_rel(ea);
        }
        if (k1 != k1c) {
            h_factors(hf, lane, k1, cd.lv, vl);
            k1c = k1;
        }
        const auto yr = __builtin_amdgcn_make_buffer_rsrc(yb + EO * (m0 + q) * hop, 0, out_left.at(q), kBufFlags);
        gemm_block<S, F32OUT>(K, u, hf, tgt, yr, oofs, tws);         // the block's first kept output sample on
    };

    // two blocks per step, so that the loads alternate between two register
    // sets instead of being copied from one to the other
    uint32_t ua[4], ub[4];
    issue(ua, 0, 0);
    int q = 0;
    for (; q + 1 < cnt; q += 2) {
        issue(ub, q + 1, CARRY ? 1 : 0);
        block(ua, q);
        if constexpr (CARRY) ub[0] = ua[3];
        issue(ua, q + 2, CARRY ? 1 : 0);
        block(ub, q + 1);
        if constexpr (CARRY) ua[0] = ub[3];
    }
    if (q < cnt) block(ua, q);
}

template <Storage S, bool F32OUT>
__global__ __launch_bounds__(kThreads) void ols_gemm_kernel(const LaunchArgs A) {
    __shared__ float vlds[kVCapG];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar control flow
    GemmConst K;
    load_consts(K, A.tw, lane);
    int v_offset = -1, lv_staged = -1, tgt = kTarget;
    const int w = blockIdx.x;
    const int end = ld_uniform(A.wg_begin, w + 1);
    for (int i = ld_uniform(A.wg_begin, w); i < end; ++i) {
        const WorkItem sp = ld_uniform(A.items, i);
        const ChannelDev cd = ld_uniform(A.ch, sp.channel);
        if (cd.v_offset != v_offset || cd.lv != lv_staged) {
            // stage V; a set with some |V(r)| > 1 lowers the block target so
            // that H_R X stays in range
            __syncthreads();
            for (int q = threadIdx.x; q < cd.lv; q += kThreads) vlds[q] = A.v[cd.v_offset + q];
            uint32_t vm = 0;
            for (int q = lane; q < cd.lv; q += 64) vm = max(vm, __float_as_uint(fabsf(A.v[cd.v_offset + q])));
            vm = wave_max(vm);
            tgt = kTarget - (vm > 0x3f800000u ? int(vm >> 23) - 126 : 0);
            __syncthreads();
            v_offset = cd.v_offset;
            lv_staged = cd.lv;
        }
        if (cd.hop == 3 * kGemmN / 4) run_span<S, F32OUT, true>(A, sp, cd, K, vlds, tgt, lane, wave);
        else run_span<S, F32OUT, false>(A, sp, cd, K, vlds, tgt, lane, wave);
    }
}

// With events, through hipExtLaunchKernel, which records the kernel's own
// start and end time in them.
template <Storage S, bool F32OUT>
hipError_t launch_g(const LaunchArgs &A, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (t0 || t1)
        hipExtLaunchKernelGGL(ols_gemm_kernel<S, F32OUT>, dim3(A.n_wg), dim3(kThreads), 0, s, t0, t1, 0, A);
    else
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

hipError_t launch_ols_gemm(const LaunchArgs &A, Storage in, bool f32_out, hipStream_t stream, hipEvent_t t0,
                           hipEvent_t t1) {
    if (A.n_items <= 0 || A.n_wg <= 0) return hipSuccess;
    if (in == Storage::F16)
        return f32_out ? launch_g<Storage::F16, true>(A, stream, t0, t1) : launch_g<Storage::F16, false>(A, stream, t0, t1);
    if (in == Storage::BF16)
        return f32_out ? launch_g<Storage::BF16, true>(A, stream, t0, t1)
                       : launch_g<Storage::BF16, false>(A, stream, t0, t1);
    return hipErrorInvalidValue;
}

}  // namespace vbw
