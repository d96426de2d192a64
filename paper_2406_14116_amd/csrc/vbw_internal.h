// vbw_internal.h -- device-table layouts shared by the plan code and the
// gfx950 kernels of the overlap-save variable-bandwidth filter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vbw {

constexpr int kMaxLog2N = 12;            // N <= 4096
constexpr int kMinLog2N = 4;             // N >= 16
constexpr int kPointsPerThread = 16;     // every thread owns 16 complex values
constexpr int kThreads = 256;            // workgroup size
constexpr int kTilePoints = kThreads * kPointsPerThread;  // 4096 values per workgroup
constexpr int kTwiddleN = 1 << kMaxLog2N;                 // one table of w_4096^r

// LDS: one padded 4096-value tile; a pad slot after every 16 values.
__host__ __device__ constexpr int lds_pad(int p) { return p + (p >> 4); }
constexpr int kLdsValues = lds_pad(kTilePoints);

// Per-channel constants (device table, 40 bytes).
struct ChannelDev {
    int64_t len;
    int32_t n;
    int32_t hop;
    int32_t lv;
    int32_t v_offset;
    int32_t sched_begin;   // first schedule entry of this channel
    int32_t sched_count;   // entries, sorted by from_block, first has from_block 0
    int64_t hist_off;      // streaming: first of this channel's N - hop history samples
};

// One bandwidth-schedule entry (16 bytes).
struct SchedDev {
    int64_t from_block;
    int32_t k1;
    int32_t pad;
};

// A run of `n_blocks` consecutive blocks of one channel.  The matrix-core
// engine takes tiles (n_blocks <= 4096 / N, one 4096-value tile); the FFT
// engine takes spans of any length (the team of one block walks through a
// contiguous part of the span).
struct WorkItem {
    int32_t channel;
    int32_t first_block;
    int32_t n_blocks;
    int32_t log2n;
};

enum class Storage : int { C64 = 0, F16 = 1, BF16 = 2, R32 = 3 };

struct LaunchArgs {
    const WorkItem *items;
    const ChannelDev *ch;
    const SchedDev *sched;
    const float *v;          // V pool, float32
    const float2 *tw;        // w_4096^r, r < 4096
    const void *const *x;    // per-channel input pointers
    void *const *y;          // per-channel output pointers
    const int32_t *wg_begin; // workgroup w owns items [wg_begin[w], wg_begin[w+1])
    const void *hist;        // streaming: history pool (storage format), else nullptr
    const int64_t *block0;   // streaming: stream block index of each channel's block 0, else nullptr
    int32_t n_items;
    int32_t n_wg;            // workgroups in the (persistent) launch
    int32_t prune;           // nonzero: stopband-pruned last forward / first inverse pass
    int32_t pad;
};

// Resident workgroups per CU of the kernel used for log2n_fixed (0: the
// kernel that dispatches on N), for sizing the persistent launch.
int ols_fft_wg_per_cu(int log2n_fixed, Storage in, bool f32_out);

// Host launchers (ols_fft.hip).  log2n_fixed = 0 selects the kernel that
// dispatches on each item's N; otherwise every item must have that N.
// t_start / t_stop (optional): events that take the kernel's own start and
// end time (hipExtLaunchKernel).
hipError_t launch_ols_fft(const LaunchArgs &args, int log2n_fixed, Storage in,
                          bool f32_out, hipStream_t stream, hipEvent_t t_start = nullptr,
                          hipEvent_t t_stop = nullptr);

// Matrix-core engine (ols_gemm.hip): N = 256, 16-bit storage only.
int ols_gemm_wg_per_cu(Storage in, bool f32_out);
hipError_t launch_ols_gemm(const LaunchArgs &args, Storage in, bool f32_out, hipStream_t stream,
                           hipEvent_t t_start = nullptr, hipEvent_t t_stop = nullptr);

// Streaming continuation (stream.hip): after a call, every channel's history
// becomes the last N - hop input samples of the call and its block counter
// advances by len / hop; reset zeroes both.
hipError_t launch_stream_update(const LaunchArgs &args, int n_channels, Storage in, void *hist, int64_t *block0,
                                hipStream_t stream);
hipError_t launch_stream_reset(void *hist, int64_t hist_bytes, int64_t *block0, int n_channels, hipStream_t stream);

// Allocation-free calls (scratch.hip): *ptr = this device's address of the
// static scratch array (VBW_NOALLOC_SCRATCH_BYTES bytes).  The first call for
// a device, which must be current, looks the address up and runs `init` on
// it once; later calls return the kept address.
hipError_t scratch_of_device(int device, unsigned char **ptr, hipError_t (*init)(unsigned char *));

// Streaming copy of `bytes` bytes (copy.hip); src and dst 16-byte aligned.
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int n_cu, hipStream_t stream);

}  // namespace vbw
