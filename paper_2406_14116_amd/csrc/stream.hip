// stream.hip -- state of a filter that continues one input stream across calls.
//
// The paper's input is one unbounded stream cut into blocks that advance by M
// samples (Sec. II).  A streaming plan filters it in chunks: a call's block 0
// needs the N - M input samples before the chunk (its history) and the band
// schedule counts blocks from the start of the stream.  After each call the
// history becomes the chunk's last N - M samples and the block counter of the
// channel advances by len / M (chunks are whole blocks, len >= N - M).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vbw_internal.h"

namespace vbw {
namespace {

template <int EI> struct Word;
template <> struct Word<8> { typedef uint2 T; };
template <> struct Word<4> { typedef uint32_t T; };

// One workgroup per channel.
template <int EI> __global__ __launch_bounds__(256) void stream_update_kernel(const LaunchArgs A, void *hist,
                                                                              int64_t *block0) {
    typedef typename Word<EI>::T W;
    const int c = blockIdx.x;
    const ChannelDev cd = A.ch[c];
    if (cd.len <= 0) return;
    const int h = cd.n - cd.hop;
    const W *x = static_cast<const W *>(A.x[c]) + (cd.len - h);
    W *dst = static_cast<W *>(hist) + cd.hist_off;
    for (int i = threadIdx.x; i < h; i += blockDim.x) dst[i] = x[i];
    if (threadIdx.x == 0) block0[c] += cd.len / cd.hop;
}

__global__ __launch_bounds__(256) void stream_reset_kernel(uint32_t *hist, int64_t words, int64_t *block0, int nch) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride) hist[i] = 0u;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nch; i += stride) block0[i] = 0;
}

}  // namespace

hipError_t launch_stream_update(const LaunchArgs &args, int n_channels, Storage in, void *hist, int64_t *block0,
                                hipStream_t stream) {
    if (n_channels <= 0) return hipSuccess;
    if (in == Storage::C64)
        hipLaunchKernelGGL(stream_update_kernel<8>, dim3(n_channels), dim3(256), 0, stream, args, hist, block0);
    else
        hipLaunchKernelGGL(stream_update_kernel<4>, dim3(n_channels), dim3(256), 0, stream, args, hist, block0);
    return hipGetLastError();
}

hipError_t launch_stream_reset(void *hist, int64_t hist_bytes, int64_t *block0, int n_channels, hipStream_t stream) {
    const int64_t words = hist_bytes / 4;
    int64_t n = words > n_channels ? words : n_channels;
    int grid = int((n + 255) / 256);
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(stream_reset_kernel, dim3(grid), dim3(256), 0, stream, static_cast<uint32_t *>(hist), words,
                       block0, n_channels);
    return hipGetLastError();
}

}  // namespace vbw
