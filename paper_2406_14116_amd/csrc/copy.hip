// copy.hip -- streaming device-to-device copy used to calibrate the achievable
// HBM bandwidth (the denominator the filter's bandwidth is compared with).
// Each workgroup copies one contiguous 32 KiB chunk with eight 16-byte
// non-temporal loads in flight per thread, and the grid covers the buffer:
// measured faster than a persistent grid-stride loop, the runtime's
// device-to-device copy and torch's copy on MI355X.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vbw_internal.h"

namespace vbw {
namespace {

typedef unsigned u4v __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 8;
constexpr int64_t kCopyChunk = int64_t(kCopyUnroll) * kCopyThreads;   // 16-byte words per workgroup

__global__ __launch_bounds__(kCopyThreads) void copy_kernel(const u4v *__restrict__ src, u4v *__restrict__ dst,
                                                            int64_t n16) {
    const int64_t b = int64_t(blockIdx.x) * kCopyChunk + threadIdx.x;
    if (int64_t(blockIdx.x + 1) * kCopyChunk <= n16) {
        u4v v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + b + u * kCopyThreads);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + b + u * kCopyThreads);
    } else {
        for (int64_t i = b; i < n16; i += kCopyThreads) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    }
}

__global__ void copy_tail(const unsigned char *src, unsigned char *dst, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int n_cu, hipStream_t stream) {
    (void)n_cu;
    if (bytes <= 0) return hipSuccess;
    const int64_t n16 = bytes / 16;
    if (n16 > 0) {
        const int64_t grid = (n16 + kCopyChunk - 1) / kCopyChunk;
        if (grid > int64_t(INT32_MAX)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(copy_kernel, dim3(unsigned(grid)), dim3(kCopyThreads), 0, stream,
                           static_cast<const u4v *>(src), static_cast<u4v *>(dst), n16);
    }
    const int64_t rem = bytes - n16 * 16;
    if (rem > 0)
        hipLaunchKernelGGL(copy_tail, dim3(1), dim3(16), 0, stream, static_cast<const unsigned char *>(src) + n16 * 16,
                           static_cast<unsigned char *>(dst) + n16 * 16, rem);
    return hipGetLastError();
}

}  // namespace vbw
