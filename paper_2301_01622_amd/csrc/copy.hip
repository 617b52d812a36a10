// Streaming device-to-device copy used for state checkpoints.  It is also
// the reference kernel whose HBM counters calibrate the traffic measurement
// of the step kernels: it reads and writes exactly `bytes` bytes.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace lbm {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte vector per thread, streamed past the caches.
__global__ __launch_bounds__(256) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(256) void k_copy1(const unsigned char *__restrict__ src, unsigned char *__restrict__ dst,
                                               int64_t begin, int64_t end)
{
    const int64_t i = begin + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < end) dst[i] = src[i];
}

} // namespace

hipError_t launch_copy(const lbm_ctx *c, const void *src, void *dst, int64_t bytes)
{
    if (bytes <= 0) return hipSuccess;
    const bool aligned = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
    int64_t n16 = aligned ? bytes / 16 : 0;
    if (n16 > 0) {
        const int64_t blocks = (n16 + 255) / 256;
        if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, c->stream, static_cast<const u32x4 *>(src),
                           static_cast<u32x4 *>(dst), n16);
    }
    const int64_t rest = bytes - n16 * 16;
    if (rest > 0) {
        const int64_t blocks = (rest + 255) / 256;
        hipLaunchKernelGGL(k_copy1, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           static_cast<const unsigned char *>(src), static_cast<unsigned char *>(dst), n16 * 16, bytes);
    }
    return hipGetLastError();
}

} // namespace lbm
