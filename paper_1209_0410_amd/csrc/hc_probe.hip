// Streaming-read probe (a measurement aid, not a step of the method), gfx950.
//
// Reads a device buffer once with coalesced 16-byte loads from a grid that
// fills the device; timing it gives the HBM read bandwidth this device
// achieves, quoted beside the published peak.  Each block folds what it read
// into one word (XOR) and writes it, so no load can be dropped.
#include <string.h>

#include "hc_internal.h"

namespace hc {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeThreads) void k_read_probe(const u32x4 *buf, uint64_t n16,
                                                              uint32_t *sink)
{
    __shared__ uint32_t part[kProbeThreads / 64];
    const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads;
    uint64_t i = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t acc = 0;
    // kProbeUnroll loads in flight per thread, each step of the grid coalesced
    for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
        u32x4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; u++)
            v[u] = __builtin_nontemporal_load(buf + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; u++) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(buf + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc ^= __shfl_xor(acc, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
#pragma unroll
        for (int w = 0; w < kProbeThreads / 64; w++) a ^= part[w];
        sink[blockIdx.x] = a;
    }
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_read_probe(const void *d_buf, size_t bytes, uint32_t *d_sink, uint32_t blocks,
                        hc_stream stream)
{
    if (!d_buf || !d_sink || ((uintptr_t)d_buf & 15) || (bytes & 15)) return HC_ERR_INVALID;
    if (blocks < 1 || blocks > 65536) return HC_ERR_INVALID;
    if (bytes == 0) return HC_OK;
    hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(kProbeThreads), 0, (hipStream_t)stream,
                       (const u32x4 *)d_buf, (uint64_t)(bytes / 16), d_sink);
    return last_hip();
}

}  // extern "C"
