// Block-level exclusive prefix sums, shared by the index build, the uneven
// search and the banded search (each translation unit gets its own copy).
#pragma once

#include "hc_internal.h"

namespace hc {

constexpr int kScanThreads = 1024;

// Exclusive prefix sum of a wave's values; *total receives the wave's sum.
static __device__ inline uint32_t wave_excl_scan(uint32_t v, uint32_t *total)
{
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// In-place exclusive prefix sum of n values by one block of kScanThreads,
// starting from carry0.
static __device__ inline void block_scan_excl(uint32_t *a, uint64_t n, uint32_t carry0)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    __shared__ uint32_t carry_s;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) carry_s = carry0;
    __syncthreads();
    for (uint64_t base = 0; base < n; base += (uint64_t)kScanThreads * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint64_t i = base + (uint64_t)tid * 4 + j;
            v[j] = i < n ? a[i] : 0u;
            s += v[j];
        }
        uint32_t wt;
        uint32_t ex = wave_excl_scan(s, &wt);
        if (lane == 0) wsum[wave] = wt;
        __syncthreads();
        if (wave == 0) {
            uint32_t t = lane < kScanThreads / 64 ? wsum[lane] : 0u;
            uint32_t tot;
            uint32_t e = wave_excl_scan(t, &tot);
            if (lane < kScanThreads / 64) wsum[lane] = e;
        }
        __syncthreads();
        uint32_t run = carry_s + wsum[wave] + ex;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint64_t i = base + (uint64_t)tid * 4 + j;
            if (i < n) a[i] = run;
            run += v[j];
        }
        __syncthreads();
        if (tid == kScanThreads - 1) carry_s = run;
        __syncthreads();
    }
}

// In-place exclusive prefix sum of n values, one block of kScanThreads.
static __global__ __launch_bounds__(kScanThreads) void k_scan_excl(uint32_t *a, uint64_t n)
{
    block_scan_excl(a, n, 0u);
}

// Multi-block form for long arrays: kScanTile values per block.
//  k_scan_tile_sums: sums[b] = the sum of tile b;
//  k_scan_excl over the sums (one block);
//  k_scan_tiles: tile b scanned in place from sums[b].
constexpr uint64_t kScanTile = (uint64_t)kScanThreads * 4;

static __global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(const uint32_t *a,
                                                                        uint64_t n,
                                                                        uint32_t *sums)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint64_t i = base + (uint64_t)tid * 4 + j;
        s += i < n ? a[i] : 0u;
    }
    uint32_t wt;
    wave_excl_scan(s, &wt);
    if (lane == 0) wsum[wave] = wt;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int i = 0; i < kScanThreads / 64; i++) t += wsum[i];
        sums[blockIdx.x] = t;
    }
}

static __global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *a, uint64_t n,
                                                                    const uint32_t *sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    const uint64_t len = n - base < kScanTile ? n - base : kScanTile;
    block_scan_excl(a + base, len, sums[blockIdx.x]);
}

// Segmented form, one block per segment: segment s (values [s len, (s + 1) len))
// is scanned from s * seg_total.  Equal to the scan of all segments at once
// when every segment sums to seg_total.
static __global__ __launch_bounds__(kScanThreads) void k_scan_excl_seg(uint32_t *a, uint64_t len,
                                                                       uint32_t seg_total)
{
    block_scan_excl(a + (uint64_t)blockIdx.x * len, len, blockIdx.x * seg_total);
}

}  // namespace hc
