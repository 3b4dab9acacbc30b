// Exact kNN over the whole database (Eq. 3, ties broken by id), gfx950.
//
// Used for recall truth and training labels, not on the search path.  A block
// holds 256 queries (one per thread, the query in registers) and streams one
// slice of the database through LDS 64 rows at a time; every thread reads the
// same row at the same time (an LDS broadcast).  Each thread keeps its best 16
// in a sorted register list; a second kernel merges the slices per query.
#include <string.h>

#include <algorithm>

#include "hc_internal.h"

namespace hc {

constexpr int kBfThreads = 256;
constexpr int kBfRows = 64;        // database rows per LDS tile
constexpr int kBfList = 16;        // register list length; k <= kBfList
constexpr int kBfTargetBlocks = 2048;

__device__ inline void bf_insert(uint64_t (&L)[kBfList], uint64_t x)
{
    if (x < L[kBfList - 1]) {
#pragma unroll
        for (int i = kBfList - 1; i > 0; i--)
            L[i] = x < L[i - 1] ? L[i - 1] : (x < L[i] ? x : L[i]);
        L[0] = x < L[0] ? x : L[0];
    }
}

__device__ inline uint64_t bf_shfl_xor(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// partial[(q * slices + s) * k + j]: the k nearest of slice s, ascending.
__global__ __launch_bounds__(kBfThreads) void k_brute_slices(const uint8_t *db, uint64_t n,
                                                             const uint8_t *queries,
                                                             uint32_t nq, uint32_t k,
                                                             uint32_t slices,
                                                             uint64_t *partial)
{
    __shared__ uint4 tile[kBfRows * 8];
    __shared__ uint32_t tile_xx[kBfRows];
    const uint32_t qt = blockIdx.x / slices, s = blockIdx.x % slices;
    const uint32_t q = qt * kBfThreads + threadIdx.x;
    const bool live = q < nq;
    uint4 qv[8];
    uint32_t qq = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        qv[i] = live ? reinterpret_cast<const uint4 *>(queries + (uint64_t)q * kDim)[i]
                     : make_uint4(0, 0, 0, 0);
        qq = __builtin_amdgcn_udot4(qv[i].x, qv[i].x, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].y, qv[i].y, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].z, qv[i].z, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].w, qv[i].w, qq, false);
    }
    uint64_t L[kBfList];
#pragma unroll
    for (int i = 0; i < kBfList; i++) L[i] = kNone;

    const uint64_t per = (n + slices - 1) / slices;
    const uint64_t r0 = (uint64_t)s * per;
    const uint64_t r1 = std::min<uint64_t>(n, r0 + per);
    for (uint64_t t0 = r0; t0 < r1; t0 += kBfRows) {
        __syncthreads();
        for (int i = threadIdx.x; i < kBfRows * 8; i += kBfThreads) {
            const uint64_t r = t0 + (i >> 3);
            tile[i] = r < r1 ? reinterpret_cast<const uint4 *>(db + r * kDim)[i & 7]
                             : make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
        if (threadIdx.x < kBfRows) {
            uint32_t xx = 0;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint4 x = tile[threadIdx.x * 8 + i];
                xx = __builtin_amdgcn_udot4(x.x, x.x, xx, false);
                xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
                xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
                xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
            }
            tile_xx[threadIdx.x] = xx;
        }
        __syncthreads();
        const int rows = (int)std::min<uint64_t>(kBfRows, r1 - t0);
        for (int r = 0; r < rows; r++) {
            uint32_t qx = 0;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint4 x = tile[r * 8 + i];
                qx = __builtin_amdgcn_udot4(qv[i].x, x.x, qx, false);
                qx = __builtin_amdgcn_udot4(qv[i].y, x.y, qx, false);
                qx = __builtin_amdgcn_udot4(qv[i].z, x.z, qx, false);
                qx = __builtin_amdgcn_udot4(qv[i].w, x.w, qx, false);
            }
            const uint32_t d = qq + tile_xx[r] - 2u * qx;
            bf_insert(L, ((uint64_t)d << 32) | (uint32_t)(t0 + r));
        }
    }
    if (live) {
        uint64_t *out = partial + ((uint64_t)q * slices + s) * k;
#pragma unroll
        for (int i = 0; i < kBfList; i++)
            if ((uint32_t)i < k) out[i] = L[i];
    }
}

// One wave per query: merges the slices' lists and keeps the k nearest.
__global__ __launch_bounds__(64) void k_brute_merge(const uint64_t *partial, uint32_t nq,
                                                    uint32_t k, uint32_t slices,
                                                    uint32_t *out_ids, uint32_t *out_dists)
{
    const uint32_t q = blockIdx.x;
    const int lane = threadIdx.x;
    uint64_t L[kBfList];
#pragma unroll
    for (int i = 0; i < kBfList; i++) L[i] = kNone;
    const uint64_t *src = partial + (uint64_t)q * slices * k;
    for (uint64_t i = lane; i < (uint64_t)slices * k; i += 64) bf_insert(L, src[i]);
    uint64_t mine = kNone;
    for (uint32_t j = 0; j < k; j++) {
        uint64_t m = L[0];
#pragma unroll
        for (int x = 32; x >= 1; x >>= 1) {
            const uint64_t o = bf_shfl_xor(m, x);
            m = o < m ? o : m;
        }
        if ((uint32_t)lane == j) mine = m;
        if (m != kNone && L[0] == m) {
#pragma unroll
            for (int i = 0; i < kBfList - 1; i++) L[i] = L[i + 1];
            L[kBfList - 1] = kNone;
        }
    }
    if ((uint32_t)lane < k) {
        out_ids[(uint64_t)q * k + lane] = (uint32_t)mine;
        out_dists[(uint64_t)q * k + lane] = (uint32_t)(mine >> 32);
    }
}

static uint32_t bf_slices(uint64_t n, uint32_t nq)
{
    const uint64_t qtiles = (nq + kBfThreads - 1) / kBfThreads;
    uint64_t s = std::max<uint64_t>(1, kBfTargetBlocks / std::max<uint64_t>(qtiles, 1));
    s = std::min<uint64_t>(s, 256);
    s = std::min<uint64_t>(s, std::max<uint64_t>(1, n / kBfRows));
    return (uint32_t)s;
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_brute_force_scratch_bytes(uint64_t n, uint32_t nq, uint32_t k, size_t *bytes)
{
    if (!bytes || n == 0 || k < 1) return HC_ERR_INVALID;
    if (k > (uint32_t)kBfList) return HC_ERR_UNSUPPORTED;
    *bytes = align256(sizeof(uint64_t) * (size_t)std::max<uint32_t>(nq, 1) *
                      bf_slices(n, nq) * k);
    return HC_OK;
}

hc_status hc_brute_force(const uint8_t *d_db, uint64_t n, const uint8_t *d_queries,
                         uint32_t nq, uint32_t k, uint32_t *d_out_ids,
                         uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                         hc_stream stream)
{
    if (!d_db || !d_queries || !d_out_ids || !d_out_dists || !d_scratch || n == 0 || k < 1)
        return HC_ERR_INVALID;
    if (((uintptr_t)d_db & 15) || ((uintptr_t)d_queries & 15) || ((uintptr_t)d_scratch & 7))
        return HC_ERR_INVALID;
    if (k > (uint32_t)kBfList || n >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;
    if (nq == 0) return HC_OK;
    size_t need = 0;
    hc_brute_force_scratch_bytes(n, nq, k, &need);
    if (scratch_bytes < need) return HC_ERR_SIZE;
    const uint32_t slices = bf_slices(n, nq);
    const uint32_t qtiles = (nq + kBfThreads - 1) / kBfThreads;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_brute_slices, dim3(qtiles * slices), dim3(kBfThreads), 0, s, d_db, n,
                       d_queries, nq, k, slices, (uint64_t *)d_scratch);
    hipLaunchKernelGGL(k_brute_merge, dim3(nq), dim3(64), 0, s, (const uint64_t *)d_scratch,
                       nq, k, slices, d_out_ids, d_out_dists);
    return last_hip();
}

}  // extern "C"
