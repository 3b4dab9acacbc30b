// Banded search for large batches with large windows (gfx950).
//
// In a batch of nq queries with windows of w entries per side, a list entry
// lies in about nq * 2w / n windows of the same curve (at n = 10^7, nq = 10^5,
// w = 27,648: ~550).  The gather search fetches the row once per window; here
// the batch is arranged so that a row is fetched once per group of queries:
//  1. every query's place in every curve (the same descent as the search);
//  2. per curve, the queries ordered by place (a counting sort on place
//     buckets of 2^kBucketShift entries);
//  3. a wavefront takes 64 consecutive queries of one curve and streams the
//     union of their windows through LDS, 64 list entries at a time (ids and
//     rows, x.x of each row); lane i keeps query i in registers and, for every
//     entry inside its own window, computes the exact squared distance (dot4)
//     and offers (distance, id) to its register top-k;
//  4. a merge takes each query's per-curve lists and keeps the k nearest
//     distinct ids.
// The candidates, distances and order are exactly those of the gather search
// (Alg. 2): only the grouping of the work differs, so the results are
// identical.  The per-pair cost is arithmetic (32 dot4 per pair); the rows
// read from HBM drop by the number of queries sharing them.
#include <string.h>

#include <algorithm>

#include "hc_device.h"
#include "hc_scan.h"

namespace hc {

constexpr int kBucketShift = 8;   // place buckets of 256 list entries
constexpr int kBandRows = 64;     // list entries per LDS tile
constexpr int kBandK = 16;        // longest list kept per query and curve

struct BandArgs {
    IndexView v;
    const uint8_t *queries;
    const Key *qkeys;
    uint32_t nq, k, w_fixed;
    const uint32_t *d_w;
    uint32_t *pos;        // [q][curves]
    uint32_t *counts;     // [curves][nbuckets] -> scanned -> cursors
    uint32_t nbuckets;
    uint32_t *order;      // [curves][nq]
    uint64_t *partial;    // [q][curves][k]
    uint32_t *out_ids, *out_dists;
};

struct BandLayout {
    size_t qkeys, pos, counts, order, partial, total;
    uint32_t nbuckets;
};

inline BandLayout band_layout(uint32_t curves, uint64_t n, uint32_t nq)
{
    BandLayout L{};
    L.nbuckets = (uint32_t)((n >> kBucketShift) + 1);
    size_t off = 0;
    L.qkeys = off;
    off = align256(off + sizeof(Key) * (size_t)nq * curves);
    L.pos = off;
    off = align256(off + sizeof(uint32_t) * (size_t)nq * curves);
    L.counts = off;
    off = align256(off + sizeof(uint32_t) * (size_t)curves * L.nbuckets);
    L.order = off;
    off = align256(off + sizeof(uint32_t) * (size_t)curves * nq);
    L.partial = off;
    off = align256(off + sizeof(uint64_t) * (size_t)nq * curves * kBandK);
    L.total = off;
    return L;
}

__global__ __launch_bounds__(256) void k_band_zero(uint32_t *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// One wavefront per query: its place in every curve, counted into buckets.
__global__ __launch_bounds__(64) void k_band_place(BandArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) {
        if (lane == c && c < (int)C) {
            a.pos[(uint64_t)q * C + c] = (uint32_t)pos[c];
            atomicAdd(&a.counts[(uint64_t)c * a.nbuckets + (pos[c] >> kBucketShift)], 1u);
        }
    }
}

// After the scan, counts[c][b] is the first order slot of bucket b of curve c
// (curve c's slots start at c * nq); each query takes the next one.
__global__ __launch_bounds__(256) void k_band_scatter(BandArgs a)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t C = a.v.curves;
    if (t >= (uint64_t)a.nq * C) return;
    const uint32_t q = (uint32_t)(t / C), c = (uint32_t)(t % C);
    const uint32_t b = a.pos[t] >> kBucketShift;
    const uint32_t slot = atomicAdd(&a.counts[(uint64_t)c * a.nbuckets + b], 1u);
    a.order[slot] = q;
}

// grid (groups, curves): a wavefront for 64 queries that are neighbours in
// curve c's order.  KR: list length (k <= KR).
template <int KR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KR >= 10 ? 3 : 4)))
void k_band(BandArgs a)
{
    __shared__ uint4 tile[kBandRows * 8];
    __shared__ uint32_t tile_xx[kBandRows];
    __shared__ uint32_t tile_id[kBandRows];
    const int lane = threadIdx.x;
    const uint32_t c = blockIdx.y;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint64_t slot = (uint64_t)blockIdx.x * 64 + lane;
    const bool live = slot < a.nq;
    const uint32_t q = live ? a.order[(uint64_t)c * a.nq + slot] : 0;

    // this lane's query and window
    uint4 qv[8];
    uint32_t qq = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        qv[i] = live ? reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim)[i]
                     : make_uint4(0, 0, 0, 0);
        qq = __builtin_amdgcn_udot4(qv[i].x, qv[i].x, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].y, qv[i].y, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].z, qv[i].z, qq, false);
        qq = __builtin_amdgcn_udot4(qv[i].w, qv[i].w, qq, false);
    }
    const uint64_t w = live ? (a.d_w ? a.d_w[q] : a.w_fixed) : 0;
    const uint64_t p = live ? a.pos[(uint64_t)q * C + c] : 0;
    const uint64_t lo = live ? (p > w ? p - w : 0) : ~0ull;
    const uint64_t hi = live ? (p + w < n ? p + w : n) : 0;
    // union of the group's windows
    uint64_t u0 = lo, u1 = hi;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o0 = shfl_xor_u64(u0, m), o1 = shfl_xor_u64(u1, m);
        u0 = o0 < u0 ? o0 : u0;
        u1 = o1 > u1 ? o1 : u1;
    }

    uint64_t L[KR];
#pragma unroll
    for (int i = 0; i < KR; i++) L[i] = kNone;
    const uint32_t *ids = a.v.ids[c];
    const int part = lane & 7, rsub = lane >> 3;
    for (uint64_t t0 = u0; t0 < u1; t0 += kBandRows) {
        const uint32_t rows = (uint32_t)std::min<uint64_t>(kBandRows, u1 - t0);
        // load: lane l takes the id of entry t0 + l; in step s, lanes 8r..8r+7
        // read the 16-byte parts of row 8s + r
        const uint32_t myid = (uint32_t)lane < rows ? ids[t0 + lane] : 0u;
        __syncthreads();
        if ((uint32_t)lane < rows) tile_id[lane] = myid;
#pragma unroll
        for (int s = 0; s < 8; s++) {
            const uint32_t r = 8 * s + rsub;
            const uint32_t rid = __shfl(myid, r, 64);
            uint4 x = make_uint4(0, 0, 0, 0);
            if (r < rows) x = *reinterpret_cast<const uint4 *>(a.v.db + (uint64_t)rid * kDim +
                                                               16 * part);
            tile[r * 8 + part] = x;
            uint32_t xx = __builtin_amdgcn_udot4(x.x, x.x, 0u, false);
            xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
            xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
            xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
            xx += __shfl_xor(xx, 1, 64);
            xx += __shfl_xor(xx, 2, 64);
            xx += __shfl_xor(xx, 4, 64);
            if (part == 0) tile_xx[r] = xx;
        }
        __syncthreads();
        for (uint32_t r = 0; r < rows; r++) {
            const uint64_t e = t0 + r;
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
            const uint64_t key = (e >= lo && e < hi) ? (((uint64_t)d << 32) | tile_id[r]) : kNone;
            // ids are distinct within one list: a plain sorted insert
            if (key < L[KR - 1]) {
#pragma unroll
                for (int i = KR - 1; i > 0; i--)
                    L[i] = key < L[i - 1] ? L[i - 1] : (key < L[i] ? key : L[i]);
                L[0] = key < L[0] ? key : L[0];
            }
        }
    }
    if (live) {
        uint64_t *out = a.partial + ((uint64_t)q * C + c) * a.k;
#pragma unroll
        for (int i = 0; i < KR; i++)
            if ((uint32_t)i < a.k) out[i] = L[i];
    }
}

// One wavefront per query: the curves' lists, repeats dropped, k nearest.
__global__ __launch_bounds__(64) void k_band_merge(BandArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    const uint64_t nkeys = (uint64_t)C * a.k;
    const uint64_t *src = a.partial + (uint64_t)q * C * a.k;
    WaveTopK<kBandK> top;
    top.init(a.k, nullptr, lane);
    for (uint64_t s = 0; s < nkeys; s += 64) {
        const uint64_t i = s + lane;
        top.push(i < nkeys ? src[i] : kNone, lane);
    }
    const uint64_t o = (uint64_t)q * a.k;
    top.finish(lane, [&](uint32_t j, uint64_t key) {
        a.out_ids[o + j] = (uint32_t)key;
        a.out_dists[o + j] = (uint32_t)(key >> 32);
    });
}

size_t band_scratch_bytes(uint32_t curves, uint64_t n, uint32_t nq)
{
    return band_layout(curves, n, nq).total;
}

// Runs the banded search with the query keys already in d_scratch.
hc_status band_search(const IndexView &v, const uint8_t *d_queries, uint32_t nq, uint32_t k,
                      uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_out_ids,
                      uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                      hipStream_t st)
{
    if (k < 1 || k > (uint32_t)kBandK) return HC_ERR_UNSUPPORTED;
    const BandLayout L = band_layout(v.curves, v.n, nq);
    if (scratch_bytes < L.total) return HC_ERR_SIZE;
    uint8_t *s = (uint8_t *)d_scratch;
    BandArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.queries = d_queries;
    a.qkeys = (const Key *)(s + L.qkeys);
    a.nq = nq;
    a.k = k;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.pos = (uint32_t *)(s + L.pos);
    a.counts = (uint32_t *)(s + L.counts);
    a.nbuckets = L.nbuckets;
    a.order = (uint32_t *)(s + L.order);
    a.partial = (uint64_t *)(s + L.partial);
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;
    const uint64_t nc = (uint64_t)v.curves * L.nbuckets;
    hipLaunchKernelGGL(k_band_zero, dim3((uint32_t)std::min<uint64_t>(4096, (nc + 255) / 256)),
                       dim3(256), 0, st, a.counts, nc);
    hipLaunchKernelGGL(k_band_place, dim3(nq), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, st, a.counts, nc);
    const uint64_t nt = (uint64_t)nq * v.curves;
    hipLaunchKernelGGL(k_band_scatter, dim3((uint32_t)((nt + 255) / 256)), dim3(256), 0, st, a);
    const dim3 grid((nq + 63) / 64, v.curves);
    if (k == 1) hipLaunchKernelGGL(k_band<1>, grid, dim3(64), 0, st, a);
    else if (k <= 4) hipLaunchKernelGGL(k_band<4>, grid, dim3(64), 0, st, a);
    else if (k <= 10) hipLaunchKernelGGL(k_band<10>, grid, dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_band<kBandK>, grid, dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_band_merge, dim3(nq), dim3(64), 0, st, a);
    return last_hip();
}

}  // namespace hc
