// Uneven batches (gfx950): every query has its own window w and its own k.
//
// The work of a query is its window slots (up to 16 w of them); a query is cut
// into work items of at most `chunk` slots (at most max_split items; the chunk
// grows for larger queries).  A persistent grid of wavefronts pops items from
// an atomic counter until the items run out; an item streams its slots through
// the same distance kernel and top-k as the plain search.  A query of one item
// writes its result directly; the items of a larger query leave partial top-k
// lists that a merge kernel combines (repeats dropped).  Bounded items keep the
// load balanced whatever the spread of w, and nothing waits on the host, so the
// whole sequence can be captured in a HIP graph.
//
// Launch sequence (one stream):
//   k_encode_rows   query keys
//   k_plan          positions, number of items per query, queue reset
//   k_scan_*        item offsets per query (base[q]; base[nq] = item count)
//   k_items         the persistent work loop
//   k_merge         queries with more than one item
#include <string.h>

#include <algorithm>

#include "hc_device.h"
#include "hc_scan.h"

namespace hc {

struct UnevenArgs {
    IndexView v;
    const uint8_t *queries;
    const Key *qkeys;
    uint32_t nq;
    const uint32_t *d_w, *d_k;
    uint32_t w_fixed, k_fixed, k_stride;
    uint32_t chunk, max_split;
    uint32_t *pos;        // [q][curves]
    uint32_t *base;       // nq + 1
    uint32_t *queue;      // 1
    uint64_t *partial;    // [item][k_stride]
    uint32_t *out_ids, *out_dists;
};

__device__ inline uint32_t query_k(const UnevenArgs &a, uint32_t q)
{
    const uint32_t k = a.d_k ? a.d_k[q] : a.k_fixed;
    return std::min<uint32_t>(std::max<uint32_t>(k, 1u), a.k_stride);
}

__device__ inline uint64_t query_w(const UnevenArgs &a, uint32_t q)
{
    return a.d_w ? a.d_w[q] : a.w_fixed;
}

// Slots of one item for a query of `total` slots.
__device__ inline uint64_t item_chunk(const UnevenArgs &a, uint64_t total)
{
    const uint64_t need = (total + a.max_split - 1) / a.max_split;
    const uint64_t c = std::max<uint64_t>(a.chunk, (need + 63) / 64 * 64);
    return c;
}

__device__ inline uint64_t window_total(const IndexView &v, const uint64_t (&pos)[kMaxCurves],
                                        uint64_t w)
{
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) {
        if (c < (int)v.curves) {
            const uint64_t lo = pos[c] > w ? pos[c] - w : 0;
            const uint64_t hi = pos[c] + w < v.n ? pos[c] + w : v.n;
            total += hi - lo;
        }
    }
    return total;
}

// One wavefront per query: positions, and the number of work items.
__global__ __launch_bounds__(64) void k_plan(UnevenArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++)
        if (lane == c && c < (int)C) a.pos[(uint64_t)q * C + c] = (uint32_t)pos[c];
    if (lane == 0) {
        const uint64_t total = window_total(a.v, pos, query_w(a, q));
        const uint64_t ch = item_chunk(a, total);
        a.base[q] = total ? (uint32_t)((total + ch - 1) / ch) : 1u;   // >= 1 item
        if (q == 0) {
            a.base[a.nq] = 0;
            *a.queue = 0;
        }
    }
}

template <int KR>
__device__ inline void run_item(const UnevenArgs &a, uint32_t q, uint32_t j, uint32_t nitems,
                                uint32_t item, uint32_t k, WindowSet *ws, TopKShared *tks,
                                int lane)
{
    const uint32_t C = a.v.curves;
    uint64_t pos[kMaxCurves];
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++)
        pos[c] = c < (int)C ? a.pos[(uint64_t)q * C + c] : 0;
    const uint64_t total = make_windows(a.v, pos, query_w(a, q), lane, ws);
    const uint64_t ch = item_chunk(a, total);
    const uint64_t s0 = std::min<uint64_t>(total, (uint64_t)j * ch);
    const uint64_t s1 = std::min<uint64_t>(total, s0 + ch);
    uint4 qv;
    uint32_t qq;
    query_part(a.queries, q, lane, qv, qq);
    WaveTopK<KR> top;
    top.init(k, tks, lane);
    stream_slots<1>(a.v.db, ws, s0, s1, qv, qq, lane, top);
    if (nitems == 1) {
        const uint64_t o = (uint64_t)q * a.k_stride;
        top.finish(lane, [&](uint32_t i, uint64_t key) {
            a.out_ids[o + i] = (uint32_t)key;
            a.out_dists[o + i] = (uint32_t)(key >> 32);
        });
        for (uint32_t i = k + lane; i < a.k_stride; i += 64) {
            a.out_ids[o + i] = kEmpty;
            a.out_dists[o + i] = kEmpty;
        }
    } else {
        uint64_t *p = a.partial + (uint64_t)item * a.k_stride;
        top.finish(lane, [&](uint32_t i, uint64_t key) { p[i] = key; });
    }
}

// Persistent work loop; every wavefront exits once the counter passes the
// item count.  BIG: some k may exceed 16 (needs the LDS top-k).
// Both forms run 4 waves per SIMD: with the 512-entry LDS buffer BIG takes
// about 8 KiB of LDS per wavefront, so 16 wavefronts fit in a CU's LDS; the few
// registers BIG spills at this budget cost less than the lost occupancy.
template <bool BIG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void k_items(UnevenArgs a)
{
    __shared__ WindowSet ws;
    TopKShared *tks = nullptr;
    if constexpr (BIG) {
        __shared__ TopKShared sh;
        tks = &sh;
    }
    const int lane = threadIdx.x;
    const uint32_t nitems_all = a.base[a.nq];
    while (true) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1u);
        item = __shfl(item, 0, 64);
        if (item >= nitems_all) break;
        // the query owning the item: base[] rises strictly (every query has an item)
        uint32_t lo = 0, hi = a.nq;      // base[lo] <= item < base[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.base[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint32_t q = lo;
        const uint32_t j = item - a.base[q];
        const uint32_t nitems = a.base[q + 1] - a.base[q];
        const uint32_t k = query_k(a, q);
        __syncthreads();
        if constexpr (BIG) {
            if (k > 16) {
                run_item<0>(a, q, j, nitems, item, k, &ws, tks, lane);
                continue;
            }
        }
        run_item<16>(a, q, j, nitems, item, k, &ws, nullptr, lane);
    }
}

// Queries with several items: their partial lists, streamed 64 keys at a time
// into the same top-k, which drops the keys seen in more than one item.
template <bool BIG>
__global__ __launch_bounds__(64) void k_merge(UnevenArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t b0 = a.base[q], nitems = a.base[q + 1] - b0;
    if (nitems <= 1) return;
    TopKShared *tks = nullptr;
    if constexpr (BIG) {
        __shared__ TopKShared sh;
        tks = &sh;
    }
    const uint32_t k = query_k(a, q);
    const uint64_t nkeys = (uint64_t)nitems * k;
    auto run = [&](auto &top) {
        for (uint64_t s = 0; s < nkeys; s += 64) {
            const uint64_t i = s + lane;
            uint64_t key = kNone;
            if (i < nkeys) key = a.partial[(uint64_t)(b0 + i / k) * a.k_stride + i % k];
            top.push(key, lane);
        }
        const uint64_t o = (uint64_t)q * a.k_stride;
        top.finish(lane, [&](uint32_t i, uint64_t key) {
            a.out_ids[o + i] = (uint32_t)key;
            a.out_dists[o + i] = (uint32_t)(key >> 32);
        });
        for (uint32_t i = k + lane; i < a.k_stride; i += 64) {
            a.out_ids[o + i] = kEmpty;
            a.out_dists[o + i] = kEmpty;
        }
    };
    if constexpr (BIG) {
        if (k > 16) {
            WaveTopK<0> top;
            top.init(k, tks, lane);
            run(top);
            return;
        }
    }
    WaveTopK<16> top;
    top.init(k, nullptr, lane);
    run(top);
}

struct UnevenLayout {
    size_t qkeys, pos, base, sums, queue, partial, total;
};

static UnevenLayout uneven_layout(uint32_t curves, uint32_t nq, uint32_t k_stride,
                                  uint32_t max_split)
{
    UnevenLayout L{};
    size_t off = 0;
    L.qkeys = off;
    off = align256(off + sizeof(Key) * (size_t)nq * curves);
    L.pos = off;
    off = align256(off + sizeof(uint32_t) * (size_t)nq * curves);
    L.base = off;
    off = align256(off + sizeof(uint32_t) * ((size_t)nq + 1));
    L.sums = off;      // tile sums of the scan of base
    off = align256(off + sizeof(uint32_t) * (((size_t)nq + 1 + kScanTile - 1) / kScanTile));
    L.queue = off;
    off = align256(off + sizeof(uint32_t));
    L.partial = off;
    off = align256(off + sizeof(uint64_t) * (size_t)nq * max_split * k_stride);
    L.total = off;
    return L;
}

static void resolve_cfg(const hc_uneven_cfg *cfg, uint32_t *chunk, uint32_t *max_split,
                        uint32_t *per_cu)
{
    *chunk = cfg && cfg->chunk_slots ? cfg->chunk_slots : kItemChunk;
    *chunk = (*chunk + 63) / 64 * 64;
    *max_split = cfg && cfg->max_split ? cfg->max_split : kItemSplit;
    *per_cu = cfg ? cfg->blocks_per_cu : 0u;
}

// Wavefronts of the persistent grid: CUs x per_cu (0 = the occupancy limit).
// The device queries run once per process and device, so a captured call
// records launches only.
template <bool BIG>
static uint32_t persistent_blocks(uint32_t per_cu)
{
    constexpr int kMaxDev = 64;
    static int cus_cache[kMaxDev], occ_cache[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
    int cus = cus_cache[dev], occ = occ_cache[dev];
    if (cus < 1 || occ < 1) {   // first call on this device (a racing repeat is harmless)
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            cus < 1)
            return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_items<BIG>, 64, 0) !=
                hipSuccess ||
            occ < 1)
            occ = 8;
        occ_cache[dev] = occ;
        cus_cache[dev] = cus;
    }
    return (uint32_t)cus * (per_cu ? per_cu : (uint32_t)occ);
}

// The work-item search of nq queries (arguments checked by the caller); with
// keys_ready the query keys are already at the start of the scratch.  ev_begin
// and ev_end, when set, are recorded around k_items.
hc_status items_search(const IndexView &v, const uint8_t *d_queries, uint32_t nq,
                       uint32_t w_fixed, const uint32_t *d_w, uint32_t k_fixed,
                       const uint32_t *d_k, uint32_t k_stride, uint32_t *d_out_ids,
                       uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                       uint32_t chunk, uint32_t max_split, uint32_t per_cu, bool keys_ready,
                       hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end)
{
    const UnevenLayout L = uneven_layout(v.curves, nq, k_stride, max_split);
    if (scratch_bytes < L.total) return HC_ERR_SIZE;
    if ((uint64_t)nq * max_split >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;

    uint8_t *s = (uint8_t *)d_scratch;
    UnevenArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.queries = d_queries;
    a.qkeys = (const Key *)(s + L.qkeys);
    a.nq = nq;
    a.d_w = d_w;
    a.d_k = d_k;
    a.w_fixed = w_fixed;
    a.k_fixed = k_fixed;
    a.k_stride = k_stride;
    a.chunk = chunk;
    a.max_split = max_split;
    a.pos = (uint32_t *)(s + L.pos);
    a.base = (uint32_t *)(s + L.base);
    a.queue = (uint32_t *)(s + L.queue);
    a.partial = (uint64_t *)(s + L.partial);
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;

    if (!keys_ready) {
        const hc_status rc = encode_rows(a.v, d_queries, nq, (Key *)(s + L.qkeys), st);
        if (rc != HC_OK) return rc;
    }
    hipLaunchKernelGGL(k_plan, dim3(nq), dim3(64), 0, st, a);
    {   // item offsets: one block per 4,096 queries, then the tile sums
        const uint64_t nb1 = (uint64_t)nq + 1;
        const uint32_t tiles = (uint32_t)((nb1 + kScanTile - 1) / kScanTile);
        uint32_t *sums = (uint32_t *)(s + L.sums);
        hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(kScanThreads), 0, st, a.base, nb1,
                           sums);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, st, sums,
                           (uint64_t)tiles);
        hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, st, a.base, nb1,
                           (const uint32_t *)sums);
    }
    const bool big = k_stride > 16;
    uint32_t blocks = big ? persistent_blocks<true>(per_cu) : persistent_blocks<false>(per_cu);
    if (blocks == 0) return HC_ERR_HIP;
    // a query has at most max_split items: a small batch needs no full grid
    blocks = (uint32_t)std::min<uint64_t>(blocks, (uint64_t)nq * max_split);
    hc_status rc = record_if(ev_begin, st);
    if (rc != HC_OK) return rc;
    if (big) hipLaunchKernelGGL(k_items<true>, dim3(blocks), dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_items<false>, dim3(blocks), dim3(64), 0, st, a);
    rc = record_if(ev_end, st);
    if (rc != HC_OK) return rc;
    if (big) hipLaunchKernelGGL(k_merge<true>, dim3(nq), dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_merge<false>, dim3(nq), dim3(64), 0, st, a);
    return last_hip();
}

size_t items_scratch_bytes(uint32_t curves, uint32_t nq, uint32_t k_stride)
{
    uint32_t chunk, max_split, per_cu;
    resolve_cfg(nullptr, &chunk, &max_split, &per_cu);
    return uneven_layout(curves, std::max<uint32_t>(nq, 1), k_stride, max_split).total;
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_uneven_scratch_bytes(const hc_index *idx, uint32_t nq, uint32_t k_stride,
                                  const hc_uneven_cfg *cfg, size_t *bytes)
{
    if (!idx || !bytes || k_stride < 1 || k_stride > HC_K_MAX) return HC_ERR_INVALID;
    uint32_t chunk, max_split, per_cu;
    resolve_cfg(cfg, &chunk, &max_split, &per_cu);
    *bytes = uneven_layout(idx->v.curves, std::max<uint32_t>(nq, 1), k_stride, max_split).total;
    return HC_OK;
}

hc_status hc_search_uneven(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                           uint32_t w_fixed, const uint32_t *d_w, uint32_t k_fixed,
                           const uint32_t *d_k, uint32_t k_stride, uint32_t *d_out_ids,
                           uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                           const hc_uneven_cfg *cfg, hc_stream stream)
{
    if (!idx || !d_queries || ((uintptr_t)d_queries & 15) || !d_out_ids || !d_out_dists)
        return HC_ERR_INVALID;
    if (k_stride < 1 || k_stride > HC_K_MAX || (!d_k && (k_fixed < 1 || k_fixed > k_stride)))
        return HC_ERR_INVALID;
    if (!d_scratch || ((uintptr_t)d_scratch & 255)) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    uint32_t chunk, max_split, per_cu;
    resolve_cfg(cfg, &chunk, &max_split, &per_cu);
    if (chunk > (1u << 30) || max_split < 1 || max_split > 4096) return HC_ERR_INVALID;
    return items_search(idx->v, d_queries, nq, w_fixed, d_w, k_fixed, d_k, k_stride, d_out_ids,
                        d_out_dists, d_scratch, scratch_bytes, chunk, max_split, per_cu, false,
                        (hipStream_t)stream, nullptr, nullptr);
}

}  // extern "C"
