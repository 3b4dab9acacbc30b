// Multicurves search (Alg. 2), gfx950.
//
// Search kernel (k_stream): one wavefront per query, no LDS for candidates.
//  1. locate the query key in every curve's sorted list (the number of keys
//     below it) by descending the 64-ary sampled-key table: at each level the
//     wave loads 64 consecutive keys (1 KiB, coalesced) for all curves at once
//     and a ballot counts those below the query key;
//  2. window: w list entries on each side of that place (Alg. 2's "depth
//     closest" entries, read as the half-list model of Sec. 4.2), clamped to
//     the list ends; the windows of all curves are streamed as one sequence;
//  3-4. per step the wave takes 64 window slots: one coalesced load of 64 ids,
//     then 8 lanes read each 128-byte row with 16-byte loads, dot4 integer
//     arithmetic gives the exact squared distance (Eq. 2), reduced over the 8
//     lanes with lane-xor shuffles;
//  5. top-k by (distance, id) over the union taken as a set: every lane keeps
//     a sorted register list that refuses a key it already holds, and the wave
//     pops its minimum k times, every lane holding that key popping it, so an
//     id met in several windows counts once.  For k > 16 candidates below the
//     current k-th distinct key collect in an LDS buffer that is bitonic-sorted
//     and merged (dropping repeats) whenever it fills.
// An id found in several windows is read again each time; at 10^7 rows this
// is 0.2% of the rows (w = 64), less than a hash of the union would cost.
//
// Set kernel (k_sets): the same key location, then the union of the windows
// built explicitly in an LDS hash -- the positions and candidate-set exports.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "hc_device.h"

namespace hc {

constexpr int kKR = 16;                 // longest register list (k <= 16)
constexpr uint32_t kBandK16 = 16;       // k the banded path takes in one pass
constexpr double kBandShare = 3.5;      // windows per list entry from which to band
constexpr double kBandMinBlocks = 512;  // banded blocks from which to band (2 per CU)
                                        // (MI355X, n = 1e7, nq = 1e5: break-even at w ~ 512)
constexpr double kBandMinRows = 256;    // the same over the row store, counting the blocks
                                        // a small batch's groups are dealt out over
                                        // (MI355X, recall-0.90 windows at n = 1e7 and 5e7:
                                        // k = 10 bands 2.4-4x faster than gather at 2,048
                                        // queries, work items are faster at 1,000)
constexpr uint32_t kMaxSetSlots = 4096; // union capacity of the set kernel
constexpr uint32_t kItemsMaxQ = 4096;   // largest batch whose scratch holds the work items
constexpr int kIdBatch = 16;            // set kernel: ids loaded before inserting

struct SearchArgs {
    IndexView v;
    const uint8_t *queries;
    const Key *qkeys;          // [q][curves]
    uint32_t nq, k, w_fixed;
    const uint32_t *d_w;
    uint32_t *out_ids, *out_dists;
    uint32_t *out_pos;         // positions export: [q][curves]
    uint32_t *out_counts;      // candidates export
    uint32_t *out_cand;
    uint32_t cand_stride;
    uint32_t cs_log2;          // set kernel: union capacity = 1 << cs_log2
    const uint32_t *only;      // search: when set, only queries q with only[q] != 0
};

// ---------------------------------------------------------------------------
// Search kernel
// ---------------------------------------------------------------------------

// G: 64-slot groups a wave loads per iteration (rows in flight per lane = 8G).
// KR: register list length (k <= KR), or 0 for the LDS path (k > 16).
// At least 5 waves per SIMD (<= 102 VGPRs) unless the 16-entry list would spill.
template <int KR, int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((KR > 10 || KR == 0) ? 4 : 5)))
void k_stream(SearchArgs a)
{
    __shared__ WindowSet ws;
    TopKShared *tks = nullptr;
    if constexpr (KR == 0) {
        __shared__ TopKShared sh;
        tks = &sh;
    }
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    if (q >= a.nq) return;
    if (a.only && !a.only[q]) return;          // the whole block
    uint4 qv;
    uint32_t qq;
    query_part(a.queries, q, lane, qv, qq);
    const uint64_t w = a.d_w ? a.d_w[q] : a.w_fixed;

    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * a.v.curves, 0, 1, lane, pos);
    const uint64_t total = make_windows(a.v, pos, w, lane, &ws);

    WaveTopK<KR> top;
    top.init(a.k, tks, lane);
    stream_slots<G>(a.v.db, &ws, 0, total, qv, qq, lane, top);
    const uint64_t o = (uint64_t)q * a.k;
    top.finish(lane, [&](uint32_t j, uint64_t key) {
        a.out_ids[o + j] = (uint32_t)key;
        a.out_dists[o + j] = (uint32_t)(key >> 32);
    });
}

// ---------------------------------------------------------------------------
// Set kernel: positions, and the union of the windows built in an LDS hash
// ---------------------------------------------------------------------------

enum { SET_POS = 0, SET_CAND = 1 };

template <int NW, int MODE>
__global__ __launch_bounds__(64 * NW) void k_sets(SearchArgs a)
{
    extern __shared__ uint32_t lds[];
    constexpr int CPW = (kMaxCurves + NW - 1) / NW;
    constexpr int NT = 64 * NW;
    __shared__ uint32_t s_pos[kMaxCurves];
    __shared__ uint64_t s_wlo[kMaxCurves], s_wn[kMaxCurves];
    __shared__ const uint32_t *s_ids[kMaxCurves];
    __shared__ uint32_t s_count;

    const uint32_t cs = 1u << a.cs_log2;
    const uint32_t tsize = 2u * cs;                  // hash slots
    uint32_t *hash = lds;
    uint32_t *list = lds + tsize;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t q = blockIdx.x;
    if (q >= a.nq) return;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;

    uint64_t cnt[CPW];
    locate<CPW>(a.v, a.qkeys + (uint64_t)q * C, wave, NW, lane, cnt);
#pragma unroll
    for (int j = 0; j < CPW; j++) {
        const uint32_t c = wave + j * NW;
        if (c < C && lane == 0) s_pos[c] = (uint32_t)cnt[j];
    }
    __syncthreads();
    if constexpr (MODE == SET_POS) {
        if (tid < (int)C) a.out_pos[(uint64_t)q * C + tid] = s_pos[tid];
        return;
    }

    if (tid < kMaxCurves) {
        const uint64_t w = a.d_w ? a.d_w[q] : a.w_fixed;
        uint64_t lo = 0, hi = 0;
        if (tid < (int)C) {
            const uint64_t p = s_pos[tid];
            lo = p > w ? p - w : 0;
            hi = p + w < n ? p + w : n;
        }
        s_wlo[tid] = lo;
        s_wn[tid] = hi - lo;
        s_ids[tid] = tid < (int)C ? a.v.ids[tid] : nullptr;
    }
    if (tid == 0) s_count = 0;
    for (uint32_t i = tid; i < tsize; i += NT) hash[i] = kEmpty;
    __syncthreads();
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) total += s_wn[c];
    if (total > a.cand_stride) {   // the union might not fit its row: flag the query
        if (tid == 0) a.out_counts[q] = 0xFFFFFFFFu;
        return;
    }
    const uint32_t cn = (uint32_t)total;
    const uint32_t hshift = 32u - (a.cs_log2 + 1u);
    for (uint32_t sb = 0; sb < cn; sb += kIdBatch * NT) {
        uint32_t idv[kIdBatch];
#pragma unroll
        for (int j = 0; j < kIdBatch; j++) {
            const uint32_t s = sb + tid + j * NT;
            idv[j] = kEmpty;
            if (s < cn) {
                uint64_t g = s;
                int c = 0;
                while (g >= s_wn[c]) {
                    g -= s_wn[c];
                    c++;
                }
                idv[j] = s_ids[c][s_wlo[c] + g];
            }
        }
#pragma unroll
        for (int j = 0; j < kIdBatch; j++) {
            const uint32_t id = idv[j];
            if (id == kEmpty) continue;
            uint32_t h = (id * 0x9E3779B1u) >> hshift;
            while (true) {
                const uint32_t prev = atomicCAS(&hash[h], kEmpty, id);
                if (prev == kEmpty || prev == id) break;
                h = (h + 1) & (tsize - 1);
            }
        }
    }
    __syncthreads();
    for (uint32_t b = 0; b < tsize; b += NT) {
        const uint32_t v = hash[b + tid];
        const bool occ = v != kEmpty;
        const uint64_t m = __ballot(occ);
        uint32_t wb = 0;
        if (lane == 0 && m) wb = atomicAdd(&s_count, (uint32_t)__popcll(m));
        wb = __shfl(wb, 0, 64);
        if (occ) list[wb + lanes_below64(m)] = v;
    }
    __syncthreads();
    const uint32_t u = s_count;
    if (tid == 0) a.out_counts[q] = u;
    for (uint32_t i = tid; i < u; i += NT) a.out_cand[(uint64_t)q * a.cand_stride + i] = list[i];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static uint32_t ceil_log2(uint64_t x)
{
    uint32_t l = 0;
    while ((1ull << l) < x) l++;
    return l;
}

template <int KR, int G>
static hc_status launch_stream(const SearchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_stream<KR, G>), dim3(a.nq), dim3(64), 0, st, a);
    return last_hip();
}

// Wavefronts of the gather kernel for k resident on the device at once
// (compute units x wavefronts per unit; 0 if the runtime cannot say).  The
// device queries run once per process, device and register-list length (a
// racing repeat is harmless).
static uint64_t gather_resident(uint32_t k)
{
    constexpr int kMaxDev = 64;
    static uint64_t cache[kMaxDev][5];
    const int kv = k == 1 ? 0 : k <= 4 ? 1 : k <= 10 ? 2 : k <= (uint32_t)kKR ? 3 : 4;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
    if (cache[dev][kv]) return cache[dev][kv];
    const void *f = kv == 0   ? reinterpret_cast<const void *>(&k_stream<1, 1>)
                    : kv == 1 ? reinterpret_cast<const void *>(&k_stream<4, 1>)
                    : kv == 2 ? reinterpret_cast<const void *>(&k_stream<10, 1>)
                    : kv == 3 ? reinterpret_cast<const void *>(&k_stream<kKR, 1>)
                              : reinterpret_cast<const void *>(&k_stream<0, 1>);
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 64, 0) != hipSuccess)
        return 0;
    cache[dev][kv] = (uint64_t)cus * (uint64_t)per;
    return cache[dev][kv];
}

// A gather search of a batch too small to keep the device's memory busy with
// one wavefront per query (under a third of the resident wavefronts) and of
// long windows (at least 4 items of slots per query) runs as work items: each
// query's windows are cut into pieces that many wavefronts stream at once,
// then merged (measured on MI355X: 10^3 queries at N = 5e7, w = 125,952 take
// 41.8 ms as items against 68.0 ms with one wavefront per query).
static bool items_route(const hc_index *idx, uint32_t nq, uint32_t k, uint64_t w,
                        size_t scratch_bytes)
{
    if (2ull * w * idx->v.curves < 4ull * kItemChunk || nq > kItemsMaxQ) return false;
    if (scratch_bytes < items_scratch_bytes(idx->v.curves, nq, k)) return false;
    return 3ull * nq < gather_resident(k);
}

// A register list as long as k (1, 4, 10 or 16) for k <= 16, the LDS buffer
// beyond.
template <int G>
static hc_status launch_search_g(const SearchArgs &a, hipStream_t st)
{
    if (a.k == 1) return launch_stream<1, G>(a, st);
    if (a.k <= 4) return launch_stream<4, G>(a, st);
    if (a.k <= 10) return launch_stream<10, G>(a, st);
    if (a.k <= (uint32_t)kKR) return launch_stream<kKR, G>(a, st);
    return launch_stream<0, G>(a, st);
}

static hc_status launch_search(const SearchArgs &a, uint64_t w_hint, hipStream_t st)
{
    // Measured on MI355X at 10^7 rows: one group with at least 5 waves per SIMD
    // is within 1% of two groups for w >= 256 and faster below.
    (void)w_hint;
    return launch_search_g<1>(a, st);
}

template <int NW, int MODE>
static hc_status launch_sets(const SearchArgs &a, hipStream_t st)
{
    const size_t lds = MODE == SET_CAND ? (size_t)12 << a.cs_log2 : 0;
    hipLaunchKernelGGL((k_sets<NW, MODE>), dim3(a.nq), dim3(64 * NW), lds, st, a);
    return last_hip();
}

// The gather search for the queries q with only[q] != 0 of a batch whose keys
// are already in qkeys (the banded path's fallback for k > 16).
hc_status gather_search_only(const IndexView &v, const uint8_t *d_queries, const Key *qkeys,
                             uint32_t nq, uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                             const uint32_t *only, uint32_t *d_out_ids, uint32_t *d_out_dists,
                             hipStream_t st)
{
    SearchArgs a;
    memset(&a, 0, sizeof(a));
    a.v = v;
    a.queries = d_queries;
    a.qkeys = qkeys;
    a.nq = nq;
    a.k = k;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;
    a.only = only;
    return launch_search(a, w_fixed, st);
}

static hc_status check_common(const hc_index *idx, const uint8_t *d_queries, void *d_scratch,
                              size_t scratch_bytes, uint32_t nq)
{
    if (!idx || !d_queries || ((uintptr_t)d_queries & 15)) return HC_ERR_INVALID;
    if (!d_scratch || ((uintptr_t)d_scratch & 15)) return HC_ERR_INVALID;
    if (scratch_bytes < sizeof(Key) * (size_t)nq * idx->v.curves) return HC_ERR_SIZE;
    return HC_OK;
}

static SearchArgs base_args(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            void *d_scratch)
{
    SearchArgs a;
    memset(&a, 0, sizeof(a));
    a.v = idx->v;
    a.queries = d_queries;
    a.qkeys = (const Key *)d_scratch;
    a.nq = nq;
    return a;
}

// Scratch of hc_search_batch_noalloc: the query keys, in a device array the
// library owns (one copy per GPU, kept until the process ends).  Host code
// never passes the array's name to a kernel or a copy: on the host it is only
// a stand-in for the symbol.  The device address comes from
// hipGetSymbolAddress, once per device, and is kept per device.
static __device__ __align__(256) uint8_t scratch[HC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The address of `scratch` on the current device.
static hc_status noalloc_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HC_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return HC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HC_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HC_OK;
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_search_scratch_bytes(const hc_index *idx, uint32_t nq, size_t *bytes)
{
    return hc_search_scratch_bytes_k(idx, nq, (uint32_t)kBandK16, bytes);
}

hc_status hc_search_scratch_bytes_k(const hc_index *idx, uint32_t nq, uint32_t k_max,
                                    size_t *bytes)
{
    if (!idx || !bytes || k_max < 1 || k_max > HC_K_MAX) return HC_ERR_INVALID;
    const uint32_t m = std::max<uint32_t>(nq, 1);
    const uint32_t kb = std::min<uint32_t>(k_max, kBandKMax);
    *bytes = std::max(align256(sizeof(Key) * (size_t)m * idx->v.curves),
                      band_scratch_bytes(idx->v.curves, idx->v.n, m, kb));
    if (m <= kItemsMaxQ)   // a small batch may run as work items (the gather path)
        *bytes = std::max(*bytes, items_scratch_bytes(idx->v.curves, m, k_max));
    return HC_OK;
}

hc_status hc_encode_queries(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            void *d_scratch, size_t scratch_bytes, hc_stream stream)
{
    if (nq == 0) return HC_OK;
    hc_status st = check_common(idx, d_queries, d_scratch, scratch_bytes, nq);
    if (st != HC_OK) return st;
    return encode_rows(idx->v, d_queries, nq, (Key *)d_scratch, (hipStream_t)stream);
}

hc_status hc_search_encoded_ex(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                               uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                               uint32_t *d_out_ids, uint32_t *d_out_dists, void *d_scratch,
                               size_t scratch_bytes, uint32_t path, hc_stream stream)
{
    if (k < 1 || k > HC_K_MAX || !d_out_ids || !d_out_dists || path > HC_PATH_BAND)
        return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hc_status st = check_common(idx, d_queries, d_scratch, scratch_bytes, nq);
    if (st != HC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t hint = d_w ? (w_fixed ? w_fixed : 64) : w_fixed;
    const bool automatic = path == HC_PATH_AUTO;
    if (automatic) hc_search_choose_path(idx, nq, k, (uint32_t)hint, scratch_bytes, &path);
    if (path == HC_PATH_BAND)
        return band_search(idx->v, d_queries, nq, k, w_fixed, d_w, d_out_ids, d_out_dists,
                           d_scratch, scratch_bytes, s, idx->kernel_begin, idx->kernel_end);
    if (automatic && items_route(idx, nq, k, hint, scratch_bytes))
        return items_search(idx->v, d_queries, nq, w_fixed, d_w, k, nullptr, k, d_out_ids,
                            d_out_dists, d_scratch, scratch_bytes, kItemChunk, kItemSplit, 0,
                            true, s, idx->kernel_begin, idx->kernel_end);
    SearchArgs a = base_args(idx, d_queries, nq, d_scratch);
    a.k = k;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;
    st = record_if(idx->kernel_begin, s);
    if (st != HC_OK) return st;
    st = launch_search(a, hint, s);
    if (st != HC_OK) return st;
    return record_if(idx->kernel_end, s);
}

hc_status hc_index_set_kernel_events(hc_index *idx, hc_event begin, hc_event end)
{
    if (!idx || !begin != !end) return HC_ERR_INVALID;
    idx->kernel_begin = (hipEvent_t)begin;
    idx->kernel_end = (hipEvent_t)end;
    return HC_OK;
}

hc_status hc_search_choose_path(const hc_index *idx, uint32_t nq, uint32_t k, uint32_t w,
                                size_t scratch_bytes, uint32_t *path)
{
    if (!idx || !path) return HC_ERR_INVALID;
    // banded when each list entry lies in enough windows of the batch (the rows
    // it saves outweigh the entries its groups stream outside windows) and the
    // batch makes enough blocks to fill the device (a small batch spreads each
    // block over a long stretch of the list, streamed by few blocks)
    const bool shared = 2.0 * (double)w * nq >= kBandShare * (double)idx->v.n;
    // over the row store a small batch's groups are dealt out over more blocks
    const bool rows = idx->v.rows[0] != nullptr;
    const double blocks = rows ? (double)band_split_blocks(idx->v.curves, nq, w, k)
                               : (double)band_blocks(idx->v.curves, nq, w);
    const bool wide = blocks >= (rows ? kBandMinRows : kBandMinBlocks);
    // k <= 16: one pass; 16 < k <= kBandKMax: two passes over the row store
    const bool k_ok = k >= 1 && (k <= kBandK16 || (k <= kBandKMax && idx->v.rows[0]));
    const bool fits = k_ok && scratch_bytes >= band_scratch_bytes(idx->v.curves, idx->v.n, nq, k);
    *path = (shared && wide && fits) ? HC_PATH_BAND : HC_PATH_GATHER;
    return HC_OK;
}

hc_status hc_search_encoded(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                            uint32_t *d_out_ids, uint32_t *d_out_dists, void *d_scratch,
                            size_t scratch_bytes, hc_stream stream)
{
    return hc_search_encoded_ex(idx, d_queries, nq, k, w_fixed, d_w, d_out_ids, d_out_dists,
                                d_scratch, scratch_bytes, HC_PATH_AUTO, stream);
}

hc_status hc_search_batch(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                          uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                          uint32_t *d_out_ids, uint32_t *d_out_dists, void *d_scratch,
                          size_t scratch_bytes, hc_stream stream)
{
    if (k < 1 || k > HC_K_MAX || !d_out_ids || !d_out_dists) return HC_ERR_INVALID;
    hc_status st = hc_encode_queries(idx, d_queries, nq, d_scratch, scratch_bytes, stream);
    if (st != HC_OK) return st;
    return hc_search_encoded(idx, d_queries, nq, k, w_fixed, d_w, d_out_ids, d_out_dists,
                             d_scratch, scratch_bytes, stream);
}

hc_status hc_search_batch_noalloc(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                                  uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                                  uint32_t *d_out_ids, uint32_t *d_out_dists,
                                  hc_stream stream)
{
    if (!idx || k < 1 || k > HC_K_MAX || !d_out_ids || !d_out_dists) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    if (sizeof(Key) * (uint64_t)nq * idx->v.curves > HC_NOALLOC_SCRATCH_BYTES)
        return HC_ERR_SIZE;
    void *s = nullptr;
    const hc_status st = noalloc_scratch(&s);
    if (st != HC_OK) return st;
    // every key the search reads is written first: nothing to clear
    const hc_status se = hc_encode_queries(idx, d_queries, nq, s, HC_NOALLOC_SCRATCH_BYTES, stream);
    if (se != HC_OK) return se;
    return hc_search_encoded_ex(idx, d_queries, nq, k, w_fixed, d_w, d_out_ids, d_out_dists, s,
                                HC_NOALLOC_SCRATCH_BYTES, HC_PATH_GATHER, stream);
}

hc_status hc_positions(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                       uint32_t *d_pos, void *d_scratch, size_t scratch_bytes,
                       hc_stream stream)
{
    if (!d_pos) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hc_status st = check_common(idx, d_queries, d_scratch, scratch_bytes, nq);
    if (st != HC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SearchArgs a = base_args(idx, d_queries, nq, d_scratch);
    st = encode_rows(a.v, d_queries, nq, (Key *)d_scratch, s);
    if (st != HC_OK) return st;
    a.out_pos = d_pos;
    return launch_sets<1, SET_POS>(a, s);
}

hc_status hc_candidates(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                        uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_counts,
                        uint32_t *d_ids, uint32_t stride, void *d_scratch,
                        size_t scratch_bytes, hc_stream stream)
{
    if (!d_counts || !d_ids) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hc_status st = check_common(idx, d_queries, d_scratch, scratch_bytes, nq);
    if (st != HC_OK) return st;
    if (stride > kMaxSetSlots) return HC_ERR_UNSUPPORTED;
    if (!d_w && (uint64_t)stride < 16ull * w_fixed) return HC_ERR_SIZE;
    hipStream_t s = (hipStream_t)stream;
    SearchArgs a = base_args(idx, d_queries, nq, d_scratch);
    st = encode_rows(a.v, d_queries, nq, (Key *)d_scratch, s);
    if (st != HC_OK) return st;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.out_counts = d_counts;
    a.out_cand = d_ids;
    a.cand_stride = stride;
    // the union must fit one table: capacity >= stride >= 16 w
    a.cs_log2 = std::max<uint32_t>(ceil_log2(std::max<uint32_t>(stride, 64)), 6);
    if ((1u << a.cs_log2) > 1024) return launch_sets<4, SET_CAND>(a, s);
    return launch_sets<1, SET_CAND>(a, s);
}

}  // extern "C"
