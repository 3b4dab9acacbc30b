// Index build (Alg. 1): per curve, the <key, id> list sorted by (key, id).
//
// The keys of one curve are encoded straight into the index buffer with ids in
// ascending order, then sorted by a stable least-significant-digit radix sort
// over the sixteen 8-bit digits of the 128-bit key.  Stability keeps equal keys
// in id order, which gives the (key, id) order.  A digit that is the same for
// every key (common: the data are small, so many high-order Hilbert bits are
// zero) is skipped.  Finally the 64-ary sampled-key table the search descends
// is extracted: level L holds key[j * 64^L].
//
// Rows appended to the database are inserted without a rebuild: their keys
// are sorted the same way and merged with each existing list (every new id is
// larger than every old one, so at an equal key the old entry comes first);
// the result is the index a full build over all rows gives, bit for bit.
#include <string.h>

#include <new>
#include <vector>

#include "hc_hilbert.h"
#include "hc_scan.h"

namespace hc {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 keys per tile

__device__ inline uint32_t key_digit(const Key &k, int d)
{
    return (uint32_t)((d < 8 ? (k.lo >> (8 * d)) : (k.hi >> (8 * (d - 8)))) & 0xFFu);
}

__device__ inline uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Keys of curve c for rows[0, count), ids id_base + i (ascending).
__global__ __launch_bounds__(256) void k_encode_curve(IndexView v, uint32_t c,
                                                      const uint8_t *rows, uint64_t count,
                                                      uint32_t id_base, Key *keys,
                                                      uint32_t *ids)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint32_t coord[kDpc];
    project16(rows + i * kDim, v, c, coord);
    keys[i] = curve_key16(coord, v.curve);
    ids[i] = id_base + (uint32_t)i;
}

// Histograms of all sixteen digits (hist[d * 256 + value]).
__global__ __launch_bounds__(256) void k_digit_hist(const Key *keys, uint64_t n,
                                                    uint32_t *hist)
{
    __shared__ uint32_t h[16 * 256];
    for (int i = threadIdx.x; i < 16 * 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const Key k = keys[i];
#pragma unroll
        for (int d = 0; d < 16; d++) atomicAdd(&h[d * 256 + key_digit(k, d)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 16 * 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Per-tile counts of digit d: counts[value * ntiles + tile].
__global__ __launch_bounds__(kSortThreads) void k_tile_hist(const Key *keys, uint64_t n,
                                                            int d, uint32_t *counts,
                                                            uint32_t ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortItems; r++) {
        const uint64_t e = base + (uint64_t)r * kSortThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[key_digit(keys[e], d)], 1u);
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit pass.  Within a tile, keys are visited in order:
// rounds of 256 consecutive keys, lanes in order, waves in order; a wave ranks
// its lanes among equal digits with ballots.
__global__ __launch_bounds__(kSortThreads) void k_scatter(const Key *src, const uint32_t *src_ids,
                                                          Key *dst, uint32_t *dst_ids,
                                                          uint64_t n, int d,
                                                          const uint32_t *offsets,
                                                          uint32_t ntiles)
{
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t wave_cnt[kWaves][256];
    __shared__ uint32_t run[256];
    const int tid = threadIdx.x, wave = tid >> 6;
    run[tid] = offsets[(uint64_t)tid * ntiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; w++) wave_cnt[w][tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        const uint64_t e = base + (uint64_t)r * kSortThreads + tid;
        const bool valid = e < n;
        Key k = {0, 0};
        uint32_t id = 0;
        if (valid) {
            k = src[e];
            id = src_ids[e];
        }
        const uint32_t dig = valid ? key_digit(k, d) : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = lanes_below(peers);
        if (valid && rank == 0) wave_cnt[wave][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[dig] + rank;
            for (int w = 0; w < wave; w++) pos += wave_cnt[w][dig];
            dst[pos] = k;
            dst_ids[pos] = id;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            add += wave_cnt[w][tid];
            wave_cnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// Merge of an existing list (old, n entries) with the sorted entries of
// appended rows (add, m entries) into out (n + m).  An appended entry goes
// after every old entry whose key is <= its key; an old entry goes after
// every appended entry whose key is < its key.
__global__ __launch_bounds__(256) void k_merge_added(const Key *old_keys, uint64_t n,
                                                     const Key *add_keys,
                                                     const uint32_t *add_ids, uint64_t m,
                                                     Key *out_keys, uint32_t *out_ids)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const Key x = add_keys[j];
    uint64_t a = 0, b = n;
    while (a < b) {
        const uint64_t mid = a + (b - a) / 2;
        if (key_less(x, old_keys[mid])) b = mid;
        else a = mid + 1;
    }
    out_keys[a + j] = x;
    out_ids[a + j] = add_ids[j];
}

__global__ __launch_bounds__(256) void k_merge_old(const Key *old_keys, const uint32_t *old_ids,
                                                   uint64_t n, const Key *add_keys, uint64_t m,
                                                   Key *out_keys, uint32_t *out_ids)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Key x = old_keys[i];
    uint64_t a = 0, b = m;
    while (a < b) {
        const uint64_t mid = a + (b - a) / 2;
        if (key_less(add_keys[mid], x)) a = mid + 1;
        else b = mid;
    }
    out_keys[i + a] = x;
    out_ids[i + a] = old_ids[i];
}

// Level L of the sampled-key table: out[j] = leaf[j * stride].
__global__ __launch_bounds__(256) void k_sample_keys(const Key *leaf, uint64_t stride,
                                                     Key *out, uint64_t len)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < len) out[j] = leaf[j * stride];
}

struct BuildScratch {
    Key *keys;
    uint32_t *ids;
    uint32_t *hist;      // 16 * 256
    uint32_t *counts;    // 256 * ntiles
    size_t total;
};

static BuildScratch build_scratch_layout(uint64_t n, uint8_t *base)
{
    const uint64_t ntiles = (n + kSortTile - 1) / kSortTile;
    BuildScratch s{};
    size_t off = 0;
    s.keys = (Key *)(base + off);
    off = align256(off + sizeof(Key) * n);
    s.ids = (uint32_t *)(base + off);
    off = align256(off + sizeof(uint32_t) * n);
    s.hist = (uint32_t *)(base + off);
    off = align256(off + sizeof(uint32_t) * 16 * 256);
    s.counts = (uint32_t *)(base + off);
    off = align256(off + sizeof(uint32_t) * 256 * ntiles);
    s.total = off;
    return s;
}

static uint32_t blocks_for(uint64_t n, uint32_t per)
{
    return (uint32_t)((n + per - 1) / per);
}

// Stable LSD radix sort of (keys, ids) by key, in place (s holds the second
// buffer).  Synchronises the stream once, to read the digit histograms.
static hc_status radix_sort(Key *keys, uint32_t *ids, uint64_t n, const BuildScratch &s,
                            hipStream_t st)
{
    const uint32_t ntiles = blocks_for(n, kSortTile);
    hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(256), 0, st, s.hist, (uint64_t)16 * 256,
                       0u);
    const uint32_t hblocks = (uint32_t)std::min<uint64_t>(1024, blocks_for(n, 256));
    hipLaunchKernelGGL(k_digit_hist, dim3(hblocks), dim3(256), 0, st, keys, n, s.hist);
    std::vector<uint32_t> hist(16 * 256);
    if (hipMemcpyAsync(hist.data(), s.hist, sizeof(uint32_t) * hist.size(),
                       hipMemcpyDeviceToHost, st) != hipSuccess)
        return HC_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return HC_ERR_HIP;

    Key *src = keys, *dst = s.keys;
    uint32_t *src_ids = ids, *dst_ids = s.ids;
    for (int d = 0; d < 16; d++) {
        bool trivial = false;
        for (int b = 0; b < 256; b++)
            if (hist[d * 256 + b] == n) trivial = true;
        if (trivial) continue;
        hipLaunchKernelGGL(k_tile_hist, dim3(ntiles), dim3(kSortThreads), 0, st, src, n, d,
                           s.counts, ntiles);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, st, s.counts,
                           (uint64_t)256 * ntiles);
        hipLaunchKernelGGL(k_scatter, dim3(ntiles), dim3(kSortThreads), 0, st, src, src_ids,
                           dst, dst_ids, n, d, s.counts, ntiles);
        std::swap(src, dst);
        std::swap(src_ids, dst_ids);
    }
    if (src != keys) {
        if (hipMemcpyAsync(keys, src, sizeof(Key) * n, hipMemcpyDeviceToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(ids, src_ids, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice,
                           st) != hipSuccess)
            return HC_ERR_HIP;
    }
    return last_hip();
}

// The sampled-key levels of curve c from its sorted keys.
static hc_status sample_levels(const IndexView &v, uint32_t c, hipStream_t st)
{
    uint64_t stride = 1;
    for (uint32_t l = 1; l <= v.levels; l++) {
        stride *= kFan;
        hipLaunchKernelGGL(k_sample_keys, dim3(blocks_for(v.len[l], 256)), dim3(256), 0, st,
                           v.lvl[c][0], stride, (Key *)v.lvl[c][l], v.len[l]);
    }
    if (v.len_sub)
        hipLaunchKernelGGL(k_sample_keys, dim3(blocks_for(v.len_sub, 256)), dim3(256), 0, st,
                           v.lvl[c][0], (uint64_t)kSub, (Key *)v.sub[c], v.len_sub);
    if (v.len_sub2)
        hipLaunchKernelGGL(k_sample_keys, dim3(blocks_for(v.len_sub2, 256)), dim3(256), 0, st,
                           v.lvl[c][0], (uint64_t)(kFan * kSub), (Key *)v.sub2[c], v.len_sub2);
    return last_hip();
}

static hc_status sort_curve(const IndexView &v, uint32_t c, Key *keys, uint32_t *ids,
                            const BuildScratch &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_encode_curve, dim3(blocks_for(v.n, 256)), dim3(256), 0, st, v, c,
                       v.db, v.n, 0u, keys, ids);
    hc_status r = radix_sort(keys, ids, v.n, s, st);
    if (r != HC_OK) return r;
    return sample_levels(v, c, st);
}

// Scratch of an insertion of m rows: the appended entries (keys, ids) and a
// radix-sort scratch for m keys.
struct InsertScratch {
    Key *keys;
    uint32_t *ids;
    BuildScratch sort;
    size_t total;
};

static InsertScratch insert_scratch_layout(uint64_t m, uint8_t *base)
{
    InsertScratch s{};
    size_t off = 0;
    s.keys = (Key *)(base + off);
    off = align256(off + sizeof(Key) * m);
    s.ids = (uint32_t *)(base + off);
    off = align256(off + sizeof(uint32_t) * m);
    s.sort = build_scratch_layout(m, base ? base + off : nullptr);
    s.total = off + s.sort.total;
    return s;
}

// Parameters of an existing index, for a new view of the same kind.
static hc_params params_of(const IndexView &v)
{
    hc_params p;
    memset(&p, 0, sizeof(p));
    p.dim = kDim;
    p.curves = v.curves;
    p.dims_per_curve = kDpc;
    p.bits = 8;
    p.perm = v.perm;
    p.curve = v.curve;
    return p;
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_index_bytes(const hc_params *p, uint64_t n, size_t *index_bytes,
                         size_t *build_scratch_bytes)
{
    hc_status st = check_params(p, nullptr, nullptr);
    if (st != HC_OK) return st;
    if (n == 0) return HC_ERR_INVALID;
    if (n >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;
    if (index_bytes) *index_bytes = make_layout(p->curves, n).total;
    if (build_scratch_bytes) *build_scratch_bytes = build_scratch_layout(n, nullptr).total;
    return HC_OK;
}

hc_status hc_insert_bytes(const hc_index *idx, uint64_t m, size_t *index_bytes,
                          size_t *scratch_bytes)
{
    if (!idx || m == 0) return HC_ERR_INVALID;
    const uint64_t n = idx->v.n + m;
    if (n < m || n >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;
    if (index_bytes) *index_bytes = make_layout(idx->v.curves, n).total;
    if (scratch_bytes) *scratch_bytes = insert_scratch_layout(m, nullptr).total;
    return HC_OK;
}

hc_status hc_insert_rows(const hc_index *idx, const uint8_t *d_db, uint64_t m, void *d_index,
                         size_t index_bytes, void *d_scratch, size_t scratch_bytes,
                         hc_stream stream, hc_index **out)
{
    if (!idx || !out || m == 0 || !d_scratch || ((uintptr_t)d_scratch & 255))
        return HC_ERR_INVALID;
    const uint64_t n0 = idx->v.n, n = n0 + m;
    if (n < m || n >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;
    // the new index is written next to the old one, never over it
    const uintptr_t a0 = (uintptr_t)idx->base, a1 = a0 + idx->bytes;
    const uintptr_t b0 = (uintptr_t)d_index, b1 = b0 + index_bytes;
    if (d_index && b0 < a1 && a0 < b1) return HC_ERR_INVALID;
    const InsertScratch s = insert_scratch_layout(m, (uint8_t *)d_scratch);
    if (scratch_bytes < s.total) return HC_ERR_SIZE;
    hc_index *h = new (std::nothrow) hc_index;
    if (!h) return HC_ERR_INVALID;
    const hc_params p = params_of(idx->v);
    hc_status st = fill_view(&p, d_db, n, d_index, index_bytes, &h->v);
    const hipStream_t hs = (hipStream_t)stream;
    for (uint32_t c = 0; st == HC_OK && c < h->v.curves; c++) {
        hipLaunchKernelGGL(k_encode_curve, dim3(blocks_for(m, 256)), dim3(256), 0, hs, h->v,
                           c, d_db + n0 * kDim, m, (uint32_t)n0, s.keys, s.ids);
        st = radix_sort(s.keys, s.ids, m, s.sort, hs);
        if (st != HC_OK) break;
        Key *keys = (Key *)h->v.lvl[c][0];
        uint32_t *ids = (uint32_t *)h->v.ids[c];
        hipLaunchKernelGGL(k_merge_old, dim3(blocks_for(n0, 256)), dim3(256), 0, hs,
                           idx->v.lvl[c][0], idx->v.ids[c], n0, (const Key *)s.keys, m, keys,
                           ids);
        hipLaunchKernelGGL(k_merge_added, dim3(blocks_for(m, 256)), dim3(256), 0, hs,
                           idx->v.lvl[c][0], n0, (const Key *)s.keys, (const uint32_t *)s.ids,
                           m, keys, ids);
        st = sample_levels(h->v, c, hs);
    }
    if (st != HC_OK) {
        delete h;
        return st;
    }
    h->base = d_index;
    h->bytes = index_bytes;
    *out = h;
    return HC_OK;
}

hc_status hc_build_index(const hc_params *p, const uint8_t *d_db, uint64_t n, void *d_index,
                         size_t index_bytes, void *d_scratch, size_t scratch_bytes,
                         hc_stream stream, hc_index **out)
{
    if (!out) return HC_ERR_INVALID;
    hc_index *h = new (std::nothrow) hc_index;
    if (!h) return HC_ERR_INVALID;
    hc_status st = fill_view(p, d_db, n, d_index, index_bytes, &h->v);
    if (st == HC_OK && (!d_scratch || ((uintptr_t)d_scratch & 255))) st = HC_ERR_INVALID;
    BuildScratch s{};
    if (st == HC_OK) {
        s = build_scratch_layout(n, (uint8_t *)d_scratch);
        if (scratch_bytes < s.total) st = HC_ERR_SIZE;
    }
    for (uint32_t c = 0; st == HC_OK && c < h->v.curves; c++)
        st = sort_curve(h->v, c, (Key *)h->v.lvl[c][0], (uint32_t *)h->v.ids[c], s,
                        (hipStream_t)stream);
    if (st != HC_OK) {
        delete h;
        return st;
    }
    h->base = d_index;
    h->bytes = index_bytes;
    *out = h;
    return HC_OK;
}

}  // extern "C"
