// Internal definitions shared by the library's translation units (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hypercurves.h"

namespace hc {

constexpr int kDim = 128;          // bytes per vector
constexpr int kDpc = 16;           // dims per curve
constexpr int kMaxCurves = 8;
constexpr int kFan = 64;           // fan-out of the sampled-key table = wave size
constexpr int kSub = 8;            // fan-out of the last two steps (8 keys = 128 B)
constexpr int kMaxLevels = 6;      // 64^6 > 2^32 rows
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kNone = ~0ull;  // packed (dist << 32 | id) of an empty slot

struct Key {                       // 128-bit key, compared as (hi, lo)
    uint64_t hi, lo;
};

// Device view of one index, passed by value to kernels.
struct IndexView {
    const uint8_t *db;
    uint64_t n;
    uint32_t curves;
    uint32_t levels;                          // D: top table is level D
    uint64_t len[kMaxLevels + 1];             // entries of level L (len[0] = n)
    const Key *lvl[kMaxCurves][kMaxLevels + 1];   // lvl[c][0] = sorted keys
    uint64_t len_sub;                         // entries of sub (0 when levels == 0)
    const Key *sub[kMaxCurves];               // every kSub-th key of curve c
    uint64_t len_sub2;                        // entries of sub2 (0 when levels < 2)
    const Key *sub2[kMaxCurves];              // every (kFan kSub)-th key of curve c
    const uint32_t *ids[kMaxCurves];
    uint16_t perm[kMaxCurves * kDpc];
    uint32_t identity;                        // perm is 16c + j
    uint32_t curve;                           // HC_CURVE_HILBERT or HC_CURVE_ZORDER
    // optional row store, curve c's entries in list order and padded to a
    // multiple of 256 entries (null when absent): the rows stored as 127 - x,
    // floor(crow / 2) and crow mod 2 with crow = sum x (x - 256), and the ids
    const uint8_t *rows[kMaxCurves];
    const int *crow2[kMaxCurves];
    const uint8_t *par[kMaxCurves];
    const uint32_t *rid[kMaxCurves];
};

}  // namespace hc

struct hc_index {
    hc::IndexView v;
    void *base;
    size_t bytes;
    // the caller's events, recorded around the search's main kernel when set
    hipEvent_t kernel_begin = nullptr, kernel_end = nullptr;
};

namespace hc {

// Layout of the index buffer: per curve, keys[n], ids[n], levels 1..D (level
// L holds every 64^L-th key), then, when D >= 1, sub[ceil(n / 8)] (every 8th
// key) and, when D >= 2, sub2[ceil(n / 512)] (every 512th key); every array
// starts on a 256-byte boundary.
struct Layout {
    uint32_t levels;
    uint64_t len[kMaxLevels + 1];
    uint64_t len_sub, len_sub2;
    size_t keys_off[kMaxCurves], ids_off[kMaxCurves];
    size_t lvl_off[kMaxCurves][kMaxLevels + 1];
    size_t sub_off[kMaxCurves], sub2_off[kMaxCurves];
    size_t total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(uint32_t curves, uint64_t n)
{
    Layout L{};
    uint32_t D = 0;
    L.len[0] = n;
    while (L.len[D] > (uint64_t)kFan && D < kMaxLevels) {
        L.len[D + 1] = (L.len[D] + kFan - 1) / kFan;
        D++;
    }
    L.levels = D;
    L.len_sub = D ? (n + kSub - 1) / kSub : 0;
    L.len_sub2 = D >= 2 ? (n + kFan * kSub - 1) / (kFan * kSub) : 0;
    size_t off = 0;
    for (uint32_t c = 0; c < curves; c++) {
        L.keys_off[c] = off;
        L.lvl_off[c][0] = off;
        off = align256(off + sizeof(Key) * n);
        L.ids_off[c] = off;
        off = align256(off + sizeof(uint32_t) * n);
        for (uint32_t l = 1; l <= D; l++) {
            L.lvl_off[c][l] = off;
            off = align256(off + sizeof(Key) * L.len[l]);
        }
        L.sub_off[c] = off;
        off = align256(off + sizeof(Key) * L.len_sub);
        L.sub2_off[c] = off;
        off = align256(off + sizeof(Key) * L.len_sub2);
    }
    L.total = off;
    return L;
}

hc_status check_params(const hc_params *p, uint16_t *perm_out, uint32_t *identity);
hc_status fill_view(const hc_params *p, const uint8_t *d_db, uint64_t n, void *d_index,
                    size_t index_bytes, IndexView *v);

// Launch helpers -----------------------------------------------------------

inline hc_status last_hip()
{
    return hipGetLastError() == hipSuccess ? HC_OK : HC_ERR_HIP;
}

// Records ev on st if it is set.
inline hc_status record_if(hipEvent_t ev, hipStream_t st)
{
    return !ev || hipEventRecord(ev, st) == hipSuccess ? HC_OK : HC_ERR_HIP;
}

// Query keys for the search kernels: keys[q*curves + c].
hc_status encode_rows(const IndexView &v, const uint8_t *rows, uint64_t nrows, Key *keys,
                      hipStream_t s);

// Gather search (hc_search.hip) of the queries q with only[q] != 0, keys in qkeys.
hc_status gather_search_only(const IndexView &v, const uint8_t *d_queries, const Key *qkeys,
                             uint32_t nq, uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                             const uint32_t *only, uint32_t *d_out_ids, uint32_t *d_out_dists,
                             hipStream_t st);

// Work-item search (hc_uneven.hip): each query's windows cut into items that
// the wavefronts of a persistent grid take from a queue, then merged.  With
// keys_ready the query keys are already at the start of d_scratch.
hc_status items_search(const IndexView &v, const uint8_t *d_queries, uint32_t nq,
                       uint32_t w_fixed, const uint32_t *d_w, uint32_t k_fixed,
                       const uint32_t *d_k, uint32_t k_stride, uint32_t *d_out_ids,
                       uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                       uint32_t chunk, uint32_t max_split, uint32_t per_cu, bool keys_ready,
                       hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end);
// its scratch with the default launch shape
size_t items_scratch_bytes(uint32_t curves, uint32_t nq, uint32_t k_stride);
constexpr uint32_t kItemChunk = 8192;   // default item size in window slots
constexpr uint32_t kItemSplit = 32;     // default items per query at most

// Banded search (hc_band.hip), query keys already at the start of d_scratch.
// Scratch for a batch of nq queries with k up to k_max (k_max > 16 adds the
// buffers of the two-pass search; it needs the row store).
size_t band_scratch_bytes(uint32_t curves, uint64_t n, uint32_t nq, uint32_t k_max);
constexpr uint32_t kBandKMax = HC_BAND_K_MAX;   // largest k the banded path takes
uint64_t band_blocks(uint32_t curves, uint32_t nq, uint32_t w);   // blocks of its main kernel
// the same when a small batch's groups are dealt out (row store)
uint64_t band_split_blocks(uint32_t curves, uint32_t nq, uint32_t w, uint32_t k);
hc_status band_search(const IndexView &v, const uint8_t *d_queries, uint32_t nq, uint32_t k,
                      uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_out_ids,
                      uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                      hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end);

__host__ __device__ inline bool key_less(const Key &a, const Key &b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

}  // namespace hc
