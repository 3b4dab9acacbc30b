// Multicurves search (Alg. 2) as one fused kernel per batch, gfx950.
//
// One workgroup per query:
//  1. locate the query key in each curve's sorted list (count of keys < qkey)
//     by descending the 64-ary sampled-key table: at every level one wave
//     loads 64 consecutive keys (1 KiB, coalesced) and a ballot counts how
//     many are below the query key; all curves of a wave descend together;
//  2. window: w list entries on each side of that position (Alg. 2, the
//     "probe-depth closest" entries, read as the half-list model of Sec. 4.2);
//  3. union of the windows' ids as a set: an open-addressing hash in LDS;
//  4. exact squared Euclidean distance of each distinct candidate (Eq. 2):
//     8 lanes read one 128-byte row with 16-byte loads, dot4 integer
//     arithmetic, a 3-step lane-xor reduction;
//  5. the k nearest by (distance, id): each lane keeps a sorted list in
//     registers; the wave then pops its global minimum k times.  For k > 16
//     the distances go to LDS and are bitonic-sorted instead.
// When the union is larger than the LDS chunk, steps 3-5 run per chunk and
// the chunk results are merged, dropping repeated ids.
#include <string.h>

#include <algorithm>

#include "hc_internal.h"

namespace hc {

constexpr int kKR = 16;                 // register list length (k <= 16 path)
constexpr uint32_t kMaxChunk = 4096;    // slots per chunk (LDS: 12 B per slot)

enum { MODE_SEARCH = 0, MODE_POS = 1, MODE_CAND = 2 };

struct SearchArgs {
    IndexView v;
    const uint8_t *queries;
    const Key *qkeys;          // [q][curves]
    uint32_t nq, k, w_fixed;
    const uint32_t *d_w;
    uint32_t *out_ids, *out_dists;
    uint32_t *out_pos;         // MODE_POS: [q][curves]
    uint32_t *out_counts;      // MODE_CAND
    uint32_t *out_cand;
    uint32_t cand_stride;
    uint32_t cs_log2;          // chunk capacity = 1 << cs_log2 slots
};

__device__ inline uint32_t lanes_below64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}

// Sum over 16 bytes of (q - x)^2 = q.q + x.x - 2 q.x with 4-byte dot products
// (all terms are exact in uint32).
__device__ inline uint32_t sqdist16(const uint4 &q, uint32_t qq, const uint4 &x)
{
    uint32_t xx = __builtin_amdgcn_udot4(x.x, x.x, 0u, false);
    xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
    xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
    xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
    uint32_t qx = __builtin_amdgcn_udot4(q.x, x.x, 0u, false);
    qx = __builtin_amdgcn_udot4(q.y, x.y, qx, false);
    qx = __builtin_amdgcn_udot4(q.z, x.z, qx, false);
    qx = __builtin_amdgcn_udot4(q.w, x.w, qx, false);
    return qq + xx - 2u * qx;
}

// Inserts x into an ascending register list (unrolled: static indexing only).
__device__ inline void list_insert(uint64_t (&L)[kKR], uint64_t x)
{
    if (x < L[kKR - 1]) {
#pragma unroll
        for (int i = kKR - 1; i > 0; i--)
            L[i] = x < L[i - 1] ? L[i - 1] : (x < L[i] ? x : L[i]);
        L[0] = x < L[0] ? x : L[0];
    }
}

// Merges two ascending lists of k packed keys (kNone = empty) into out,
// keeping the first k distinct keys.  Run by one thread.
__device__ inline void merge_distinct(const uint64_t *a, const uint64_t *b, uint32_t k,
                                      uint64_t *out)
{
    uint32_t i = 0, j = 0;
    for (uint32_t o = 0; o < k; o++) {
        const uint64_t x = i < k ? a[i] : kNone;
        const uint64_t y = j < k ? b[j] : kNone;
        if (x < y) {
            out[o] = x;
            i++;
        } else if (y < x) {
            out[o] = y;
            j++;
        } else {
            out[o] = x;   // equal: the same candidate seen in two chunks
            i++;
            j++;
        }
    }
}

template <int NW, bool BIGK, int MODE>
__global__ __launch_bounds__(64 * NW) void k_search(SearchArgs a)
{
    extern __shared__ uint32_t lds[];
    constexpr int CPW = (kMaxCurves + NW - 1) / NW;   // curves per wave
    constexpr int NT = 64 * NW;
    __shared__ uint32_t s_pos[kMaxCurves];
    __shared__ uint32_t s_count;
    constexpr int KCAP = BIGK ? HC_K_MAX : kKR;      // longest running list
    __shared__ uint64_t s_run[KCAP];
    __shared__ uint64_t s_tmp[KCAP];
    __shared__ uint64_t s_out[KCAP];
    __shared__ uint64_t s_wave[NW][kKR];

    const uint32_t cs = 1u << a.cs_log2;
    const uint32_t tsize = 2u * cs;                  // hash slots
    uint32_t *hash = lds;
    uint32_t *list = lds + tsize;
    uint64_t *ckeys = reinterpret_cast<uint64_t *>(lds);   // overlays hash

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t q = blockIdx.x;
    if (q >= a.nq) return;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint32_t D = a.v.levels;

    // ---- 1. position of the query key in each curve --------------------
    {
        Key qk[CPW];
        uint64_t cnt[CPW];
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const uint32_t c = wave + j * NW;
            if (c < C) qk[j] = a.qkeys[(uint64_t)q * C + c];
            else qk[j] = Key{0, 0};
        }
        {   // top table: at most 64 entries
            Key kk[CPW];
            const bool valid = (uint64_t)lane < a.v.len[D];
#pragma unroll
            for (int j = 0; j < CPW; j++) {
                const uint32_t c = wave + j * NW;
                kk[j] = (c < C && valid) ? a.v.lvl[c][D][lane] : Key{~0ull, ~0ull};
            }
#pragma unroll
            for (int j = 0; j < CPW; j++) {
                const bool less = (wave + j * NW < C) && valid && key_less(kk[j], qk[j]);
                cnt[j] = (uint64_t)__popcll(__ballot(less));
            }
        }
        for (int L = (int)D; L >= 1; L--) {
            // cnt = entries of level L below qkey; the answer at level L-1 lies
            // in the 64 entries starting at 64*(cnt-1) (entry 64*cnt is >= qkey).
            Key kk[CPW];
            uint64_t base[CPW];
            const uint64_t len = a.v.len[L - 1];
#pragma unroll
            for (int j = 0; j < CPW; j++) {
                const uint32_t c = wave + j * NW;
                base[j] = cnt[j] ? (cnt[j] - 1) * kFan : 0;
                const uint64_t idx = base[j] + lane;
                kk[j] = (c < C && cnt[j] && idx < len) ? a.v.lvl[c][L - 1][idx]
                                                      : Key{~0ull, ~0ull};
            }
#pragma unroll
            for (int j = 0; j < CPW; j++) {
                const uint32_t c = wave + j * NW;
                const uint64_t idx = base[j] + lane;
                const bool less = c < C && cnt[j] && idx < len && key_less(kk[j], qk[j]);
                const uint64_t m = __ballot(less);
                cnt[j] = cnt[j] ? base[j] + (uint64_t)__popcll(m) : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const uint32_t c = wave + j * NW;
            if (c < C && lane == 0) s_pos[c] = (uint32_t)cnt[j];
        }
    }
    __syncthreads();
    if constexpr (MODE == MODE_POS) {
        if (tid < (int)C) a.out_pos[(uint64_t)q * C + tid] = s_pos[tid];
        return;
    }

    // ---- 2. windows ------------------------------------------------------
    __shared__ uint64_t s_wlo[kMaxCurves], s_wn[kMaxCurves];
    __shared__ const uint32_t *s_ids[kMaxCurves];
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
    __syncthreads();
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) total += s_wn[c];
    if constexpr (MODE == MODE_CAND) {
        if (total > cs) {   // the union does not fit one chunk: flag the query
            if (tid == 0) a.out_counts[q] = 0xFFFFFFFFu;
            return;
        }
    }

    // query bytes for this lane's 16-byte part of a row
    const int part = lane & 7;
    const uint4 qv = *reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim + 16 * part);
    const uint32_t qq = __builtin_amdgcn_udot4(qv.x, qv.x, 0u, false) +
                        __builtin_amdgcn_udot4(qv.y, qv.y, 0u, false) +
                        __builtin_amdgcn_udot4(qv.z, qv.z, 0u, false) +
                        __builtin_amdgcn_udot4(qv.w, qv.w, 0u, false);

    const uint32_t k = a.k;
    for (uint32_t i = tid; i < k; i += NT) s_run[i] = kNone;
    const uint32_t hshift = 32u - (a.cs_log2 + 1u);

    for (uint64_t c0 = 0; c0 < total; c0 += cs) {
        const uint32_t cn = (uint32_t)std::min<uint64_t>(cs, total - c0);
        // ---- 3. union of the window ids (distinct within the chunk) -----
        for (uint32_t i = tid; i < tsize; i += NT) hash[i] = kEmpty;
        if (tid == 0) s_count = 0;
        __syncthreads();
        for (uint32_t s = tid; s < cn; s += NT) {
            uint64_t g = c0 + s;
            int c = 0;
            while (g >= s_wn[c]) {
                g -= s_wn[c];
                c++;
            }
            const uint32_t id = s_ids[c][s_wlo[c] + g];
            uint32_t h = (id * 0x9E3779B1u) >> hshift;
            while (true) {
                const uint32_t prev = atomicCAS(&hash[h], kEmpty, id);
                if (prev == kEmpty || prev == id) break;
                h = (h + 1) & (tsize - 1);
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
        if constexpr (MODE == MODE_CAND) {
            if (tid == 0) a.out_counts[q] = u;
            for (uint32_t i = tid; i < u; i += NT)
                a.out_cand[(uint64_t)q * a.cand_stride + i] = list[i];
            return;
        }

        // ---- 4. distances, 64 rows per wave step --------------------------
        uint64_t L[kKR];
#pragma unroll
        for (int i = 0; i < kKR; i++) L[i] = kNone;
        for (uint32_t g = wave; g * 64u < u; g += NW) {
            const uint32_t row0 = g * 64u;
            uint32_t rid[8];
            uint4 x[8];
#pragma unroll
            for (int s = 0; s < 8; s++) {
                const uint32_t r = row0 + s * 8 + (lane >> 3);
                rid[s] = r < u ? list[r] : 0u;
            }
#pragma unroll
            for (int s = 0; s < 8; s++) {
                const uint32_t r = row0 + s * 8 + (lane >> 3);
                x[s] = r < u ? *reinterpret_cast<const uint4 *>(a.v.db + (uint64_t)rid[s] * kDim +
                                                                16 * part)
                             : make_uint4(0, 0, 0, 0);
            }
            uint32_t mine = 0, myid = 0;
#pragma unroll
            for (int s = 0; s < 8; s++) {
                uint32_t d = sqdist16(qv, qq, x[s]);
                d += __shfl_xor(d, 1, 64);
                d += __shfl_xor(d, 2, 64);
                d += __shfl_xor(d, 4, 64);
                if (part == s) {
                    mine = d;
                    myid = rid[s];
                }
            }
            const uint32_t myrow = row0 + part * 8 + (lane >> 3);
            const uint64_t key = myrow < u ? (((uint64_t)mine << 32) | myid) : kNone;
            if constexpr (BIGK) {
                if (myrow < u) ckeys[myrow] = key;
            } else {
                list_insert(L, key);
            }
        }

        // ---- 5. k nearest of the chunk, merged into the running list ------
        if constexpr (!BIGK) {
            uint64_t mykey = kNone;
            for (uint32_t j = 0; j < k; j++) {
                const uint64_t m = wave_min_u64(L[0]);
                if ((uint32_t)lane == j) mykey = m;
                if (m != kNone && L[0] == m) {
#pragma unroll
                    for (int i = 0; i < kKR - 1; i++) L[i] = L[i + 1];
                    L[kKR - 1] = kNone;
                }
            }
            if (NW == 1 && c0 == 0 && cn == total) {
                // the whole union fit in one chunk: write the result directly
                if ((uint32_t)lane < k) {
                    a.out_ids[(uint64_t)q * k + lane] = (uint32_t)mykey;
                    a.out_dists[(uint64_t)q * k + lane] = (uint32_t)(mykey >> 32);
                }
                return;
            }
            if ((uint32_t)lane < k) s_wave[wave][lane] = mykey;
            __syncthreads();
            if (tid == 0) {
                for (int wv = 0; wv < NW; wv++) {
                    merge_distinct(s_run, s_wave[wv], k, s_out);
                    for (uint32_t i = 0; i < k; i++) s_run[i] = s_out[i];
                }
            }
            __syncthreads();
        } else {
            __syncthreads();
            uint32_t p2 = 1;
            while (p2 < u) p2 <<= 1;
            for (uint32_t i = u + tid; i < p2; i += NT) ckeys[i] = kNone;
            __syncthreads();
            for (uint32_t size = 2; size <= p2; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t i = tid; i < p2 / 2; i += NT) {
                        const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
                        const uint32_t hi = lo + stride;
                        const bool up = (lo & size) == 0;
                        const uint64_t x0 = ckeys[lo], x1 = ckeys[hi];
                        if ((x0 > x1) == up) {
                            ckeys[lo] = x1;
                            ckeys[hi] = x0;
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t i = tid; i < k; i += NT) s_tmp[i] = i < u ? ckeys[i] : kNone;
            __syncthreads();
            if (tid == 0) {
                merge_distinct(s_run, s_tmp, k, s_out);
                for (uint32_t i = 0; i < k; i++) s_run[i] = s_out[i];
            }
            __syncthreads();
        }
    }
    if constexpr (MODE == MODE_CAND) {
        // empty union: no chunk ran
        if (tid == 0) a.out_counts[q] = 0;
        return;
    }
    for (uint32_t i = tid; i < k; i += NT) {
        const uint64_t key = s_run[i];
        a.out_ids[(uint64_t)q * k + i] = (uint32_t)key;
        a.out_dists[(uint64_t)q * k + i] = (uint32_t)(key >> 32);
    }
}

struct LaunchShape {
    int nw;
    uint32_t cs_log2;
};

static uint32_t ceil_log2(uint64_t x)
{
    uint32_t l = 0;
    while ((1ull << l) < x) l++;
    return l;
}

// Chunk capacity and waves per query from the (typical) window w.
static LaunchShape pick_shape(uint64_t w_hint, uint32_t max_slots)
{
    const uint64_t slots = std::max<uint64_t>(16 * std::max<uint64_t>(w_hint, 1), 64);
    LaunchShape s;
    s.nw = slots > 1024 ? 4 : 1;
    uint64_t cs = std::min<uint64_t>(slots, max_slots);
    cs = std::max<uint64_t>(cs, 64u * s.nw);
    s.cs_log2 = ceil_log2(cs);
    return s;
}

template <int NW, bool BIGK, int MODE>
static hc_status launch(const SearchArgs &a, hipStream_t st)
{
    const size_t lds = (size_t)12 << a.cs_log2;
    hipLaunchKernelGGL((k_search<NW, BIGK, MODE>), dim3(a.nq), dim3(64 * NW), lds, st, a);
    return last_hip();
}

template <int MODE>
static hc_status launch_mode(const SearchArgs &a, int nw, bool bigk, hipStream_t st)
{
    if (nw == 1) return bigk ? launch<1, true, MODE>(a, st) : launch<1, false, MODE>(a, st);
    return bigk ? launch<4, true, MODE>(a, st) : launch<4, false, MODE>(a, st);
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

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_search_scratch_bytes(const hc_index *idx, uint32_t nq, size_t *bytes)
{
    if (!idx || !bytes) return HC_ERR_INVALID;
    *bytes = align256(sizeof(Key) * (size_t)std::max<uint32_t>(nq, 1) * idx->v.curves);
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

hc_status hc_search_encoded(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                            uint32_t *d_out_ids, uint32_t *d_out_dists, void *d_scratch,
                            size_t scratch_bytes, hc_stream stream)
{
    if (k < 1 || k > HC_K_MAX || !d_out_ids || !d_out_dists) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hc_status st = check_common(idx, d_queries, d_scratch, scratch_bytes, nq);
    if (st != HC_OK) return st;
    SearchArgs a = base_args(idx, d_queries, nq, d_scratch);
    a.k = k;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;
    const uint64_t hint = d_w ? (w_fixed ? w_fixed : 64) : w_fixed;
    LaunchShape sh = pick_shape(hint, kMaxChunk);
    a.cs_log2 = sh.cs_log2;
    return launch_mode<MODE_SEARCH>(a, sh.nw, k > (uint32_t)kKR, (hipStream_t)stream);
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
    a.cs_log2 = 6;
    return launch_mode<MODE_POS>(a, 1, false, s);
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
    if (stride > kMaxChunk) return HC_ERR_UNSUPPORTED;
    if (!d_w && (uint64_t)stride < 16ull * w_fixed) return HC_ERR_SIZE;
    hipStream_t s = (hipStream_t)stream;
    SearchArgs a = base_args(idx, d_queries, nq, d_scratch);
    st = encode_rows(a.v, d_queries, nq, (Key *)d_scratch, s);
    if (st != HC_OK) return st;
    a.w_fixed = d_w ? std::min<uint32_t>(w_fixed, stride / 16) : w_fixed;
    a.d_w = d_w;
    a.out_counts = d_counts;
    a.out_cand = d_ids;
    a.cand_stride = stride;
    // one chunk must hold the whole union: capacity >= stride >= 16 w
    a.cs_log2 = std::max<uint32_t>(ceil_log2(std::max<uint32_t>(stride, 64)), 6);
    return launch_mode<MODE_CAND>(a, 1, false, s);
}

}  // extern "C"
