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

#include "hc_device.h"

namespace hc {

constexpr int kKR = 16;                 // longest register list (k <= 16)
constexpr int kBuf = 1024;              // LDS buffer of the k > 16 path
constexpr uint32_t kMaxSetSlots = 4096; // union capacity of the set kernel
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
};

// Sum over 16 bytes of (q - x)^2 = q.q + x.x - 2 q.x with 4-byte dot products
// (every term is exact in uint32).
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

// Inserts x into an ascending register list unless the list holds it already
// (unrolled: static register indexing only).
template <int KR>
__device__ inline void insert_distinct(uint64_t (&L)[KR], uint64_t x)
{
    if (x < L[KR - 1]) {
        bool dup = false;
#pragma unroll
        for (int i = 0; i < KR; i++) dup |= (L[i] == x);
        if (!dup) {
#pragma unroll
            for (int i = KR - 1; i > 0; i--)
                L[i] = x < L[i - 1] ? L[i - 1] : (x < L[i] ? x : L[i]);
            L[0] = x < L[0] ? x : L[0];
        }
    }
}

// Merges two ascending lists (kNone = empty) into the first k distinct keys.
// Either list may repeat a key.  Run by one lane.
__device__ inline void merge_distinct(const uint64_t *a, uint32_t na, const uint64_t *b,
                                      uint32_t nb, uint32_t k, uint64_t *out)
{
    uint32_t i = 0, j = 0, o = 0;
    uint64_t last = kNone;
    while (o < k) {
        const uint64_t x = i < na ? a[i] : kNone;
        const uint64_t y = j < nb ? b[j] : kNone;
        const uint64_t m = x < y ? x : y;
        if (m == kNone) break;
        if (x == m) i++;
        if (y == m) j++;
        if (m != last) {
            out[o++] = m;
            last = m;
        }
    }
    for (; o < k; o++) out[o] = kNone;
}

// ---------------------------------------------------------------------------
// Search kernel
// ---------------------------------------------------------------------------

// G: 64-slot groups a wave loads per iteration (rows in flight per lane = 8G).
// At least 5 waves per SIMD (<= 102 VGPRs) unless the 16-entry list would spill.
template <int KR, int G, bool BIGK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((KR > 10 || BIGK) ? 4 : 5)))
void k_stream(SearchArgs a)
{
    __shared__ const uint32_t *s_base[kMaxCurves + 1];   // &ids_c[lo_c]
    __shared__ uint64_t s_off[kMaxCurves + 1];           // window prefix sums
    __shared__ uint64_t s_buf[BIGK ? kBuf : 1];
    __shared__ uint64_t s_run[BIGK ? HC_K_MAX : 1];
    __shared__ uint64_t s_out[BIGK ? HC_K_MAX : 1];

    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    if (q >= a.nq) return;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint32_t k = a.k;

    // this lane's 16-byte part of the query row
    const int part = lane & 7;
    const uint4 qv = *reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim + 16 * part);
    const uint32_t qq = __builtin_amdgcn_udot4(qv.x, qv.x, 0u, false) +
                        __builtin_amdgcn_udot4(qv.y, qv.y, 0u, false) +
                        __builtin_amdgcn_udot4(qv.z, qv.z, 0u, false) +
                        __builtin_amdgcn_udot4(qv.w, qv.w, 0u, false);
    const uint64_t w = a.d_w ? a.d_w[q] : a.w_fixed;

    // ---- 1-2. positions and windows ----------------------------------------
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) {
        uint64_t lo = 0, cnt = 0;
        if (c < (int)C) {
            lo = pos[c] > w ? pos[c] - w : 0;
            const uint64_t hi = pos[c] + w < n ? pos[c] + w : n;
            cnt = hi - lo;
        }
        if (lane == c) {
            s_base[c] = c < (int)C ? a.v.ids[c] + lo : nullptr;
            s_off[c] = total;
        }
        total += cnt;
    }
    if (lane == kMaxCurves) {
        s_base[kMaxCurves] = nullptr;
        s_off[kMaxCurves] = total;
    }
    __syncthreads();
    uint64_t off[kMaxCurves];   // uniform copies of the prefix sums
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) off[c] = s_off[c];

    uint64_t L[KR];
#pragma unroll
    for (int i = 0; i < KR; i++) L[i] = kNone;
    uint32_t nbuf = 0;          // BIGK: keys in s_buf
    uint64_t tau = kNone;       // BIGK: k-th distinct key so far
    if constexpr (BIGK) {
        for (uint32_t i = lane; i < k; i += 64) s_run[i] = kNone;
    }

    auto flush = [&]() {
        // sort the buffer, merge it into the running list, tighten tau
        __syncthreads();
        for (uint32_t i = nbuf + lane; i < (uint32_t)kBuf; i += 64) s_buf[i] = kNone;
        __syncthreads();
        for (uint32_t size = 2; size <= (uint32_t)kBuf; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t i = lane; i < (uint32_t)kBuf / 2; i += 64) {
                    const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
                    const uint32_t hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t x0 = s_buf[lo], x1 = s_buf[hi];
                    if ((x0 > x1) == up) {
                        s_buf[lo] = x1;
                        s_buf[hi] = x0;
                    }
                }
                __syncthreads();
            }
        }
        if (lane == 0) {
            merge_distinct(s_run, k, s_buf, nbuf, k, s_out);
            for (uint32_t i = 0; i < k; i++) s_run[i] = s_out[i];
        }
        __syncthreads();
        tau = s_run[k - 1];
        nbuf = 0;
    };

    // ---- 3-5. stream the window slots -------------------------------------
    for (uint64_t base = 0; base < total; base += 64 * G) {
        // ids of the G*64 slots: lane l loads slot base + 64 g + l (coalesced)
        uint32_t myid[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const uint64_t s = base + 64 * g + lane;
            myid[g] = 0;
            if (s < total) {
                int c = 0;
#pragma unroll
                for (int j = 1; j < kMaxCurves; j++) c += s >= off[j] ? 1 : 0;
                myid[g] = s_base[c][s - s_off[c]];
            }
        }
        // rows: in step t of group g, lanes 8r..8r+7 read row (g, 8t + r)
        uint4 x[8 * G];
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const uint32_t rid = __shfl(myid[g], 8 * t + (lane >> 3), 64);
                const uint64_t s = base + 64 * g + 8 * t + (lane >> 3);
                x[8 * g + t] = s < total
                    ? *reinterpret_cast<const uint4 *>(a.v.db + (uint64_t)rid * kDim + 16 * part)
                    : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
        for (int g = 0; g < G; g++) {
            uint32_t mine = 0;
#pragma unroll
            for (int t = 0; t < 8; t++) {
                uint32_t d = sqdist16(qv, qq, x[8 * g + t]);
                d += __shfl_xor(d, 1, 64);
                d += __shfl_xor(d, 2, 64);
                d += __shfl_xor(d, 4, 64);
                if (part == t) mine = d;
            }
            const uint32_t mid = __shfl(myid[g], 8 * part + (lane >> 3), 64);
            // this lane now holds slot base + 64 g + 8 part + (lane >> 3)
            const uint64_t s = base + 64 * g + 8 * part + (lane >> 3);
            const uint64_t key = s < total ? (((uint64_t)mine << 32) | mid) : kNone;
            if constexpr (!BIGK) {
                insert_distinct<KR>(L, key);
            } else {
                const bool pass = key < tau;
                const uint64_t m = __ballot(pass);
                if (pass) s_buf[nbuf + lanes_below64(m)] = key;
                nbuf += (uint32_t)__popcll(m);
                if (nbuf > (uint32_t)(kBuf - 64)) flush();
            }
        }
    }

    if constexpr (!BIGK) {
        uint64_t mykey = kNone;
        for (uint32_t j = 0; j < k; j++) {
            const uint64_t m = wave_min_u64(L[0]);
            if ((uint32_t)lane == j) mykey = m;
            if (m != kNone && L[0] == m) {   // every lane holding m pops it
#pragma unroll
                for (int i = 0; i < KR - 1; i++) L[i] = L[i + 1];
                L[KR - 1] = kNone;
            }
        }
        if ((uint32_t)lane < k) {
            a.out_ids[(uint64_t)q * k + lane] = (uint32_t)mykey;
            a.out_dists[(uint64_t)q * k + lane] = (uint32_t)(mykey >> 32);
        }
    } else {
        if (nbuf) flush();
        for (uint32_t i = lane; i < k; i += 64) {
            const uint64_t key = s_run[i];
            a.out_ids[(uint64_t)q * k + i] = (uint32_t)key;
            a.out_dists[(uint64_t)q * k + i] = (uint32_t)(key >> 32);
        }
    }
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

template <int KR, int G, bool BIGK>
static hc_status launch_stream(const SearchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_stream<KR, G, BIGK>), dim3(a.nq), dim3(64), 0, st, a);
    return last_hip();
}

// A register list as long as k (1, 4, 10 or 16) for k <= 16, the LDS buffer
// beyond.
template <int G>
static hc_status launch_search_g(const SearchArgs &a, hipStream_t st)
{
    if (a.k == 1) return launch_stream<1, G, false>(a, st);
    if (a.k <= 4) return launch_stream<4, G, false>(a, st);
    if (a.k <= 10) return launch_stream<10, G, false>(a, st);
    if (a.k <= (uint32_t)kKR) return launch_stream<kKR, G, false>(a, st);
    return launch_stream<1, G, true>(a, st);
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
    return launch_search(a, hint, (hipStream_t)stream);
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
