// Banded search for large batches with large windows (gfx950).
//
// In a batch of nq queries with windows of w entries per side, a list entry
// lies in about nq * 2w / n windows of the same curve (at n = 10^7, nq = 10^5,
// w = 27,648: ~550).  The gather search fetches the row once per window; here
// the batch is arranged so that a row is fetched once per group of queries:
//  1. every query's place in every curve (the same descent as the search);
//  2. per curve, the queries ordered by place (a counting sort on place
//     buckets of 2^kBucketShift entries);
//  3. a block takes 256 consecutive queries of one curve (128 below
//     kBandWideW) and streams the union of their windows through LDS, 128
//     (64) list entries at a time: gathered by id and transformed on the way
//     (k_band), or copied from the row store by LDS DMA (k_band_dma); the
//     distances of 32 queries against the tile's rows come from the matrix
//     cores (below), and every entry inside a query's own window is offered,
//     as (distance, id), to that query's register top-k;
//  4. a merge takes each query's per-curve lists and keeps the k nearest
//     distinct ids.
// The candidates, distances and order are exactly those of the gather search
// (Alg. 2): only the grouping of the work differs, so the results are
// identical.  The rows read from HBM drop by the number of queries sharing
// them, and the per-pair arithmetic moves to the matrix cores.
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "hc_device.h"
#include "hc_scan.h"

namespace hc {

constexpr int kBucketShift = 8;   // place buckets of 256 list entries
constexpr int kBandK = 16;        // longest list kept per query and curve
constexpr uint32_t kMaxSplit = 4; // blocks a group's union may be split over
constexpr uint64_t kBandFillBlocks = 512;   // blocks that fill MI355X (2 per CU)
constexpr uint32_t kMQ = 32;             // queries per wavefront
// a large batch's last round: the query slots whose groups may be dealt out
// (at most half the resident blocks of 256 queries, or of 128 at 4 blocks per CU)
constexpr uint32_t kTailQ = 65536;

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
    uint64_t *partial;    // [q][curves][k] (k > 16, first pass: [q][curves][2 kBandK])
    uint32_t *bound;      // [q]: least k-th distance of the curves done so far
    uint32_t *out_ids, *out_dists;
    // k > 16 (two passes): the threshold key of each query, the number of
    // pairs at or below it collected in buf ([q][cap]), and the queries left
    // to the gather kernel
    uint64_t *theta;
    uint32_t *cnt;
    uint64_t *buf;
    uint32_t cap;
    uint32_t *redo;
    uint32_t tight;       // first pass: a half also drops pairs above the other half's 16th
    uint32_t split;       // row-store kernel: blocks per group (the union's tiles dealt out)
    uint32_t split_from;  // groups (curve-major) below it take one block each
    uint32_t pstride;     // lists per query and curve in partial (split, or 1 with a tail)
    uint64_t *tail;       // lists of the dealt-out groups when split_from > 0:
                          // [group - split_from][split][query of the group][k]
};

constexpr uint32_t kBandCap = 1024;   // k > 16: pairs collected per query (buffer entries)
constexpr uint32_t kBandTightK = 32;  // k > 16 up to this: the first pass's halves share a bound

// Blocks a group's union is dealt out over: the least number that gives the
// grid kBandFillBlocks blocks (two per CU), at most kMaxSplit.  Larger groups
// give fewer blocks, so the 256-query groups bound it for any window.  The
// two passes of k > 16 run one block per CU and split only a batch of fewer
// than 256 groups: every split block builds its lists from nothing, which
// costs more than the rounds it saves once the groups fill the device
// (MI355X, N = 1e7, w = 27,648, k = 100: 8,192 queries in 256 blocks 31.4 ms,
// split over 512 45.8 ms; 4,096 queries in 128 blocks 40.0 ms, split over 256
// 31.7 ms, over 512 21.8 ms; N = 1e8, w = 241,664: 6,000 queries 213.8 ms,
// split over 564 blocks 117.7 ms).
inline uint32_t band_split(uint32_t curves, uint32_t nq, uint32_t block_q,
                           uint32_t k = 1)
{
    const uint64_t blocks = ((uint64_t)nq + block_q - 1) / block_q * curves;
    if (k > (uint32_t)kBandK && blocks >= kBandFillBlocks / 2) return 1;
    uint32_t sp = 1;
    while (sp < kMaxSplit && blocks * sp < kBandFillBlocks) sp++;
    return sp;
}

struct BandLayout {
    size_t qkeys, pos, counts, order, partial, tail, bound, theta, cnt, redo, buf, total;
    uint32_t nbuckets;
};

// k_max > 16 adds the two-pass buffers: 2 * kBandK first-pass entries per
// query and curve, the threshold, the counters and kBandCap collected pairs
// per query (8 KiB).
inline BandLayout band_layout(uint32_t curves, uint64_t n, uint32_t nq, uint32_t k_max)
{
    const bool two = k_max > (uint32_t)kBandK;
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
    off = align256(off + sizeof(uint64_t) * (size_t)nq * curves * band_split(curves, nq, 256) *
                         (two ? 2 * kBandK : kBandK));
    L.tail = off;
    if (!two)
        off = align256(off + sizeof(uint64_t) * std::min<size_t>((size_t)nq * curves, kTailQ) *
                             kMaxSplit * kBandK);
    L.bound = off;
    off = align256(off + sizeof(uint32_t) * (size_t)nq);
    L.theta = L.cnt = L.redo = L.buf = 0;
    if (two) {
        L.theta = off;
        off = align256(off + sizeof(uint64_t) * (size_t)nq);
        L.cnt = off;
        off = align256(off + sizeof(uint32_t) * (size_t)nq);
        L.redo = off;
        off = align256(off + sizeof(uint32_t) * (size_t)nq);
        L.buf = off;
        off = align256(off + sizeof(uint64_t) * (size_t)nq * kBandCap);
    }
    L.total = off;
    return L;
}

__global__ __launch_bounds__(256) void k_band_fill(uint32_t *p, uint64_t n, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
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

// ---------------------------------------------------------------------------
// Distances on the matrix cores.  For a query q and a row x (bytes 0..255),
//   sum (q - x)^2 = crow(x) + cq(q) + 2 * sum (127 - x_j)(q_j - 128)
// with crow(x) = sum x_j (x_j - 256) and cq(q) = sum q_j^2 - 254 sum q_j + 128 * 2 * 127 * 128.
// Both factors of the last sum are signed bytes (127 - x = x ^ 0x7F,
// q - 128 = q ^ 0x80), so a 32 x 32 tile of those sums, rows by queries, is
// one chain of four v_mfma_i32_32x32x32_i8 (K = 128).  Every term is an
// exact integer: the distance is the same uint32 as the byte-wise one.
//
// Block: NW wavefronts, 32 queries each, consecutive in curve c's order.  The
// block streams the union of its queries' windows through LDS, 16 NW entries
// per tile (rows stored as 127 - x, 16-byte parts XOR-swizzled against bank
// conflicts; crow and the id of each row beside them).  Lane l of a wavefront
// holds query l % 32 as the B operand; the tile's rows are the A operand; the
// result gives lane l the sums of its query with 16 of every 32 rows (the
// rows 8g + 4h + j, h = l / 32).  So every query has two lanes, each keeping a
// list of the nearest entries among its half of the rows; the halves are
// merged at the end.  The accumulator starts at floor(crow / 2), so the
// product gives h = floor(crow / 2) + sum (127 - x)(q - 128) and the distance
// is 2h + (crow mod 2) + cq: h <= floor((bound - cq) / 2) holds for every
// distance within the bound, so h alone screens the pairs (four at a time).
// Only a pair that passes pays for the exact distance, the window test, the id
// and the insertion (ties are settled by the id there).
// ---------------------------------------------------------------------------

// Wavefronts per block: 8 shares each streamed row among 256 queries (large
// windows, where the rows dominate); 4 keeps blocks small and many (windows
// below kBandWideW, where a block's union is mostly the span of its places).
constexpr uint32_t kBandWideW = 8192;

// queries per block of the banded kernels for a window w
__host__ __device__ constexpr uint32_t band_block_q(uint32_t w)
{
    return w < kBandWideW ? 4 * kMQ : 8 * kMQ;
}
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// 16-byte part c of tile row r; the XOR spreads the rows read together by
// one ds_read_b128 over all banks.
__device__ inline uint32_t mslot(uint32_t r, uint32_t c) { return r * 8 + (c ^ ((r >> 1) & 7)); }

__device__ inline uint4 xor4(uint4 v, uint32_t m)
{
    return make_uint4(v.x ^ m, v.y ^ m, v.z ^ m, v.w ^ m);
}

template <int KR>
__device__ inline int list_bound(const uint64_t (&L)[KR], int cq)
{
    return L[KR - 1] == kNone ? INT32_MAX : (int)(uint32_t)(L[KR - 1] >> 32) - cq;
}

// 1-D grid of groups * curves blocks, curve-major: the curves are worked
// through one after another, so that most blocks start with a bound on the
// k-th distance of their queries from the curves already done.  Any such
// bound is safe: a curve's list holds k distinct candidates of the union, so
// the final k-th distance is at most its k-th distance, and a sum above the
// bound cannot reach the result.  The results do not depend on the timing.
template <int KR, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(KR > 10 ? 3 : 4)))
void k_band(BandArgs a)
{
    constexpr int kMW = NW;
    constexpr int kMRows = 16 * NW;         // list entries per tile: 4 loader threads a row
    constexpr int kMBlockQ = NW * kMQ;
    static_assert(kMRows % 32 == 0, "a tile holds whole 32-row blocks");
    __shared__ uint4 tile[kMRows * 8];
    __shared__ __align__(16) int tile_c[kMRows];     // floor(crow / 2)
    __shared__ uint8_t tile_p[kMRows];               // crow mod 2
    __shared__ uint32_t tile_id[kMRows];
    __shared__ uint32_t wspan[2][kMW];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int h = lane >> 5, qn = lane & 31;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint32_t groups = (a.nq + kMBlockQ - 1) / kMBlockQ;
    const uint32_t grp = blockIdx.x % groups, c = blockIdx.x / groups;

    // this lane's query: B operand (16-byte parts 2s + h), cq, window
    const uint64_t slot = (uint64_t)grp * kMBlockQ + (uint64_t)wv * kMQ + qn;
    const bool live = slot < a.nq;
    const uint32_t q = live ? a.order[(uint64_t)c * a.nq + slot] : 0;
    v4i bq[4];
    uint32_t qq = 0, sq = 0;
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const uint4 v = live ? qrow[2 * s + h] : make_uint4(0, 0, 0, 0);
            qq = __builtin_amdgcn_udot4(v.x, v.x, qq, false);
            qq = __builtin_amdgcn_udot4(v.y, v.y, qq, false);
            qq = __builtin_amdgcn_udot4(v.z, v.z, qq, false);
            qq = __builtin_amdgcn_udot4(v.w, v.w, qq, false);
            sq = __builtin_amdgcn_udot4(v.x, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.y, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.z, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.w, 0x01010101u, sq, false);
            const uint4 b = xor4(v, 0x80808080u);
            bq[s] = v4i{(int)b.x, (int)b.y, (int)b.z, (int)b.w};
        }
    }
    qq += __shfl_xor(qq, 32, 64);
    sq += __shfl_xor(sq, 32, 64);
    const int cq = (int)(qq - 254u * sq + 4161536u);
    // list places fit 32 bits (n < 2^32 - 1)
    uint32_t lo, hi;
    {
        const uint64_t w = live ? (a.d_w ? a.d_w[q] : a.w_fixed) : 0;
        const uint64_t p = live ? a.pos[(uint64_t)q * C + c] : 0;
        lo = live ? (uint32_t)(p > w ? p - w : 0) : 0xFFFFFFFFu;
        hi = live ? (uint32_t)(p + w < n ? p + w : n) : 0u;
    }

    // unions of the wavefront's and of the block's windows
    uint32_t u0 = lo, u1 = hi;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t o0 = __shfl_xor(u0, m, 64), o1 = __shfl_xor(u1, m, 64);
        u0 = o0 < u0 ? o0 : u0;
        u1 = o1 > u1 ? o1 : u1;
    }
    if (lane == 0) {
        wspan[0][wv] = u0;
        wspan[1][wv] = u1;
    }
    __syncthreads();
    uint32_t U0 = 0xFFFFFFFFu, U1 = 0;
#pragma unroll
    for (int i = 0; i < kMW; i++) {
        U0 = wspan[0][i] < U0 ? wspan[0][i] : U0;
        U1 = wspan[1][i] > U1 ? wspan[1][i] : U1;
    }

    uint64_t L[KR];
#pragma unroll
    for (int i = 0; i < KR; i++) L[i] = kNone;
    // bound from the other curves, in the sum's terms (sum = distance - cq)
    // It is re-read every 8 tiles and taken into account one tile later, so
    // that the read's latency hides behind a tile of work.
    int ext = INT32_MAX;
    uint32_t bread = kEmpty;
    auto read_bound = [&]() {
        bread = live ? __hip_atomic_load(a.bound + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : kEmpty;
    };
    auto take_bound = [&]() {
        if (bread != kEmpty) {
            const int e = (int)bread - cq;
            ext = e < ext ? e : ext;
        }
    };
    read_bound();
    take_bound();

    // Tiles are taken from the middle of the union outwards: the entries
    // nearest the queries' places come first and fill the lists with close
    // candidates early, so that fewer later sums pass the list bound.
    const uint32_t T = U0 < U1 ? (uint32_t)(((uint64_t)U1 - U0 + kMRows - 1) / kMRows) : 0u;
    const uint32_t jm = T ? (uint32_t)(((U1 - U0) / 2) / kMRows) : 0u;
    const uint32_t nleft = jm, nright = T ? T - 1 - jm : 0u;
    const uint32_t nboth = nleft < nright ? nleft : nright;
    auto tile_start = [&](uint32_t i) -> uint32_t {
        uint32_t j;
        if (i <= 2 * nboth) j = (i & 1) ? jm + (i + 1) / 2 : jm - i / 2;
        else j = nright > nleft ? jm + (i - nboth) : jm - (i - nboth);
        return U0 + j * kMRows;
    };

    // loader: thread t fills 32 bytes (parts 2f, 2f + 1) of tile row t / 4;
    // the ids run two tiles ahead of the rows, the rows one tile ahead of the
    // matrix work.  Rows past the union (the last tile's tail) read a valid
    // row: they lie outside every window and are never offered.
    const uint32_t *ids = a.v.ids[c];
    const uint32_t lr = (uint32_t)tid >> 2, lf = (uint32_t)tid & 3;
    auto load_id = [&](uint32_t i) -> uint32_t {
        const uint64_t e = (uint64_t)tile_start(i) + lr;
        return e < U1 ? ids[e] : kEmpty;
    };
    uint4 x0 = make_uint4(0, 0, 0, 0), x1 = x0;
    auto load_row = [&](uint32_t id) {
        const uint64_t r = id != kEmpty ? id : 0u;
        const uint4 *src = reinterpret_cast<const uint4 *>(a.v.db + r * kDim) + 2 * lf;
        x0 = src[0];
        x1 = src[1];
    };
    uint32_t xid = T > 0 ? load_id(0) : kEmpty;
    uint32_t id_next = T > 1 ? load_id(1) : kEmpty;
    if (T > 0) load_row(xid);

    for (uint32_t i = 0; i < T; i++) {
        const uint32_t t0 = tile_start(i);
        {
            uint32_t xx = 0, sx = 0;
            const uint32_t parts[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
            for (int m = 0; m < 8; m++) {
                xx = __builtin_amdgcn_udot4(parts[m], parts[m], xx, false);
                sx = __builtin_amdgcn_udot4(parts[m], 0x01010101u, sx, false);
            }
            xx += __shfl_xor(xx, 1, 64);
            sx += __shfl_xor(sx, 1, 64);
            xx += __shfl_xor(xx, 2, 64);
            sx += __shfl_xor(sx, 2, 64);
            __syncthreads();
            tile[mslot(lr, 2 * lf)] = xor4(x0, 0x7F7F7F7Fu);
            tile[mslot(lr, 2 * lf + 1)] = xor4(x1, 0x7F7F7F7Fu);
            if (lf == 0) {
                const int crow = (int)(xx - 256u * sx);
                tile_c[lr] = crow >> 1;
                tile_p[lr] = (uint8_t)(crow & 1);
                tile_id[lr] = xid;
            }
            if ((i & 7) == 0 && i) take_bound();
            __syncthreads();
            if ((i & 7) == 7) read_bound();
            if (i + 1 < T) {
                xid = id_next;
                load_row(xid);
            }
            if (i + 2 < T) id_next = load_id(i + 2);
        }
        if (!(t0 < u1 && (uint64_t)t0 + kMRows > u0)) continue;       // wavefront-uniform

        // this lane's bound: its list, the other half's list, the other curves
        const int own = list_bound(L, cq);
        int th = own;
        {
            const int other = __shfl_xor(own, 32, 64);
            th = other < th ? other : th;
            th = ext < th ? ext : th;
        }
        // the window as tile rows [rlo, rhi)
        const uint32_t rlo = lo > t0 ? std::min<uint32_t>(lo - t0, kMRows) : 0u;
        const uint32_t rhi = hi > t0 ? std::min<uint32_t>(hi - t0, kMRows) : 0u;
        if (!live || rlo >= rhi) th = INT32_MIN;
        int hb = th >> 1;       // screen: h <= floor(bound / 2)
        // A passing pair waits in a pending slot (its h and tile row) and is
        // inserted at the end of the tile, when the whole wavefront inserts at
        // once; a lane inserts early only when a second pair passes.
        int pend_h = 0;
        uint32_t pend_r = kNoRow;
        auto insert_pending = [&]() {
            const int t = 2 * pend_h + (int)tile_p[pend_r];
            const uint64_t key = ((uint64_t)(uint32_t)(t + cq) << 32) | tile_id[pend_r];
            if (key < L[KR - 1]) {
#pragma unroll
                for (int m = KR - 1; m > 0; m--)
                    L[m] = key < L[m - 1] ? L[m - 1] : (key < L[m] ? key : L[m]);
                L[0] = key < L[0] ? key : L[0];
                const int b = list_bound(L, cq);
                th = b < th ? b : th;
                hb = th >> 1;
            }
            pend_r = kNoRow;
        };
#pragma unroll 1
        for (uint32_t rb = 0; rb < kMRows / 32; rb++) {
            // accumulator rows of this lane: 8g + 4h + j; start at floor(crow / 2)
            v16i acc;
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const int4 cr = *reinterpret_cast<const int4 *>(&tile_c[rb * 32 + 8 * g + 4 * h]);
                acc[4 * g] = cr.x;
                acc[4 * g + 1] = cr.y;
                acc[4 * g + 2] = cr.z;
                acc[4 * g + 3] = cr.w;
            }
            const uint32_t ar = rb * 32 + qn;
            if constexpr (KR <= 10) {
                // the four A operands are read before the chain, so that their
                // LDS latencies overlap (the longest list has no registers for it)
                uint4 av[4];
#pragma unroll
                for (int s = 0; s < 4; s++) av[s] = tile[mslot(ar, 2 * s + h)];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < 4; s++)
                    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        v4i{(int)av[s].x, (int)av[s].y, (int)av[s].z, (int)av[s].w}, bq[s],
                        acc, 0, 0, 0);
            } else {
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    const uint4 av = tile[mslot(ar, 2 * s + h)];
                    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        v4i{(int)av.x, (int)av.y, (int)av.z, (int)av.w}, bq[s], acc, 0, 0, 0);
                }
            }
            int hm[4];
#pragma unroll
            for (int g = 0; g < 4; g++)
                hm[g] = std::min(std::min(acc[4 * g], acc[4 * g + 1]),
                                 std::min(acc[4 * g + 2], acc[4 * g + 3]));
            if (std::min(std::min(hm[0], hm[1]), std::min(hm[2], hm[3])) > hb) continue;
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const uint32_t r0 = rb * 32 + 8 * g + 4 * h;
                if (hm[g] <= hb) {       // rare once the lists are full
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        if (acc[4 * g + j] <= hb && r0 + j - rlo < rhi - rlo) {
                            if (pend_r != kNoRow) insert_pending();
                            pend_h = acc[4 * g + j];
                            pend_r = r0 + j;
                        }
                    }
                }
            }
        }
        if (pend_r != kNoRow) insert_pending();
    }

    // lane qn takes the other half's list (rows of one list: ids distinct)
#pragma unroll
    for (int i = 0; i < KR; i++) {
        const uint64_t o = shfl_xor_u64(L[i], 32);
        if (h == 0 && o < L[KR - 1]) {
#pragma unroll
            for (int j = KR - 1; j > 0; j--)
                L[j] = o < L[j - 1] ? L[j - 1] : (o < L[j] ? o : L[j]);
            L[0] = o < L[0] ? o : L[0];
        }
    }
    if (live && h == 0) {
        uint64_t *out = a.partial + ((uint64_t)q * C + c) * a.k;
        uint64_t kth = kNone;
#pragma unroll
        for (int i = 0; i < KR; i++) {
            if ((uint32_t)i < a.k) out[i] = L[i];
            if ((uint32_t)i == a.k - 1) kth = L[i];
        }
        if (kth != kNone) atomicMin(a.bound + q, (uint32_t)(kth >> 32));
    }
}

// ---------------------------------------------------------------------------
// Banded search from the row store, tiles copied straight into LDS.
//
// The same work and the same results as k_band, but a tile's rows, their
// floor(crow / 2), crow mod 2 and list ids come from the row store by LDS DMA
// (global_load_lds_dwordx4: lane l of one instruction writes its 16 bytes at
// the instruction's LDS base + 16 l).  No registers hold a tile on its way.
// Tiles go in groups of kTPB through two sets of stages: while group g is
// worked on, group g + 1 is in flight into the stages group g - 1 used; one
// wait and one barrier per group.  Tiles are aligned to their size in the
// list (the row store is padded to a multiple of 256 entries), which keeps
// every 16-byte copy aligned and inside the store.
//
// The compiler does not follow LDS DMA closely enough (it would wait for
// every copy in flight before any LDS read), so the reads of staged data are
// ds_read instructions with explicit lgkmcnt waits, and the vmcnt waits are
// explicit too.
// ---------------------------------------------------------------------------
constexpr int kTPB = 2;                 // tiles per barrier
constexpr int kStages = 2 * kTPB;

template <int NW>
struct BandStage {
    static constexpr int R = 16 * NW;   // list entries per tile
    uint4 rows[R * 8];                   // 127 - x, 16-byte parts at mslot(r, part)
    int crow2[R];                        // floor(crow / 2)
    uint32_t rid[R];                     // list ids
    uint8_t par[R];                      // crow mod 2
};

typedef __attribute__((address_space(3))) void lds_void;

__device__ inline uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(const lds_void *)p;
}

// 16 bytes per lane from global memory to LDS at lds + 16 * lane
__device__ inline void dma16(const void *g, void *lds)
{
    __builtin_amdgcn_global_load_lds(g, (lds_void *)lds, 16, 0, 0);
}

// 4 bytes per lane from global memory to LDS at lds + 4 * lane
__device__ inline void dma4(const void *g, void *lds)
{
    __builtin_amdgcn_global_load_lds(g, (lds_void *)lds, 4, 0, 0);
}

template <int OFF>
__device__ inline v4i lds_b128(uint32_t addr)
{
    v4i r;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(r) : "v"(addr), "i"(OFF));
    return r;
}

__device__ inline uint32_t lds_b32(uint32_t addr)
{
    uint32_t r;
    asm volatile("ds_read_b32 %0, %1" : "=v"(r) : "v"(addr));
    return r;
}

__device__ inline uint32_t lds_u8(uint32_t addr)
{
    uint32_t r;
    asm volatile("ds_read_u8 %0, %1" : "=v"(r) : "v"(addr));
    return r;
}

// f(integral_constant<uint32_t, i>) for i = 0 .. N - 1, in order
template <int N, class F>
__device__ inline void unroll_blocks(F &f)
{
    if constexpr (N > 0) {
        unroll_blocks<N - 1>(f);
        f(std::integral_constant<uint32_t, N - 1>{});
    }
}

// Modes of the row-store kernel:
//  kBandLists:  every query keeps its k (<= 16) nearest of the curve's window,
//               with the bound shared between curves (the search for k <= 16);
//  kBandHalves: every lane keeps the 16 nearest of its half of the rows and
//               both halves are written out, no bound shared (first pass for
//               k > 16: 32 candidates per curve, the source of the threshold);
//  kBandThresh: every pair of the window at or below the query's threshold
//               key is appended to the query's buffer (second pass for k > 16).
constexpr int kBandLists = 0, kBandHalves = 1, kBandThresh = 2;

// SPLIT: the union of each group from a.split_from on (curve-major; all of
// them in a small batch, the last round's in a large one) is dealt out over
// a.split blocks; without it the block decomposition folds to one block per
// group.
template <int KR, int NW, int MODE, bool SPLIT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(KR > 10 ? 3 : 4)))
void k_band_dma(BandArgs a)
{
    constexpr int R = 16 * NW;
    constexpr int kBlockQ = NW * kMQ;
    static_assert(R % 32 == 0 && R / 16 >= 1 && NW >= 3, "tile shape");
    __shared__ BandStage<NW> st[kStages];
    __shared__ uint32_t bslot[NW][kMQ];
    __shared__ uint32_t wspan[2][NW];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, qn = lane & 31;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint32_t groups = (a.nq + kBlockQ - 1) / kBlockQ;
    // curve-major; the split blocks of a group are neighbours and take the
    // tiles of its union in turn (tile i of the middle-out order to block
    // i mod split), so each sees every wavefront busy about as often
    const uint32_t S = SPLIT ? a.split : 1u, F = SPLIT ? a.split_from : 0u;
    const uint32_t bid = blockIdx.x;
    const bool whole = bid < F;
    const uint32_t pair = whole ? bid : F + (bid - F) / S;
    const uint32_t nsplit = whole ? 1u : S, sub = whole ? 0u : (bid - F) % S;
    const uint32_t c = pair / groups, grp = pair % groups;

    const uint64_t slot = (uint64_t)grp * kBlockQ + (uint64_t)wv * kMQ + qn;
    const bool live = slot < a.nq;
    const uint32_t q = live ? a.order[(uint64_t)c * a.nq + slot] : 0;
    v4i bq[4];
    uint32_t qq = 0, sq = 0;
    {
        const uint4 *qrow = reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const uint4 v = live ? qrow[2 * s + h] : make_uint4(0, 0, 0, 0);
            qq = __builtin_amdgcn_udot4(v.x, v.x, qq, false);
            qq = __builtin_amdgcn_udot4(v.y, v.y, qq, false);
            qq = __builtin_amdgcn_udot4(v.z, v.z, qq, false);
            qq = __builtin_amdgcn_udot4(v.w, v.w, qq, false);
            sq = __builtin_amdgcn_udot4(v.x, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.y, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.z, 0x01010101u, sq, false);
            sq = __builtin_amdgcn_udot4(v.w, 0x01010101u, sq, false);
            const uint4 b = xor4(v, 0x80808080u);
            bq[s] = v4i{(int)b.x, (int)b.y, (int)b.z, (int)b.w};
        }
    }
    qq += __shfl_xor(qq, 32, 64);
    sq += __shfl_xor(sq, 32, 64);
    const int cq = (int)(qq - 254u * sq + 4161536u);
    uint32_t lo, hi;
    {
        const uint64_t w = live ? (a.d_w ? a.d_w[q] : a.w_fixed) : 0;
        const uint64_t p = live ? a.pos[(uint64_t)q * C + c] : 0;
        lo = live ? (uint32_t)(p > w ? p - w : 0) : 0xFFFFFFFFu;
        hi = live ? (uint32_t)(p + w < n ? p + w : n) : 0u;
    }
    uint32_t u0 = lo, u1 = hi;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t o0 = __shfl_xor(u0, m, 64), o1 = __shfl_xor(u1, m, 64);
        u0 = o0 < u0 ? o0 : u0;
        u1 = o1 > u1 ? o1 : u1;
    }
    u0 = __builtin_amdgcn_readfirstlane(u0);
    u1 = __builtin_amdgcn_readfirstlane(u1);
    if (lane == 0) {
        wspan[0][wv] = u0;
        wspan[1][wv] = u1;
    }
    __syncthreads();
    uint32_t U0 = 0xFFFFFFFFu, U1 = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        U0 = wspan[0][i] < U0 ? wspan[0][i] : U0;
        U1 = wspan[1][i] > U1 ? wspan[1][i] : U1;
    }
    U0 = __builtin_amdgcn_readfirstlane(U0);
    U1 = __builtin_amdgcn_readfirstlane(U1);

    uint64_t L[KR];
#pragma unroll
    for (int i = 0; i < KR; i++) L[i] = kNone;
    // bound from the other curves in the sum's terms; later reads come by
    // DMA into bslot every 8 tiles
    int ext = INT32_MAX;
    uint64_t theta = kNone;     // kBandThresh: the query's threshold key
    // the bound is shared between curves in the one-pass search, and in the
    // first pass of k <= 32 (a.tight), where it is the k-th of a curve's 32
    // candidates
    const bool shared = MODE == kBandLists || (MODE == kBandHalves && a.tight);
    if (shared) {
        const uint32_t b = live ? __hip_atomic_load(a.bound + q, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT)
                                : kEmpty;
        if (b != kEmpty) ext = (int)b - cq;
        // taken now, before any copy is in flight (waiting for it later would
        // wait for the copies too)
        asm volatile("" : "+v"(ext)::"memory");
    } else if (MODE == kBandThresh) {
        // no threshold (fewer than k distinct candidates in the first pass):
        // nothing is collected and the gather kernel answers the query
        theta = live ? a.theta[q] : kNone;
        ext = theta == kNone ? INT32_MIN : (int)(uint32_t)(theta >> 32) - cq;
        asm volatile("" : "+v"(ext)::"memory");
    }

    // tiles of R entries aligned in the list, middle of the union outwards
    const uint32_t A0 = U0 < U1 ? (U0 & ~(uint32_t)(R - 1)) : 0u;
    const uint32_t T = U0 < U1 ? (U1 - A0 + R - 1) / R : 0u;
    const uint32_t jm = T ? ((U1 - A0) / 2) / R : 0u;
    const uint32_t nleft = jm, nright = T ? T - 1 - jm : 0u;
    const uint32_t nboth = nleft < nright ? nleft : nright;
    auto tile_start = [&](uint32_t i) -> uint32_t {
        uint32_t j;
        if (i <= 2 * nboth) j = (i & 1) ? jm + (i + 1) / 2 : jm - i / 2;
        else j = nright > nleft ? jm + (i - nboth) : jm - (i - nboth);
        return A0 + j * R;
    };

    const uint8_t *rows_c = a.v.rows[c];
    const int *crow2_c = a.v.crow2[c];
    const uint32_t *rid_c = a.v.rid[c];
    const uint8_t *par_c = a.v.par[c];
    // a tile's copies: each wavefront two 1 KiB parts of the rows, and
    // wavefronts 0, 1, 2 the crow2, id and parity parts
    auto issue = [&](uint32_t j, uint32_t sj) {
        BandStage<NW> &S = st[sj];
        const uint64_t e0 = tile_start(j * nsplit + sub);
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const uint32_t m = 2 * wv + k;
            const uint32_t r = 8 * m + ((uint32_t)lane >> 3);
            const uint32_t part = ((uint32_t)lane & 7) ^ ((r >> 1) & 7);
            dma16(rows_c + (e0 + r) * kDim + part * 16, &S.rows[64 * m]);
        }
        if (wv == 0) {
            if (lane < R / 4) dma16(crow2_c + e0 + 4 * lane, &S.crow2[0]);
        } else if (wv == 1) {
            if (lane < R / 4) dma16(rid_c + e0 + 4 * lane, &S.rid[0]);
        } else if (wv == 2) {
            if (lane < R / 16) dma16(par_c + e0 + 16 * lane, &S.par[0]);
        }
    };

    // this lane's A operand parts within a 32-row block: row qn, parts 2s + h
    uint32_t aoff[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; s4++)
        aoff[s4] = (uint32_t)qn * 128 + ((uint32_t)(2 * s4 + h) ^ (((uint32_t)qn >> 1) & 7)) * 16;

    // tile i of the union, from stage si
    auto do_tile = [&](uint32_t i, uint32_t si) {
        const uint32_t t0 = tile_start(i * nsplit + sub);
        if (!(t0 < u1 && (uint64_t)t0 + R > u0)) return;       // wavefront-uniform
        {
            BandStage<NW> &S = st[si];
            const uint32_t rows_l = lds_addr(&S.rows[0]);
            const uint32_t crow_l = lds_addr(&S.crow2[0]) + 16 * h;
            const uint32_t rid_l = lds_addr(&S.rid[0]), par_l = lds_addr(&S.par[0]);

            int th = ext;
            if (MODE == kBandLists) {
                const int own = list_bound(L, cq);
                const int other = __shfl_xor(own, 32, 64);
                th = own < th ? own : th;
                th = other < th ? other : th;
            } else if (MODE == kBandHalves) {
                // the two halves' lists then hold about the curve's 16 nearest:
                // 16 distinct per curve, enough for a threshold when k is
                // small (a.tight), and fewer insertions
                const int own = list_bound(L, cq);
                th = own < th ? own : th;
                if (a.tight) {
                    const int other = __shfl_xor(own, 32, 64);
                    th = other < th ? other : th;
                }
            }
            const uint32_t rlo = lo > t0 ? std::min<uint32_t>(lo - t0, R) : 0u;
            const uint32_t rhi = hi > t0 ? std::min<uint32_t>(hi - t0, R) : 0u;
            if (!live || rlo >= rhi) th = INT32_MIN;
            int hb = th >> 1;
            int pend_h = 0;
            uint32_t pend_r = kNoRow;
            auto insert_pending = [&]() {
                uint32_t p = lds_u8(par_l + pend_r), id = lds_b32(rid_l + 4 * pend_r);
                asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(p), "+v"(id));
                const int t = 2 * pend_h + (int)p;
                const uint64_t key = ((uint64_t)(uint32_t)(t + cq) << 32) | id;
                if (MODE == kBandThresh) {
                    if (key <= theta) {
                        const uint32_t at = atomicAdd(a.cnt + q, 1u);
                        if (at < a.cap) a.buf[(uint64_t)q * a.cap + at] = key;
                    }
                } else if (key < L[KR - 1]) {
#pragma unroll
                    for (int m = KR - 1; m > 0; m--)
                        L[m] = key < L[m - 1] ? L[m - 1] : (key < L[m] ? key : L[m]);
                    L[0] = key < L[0] ? key : L[0];
                    const int b = list_bound(L, cq);
                    th = b < th ? b : th;
                    hb = th >> 1;
                }
                pend_r = kNoRow;
            };
            // this lane's A operand addresses and crow2 address in this stage
            const uint32_t ab0 = rows_l + aoff[0], ab1 = rows_l + aoff[1], ab2 = rows_l + aoff[2],
                           ab3 = rows_l + aoff[3];
            // one 32-row block; RB is a compile-time constant, so that the block's
            // LDS offsets are immediates
            auto block32 = [&](auto rbc) {
                constexpr uint32_t RB = decltype(rbc)::value;
                v4i c0 = lds_b128<RB * 128>(crow_l), c1 = lds_b128<RB * 128 + 32>(crow_l),
                    c2 = lds_b128<RB * 128 + 64>(crow_l), c3 = lds_b128<RB * 128 + 96>(crow_l);
                v4i a0 = lds_b128<RB * 4096>(ab0), a1 = lds_b128<RB * 4096>(ab1),
                    a2 = lds_b128<RB * 4096>(ab2), a3 = lds_b128<RB * 4096>(ab3);
                asm volatile("s_waitcnt lgkmcnt(3)" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(a0));
                v16i acc = v16i{c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w,
                                c2.x, c2.y, c2.z, c2.w, c3.x, c3.y, c3.z, c3.w};
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, bq[0], acc, 0, 0, 0);
                asm volatile("s_waitcnt lgkmcnt(2)" : "+v"(a1));
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, bq[1], acc, 0, 0, 0);
                asm volatile("s_waitcnt lgkmcnt(1)" : "+v"(a2));
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, bq[2], acc, 0, 0, 0);
                asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(a3));
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a3, bq[3], acc, 0, 0, 0);
                const int m0 = std::min(std::min(acc[0], acc[1]), acc[2]);
                const int m1 = std::min(std::min(acc[3], acc[4]), acc[5]);
                const int m2 = std::min(std::min(acc[6], acc[7]), acc[8]);
                const int m3 = std::min(std::min(acc[9], acc[10]), acc[11]);
                const int m4 = std::min(std::min(acc[12], acc[13]), acc[14]);
                const int mm = std::min(std::min(std::min(m0, m1), m2),
                                        std::min(std::min(m3, m4), acc[15]));
                if (mm > hb) return;        // rare once the lists are full
                int hm[4];
#pragma unroll
                for (int g = 0; g < 4; g++)
                    hm[g] = std::min(std::min(acc[4 * g], acc[4 * g + 1]),
                                     std::min(acc[4 * g + 2], acc[4 * g + 3]));
#pragma unroll
                for (int g = 0; g < 4; g++) {
                    const uint32_t r0 = RB * 32 + 8 * g + 4 * h;
                    if (hm[g] <= hb) {
#pragma unroll
                        for (int j = 0; j < 4; j++) {
                            if (acc[4 * g + j] <= hb && r0 + j - rlo < rhi - rlo) {
                                if (pend_r != kNoRow) insert_pending();
                                pend_h = acc[4 * g + j];
                                pend_r = r0 + j;
                            }
                        }
                    }
                }
            };
            unroll_blocks<R / 32>(block32);
            if (pend_r != kNoRow) insert_pending();
        }
    };

    // Groups of kTPB tiles in ping-pong stages: group g sits in stages
    // (g & 1) * kTPB + j.  Group g + 1 is issued right after group g's
    // barrier, into the stages group g - 1 used, so one wait (everything
    // issued so far) and one barrier serve kTPB tiles.  The bound copied
    // with group g + 1 (every 4 groups) is read with it.
    const uint32_t TS = T > sub ? (T - 1 - sub) / nsplit + 1 : 0u;   // this block's tiles
    const uint32_t NG = (TS + kTPB - 1) / kTPB;
    auto issue_group = [&](uint32_t g) {
#pragma unroll
        for (int j = 0; j < kTPB; j++) {
            const uint32_t t = g * kTPB + j;
            if (t < TS) issue(t, (g & 1) * kTPB + j);
        }
    };
    if (NG > 0) issue_group(0);
    for (uint32_t g = 0; g < NG; g++) {
        __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
        __builtin_amdgcn_s_barrier();
        if (shared && g >= 1 && ((g - 1) & 3) == 3) {
            uint32_t b = lds_b32(lds_addr(&bslot[wv][qn]));
            asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(b));
            if (live && b != kEmpty) {
                const int e = (int)b - cq;
                ext = e < ext ? e : ext;
            }
        }
        if (g + 1 < NG) {
            if (shared && (g & 3) == 3 && lane < kMQ)
                dma4(a.bound + q, &bslot[wv][0]);
            asm volatile("" ::: "memory");
            issue_group(g + 1);
        }
#pragma unroll
        for (int j = 0; j < kTPB; j++) {
            const uint32_t t = g * kTPB + j;
            if (t < TS) do_tile(t, (g & 1) * kTPB + j);
        }
    }

    if (MODE == kBandThresh) return;
    if (MODE == kBandHalves) {
        // both halves' lists: entries [16 h, 16 h + 16) of the query's 32 for curve c
        if (live) {
            uint64_t *out = a.partial + (((uint64_t)q * C + c) * a.pstride + sub) * (2 * kBandK) +
                            kBandK * h;
#pragma unroll
            for (int i = 0; i < KR; i++) out[i] = L[i];
        }
        if (a.tight) {
            // the k-th of the two halves' lists (32 distinct ids of the
            // union, in this block's rows of the curve): a key's rank is its
            // index plus the other list's keys below it.  These 32 stay among
            // the threshold's candidates, so the threshold exists and is at
            // or below this bound; and the union's k nearest are at or below it
            uint64_t M[KR];
#pragma unroll
            for (int i = 0; i < KR; i++) M[i] = shfl_xor_u64(L[i], 32);
            uint64_t kth = kNone;
#pragma unroll
            for (int i = 0; i < KR; i++) {
                uint32_t below_l = 0, below_m = 0;
#pragma unroll
                for (int j = 0; j < KR; j++) {
                    below_l += M[j] < L[i] ? 1u : 0u;
                    below_m += L[j] < M[i] ? 1u : 0u;
                }
                if (i + below_l == a.k - 1 && L[i] != kNone) kth = L[i];
                if (i + below_m == a.k - 1 && M[i] != kNone) kth = M[i];
            }
            if (live && h == 0 && kth != kNone) atomicMin(a.bound + q, (uint32_t)(kth >> 32));
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < KR; i++) {
        const uint64_t o = shfl_xor_u64(L[i], 32);
        if (h == 0 && o < L[KR - 1]) {
#pragma unroll
            for (int j = KR - 1; j > 0; j--)
                L[j] = o < L[j - 1] ? L[j - 1] : (o < L[j] ? o : L[j]);
            L[0] = o < L[0] ? o : L[0];
        }
    }
    if (live && h == 0) {
        // a dealt-out group of a large batch's last round: its own lists,
        // merged by k_band_tail_merge
        uint64_t *out = (SPLIT && a.tail && !whole)
            ? a.tail + ((uint64_t)((pair - F) * S + sub) * kBlockQ + (slot - (uint64_t)grp * kBlockQ)) * a.k
            : a.partial + (((uint64_t)q * C + c) * a.pstride + sub) * a.k;
        uint64_t kth = kNone;
#pragma unroll
        for (int i = 0; i < KR; i++) {
            if ((uint32_t)i < a.k) out[i] = L[i];
            if ((uint32_t)i == a.k - 1) kth = L[i];
        }
        if (kth != kNone) atomicMin(a.bound + q, (uint32_t)(kth >> 32));
    }
}

// One wavefront per query: the curves' lists, repeats dropped, k nearest.
// Each curve's list is ascending with distinct ids, so the result is a merge
// of their heads: the wavefront copies the C lists into LDS (one coalesced
// load), then lane c < C follows the head of list c; per output the smallest
// head is taken and every lane holding that key advances (a repeated id has
// the same key in every curve, so it is taken once).
constexpr int kMergeWaves = 4;
__global__ __launch_bounds__(64 * kMergeWaves) void k_band_merge(BandArgs a)
{
    __shared__ uint64_t lists[kMergeWaves][kMaxCurves * kMaxSplit * kBandK];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t q = blockIdx.x * kMergeWaves + wv;
    if (q >= a.nq) return;                 // the whole wavefront; no barrier follows
    const uint32_t C = a.v.curves * a.pstride, k = a.k;   // lists: per curve and split block
    const uint32_t nkeys = C * k;
    const uint64_t *src = a.partial + (uint64_t)q * nkeys;
    uint64_t *ls = lists[wv];
    for (uint32_t i = lane; i < nkeys; i += 64) ls[i] = src[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool mine = (uint32_t)lane < C;
    uint32_t hc = 0;
    uint64_t head = mine ? ls[lane * k] : kNone;
    const uint64_t o = (uint64_t)q * k;
    for (uint32_t j = 0; j < k; j++) {
        uint64_t m = head;                 // minimum over lanes 0..15 (C <= 16)
#pragma unroll
        for (int x = 1; x < kMaxCurves * (int)kMaxSplit; x <<= 1) {
            const uint64_t y = shfl_xor_u64(m, x);
            m = y < m ? y : m;
        }
        if (lane == 0) {
            a.out_ids[o + j] = (uint32_t)m;
            a.out_dists[o + j] = (uint32_t)(m >> 32);
        }
        if (mine && head == m && m != kNone) {
            hc++;
            head = hc < k ? ls[lane * k + hc] : kNone;
        }
    }
}

// A large batch's last round, after the main kernel: one thread per query
// slot of a dealt-out group merges the group's split lists for that query
// into its list for the curve.  The split blocks took disjoint tiles of the
// curve's union, so the lists hold distinct ids and the merge keeps the k
// smallest heads.
__global__ __launch_bounds__(256) void k_band_tail_merge(BandArgs a, uint32_t block_q,
                                                         uint64_t nslots)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const uint32_t S = a.split, k = a.k, C = a.v.curves;
    const uint32_t groups = (a.nq + block_q - 1) / block_q;
    const uint32_t tp = (uint32_t)(t / block_q), i = (uint32_t)(t % block_q);
    const uint32_t pair = a.split_from + tp, c = pair / groups, grp = pair % groups;
    const uint64_t slot = (uint64_t)grp * block_q + i;
    if (slot >= a.nq) return;
    const uint32_t q = a.order[(uint64_t)c * a.nq + slot];
    const uint64_t *src = a.tail + ((uint64_t)tp * S * block_q + i) * k;
    const uint64_t sstep = (uint64_t)block_q * k;      // from one split list to the next
    uint32_t hd[kMaxSplit];
    uint64_t key[kMaxSplit];
#pragma unroll
    for (uint32_t s = 0; s < kMaxSplit; s++) {
        hd[s] = 0;
        key[s] = s < S ? src[s * sstep] : kNone;
    }
    uint64_t *out = a.partial + ((uint64_t)q * C + c) * k;
    for (uint32_t j = 0; j < k; j++) {
        uint64_t m = key[0];
#pragma unroll
        for (uint32_t s = 1; s < kMaxSplit; s++) m = key[s] < m ? key[s] : m;
        out[j] = m;
#pragma unroll
        for (uint32_t s = 0; s < kMaxSplit; s++) {
            if (key[s] == m && m != kNone) {
                hd[s]++;
                key[s] = hd[s] < k ? src[s * sstep + hd[s]] : kNone;
            }
        }
    }
}

// k > 16, between the passes: one wavefront per query takes the k nearest
// distinct keys among the first pass's 32 C candidates (all members of the
// query's union), and the k-th of them is the threshold: the union's k
// nearest are all at or below it.  Fewer than k distinct candidates leave no
// threshold (kNone).  Clears the query's counter and fallback flag.
__global__ __launch_bounds__(64) void k_band_theta(BandArgs a)
{
    __shared__ TopKShared sh;
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t m = a.v.curves * a.pstride * 2 * kBandK;
    const uint64_t *src = a.partial + (uint64_t)q * m;
    WaveTopK<0> tk;
    tk.init(a.k, &sh, lane);
    for (uint32_t i0 = 0; i0 < m; i0 += 64) {
        const uint32_t i = i0 + (uint32_t)lane;
        tk.push(i < m ? src[i] : kNone, lane);
    }
    tk.finish(lane, [&](uint32_t j, uint64_t key) {
        if (j == a.k - 1) a.theta[q] = key;
    });
    if (lane == 0) {
        a.cnt[q] = 0;
        a.redo[q] = 0;
    }
}

// k > 16, after the second pass: one wavefront per query keeps the k nearest
// distinct keys of the pairs collected at or below the threshold (a key met
// in several curves' windows is taken once).  They are the query's result:
// every member of the union at or below the threshold was collected, and the
// union's k nearest are among them.  A query without a threshold or whose
// pairs overflowed the buffer is flagged for the gather kernel.
__global__ __launch_bounds__(64) void k_band_select(BandArgs a)
{
    __shared__ TopKShared sh;
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t cnt = a.cnt[q];
    if (a.theta[q] == kNone || cnt > a.cap) {        // the whole wavefront
        if (lane == 0) a.redo[q] = 1;
        return;
    }
    const uint64_t *src = a.buf + (uint64_t)q * a.cap;
    WaveTopK<0> tk;
    tk.init(a.k, &sh, lane);
    for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
        const uint32_t i = i0 + (uint32_t)lane;
        tk.push(i < cnt ? src[i] : kNone, lane);
    }
    const uint64_t o = (uint64_t)q * a.k;
    tk.finish(lane, [&](uint32_t j, uint64_t key) {
        a.out_ids[o + j] = (uint32_t)key;
        a.out_dists[o + j] = (uint32_t)(key >> 32);
    });
}

// Row store of curve c: 8 lanes per list entry, each 16 bytes of the row
// (127 - x) and its part of crow, reduced over the 8 lanes.  Entries from n
// to the padded length get zero rows and crow, and no id.
__global__ __launch_bounds__(256) void k_rowstore(IndexView v, uint32_t c, uint64_t npad,
                                                  uint8_t *rows, int *crow2, uint8_t *par,
                                                  uint32_t *rid)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t e = t >> 3;
    const uint32_t part = (uint32_t)t & 7;
    const bool valid = e < v.n;
    const uint32_t id = valid ? v.ids[c][e] : 0u;
    const uint4 x = valid ? reinterpret_cast<const uint4 *>(v.db + (uint64_t)id * kDim)[part]
                          : make_uint4(0x7F7F7F7Fu, 0x7F7F7F7Fu, 0x7F7F7F7Fu, 0x7F7F7F7Fu);
    uint32_t xx = __builtin_amdgcn_udot4(x.x, x.x, 0u, false);
    xx = __builtin_amdgcn_udot4(x.y, x.y, xx, false);
    xx = __builtin_amdgcn_udot4(x.z, x.z, xx, false);
    xx = __builtin_amdgcn_udot4(x.w, x.w, xx, false);
    uint32_t sx = __builtin_amdgcn_udot4(x.x, 0x01010101u, 0u, false);
    sx = __builtin_amdgcn_udot4(x.y, 0x01010101u, sx, false);
    sx = __builtin_amdgcn_udot4(x.z, 0x01010101u, sx, false);
    sx = __builtin_amdgcn_udot4(x.w, 0x01010101u, sx, false);
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        xx += __shfl_xor(xx, m, 64);
        sx += __shfl_xor(sx, m, 64);
    }
    if (e < npad) {
        reinterpret_cast<uint4 *>(rows + e * kDim)[part] = xor4(x, 0x7F7F7F7Fu);
        if (part == 0) {
            const int crow = valid ? (int)(xx - 256u * sx) : 0;
            crow2[e] = crow >> 1;
            par[e] = (uint8_t)(crow & 1);
            rid[e] = valid ? id : kEmpty;
        }
    }
}

constexpr uint64_t kRowPad = 256;   // row store entries per curve: a multiple of this

struct RowStoreLayout {
    uint64_t npad;
    size_t rows_off[kMaxCurves], crow_off[kMaxCurves], par_off[kMaxCurves],
        rid_off[kMaxCurves], total;
};

static RowStoreLayout rowstore_layout(uint32_t curves, uint64_t n)
{
    RowStoreLayout L{};
    L.npad = (n + kRowPad - 1) / kRowPad * kRowPad;
    size_t off = 0;
    for (uint32_t c = 0; c < curves; c++) {
        L.rows_off[c] = off;
        off = align256(off + (size_t)kDim * L.npad);
        L.crow_off[c] = off;
        off = align256(off + sizeof(int) * L.npad);
        L.par_off[c] = off;
        off = align256(off + L.npad);
        L.rid_off[c] = off;
        off = align256(off + sizeof(uint32_t) * L.npad);
    }
    L.total = off;
    return L;
}

size_t band_scratch_bytes(uint32_t curves, uint64_t n, uint32_t nq, uint32_t k_max)
{
    return band_layout(curves, n, nq, k_max).total;
}

template <int NW, bool SPLIT>
static void launch_dma_lists(uint32_t k, dim3 grid, dim3 block, const BandArgs &a, hipStream_t st)
{
    if (k == 1) hipLaunchKernelGGL((k_band_dma<1, NW, kBandLists, SPLIT>), grid, block, 0, st, a);
    else if (k <= 4)
        hipLaunchKernelGGL((k_band_dma<4, NW, kBandLists, SPLIT>), grid, block, 0, st, a);
    else if (k <= 10)
        hipLaunchKernelGGL((k_band_dma<10, NW, kBandLists, SPLIT>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_band_dma<kBandK, NW, kBandLists, SPLIT>), grid, block, 0, st, a);
}

// Blocks of the row-store kernel for k that are resident on the device at
// once (compute units x blocks per unit); 0 if the runtime cannot say.  The
// device queries run once per process, device and list length (a racing
// repeat is harmless).
template <int NW>
static uint64_t band_resident(uint32_t k)
{
    constexpr int kMaxDev = 64;
    static uint64_t cache[kMaxDev][4];
    const int kv = k == 1 ? 0 : k <= 4 ? 1 : k <= 10 ? 2 : 3;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
    if (cache[dev][kv]) return cache[dev][kv];
    const void *f = kv == 0   ? reinterpret_cast<const void *>(&k_band_dma<1, NW, kBandLists, true>)
                    : kv == 1 ? reinterpret_cast<const void *>(&k_band_dma<4, NW, kBandLists, true>)
                    : kv == 2 ? reinterpret_cast<const void *>(&k_band_dma<10, NW, kBandLists, true>)
                              : reinterpret_cast<const void *>(&k_band_dma<kBandK, NW, kBandLists, true>);
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 64 * NW, 0) != hipSuccess)
        return 0;
    cache[dev][kv] = (uint64_t)cus * (uint64_t)per;
    return cache[dev][kv];
}

template <int NW>
static void launch_band(const IndexView &v, uint32_t k, uint32_t nq, const BandArgs &a,
                        hipStream_t st)
{
    const uint32_t blocks = (uint32_t)(((uint64_t)nq + NW * kMQ - 1) / (NW * kMQ)) * v.curves;
    const dim3 block(64 * NW);
    if (v.rows[0]) {
        const dim3 grid(a.split_from + (blocks - a.split_from) * a.split);
        if (a.split > 1) launch_dma_lists<NW, true>(k, grid, block, a, st);
        else launch_dma_lists<NW, false>(k, grid, block, a, st);
    } else {
        const dim3 grid(blocks);
        if (k == 1) hipLaunchKernelGGL((k_band<1, NW>), grid, block, 0, st, a);
        else if (k <= 4) hipLaunchKernelGGL((k_band<4, NW>), grid, block, 0, st, a);
        else if (k <= 10) hipLaunchKernelGGL((k_band<10, NW>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_band<kBandK, NW>), grid, block, 0, st, a);
    }
}

// The two passes of k > 16 (row store only): 16 nearest per lane half, then
// every pair at or below the threshold.
template <int NW>
static void launch_band_two(const IndexView &v, uint32_t nq, const BandArgs &a, int mode,
                            hipStream_t st)
{
    const uint32_t blocks = (uint32_t)(((uint64_t)nq + NW * kMQ - 1) / (NW * kMQ)) * v.curves;
    const dim3 grid(blocks * a.split), block(64 * NW);
    const bool sp = a.split > 1;
    if (mode == kBandHalves && sp)
        hipLaunchKernelGGL((k_band_dma<kBandK, NW, kBandHalves, true>), grid, block, 0, st, a);
    else if (mode == kBandHalves)
        hipLaunchKernelGGL((k_band_dma<kBandK, NW, kBandHalves, false>), grid, block, 0, st, a);
    else if (sp)
        hipLaunchKernelGGL((k_band_dma<1, NW, kBandThresh, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_band_dma<1, NW, kBandThresh, false>), grid, block, 0, st, a);
}

uint64_t band_blocks(uint32_t curves, uint32_t nq, uint32_t w)
{
    const uint64_t q = w < kBandWideW ? 4 * kMQ : 8 * kMQ;
    return ((uint64_t)nq + q - 1) / q * curves;
}

uint64_t band_split_blocks(uint32_t curves, uint32_t nq, uint32_t w, uint32_t k)
{
    return band_blocks(curves, nq, w) * band_split(curves, nq, band_block_q(w), k);
}

// Runs the banded search with the query keys already in d_scratch.  w_fixed
// is the window, or with per-query windows a typical one (the block size
// follows it).  ev_begin / ev_end (may be null) are recorded around the
// banded kernel.
hc_status band_search(const IndexView &v, const uint8_t *d_queries, uint32_t nq, uint32_t k,
                      uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_out_ids,
                      uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                      hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end)
{
    const bool two = k > (uint32_t)kBandK;
    if (k < 1 || k > kBandKMax || (two && !v.rows[0])) return HC_ERR_UNSUPPORTED;
    const BandLayout L = band_layout(v.curves, v.n, nq, k);
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
    a.bound = (uint32_t *)(s + L.bound);
    a.out_ids = d_out_ids;
    a.out_dists = d_out_dists;
    if (two) {
        a.theta = (uint64_t *)(s + L.theta);
        a.cnt = (uint32_t *)(s + L.cnt);
        a.redo = (uint32_t *)(s + L.redo);
        a.buf = (uint64_t *)(s + L.buf);
        a.cap = kBandCap;
        a.tight = k <= kBandTightK;
    }
    // a small batch makes few groups; over the row store each group's union
    // is then dealt out over up to kMaxSplit blocks, so that the grid fills
    // the device (band_split)
    // A large batch ends with a partial round of blocks; when it is at most
    // half a round, its groups are dealt out the same way (on the blocks that
    // would stand idle) and their lists merged after the main kernel.
    const uint32_t bq = band_block_q(w_fixed);
    a.split = 1;
    a.split_from = 0;
    a.pstride = 1;
    a.tail = nullptr;
    uint64_t tail_slots = 0;
    if (v.rows[0]) {
        const uint32_t sp = band_split(v.curves, nq, bq, k);
        const uint64_t P = ((uint64_t)nq + bq - 1) / bq * v.curves;
        const uint64_t res = sp > 1 || two ? 0
                             : bq == 4 * kMQ ? band_resident<4>(k) : band_resident<8>(k);
        const uint64_t Lt = res ? P % res : 0;
        if (sp > 1) {
            a.split = sp;
            a.pstride = sp;
        } else if (P >= res && Lt > 0 && 2 * Lt <= res &&
                   Lt * bq <= std::min<uint64_t>((uint64_t)nq * v.curves, kTailQ)) {
            a.split = (uint32_t)std::min<uint64_t>(kMaxSplit, res / Lt);
            a.split_from = (uint32_t)(P - Lt);
            a.tail = (uint64_t *)(s + L.tail);
            tail_slots = Lt * bq;
        }
    }
    const uint64_t nc = (uint64_t)v.curves * L.nbuckets;
    hipLaunchKernelGGL(k_band_fill, dim3((uint32_t)std::min<uint64_t>(4096, (nc + 255) / 256)),
                       dim3(256), 0, st, a.counts, nc, 0u);
    hipLaunchKernelGGL(k_band_fill, dim3((uint32_t)std::min<uint64_t>(4096, (nq + 255) / 256)),
                       dim3(256), 0, st, a.bound, (uint64_t)nq, kEmpty);
    hipLaunchKernelGGL(k_band_place, dim3(nq), dim3(64), 0, st, a);
    // each curve's buckets count every query once: one block per curve
    hipLaunchKernelGGL(k_scan_excl_seg, dim3(v.curves), dim3(kScanThreads), 0, st, a.counts,
                       (uint64_t)L.nbuckets, nq);
    const uint64_t nt = (uint64_t)nq * v.curves;
    hipLaunchKernelGGL(k_band_scatter, dim3((uint32_t)((nt + 255) / 256)), dim3(256), 0, st, a);
    hc_status rs = record_if(ev_begin, st);
    if (rs != HC_OK) return rs;
    if (two) {
        // first pass, threshold, second pass; then the selection and, for
        // the queries it flags, the gather kernel
        if (w_fixed < kBandWideW) launch_band_two<4>(v, nq, a, kBandHalves, st);
        else launch_band_two<8>(v, nq, a, kBandHalves, st);
        hipLaunchKernelGGL(k_band_theta, dim3(nq), dim3(64), 0, st, a);
        if (w_fixed < kBandWideW) launch_band_two<4>(v, nq, a, kBandThresh, st);
        else launch_band_two<8>(v, nq, a, kBandThresh, st);
        rs = record_if(ev_end, st);
        if (rs != HC_OK) return rs;
        hipLaunchKernelGGL(k_band_select, dim3(nq), dim3(64), 0, st, a);
        rs = last_hip();
        if (rs != HC_OK) return rs;
        return gather_search_only(v, d_queries, a.qkeys, nq, k, w_fixed, d_w, a.redo,
                                  d_out_ids, d_out_dists, st);
    }
    if (w_fixed < kBandWideW) launch_band<4>(v, k, nq, a, st);
    else launch_band<8>(v, k, nq, a, st);
    rs = record_if(ev_end, st);
    if (rs != HC_OK) return rs;
    if (tail_slots)
        hipLaunchKernelGGL(k_band_tail_merge, dim3((uint32_t)((tail_slots + 255) / 256)),
                           dim3(256), 0, st, a, bq, tail_slots);
    hipLaunchKernelGGL(k_band_merge, dim3((nq + kMergeWaves - 1) / kMergeWaves),
                       dim3(64 * kMergeWaves), 0, st, a);
    return last_hip();
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_rowstore_bytes(const hc_index *idx, size_t *bytes)
{
    if (!idx || !bytes) return HC_ERR_INVALID;
    *bytes = rowstore_layout(idx->v.curves, idx->v.n).total;
    return HC_OK;
}

hc_status hc_rowstore_build(hc_index *idx, void *d_rows, size_t bytes, hc_stream stream)
{
    if (!idx || !d_rows || ((uintptr_t)d_rows & 255)) return HC_ERR_INVALID;
    const RowStoreLayout L = rowstore_layout(idx->v.curves, idx->v.n);
    if (bytes < L.total) return HC_ERR_SIZE;
    const uint64_t threads = L.npad * 8;
    uint8_t *base = (uint8_t *)d_rows;
    for (uint32_t c = 0; c < idx->v.curves; c++) {
        hipLaunchKernelGGL(k_rowstore, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0,
                           (hipStream_t)stream, idx->v, c, L.npad, base + L.rows_off[c],
                           (int *)(base + L.crow_off[c]), base + L.par_off[c],
                           (uint32_t *)(base + L.rid_off[c]));
    }
    const hc_status st = last_hip();
    if (st != HC_OK) return st;
    for (uint32_t c = 0; c < idx->v.curves; c++) {
        idx->v.rows[c] = base + L.rows_off[c];
        idx->v.crow2[c] = (const int *)(base + L.crow_off[c]);
        idx->v.par[c] = base + L.par_off[c];
        idx->v.rid[c] = (const uint32_t *)(base + L.rid_off[c]);
    }
    return HC_OK;
}

hc_status hc_rowstore_detach(hc_index *idx)
{
    if (!idx) return HC_ERR_INVALID;
    for (uint32_t c = 0; c < kMaxCurves; c++) {
        idx->v.rows[c] = nullptr;
        idx->v.crow2[c] = nullptr;
        idx->v.par[c] = nullptr;
        idx->v.rid[c] = nullptr;
    }
    return HC_OK;
}

}  // extern "C"
