// Device helpers shared by the search and learned-depth kernels (gfx950).
#pragma once

#include "hc_internal.h"

namespace hc {

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

__device__ inline uint64_t readlane_u64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
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

// Number of keys below the query key in each curve c < C, for the curves
// c = first + j * step (j < CPW) handled by the calling wave.  Wave-uniform
// control flow; cnt[j] is the position of curve first + j * step.
// The table's upper levels, down to level 2 (every 4096th key), are read 64
// keys wide (1 KiB per curve, cache hits); the last four steps, through every
// 512th key, level 1, every 8th key and the keys, read 8 keys (128 B) per
// curve, lane 8j + r holding key r of curve j's block: one load serves every
// curve, and the bytes from beyond the cache drop from 2 KiB to 512 B per
// curve.
// Every load is issued unconditionally from an address inside the table
// (entry 0 of curve 0 standing in for slots that do not exist) and masked
// afterwards, so that the loads of all curves at one level are in flight
// together: a level costs one memory latency, not one per curve.
// Ties the 8 loaded keys together: every load is issued before the first of
// them is compared (the compiler would otherwise load, wait and compare one
// curve at a time).
template <int CPW>
__device__ inline void keys_landed(Key (&kk)[CPW])
{
    if constexpr (CPW == 8) {
        asm volatile(""
                     : "+v"(kk[0].hi), "+v"(kk[0].lo), "+v"(kk[1].hi), "+v"(kk[1].lo),
                       "+v"(kk[2].hi), "+v"(kk[2].lo), "+v"(kk[3].hi), "+v"(kk[3].lo),
                       "+v"(kk[4].hi), "+v"(kk[4].lo), "+v"(kk[5].hi), "+v"(kk[5].lo),
                       "+v"(kk[6].hi), "+v"(kk[6].lo), "+v"(kk[7].hi), "+v"(kk[7].lo));
    }
}

// a < b on 128-bit keys without short-circuit control flow
__device__ inline bool key_less_nb(const Key &a, const Key &b)
{
    return (a.hi < b.hi) | ((a.hi == b.hi) & (a.lo < b.lo));
}

template <int CPW>
__device__ inline void locate(const IndexView &v, const Key *qk_row, uint32_t first,
                              uint32_t step, int lane, uint64_t (&cnt)[CPW])
{
    const uint32_t C = v.curves;
    const uint32_t D = v.levels;
    Key qk[CPW];
    bool on[CPW];
    uint32_t cc[CPW];
#pragma unroll
    for (int j = 0; j < CPW; j++) {
        const uint32_t c = first + j * step;
        on[j] = c < C;
        cc[j] = on[j] ? c : 0u;
        qk[j] = qk_row[cc[j]];
    }
    {   // top table: at most 64 entries
        Key kk[CPW];
        const bool valid = (uint64_t)lane < v.len[D];
        const uint32_t li = valid ? (uint32_t)lane : 0u;
#pragma unroll
        for (int j = 0; j < CPW; j++) kk[j] = v.lvl[cc[j]][D][li];
        keys_landed(kk);
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const bool less = on[j] & valid & key_less_nb(kk[j], qk[j]);
            cnt[j] = (uint64_t)__popcll(__ballot(less));
        }
    }
    // 64 keys wide down to level 2 (its cnt), or to the top table
    for (int L = (int)D; L >= 3; L--) {
        // cnt = entries of level L below qkey, so the answer at level L-1 lies in
        // the 64 entries from 64*(cnt-1) (entry 64*cnt is >= qkey); cnt = 0
        // means every key is >= qkey.
        Key kk[CPW];
        uint64_t base[CPW];
        bool ok[CPW];
        const uint64_t len = v.len[L - 1];
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            base[j] = cnt[j] ? (cnt[j] - 1) * kFan : 0;
            const uint64_t idx = base[j] + lane;
            ok[j] = on[j] & (cnt[j] != 0) & (idx < len);
            kk[j] = v.lvl[cc[j]][L - 1][ok[j] ? idx : 0];
        }
        keys_landed(kk);
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const bool less = ok[j] & key_less_nb(kk[j], qk[j]);
            const uint64_t m = __ballot(less);
            cnt[j] = cnt[j] ? base[j] + (uint64_t)__popcll(m) : 0;
        }
    }
    if (D == 0) return;   // the top table was the list itself
    // Then 8 keys wide, lane 8j + r on key r of curve j's block: from level 2
    // through every 512th key, level 1 and every 8th key to the keys (from
    // level 1 when it is the top table).  The same rule: c entries of the
    // coarser level below the key put the answer in the 8 entries from
    // 8 (c - 1) of the finer one.
    const int jl = lane >> 3, r = lane & 7;
    uint64_t c = 0;
    Key mq = qk[0];
    const Key *f2 = v.sub2[cc[0]], *f1 = v.lvl[cc[0]][1];
    const Key *f0 = v.sub[cc[0]], *fk = v.lvl[cc[0]][0];
    bool lon = false;
#pragma unroll
    for (int j = 0; j < CPW; j++) {
        if (jl == j) {
            c = cnt[j];
            mq = qk[j];
            f2 = v.sub2[cc[j]];
            f1 = v.lvl[cc[j]][1];
            f0 = v.sub[cc[j]];
            fk = v.lvl[cc[j]][0];
            lon = on[j];
        }
    }
    auto step8 = [&](const Key *fine, uint64_t len) {
        const uint64_t base = c ? (c - 1) * kSub : 0;
        const bool ok = lon & (c != 0) & (base + r < len);
        const Key k = fine[ok ? base + r : 0];
        const uint64_t m = __ballot(ok & key_less_nb(k, mq));
        c = c ? base + (uint64_t)__popcll((m >> (8 * jl)) & 0xFFull) : 0;
    };
    if (D >= 2) {
        step8(f2, v.len_sub2);
        step8(f1, v.len[1]);
    }
    step8(f0, v.len_sub);
    step8(fk, v.n);
#pragma unroll
    for (int j = 0; j < CPW; j++) cnt[j] = readlane_u64(c, 8 * j);
}

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

constexpr int kBuf = 512;    // LDS buffer of the k > 16 top-k (entries, a power of two)

// LDS of one wavefront's top-k for k > 16.
struct TopKShared {
    uint64_t buf[kBuf];
    uint64_t run[HC_K_MAX];
    uint64_t out[HC_K_MAX];
};

// The k smallest distinct packed keys (dist << 32 | id) pushed by a wavefront,
// 64 keys (one per lane) per push.
//  KR > 0: every lane keeps an ascending register list of KR keys that refuses
//          a key it holds; k <= KR.
//  KR = 0: keys below the current k-th distinct key collect in an LDS buffer
//          that is bitonic-sorted and merged into the running list when full.
template <int KR>
struct WaveTopK {
    static constexpr int NL = KR > 0 ? KR : 1;
    uint64_t L[NL];
    uint32_t k, nbuf;
    uint64_t tau;
    TopKShared *sh;

    __device__ void init(uint32_t k_, TopKShared *sh_, int lane)
    {
        k = k_;
        sh = sh_;
        nbuf = 0;
        tau = kNone;
#pragma unroll
        for (int i = 0; i < NL; i++) L[i] = kNone;
        if (KR == 0) {
            for (uint32_t i = lane; i < k; i += 64) sh->run[i] = kNone;
            __syncthreads();
        }
    }

    // Number of entries of the ascending array a[0, n) below x (LDS).
    static __device__ uint32_t below(const uint64_t *a, uint32_t n, uint64_t x)
    {
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    }

    // Wave-collective (the block is this one wavefront).  The buffer is sorted
    // (bitonic, over the next power of two above its fill), its repeats and the
    // keys already in the running list are dropped, and the two ascending lists
    // are merged by rank: a key's place in the result is its index plus the
    // number of keys of the other list below it.
    __device__ void flush(int lane)
    {
        uint32_t sz = 2;
        while (sz < nbuf) sz <<= 1;
        __syncthreads();
        for (uint32_t i = nbuf + lane; i < sz; i += 64) sh->buf[i] = kNone;
        __syncthreads();
        for (uint32_t size = 2; size <= sz; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t i = lane; i < sz / 2; i += 64) {
                    const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
                    const uint32_t hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t x0 = sh->buf[lo], x1 = sh->buf[hi];
                    if ((x0 > x1) == up) {
                        sh->buf[lo] = x1;
                        sh->buf[hi] = x0;
                    }
                }
                __syncthreads();
            }
        }
        // valid entries of the running list (ascending, distinct, kNone after)
        const uint32_t nr = below(sh->run, k, kNone);
        // compact the buffer in place to its distinct keys not in the list; a
        // round reads all of its 64 entries before any is written, and carries
        // its last original entry to the next round
        uint32_t nb2 = 0;
        uint64_t prev_last = kNone;
        for (uint32_t base = 0; base < nbuf; base += 64) {
            const uint32_t i = base + lane;
            const uint64_t x = i < nbuf ? sh->buf[i] : kNone;
            uint64_t prev = i > base ? sh->buf[i - 1] : prev_last;
            const bool first = i == 0 || prev != x;
            const uint32_t r = below(sh->run, nr, x);
            const bool in_run = r < nr && sh->run[r] == x;
            const bool keep = i < nbuf && x != kNone && first && !in_run;
            prev_last = __shfl(x, 63, 64);
            const uint64_t m = __ballot(keep);
            __syncthreads();
            if (keep) sh->buf[nb2 + lanes_below64(m)] = x;
            nb2 += (uint32_t)__popcll(m);
            __syncthreads();
        }
        for (uint32_t j = lane; j < nr; j += 64) {
            const uint64_t x = sh->run[j];
            const uint32_t r = j + below(sh->buf, nb2, x);
            if (r < k) sh->out[r] = x;
        }
        for (uint32_t i = lane; i < nb2; i += 64) {
            const uint64_t x = sh->buf[i];
            const uint32_t r = i + below(sh->run, nr, x);
            if (r < k) sh->out[r] = x;
        }
        for (uint32_t o = nr + nb2 + lane; o < k; o += 64) sh->out[o] = kNone;
        __syncthreads();
        for (uint32_t i = lane; i < k; i += 64) sh->run[i] = sh->out[i];
        __syncthreads();
        tau = sh->run[k - 1];
        nbuf = 0;
    }

    // wave-collective
    __device__ void push(uint64_t key, int lane)
    {
        if constexpr (KR > 0) {
            insert_distinct<NL>(L, key);
        } else {
            const bool pass = key < tau;
            const uint64_t m = __ballot(pass);
            if (pass) sh->buf[nbuf + lanes_below64(m)] = key;
            nbuf += (uint32_t)__popcll(m);
            if (nbuf > (uint32_t)(kBuf - 64)) flush(lane);
        }
    }

    // wave-collective: key j of the result (kNone = empty) for j < k goes to
    // write(j, key), called by one lane per j.
    template <class F>
    __device__ void finish(int lane, F write)
    {
        if constexpr (KR > 0) {
            uint64_t mykey = kNone;
            for (uint32_t j = 0; j < k; j++) {
                const uint64_t m = wave_min_u64(L[0]);
                if ((uint32_t)lane == j) mykey = m;
                if (m != kNone && L[0] == m) {   // every lane holding m pops it
#pragma unroll
                    for (int i = 0; i < NL - 1; i++) L[i] = L[i + 1];
                    L[NL - 1] = kNone;
                }
            }
            if ((uint32_t)lane < k) write((uint32_t)lane, mykey);
        } else {
            if (nbuf) flush(lane);
            for (uint32_t i = lane; i < k; i += 64) write(i, sh->run[i]);
        }
    }
};

// The window slots of one query, all curves concatenated: curve c's window
// starts at list place lo_c and occupies slots [off_c, off_{c+1}).
struct WindowSet {
    const uint32_t *base[kMaxCurves + 1];   // &ids_c[lo_c]
    uint64_t off[kMaxCurves + 1];
};

// Fills ws (LDS) from the query's positions; returns the number of slots.
// Wave-collective (writes by lanes 0..8, then a barrier).
__device__ inline uint64_t make_windows(const IndexView &v, const uint64_t (&pos)[kMaxCurves],
                                        uint64_t w, int lane, WindowSet *ws)
{
    uint64_t total = 0;
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) {
        uint64_t lo = 0, cnt = 0;
        if (c < (int)v.curves) {
            lo = pos[c] > w ? pos[c] - w : 0;
            const uint64_t hi = pos[c] + w < v.n ? pos[c] + w : v.n;
            cnt = hi - lo;
        }
        if (lane == c) {
            ws->base[c] = c < (int)v.curves ? v.ids[c] + lo : nullptr;
            ws->off[c] = total;
        }
        total += cnt;
    }
    if (lane == kMaxCurves) {
        ws->base[kMaxCurves] = nullptr;
        ws->off[kMaxCurves] = total;
    }
    __syncthreads();
    return total;
}

// Streams slots [s0, s1) of a query's windows through the distance kernel:
// per step, one coalesced load of 64 window ids, then 8 lanes per 128-byte
// row (16-byte loads), dot4 arithmetic and a 3-step lane-xor reduction; each
// lane ends up with one slot's packed key, handed to sink.push (kNone past s1).
// The next step's ids are loaded together with this step's rows, so a step
// waits for one memory latency, not two.
template <int G, class Sink>
__device__ inline void stream_slots(const uint8_t *db, const WindowSet *ws, uint64_t s0,
                                    uint64_t s1, const uint4 &qv, uint32_t qq, int lane,
                                    Sink &sink)
{
    const int part = lane & 7;
    uint64_t off[kMaxCurves];   // uniform copies of the prefix sums
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) off[c] = ws->off[c];
    auto load_ids = [&](uint64_t base, uint32_t (&ids)[G]) {
#pragma unroll
        for (int g = 0; g < G; g++) {
            const uint64_t s = base + 64 * g + lane;
            ids[g] = 0;
            if (s < s1) {
                int c = 0;
#pragma unroll
                for (int j = 1; j < kMaxCurves; j++) c += s >= off[j] ? 1 : 0;
                ids[g] = ws->base[c][s - ws->off[c]];
            }
        }
    };
    uint32_t next[G];
    load_ids(s0, next);
    for (uint64_t base = s0; base < s1; base += 64 * G) {
        uint32_t myid[G];
#pragma unroll
        for (int g = 0; g < G; g++) myid[g] = next[g];
        load_ids(base + 64 * G, next);
        // in step t of group g, lanes 8r..8r+7 read the row of slot 64 g + 8 t + r
        uint4 x[8 * G];
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const uint32_t rid = __shfl(myid[g], 8 * t + (lane >> 3), 64);
                const uint64_t s = base + 64 * g + 8 * t + (lane >> 3);
                x[8 * g + t] = s < s1
                    ? *reinterpret_cast<const uint4 *>(db + (uint64_t)rid * kDim + 16 * part)
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
            sink.push(s < s1 ? (((uint64_t)mine << 32) | mid) : kNone, lane);
        }
    }
}

// This lane's 16-byte part of query row q, and that part's q.q.
__device__ inline void query_part(const uint8_t *queries, uint32_t q, int lane, uint4 &qv,
                                  uint32_t &qq)
{
    qv = *reinterpret_cast<const uint4 *>(queries + (uint64_t)q * kDim + 16 * (lane & 7));
    qq = __builtin_amdgcn_udot4(qv.x, qv.x, 0u, false) +
         __builtin_amdgcn_udot4(qv.y, qv.y, 0u, false) +
         __builtin_amdgcn_udot4(qv.z, qv.z, 0u, false) +
         __builtin_amdgcn_udot4(qv.w, qv.w, 0u, false);
}

}  // namespace hc
