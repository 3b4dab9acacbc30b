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
template <int CPW>
__device__ inline void locate(const IndexView &v, const Key *qk_row, uint32_t first,
                              uint32_t step, int lane, uint64_t (&cnt)[CPW])
{
    const uint32_t C = v.curves;
    const uint32_t D = v.levels;
    Key qk[CPW];
#pragma unroll
    for (int j = 0; j < CPW; j++) {
        const uint32_t c = first + j * step;
        qk[j] = c < C ? qk_row[c] : Key{0, 0};
    }
    {   // top table: at most 64 entries
        Key kk[CPW];
        const bool valid = (uint64_t)lane < v.len[D];
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const uint32_t c = first + j * step;
            kk[j] = (c < C && valid) ? v.lvl[c][D][lane] : Key{~0ull, ~0ull};
        }
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const bool less = (first + j * step < C) && valid && key_less(kk[j], qk[j]);
            cnt[j] = (uint64_t)__popcll(__ballot(less));
        }
    }
    for (int L = (int)D; L >= 1; L--) {
        // cnt = entries of level L below qkey, so the answer at level L-1 lies in
        // the 64 entries from 64*(cnt-1) (entry 64*cnt is >= qkey); cnt = 0
        // means every key is >= qkey.
        Key kk[CPW];
        uint64_t base[CPW];
        const uint64_t len = v.len[L - 1];
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const uint32_t c = first + j * step;
            base[j] = cnt[j] ? (cnt[j] - 1) * kFan : 0;
            const uint64_t idx = base[j] + lane;
            kk[j] = (c < C && cnt[j] && idx < len) ? v.lvl[c][L - 1][idx] : Key{~0ull, ~0ull};
        }
#pragma unroll
        for (int j = 0; j < CPW; j++) {
            const uint32_t c = first + j * step;
            const uint64_t idx = base[j] + lane;
            const bool less = c < C && cnt[j] && idx < len && key_less(kk[j], qk[j]);
            const uint64_t m = __ballot(less);
            cnt[j] = cnt[j] ? base[j] + (uint64_t)__popcll(m) : 0;
        }
    }
}

}  // namespace hc
