// Learned probe depth (gfx950).  The paper's probe depth is one fixed knob for
// every query; here a small MLP predicts each query's window w from cheap
// features of its neighbourhood in the curves, trained on labels that say how
// large a window recovers the exact kNN (Eq. 3).
//
//  k_ranks        inverse permutation of every list (place of an id in curve c)
//  k_labels       smallest per-side window whose union holds the exact top-k
//  k_union_sizes  size of a query's candidate set (union of Alg. 2) for any w
//  k_features     24 features per query (one wavefront per query)
//  k_mlp_infer    24 -> 64 -> 64 -> 1 ReLU MLP, BF16 weights staged in LDS as
//                 FP32, FP32 arithmetic; w = clamp(ceil(2^(y + delta)))
//  k_mlp_sample / k_mlp_grad / k_adam
//                 training: per-sample forward and backward, a per-parameter
//                 reduction over the batch in a fixed order (deterministic),
//                 and Adam on FP32 master weights with a BF16 copy.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "hc_device.h"

namespace hc {

constexpr int kIn = HC_FEATURES;    // 24
constexpr int kH1 = 64, kH2 = 64;
constexpr int kNP = HC_MLP_PARAMS;  // 5825
// parameter offsets: W1[h1][in], b1[h1], W2[h2][h1], b2[h2], W3[h2], b3
constexpr int oW1 = 0, oB1 = oW1 + kH1 * kIn, oW2 = oB1 + kH1, oB2 = oW2 + kH2 * kH1,
              oW3 = oB2 + kH2, oB3 = oW3 + kH2;
static_assert(oB3 + 1 == kNP, "parameter count");

__device__ inline float bf16_to_f32(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

// Round to nearest even; NaN stays NaN.
__device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// log2(1 + g) for a 128-bit g = (hi, lo), in FP32 without overflow.
__device__ inline float log2_1p_u128(uint64_t hi, uint64_t lo)
{
    if (hi == 0) return log2f(1.0f + (float)lo);
    return 64.0f + log2f((float)hi + (float)lo * 5.421010862427522e-20f);   // 2^-64
}

__device__ inline void sub128(uint64_t ahi, uint64_t alo, uint64_t bhi, uint64_t blo,
                              uint64_t &hi, uint64_t &lo)
{
    lo = alo - blo;
    hi = ahi - bhi - (alo < blo ? 1 : 0);
}

__device__ inline uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = shfl_xor_u64(v, m);
        v = o > v ? o : v;
    }
    return v;
}

struct LearnArgs {
    IndexView v;
    const uint8_t *queries;
    const Key *qkeys;
    uint32_t nq, k, w_fixed;
    const uint32_t *d_k, *d_w, *rank, *truth;
    uint32_t *out_u32;
    float *feat;
};

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_ranks(IndexView v, uint32_t *rank)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= v.n * v.curves) return;
    const uint32_t c = (uint32_t)(t / v.n);
    const uint64_t r = t - (uint64_t)c * v.n;
    rank[(uint64_t)v.ids[c][r] * v.curves + c] = (uint32_t)r;
}

// label[q] = max over the exact top-k ids j of min over curves of r_c(j),
// r_c(j) = pos_c - rank_c(j) below the query's place, rank_c(j) - pos_c + 1
// at or above it: the window w takes j from curve c iff r_c(j) <= w.
__global__ __launch_bounds__(64) void k_labels(LearnArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
    uint64_t need = 0;
    for (uint32_t j = lane; j < a.k; j += 64) {
        const uint32_t id = a.truth[(uint64_t)q * a.k + j];
        if (id == kEmpty) continue;
        uint64_t best = ~0ull;
#pragma unroll
        for (int c = 0; c < kMaxCurves; c++) {
            if (c < (int)C) {
                const uint64_t rk = a.rank[(uint64_t)id * C + c];
                const uint64_t r = rk < pos[c] ? pos[c] - rk : rk - pos[c] + 1;
                best = r < best ? r : best;
            }
        }
        need = best > need ? best : need;
    }
    need = wave_max_u64(need);
    if (lane == 0) a.out_u32[q] = (uint32_t)std::min<uint64_t>(need, 0xFFFFFFFFull);
}

// A slot (curve c, list place r) is new unless its id lies in the window of a
// curve c' < c; the count of new slots is the size of the union.
__global__ __launch_bounds__(64) void k_union_sizes(LearnArgs a)
{
    __shared__ const uint32_t *s_base[kMaxCurves + 1];
    __shared__ uint64_t s_off[kMaxCurves + 1];
    __shared__ uint32_t s_curve_lo[kMaxCurves], s_curve_hi[kMaxCurves];
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    const uint64_t n = a.v.n;
    const uint64_t w = a.d_w ? a.d_w[q] : a.w_fixed;
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
    uint64_t total = 0;
    uint64_t wlo[kMaxCurves], whi[kMaxCurves];
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) {
        wlo[c] = 0;
        whi[c] = 0;
        if (c < (int)C) {
            wlo[c] = pos[c] > w ? pos[c] - w : 0;
            whi[c] = pos[c] + w < n ? pos[c] + w : n;
        }
        if (lane == c) {
            s_base[c] = c < (int)C ? a.v.ids[c] + wlo[c] : nullptr;
            s_off[c] = total;
            s_curve_lo[c] = (uint32_t)wlo[c];
            s_curve_hi[c] = (uint32_t)whi[c];
        }
        total += whi[c] - wlo[c];
    }
    if (lane == kMaxCurves) {
        s_base[kMaxCurves] = nullptr;
        s_off[kMaxCurves] = total;
    }
    __syncthreads();
    uint64_t off[kMaxCurves];
#pragma unroll
    for (int c = 0; c < kMaxCurves; c++) off[c] = s_off[c];
    uint64_t fresh = 0;
    for (uint64_t base = 0; base < total; base += 64) {
        const uint64_t s = base + lane;
        bool is_new = false;
        if (s < total) {
            int c = 0;
#pragma unroll
            for (int j = 1; j < kMaxCurves; j++) c += s >= off[j] ? 1 : 0;
            const uint32_t id = s_base[c][s - s_off[c]];
            is_new = true;
            for (int e = 0; e < c; e++) {
                const uint32_t rk = a.rank[(uint64_t)id * C + e];
                if (rk >= s_curve_lo[e] && rk < s_curve_hi[e]) is_new = false;
            }
        }
        fresh += (uint64_t)__popcll(__ballot(is_new));
    }
    if (lane == 0) a.out_u32[q] = (uint32_t)fresh;
}

// Features: lane = 8 c + t handles curve c, task t.
//   t < 6: log2(1 + |key_c[pos_c + o'] - qkey_c|), o in {-64,-8,-1,+1,+8,+64},
//          o' = o below the query's place, o - 1 at or above it
//   t = 6: log2(1 + squared distance to the entry at pos_c)
//   t = 7: log2(1 + key_c[pos_c + s - 1] - key_c[pos_c - s]), s in {1, 8, 64}
// (list places clamped to [0, n-1]), then min / mean / max over the curves.
__global__ __launch_bounds__(64) void k_features(LearnArgs a)
{
    const int lane = threadIdx.x;
    const uint32_t q = blockIdx.x;
    const uint32_t C = a.v.curves;
    const int64_t n = (int64_t)a.v.n;
    uint64_t pos[kMaxCurves];
    locate<kMaxCurves>(a.v, a.qkeys + (uint64_t)q * C, 0, 1, lane, pos);
    const int c = lane >> 3, t = lane & 7;
    const bool live = c < (int)C;
    int64_t p = 0;
#pragma unroll
    for (int j = 0; j < kMaxCurves; j++)
        if (j == c) p = (int64_t)pos[j];
    auto clampi = [n](int64_t x) { return x < 0 ? 0 : (x > n - 1 ? n - 1 : x); };
    float gap = INFINITY, dist = 0.0f;
    float span[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (live) {
        const Key *keys = a.v.lvl[c][0];
        const Key qk = a.qkeys[(uint64_t)q * C + c];
        if (t < 6) {
            const int offs[6] = {-64, -8, -1, 0, 7, 63};   // o' of o = -64..+64
            const Key kk = keys[clampi(p + offs[t])];
            uint64_t hi, lo;
            if (key_less(kk, qk)) sub128(qk.hi, qk.lo, kk.hi, kk.lo, hi, lo);
            else sub128(kk.hi, kk.lo, qk.hi, qk.lo, hi, lo);
            gap = log2_1p_u128(hi, lo);
        } else if (t == 6) {
            const uint32_t id = a.v.ids[c][clampi(p)];
            const uint4 *row = reinterpret_cast<const uint4 *>(a.v.db + (uint64_t)id * kDim);
            const uint4 *qr = reinterpret_cast<const uint4 *>(a.queries + (uint64_t)q * kDim);
            uint32_t d = 0;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const uint4 x = row[i], y = qr[i];
                const uint32_t xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    d = __builtin_amdgcn_udot4(xs[b], xs[b], d, false);
                    d = __builtin_amdgcn_udot4(ys[b], ys[b], d, false);
                    d -= 2u * __builtin_amdgcn_udot4(xs[b], ys[b], 0u, false);
                }
            }
            dist = log2f(1.0f + (float)d);
        } else {
            const int sp[3] = {1, 8, 64};
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const Key ka = keys[clampi(p - sp[i])];
                const Key kb = keys[clampi(p + sp[i] - 1)];
                uint64_t hi, lo;
                sub128(kb.hi, kb.lo, ka.hi, ka.lo, hi, lo);
                span[i] = log2_1p_u128(hi, lo);
            }
        }
    }
    // reduce over the curves: lanes t, t + 8, ..., t + 56
    float mn = gap, sum = live && t < 6 ? gap : 0.0f;
#pragma unroll
    for (int m = 8; m <= 32; m <<= 1) {
        mn = fminf(mn, __shfl_xor(mn, m, 64));
        sum += __shfl_xor(sum, m, 64);
#pragma unroll
        for (int i = 0; i < 3; i++) span[i] = fmaxf(span[i], __shfl_xor(span[i], m, 64));
    }
    float *f = a.feat + (uint64_t)q * kIn;
    if (c == 0 && t < 6) {
        f[t] = mn;
        f[6 + t] = sum / (float)C;
    }
    if (live && t == 6) f[12 + c] = dist;
    if (lane == 7) {
        f[21] = span[0];
        f[22] = span[1];
        f[23] = span[2];
        const uint32_t kq = a.d_k ? a.d_k[q] : a.k;
        f[20] = log2f((float)kq);
    }
    if (C < kMaxCurves && lane >= (int)C && lane < kMaxCurves) f[12 + lane] = 0.0f;
}

// ---------------------------------------------------------------------------
// MLP
// ---------------------------------------------------------------------------

struct MlpArgs {
    const uint16_t *params;   // BF16, kNP
    const float *norm;        // mean[24], std[24] or NULL
    const float *x;           // [rows][24] raw features
    const uint32_t *idx;      // batch rows, NULL = 0..batch-1
    const float *target;      // [rows]
    uint32_t batch;
    float delta;
    uint32_t w_min, w_max, w_fallback;
    uint32_t *w_out;
    float *y_out;
    float *scratch;           // [batch][kRow] per-sample records
    float *grad, *loss;
};

// per-sample record: xn[24] a1[64] d1[64] a2[64] d2[64] d3 loss
constexpr int kRow = kIn + 4 * 64 + 2;
constexpr int rXn = 0, rA1 = kIn, rD1 = rA1 + 64, rA2 = rD1 + 64, rD2 = rA2 + 64,
              rD3 = rD2 + 64, rLoss = rD3 + 1;

__device__ inline void stage_params(const uint16_t *params, float *w)
{
    for (int i = threadIdx.x; i < kNP; i += blockDim.x) w[i] = bf16_to_f32(params[i]);
    __syncthreads();
}

__device__ inline void load_x(const MlpArgs &a, uint32_t row, float (&x)[kIn])
{
    const float *src = a.x + (uint64_t)row * kIn;
#pragma unroll
    for (int i = 0; i < kIn; i++) {
        const float v = src[i];
        x[i] = a.norm ? (v - a.norm[i]) / a.norm[kIn + i] : v;
    }
}

__device__ inline float forward(const float *w, const float (&x)[kIn], float (&a1)[kH1],
                                uint64_t &mask2, float *rec)
{
#pragma unroll
    for (int o = 0; o < kH1; o++) {
        float s = w[oB1 + o];
#pragma unroll
        for (int i = 0; i < kIn; i++) s = fmaf(w[oW1 + o * kIn + i], x[i], s);
        a1[o] = s > 0.0f ? s : 0.0f;
    }
    float y = w[oB3];
    mask2 = 0;
    for (int o = 0; o < kH2; o++) {
        float s = w[oB2 + o];
#pragma unroll
        for (int i = 0; i < kH1; i++) s = fmaf(w[oW2 + o * kH1 + i], a1[i], s);
        const float r = s > 0.0f ? s : 0.0f;
        if (s > 0.0f) mask2 |= 1ull << o;
        if (rec) rec[rA2 + o] = r;
        y = fmaf(w[oW3 + o], r, y);
    }
    return y;
}

__global__ __launch_bounds__(256) void k_mlp_infer(MlpArgs a)
{
    __shared__ float w[kNP];
    stage_params(a.params, w);
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    const uint32_t row = a.idx ? a.idx[b] : b;
    float x[kIn], a1[kH1];
    uint64_t m2;
    load_x(a, row, x);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < kIn; i++) finite = finite && isfinite(x[i]);
    const float y = forward(w, x, a1, m2, nullptr);
    if (a.y_out) a.y_out[b] = finite ? y : NAN;
    if (a.w_out) {
        const float t = y + a.delta;
        uint32_t out;
        if (!finite || !isfinite(t)) {
            out = a.w_fallback;
        } else {
            const float e = exp2f(t);
            if (e >= (float)a.w_max) out = a.w_max;
            else if (e <= (float)a.w_min) out = a.w_min;
            else out = std::min<uint32_t>(std::max<uint32_t>((uint32_t)ceilf(e), a.w_min), a.w_max);
        }
        a.w_out[b] = out;
    }
}

// Inference for small batches: one wavefront per sample, lane j computing
// hidden unit j of each layer with the terms in the same order as forward(),
// so the outputs are bit-identical to k_mlp_infer's.
constexpr int kInferWaves = 4;
static_assert(kH1 == 64 && kH2 == 64, "one lane per hidden unit");
__global__ __launch_bounds__(64 * kInferWaves) void k_mlp_infer_wave(MlpArgs a)
{
    __shared__ float w[kNP];
    __shared__ float hs[kInferWaves][kH1 + kH2];
    stage_params(a.params, w);      // block barrier: before any wavefront leaves
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t b = blockIdx.x * kInferWaves + wv;
    if (b >= a.batch) return;
    const uint32_t row = a.idx ? a.idx[b] : b;
    float x[kIn];
    load_x(a, row, x);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < kIn; i++) finite = finite && isfinite(x[i]);
    float *h = hs[wv];
    {
        float s = w[oB1 + lane];
#pragma unroll
        for (int i = 0; i < kIn; i++) s = fmaf(w[oW1 + lane * kIn + i], x[i], s);
        h[lane] = s > 0.0f ? s : 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
        float s = w[oB2 + lane];
#pragma unroll 8
        for (int i = 0; i < kH1; i++) s = fmaf(w[oW2 + lane * kH1 + i], h[i], s);
        h[kH1 + lane] = s > 0.0f ? s : 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float y = w[oB3];
#pragma unroll 8
    for (int o = 0; o < kH2; o++) y = fmaf(w[oW3 + o], h[kH1 + o], y);
    if (lane != 0) return;
    if (a.y_out) a.y_out[b] = finite ? y : NAN;
    if (a.w_out) {
        const float t = y + a.delta;
        uint32_t out;
        if (!finite || !isfinite(t)) {
            out = a.w_fallback;
        } else {
            const float e = exp2f(t);
            if (e >= (float)a.w_max) out = a.w_max;
            else if (e <= (float)a.w_min) out = a.w_min;
            else out = std::min<uint32_t>(std::max<uint32_t>((uint32_t)ceilf(e), a.w_min), a.w_max);
        }
        a.w_out[b] = out;
    }
}

// Forward and backward of one sample; the record feeds k_mlp_grad.
// loss = mean over the batch of (y - target)^2.
__global__ __launch_bounds__(256) void k_mlp_sample(MlpArgs a)
{
    __shared__ float w[kNP];
    stage_params(a.params, w);
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    const uint32_t row = a.idx ? a.idx[b] : b;
    float *rec = a.scratch + (uint64_t)b * kRow;
    float x[kIn], a1[kH1];
    load_x(a, row, x);
#pragma unroll
    for (int i = 0; i < kIn; i++) rec[rXn + i] = x[i];
    uint64_t m2;
    const float y = forward(w, x, a1, m2, rec);
    uint64_t m1 = 0;
#pragma unroll
    for (int i = 0; i < kH1; i++) {
        rec[rA1 + i] = a1[i];
        if (a1[i] > 0.0f) m1 |= 1ull << i;
    }
    const float e = y - a.target[row];
    const float d3 = 2.0f * e / (float)a.batch;
    rec[rD3] = d3;
    rec[rLoss] = e * e;
    float d2[kH2];
#pragma unroll
    for (int o = 0; o < kH2; o++) {
        d2[o] = ((m2 >> o) & 1) ? w[oW3 + o] * d3 : 0.0f;
        rec[rD2 + o] = d2[o];
    }
    for (int i = 0; i < kH1; i++) {
        float s = 0.0f;
#pragma unroll
        for (int o = 0; o < kH2; o++) s = fmaf(w[oW2 + o * kH1 + i], d2[o], s);
        rec[rD1 + i] = ((m1 >> i) & 1) ? s : 0.0f;
    }
}

// grad[p] = sum over the batch, in sample order, of (output delta) x (input);
// thread kNP sums the loss.
__global__ __launch_bounds__(256) void k_mlp_grad(MlpArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    int dfield, ifield;   // record offsets of the delta and of the input (-1 = bias)
    if (p < oB1) {
        dfield = rD1 + p / kIn;
        ifield = rXn + p % kIn;
    } else if (p < oW2) {
        dfield = rD1 + (p - oB1);
        ifield = -1;
    } else if (p < oB2) {
        dfield = rD2 + (p - oW2) / kH1;
        ifield = rA1 + (p - oW2) % kH1;
    } else if (p < oW3) {
        dfield = rD2 + (p - oB2);
        ifield = -1;
    } else if (p < oB3) {
        dfield = rD3;
        ifield = rA2 + (p - oW3);
    } else if (p == oB3) {
        dfield = rD3;
        ifield = -1;
    } else {
        dfield = rLoss;
        ifield = -1;
    }
    float s = 0.0f;
    for (uint32_t b = 0; b < a.batch; b++) {
        const float *rec = a.scratch + (uint64_t)b * kRow;
        const float d = rec[dfield];
        s = ifield < 0 ? s + d : fmaf(d, rec[ifield], s);
    }
    if (p < kNP) a.grad[p] = s;
    else if (a.loss) *a.loss = s / (float)a.batch;
}

__global__ __launch_bounds__(256) void k_adam(float *master, float *m, float *v, const float *g,
                                              uint32_t np, float lr, float beta1, float beta2,
                                              float eps, float c1, float c2, uint16_t *out_bf16)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = th;
    if (out_bf16) out_bf16[i] = f32_to_bf16(th);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *src, uint32_t n, uint16_t *dst)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f32_to_bf16(src[i]);
}

// Training targets: y = log2(clamp(label, w_min, w_max)), the label's log
// taken in FP64 and rounded to FP32.
__global__ __launch_bounds__(256) void k_targets(const uint32_t *labels, uint32_t nq,
                                                 uint32_t w_min, uint32_t w_max, float *y)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nq) return;
    uint32_t l = labels[i];
    l = l < w_min ? w_min : (l > w_max ? w_max : l);
    y[i] = (float)log2((double)l);
}

// Standardisation of one feature per block: mean and standard deviation
// (divisor rows - 1) over the rows, summed in FP64 in a fixed order (thread t
// takes rows t, t + 256, ..., then a fixed tree), so the result is
// deterministic.  A deviation below 1e-3 (a feature that does not vary) is
// replaced by 1, so that unseen values stay moderate.
constexpr int kNormThreads = 256;
__global__ __launch_bounds__(kNormThreads) void k_feature_norm(const float *x, uint32_t rows,
                                                               float *norm)
{
    __shared__ double sh[kNormThreads];
    const uint32_t f = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (uint32_t r = t; r < rows; r += kNormThreads) s += (double)x[(uint64_t)r * kIn + f];
    sh[t] = s;
    __syncthreads();
    for (int m = kNormThreads / 2; m > 0; m >>= 1) {
        if ((int)t < m) sh[t] += sh[t + m];
        __syncthreads();
    }
    const double mean = sh[0] / (double)rows;
    __syncthreads();
    double v = 0.0;
    for (uint32_t r = t; r < rows; r += kNormThreads) {
        const double d = (double)x[(uint64_t)r * kIn + f] - mean;
        v += d * d;
    }
    sh[t] = v;
    __syncthreads();
    for (int m = kNormThreads / 2; m > 0; m >>= 1) {
        if ((int)t < m) sh[t] += sh[t + m];
        __syncthreads();
    }
    if (t == 0) {
        double sd = rows > 1 ? sqrt(sh[0] / (double)(rows - 1)) : 0.0;
        if (!(sd >= 1e-3)) sd = 1.0;
        norm[f] = (float)mean;
        norm[kIn + f] = (float)sd;
    }
}

static hc_status learn_common(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                              void *d_scratch, size_t scratch_bytes, hipStream_t s,
                              LearnArgs *a)
{
    if (!idx || !d_queries || ((uintptr_t)d_queries & 15)) return HC_ERR_INVALID;
    if (!d_scratch || ((uintptr_t)d_scratch & 15)) return HC_ERR_INVALID;
    if (scratch_bytes < sizeof(Key) * (size_t)nq * idx->v.curves) return HC_ERR_SIZE;
    memset(a, 0, sizeof(*a));
    a->v = idx->v;
    a->queries = d_queries;
    a->qkeys = (const Key *)d_scratch;
    a->nq = nq;
    return encode_rows(idx->v, d_queries, nq, (Key *)d_scratch, s);
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_index_ranks(const hc_index *idx, uint32_t *d_rank, hc_stream stream)
{
    if (!idx || !d_rank || ((uintptr_t)d_rank & 3)) return HC_ERR_INVALID;
    const uint64_t work = idx->v.n * idx->v.curves;
    hipLaunchKernelGGL(k_ranks, dim3((uint32_t)((work + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, idx->v, d_rank);
    return last_hip();
}

hc_status hc_labels(const hc_index *idx, const uint32_t *d_rank, const uint8_t *d_queries,
                    uint32_t nq, uint32_t k, const uint32_t *d_truth_ids, uint32_t *d_labels,
                    void *d_scratch, size_t scratch_bytes, hc_stream stream)
{
    if (!d_rank || !d_truth_ids || !d_labels || k < 1) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hipStream_t s = (hipStream_t)stream;
    LearnArgs a;
    hc_status st = learn_common(idx, d_queries, nq, d_scratch, scratch_bytes, s, &a);
    if (st != HC_OK) return st;
    a.k = k;
    a.rank = d_rank;
    a.truth = d_truth_ids;
    a.out_u32 = d_labels;
    hipLaunchKernelGGL(k_labels, dim3(nq), dim3(64), 0, s, a);
    return last_hip();
}

hc_status hc_union_sizes(const hc_index *idx, const uint32_t *d_rank, const uint8_t *d_queries,
                         uint32_t nq, uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_counts,
                         void *d_scratch, size_t scratch_bytes, hc_stream stream)
{
    if (!d_rank || !d_counts) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hipStream_t s = (hipStream_t)stream;
    LearnArgs a;
    hc_status st = learn_common(idx, d_queries, nq, d_scratch, scratch_bytes, s, &a);
    if (st != HC_OK) return st;
    a.w_fixed = w_fixed;
    a.d_w = d_w;
    a.rank = d_rank;
    a.out_u32 = d_counts;
    hipLaunchKernelGGL(k_union_sizes, dim3(nq), dim3(64), 0, s, a);
    return last_hip();
}

hc_status hc_features(const hc_index *idx, const uint8_t *d_queries, uint32_t nq, uint32_t k,
                      const uint32_t *d_k, float *d_feat, void *d_scratch, size_t scratch_bytes,
                      hc_stream stream)
{
    if (!d_feat || ((uintptr_t)d_feat & 3) || (!d_k && k < 1)) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hipStream_t s = (hipStream_t)stream;
    LearnArgs a;
    hc_status st = learn_common(idx, d_queries, nq, d_scratch, scratch_bytes, s, &a);
    if (st != HC_OK) return st;
    a.k = k;
    a.d_k = d_k;
    a.feat = d_feat;
    hipLaunchKernelGGL(k_features, dim3(nq), dim3(64), 0, s, a);
    return last_hip();
}

hc_status hc_mlp_infer(const uint16_t *d_params_bf16, const float *d_norm, const float *d_feat,
                       uint32_t nq, float delta, uint32_t w_min, uint32_t w_max,
                       uint32_t w_fallback, uint32_t *d_w_out, float *d_y_out, hc_stream stream)
{
    if (!d_params_bf16 || !d_feat || (!d_w_out && !d_y_out)) return HC_ERR_INVALID;
    if (w_min > w_max) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    MlpArgs a;
    memset(&a, 0, sizeof(a));
    a.params = d_params_bf16;
    a.norm = d_norm;
    a.x = d_feat;
    a.batch = nq;
    a.delta = delta;
    a.w_min = w_min;
    a.w_max = w_max;
    a.w_fallback = w_fallback;
    a.w_out = d_w_out;
    a.y_out = d_y_out;
    // small batches (the serving loop's): a wavefront per sample; large ones:
    // a thread per sample
    if (nq <= 2048)
        hipLaunchKernelGGL(k_mlp_infer_wave, dim3((nq + kInferWaves - 1) / kInferWaves),
                           dim3(64 * kInferWaves), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_mlp_infer, dim3((nq + 255) / 256), dim3(256), 0,
                           (hipStream_t)stream, a);
    return last_hip();
}

hc_status hc_mlp_train_scratch_bytes(uint32_t batch, size_t *bytes)
{
    if (!bytes || batch < 1) return HC_ERR_INVALID;
    *bytes = align256(sizeof(float) * (size_t)batch * kRow);
    return HC_OK;
}

hc_status hc_mlp_forward(const uint16_t *d_params_bf16, const float *d_norm, const float *d_x,
                         const uint32_t *d_idx, uint32_t batch, float *d_y, hc_stream stream)
{
    if (!d_params_bf16 || !d_x || !d_y) return HC_ERR_INVALID;
    if (batch == 0) return HC_OK;
    MlpArgs a;
    memset(&a, 0, sizeof(a));
    a.params = d_params_bf16;
    a.norm = d_norm;
    a.x = d_x;
    a.idx = d_idx;
    a.batch = batch;
    a.y_out = d_y;
    hipLaunchKernelGGL(k_mlp_infer, dim3((batch + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       a);
    return last_hip();
}

hc_status hc_mlp_backward(const uint16_t *d_params_bf16, const float *d_norm, const float *d_x,
                          const float *d_target, const uint32_t *d_idx, uint32_t batch,
                          float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes,
                          hc_stream stream)
{
    if (!d_params_bf16 || !d_x || !d_target || !d_grad || !d_scratch || batch < 1)
        return HC_ERR_INVALID;
    size_t need = 0;
    hc_mlp_train_scratch_bytes(batch, &need);
    if (scratch_bytes < need) return HC_ERR_SIZE;
    MlpArgs a;
    memset(&a, 0, sizeof(a));
    a.params = d_params_bf16;
    a.norm = d_norm;
    a.x = d_x;
    a.idx = d_idx;
    a.target = d_target;
    a.batch = batch;
    a.scratch = (float *)d_scratch;
    a.grad = d_grad;
    a.loss = d_loss;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_sample, dim3((batch + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_mlp_grad, dim3((kNP + 1 + 255) / 256), dim3(256), 0, s, a);
    return last_hip();
}

hc_status hc_adam_step(float *d_master, float *d_m, float *d_v, const float *d_grad, uint32_t np,
                       uint32_t t, float lr, float beta1, float beta2, float eps,
                       uint16_t *d_params_bf16, hc_stream stream)
{
    if (!d_master || !d_m || !d_v || !d_grad || t < 1) return HC_ERR_INVALID;
    if (np == 0) return HC_OK;
    const float c1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       d_master, d_m, d_v, d_grad, np, lr, beta1, beta2, eps, c1, c2,
                       d_params_bf16);
    return last_hip();
}

hc_status hc_mlp_targets(const uint32_t *d_labels, uint32_t nq, uint32_t w_min, uint32_t w_max,
                         float *d_y, hc_stream stream)
{
    if (!d_labels || !d_y || w_min < 1 || w_min > w_max) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    hipLaunchKernelGGL(k_targets, dim3((nq + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       d_labels, nq, w_min, w_max, d_y);
    return last_hip();
}

hc_status hc_feature_norm(const float *d_feat, uint32_t rows, float *d_norm, hc_stream stream)
{
    if (!d_feat || !d_norm || rows < 1) return HC_ERR_INVALID;
    hipLaunchKernelGGL(k_feature_norm, dim3(kIn), dim3(kNormThreads), 0, (hipStream_t)stream,
                       d_feat, rows, d_norm);
    return last_hip();
}

hc_status hc_to_bf16(const float *d_src, uint32_t n, uint16_t *d_dst, hc_stream stream)
{
    if (!d_src || !d_dst) return HC_ERR_INVALID;
    if (n == 0) return HC_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       d_src, n, d_dst);
    return last_hip();
}

}  // extern "C"
