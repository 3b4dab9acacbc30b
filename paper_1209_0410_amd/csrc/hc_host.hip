// Host-core search for the cooperative CPU/GPU scheduler (Sec. 6, Alg. 3):
// the same Alg. 2 on copies of the curve lists in host memory, so that a few
// ready requests can be answered by host cores while the GPU is idle or busy.
// One call searches its queries on the calling thread; callers run calls on
// as many threads as they give the scheduler.  Results equal the GPU
// search's bit for bit: same keys, same positional windows, the union as a
// set, uint32 squared distances, (distance, id) order.
#include <string.h>

#include <algorithm>
#include <vector>

#include "hc_hilbert.h"

namespace hc {

// Host copy layout: keys of every curve ([curve][n], 16 B), then ids
// ([curve][n], 4 B).
struct HostLists {
    const Key *keys;
    const uint32_t *ids;
};

static HostLists host_lists(const IndexView &v, const void *h_index)
{
    HostLists L;
    L.keys = (const Key *)h_index;
    L.ids = (const uint32_t *)((const uint8_t *)h_index + sizeof(Key) * v.n * v.curves);
    return L;
}

static uint64_t host_lower_bound(const Key *keys, uint64_t n, const Key &q)
{
    uint64_t a = 0, b = n;
    while (a < b) {
        const uint64_t mid = a + (b - a) / 2;
        if (key_less(keys[mid], q)) a = mid + 1;
        else b = mid;
    }
    return a;
}

static uint32_t host_sqdist(const uint8_t *a, const uint8_t *b)
{
    uint32_t s = 0;
    for (int i = 0; i < kDim; i++) {
        const int d = (int)a[i] - (int)b[i];
        s += (uint32_t)(d * d);
    }
    return s;
}

static void host_one(const IndexView &v, const HostLists &L, const uint8_t *h_db,
                     const uint8_t *q, uint32_t k, uint64_t w, uint32_t k_stride,
                     uint32_t *out_ids, uint32_t *out_dists, std::vector<uint32_t> &cand,
                     std::vector<uint64_t> &keyd)
{
    cand.clear();
    for (uint32_t c = 0; c < v.curves; c++) {
        uint32_t coord[kDpc];
        project16(q, v, c, coord);
        const Key qk = curve_key16(coord, v.curve);
        const uint64_t p = host_lower_bound(L.keys + c * v.n, v.n, qk);
        const uint64_t lo = p > w ? p - w : 0, hi = p + w < v.n ? p + w : v.n;
        const uint32_t *ids = L.ids + c * v.n;
        cand.insert(cand.end(), ids + lo, ids + hi);
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    keyd.resize(cand.size());
    for (size_t i = 0; i < cand.size(); i++)
        keyd[i] = ((uint64_t)host_sqdist(q, h_db + (uint64_t)cand[i] * kDim) << 32) | cand[i];
    const size_t m = std::min<size_t>(k, keyd.size());
    std::partial_sort(keyd.begin(), keyd.begin() + m, keyd.end());
    for (uint32_t j = 0; j < k_stride; j++) {
        const bool have = j < m;
        out_ids[j] = have ? (uint32_t)keyd[j] : kEmpty;
        out_dists[j] = have ? (uint32_t)(keyd[j] >> 32) : kEmpty;
    }
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_status hc_host_index_bytes(const hc_index *idx, size_t *bytes)
{
    if (!idx || !bytes) return HC_ERR_INVALID;
    *bytes = (sizeof(Key) + sizeof(uint32_t)) * (size_t)idx->v.n * idx->v.curves;
    return HC_OK;
}

hc_status hc_host_index_copy(const hc_index *idx, void *h_index, size_t bytes, hc_stream stream)
{
    size_t need = 0;
    if (hc_host_index_bytes(idx, &need) != HC_OK || !h_index) return HC_ERR_INVALID;
    if (bytes < need) return HC_ERR_SIZE;
    const IndexView &v = idx->v;
    const HostLists L = host_lists(v, h_index);
    const hipStream_t st = (hipStream_t)stream;
    for (uint32_t c = 0; c < v.curves; c++) {
        if (hipMemcpyAsync((void *)(L.keys + c * v.n), v.lvl[c][0], sizeof(Key) * v.n,
                           hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync((void *)(L.ids + c * v.n), v.ids[c], sizeof(uint32_t) * v.n,
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            return HC_ERR_HIP;
    }
    return hipStreamSynchronize(st) == hipSuccess ? HC_OK : HC_ERR_HIP;
}

hc_status hc_host_search(const hc_index *idx, const void *h_index, const uint8_t *h_db,
                         const uint8_t *h_queries, uint32_t nq, uint32_t w_fixed,
                         const uint32_t *h_w, uint32_t k_fixed, const uint32_t *h_k,
                         uint32_t k_stride, uint32_t *h_out_ids, uint32_t *h_out_dists)
{
    if (!idx || !h_index || !h_db || !h_out_ids || !h_out_dists) return HC_ERR_INVALID;
    if (k_stride < 1 || k_stride > HC_K_MAX) return HC_ERR_INVALID;
    if (!h_k && (k_fixed < 1 || k_fixed > k_stride)) return HC_ERR_INVALID;
    if (nq == 0) return HC_OK;
    if (!h_queries) return HC_ERR_INVALID;
    const IndexView &v = idx->v;
    const HostLists L = host_lists(v, h_index);
    std::vector<uint32_t> cand;
    std::vector<uint64_t> keyd;
    for (uint32_t i = 0; i < nq; i++) {
        uint32_t k = h_k ? h_k[i] : k_fixed;
        k = std::min(std::max(k, 1u), k_stride);
        const uint64_t w = h_w ? h_w[i] : w_fixed;
        host_one(v, L, h_db, h_queries + (uint64_t)i * kDim, k, w, k_stride,
                 h_out_ids + (uint64_t)i * k_stride, h_out_dists + (uint64_t)i * k_stride,
                 cand, keyd);
    }
    return HC_OK;
}

}  // extern "C"
