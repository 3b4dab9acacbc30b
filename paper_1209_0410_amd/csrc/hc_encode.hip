// Hilbert key encoding (Sec. 2.2.1; Alg. 1 and Alg. 2, projection + C^-1),
// parameter checks and the index handle.
#include <string.h>

#include <new>

#include "hc_hilbert.h"

namespace hc {

hc_status check_params(const hc_params *p, uint16_t *perm_out, uint32_t *identity)
{
    if (!p) return HC_ERR_INVALID;
    if (p->dim != (uint32_t)kDim || p->dims_per_curve != (uint32_t)kDpc || p->bits != 8)
        return HC_ERR_UNSUPPORTED;
    if (p->curves < 1 || p->curves > (uint32_t)kMaxCurves) return HC_ERR_UNSUPPORTED;
    if (p->curve != HC_CURVE_HILBERT && p->curve != HC_CURVE_ZORDER) return HC_ERR_UNSUPPORTED;
    uint32_t ident = 1;
    for (uint32_t i = 0; i < p->curves * kDpc; i++) {
        uint16_t d = p->perm ? p->perm[i] : (uint16_t)i;
        if (d >= kDim) return HC_ERR_INVALID;
        if (d != i) ident = 0;
        if (perm_out) perm_out[i] = d;
    }
    if (identity) *identity = ident;
    return HC_OK;
}

hc_status fill_view(const hc_params *p, const uint8_t *d_db, uint64_t n, void *d_index,
                    size_t index_bytes, IndexView *v)
{
    memset(v, 0, sizeof(*v));
    hc_status st = check_params(p, v->perm, &v->identity);
    if (st != HC_OK) return st;
    if (!d_db || !d_index || n == 0) return HC_ERR_INVALID;
    if (n >= 0xFFFFFFFFull) return HC_ERR_UNSUPPORTED;
    if (((uintptr_t)d_db & 15) || ((uintptr_t)d_index & 255)) return HC_ERR_INVALID;
    Layout L = make_layout(p->curves, n);
    if (index_bytes < L.total) return HC_ERR_SIZE;
    v->db = d_db;
    v->n = n;
    v->curves = p->curves;
    v->curve = p->curve;
    v->levels = L.levels;
    for (uint32_t l = 0; l <= L.levels; l++) v->len[l] = L.len[l];
    v->len_sub = L.len_sub;
    v->len_sub2 = L.len_sub2;
    uint8_t *base = (uint8_t *)d_index;
    for (uint32_t c = 0; c < p->curves; c++) {
        for (uint32_t l = 0; l <= L.levels; l++)
            v->lvl[c][l] = (const Key *)(base + L.lvl_off[c][l]);
        v->ids[c] = (const uint32_t *)(base + L.ids_off[c]);
        v->sub[c] = (const Key *)(base + L.sub_off[c]);
        v->sub2[c] = (const Key *)(base + L.sub2_off[c]);
    }
    return HC_OK;
}

// One thread per (row, curve): keys[row * curves + c].
__global__ __launch_bounds__(256) void k_encode_rows(IndexView v, const uint8_t *rows,
                                                     uint64_t nrows, Key *keys)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * v.curves) return;
    const uint64_t r = t / v.curves;
    const uint32_t c = (uint32_t)(t - r * v.curves);
    uint32_t coord[kDpc];
    project16(rows + r * kDim, v, c, coord);
    keys[t] = curve_key16(coord, v.curve);
}

hc_status encode_rows(const IndexView &v, const uint8_t *rows, uint64_t nrows, Key *keys,
                      hipStream_t s)
{
    if (nrows == 0) return HC_OK;
    const uint64_t work = nrows * v.curves;
    const uint64_t blocks = (work + 255) / 256;
    hipLaunchKernelGGL(k_encode_rows, dim3((uint32_t)blocks), dim3(256), 0, s, v, rows,
                       nrows, keys);
    return last_hip();
}

}  // namespace hc

using namespace hc;

extern "C" {

const char *hc_status_str(hc_status s)
{
    switch (s) {
    case HC_OK: return "ok";
    case HC_ERR_INVALID: return "invalid argument";
    case HC_ERR_SIZE: return "buffer too small";
    case HC_ERR_HIP: return "HIP error";
    case HC_ERR_UNSUPPORTED: return "unsupported shape";
    }
    return "unknown status";
}

hc_status hc_encode_keys(const hc_params *p, const uint8_t *d_rows, uint64_t nrows,
                         uint64_t *d_keys, hc_stream stream)
{
    IndexView v;
    memset(&v, 0, sizeof(v));
    hc_status st = check_params(p, v.perm, &v.identity);
    if (st != HC_OK) return st;
    if (nrows == 0) return HC_OK;
    if (!d_rows || !d_keys || ((uintptr_t)d_rows & 15) || ((uintptr_t)d_keys & 15))
        return HC_ERR_INVALID;
    if (nrows > (1ull << 40)) return HC_ERR_UNSUPPORTED;
    v.curves = p->curves;
    v.curve = p->curve;
    return encode_rows(v, d_rows, nrows, (Key *)d_keys, (hipStream_t)stream);
}

hc_status hc_index_destroy(hc_index *idx)
{
    if (!idx) return HC_ERR_INVALID;
    delete idx;
    return HC_OK;
}

hc_status hc_index_curve(const hc_index *idx, uint32_t c, const uint64_t **d_keys,
                         const uint32_t **d_ids)
{
    if (!idx || c >= idx->v.curves) return HC_ERR_INVALID;
    if (d_keys) *d_keys = (const uint64_t *)idx->v.lvl[c][0];
    if (d_ids) *d_ids = idx->v.ids[c];
    return HC_OK;
}

hc_status hc_index_info(const hc_index *idx, uint64_t *n, uint32_t *curves)
{
    if (!idx) return HC_ERR_INVALID;
    if (n) *n = idx->v.n;
    if (curves) *curves = idx->v.curves;
    return HC_OK;
}

hc_status hc_index_attach(const hc_params *p, const uint8_t *d_db, uint64_t n,
                          void *d_index, size_t index_bytes, hc_index **out)
{
    if (!out) return HC_ERR_INVALID;
    hc_index *h = new (std::nothrow) hc_index;
    if (!h) return HC_ERR_INVALID;
    hc_status st = fill_view(p, d_db, n, d_index, index_bytes, &h->v);
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
