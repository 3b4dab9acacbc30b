/*
 * hc_oracle.c -- plain CPU oracle for the Multicurves search path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library; both sides only see the same seeded inputs.
 *
 * Every routine is the slow, obviously-correct form of one step of the method
 * (Teodoro et al., "Approximate similarity search for online multimedia
 * services on distributed CPU-GPU platforms", arXiv 1209.0410):
 *
 *   hco_hilbert_encode / _decode  Sec. 2.2.1 (extended-key C^-1 of a d-dim
 *                                 point of m-bit coordinates, d*m key bits;
 *                                 Hilbert curve computed by the iterative
 *                                 Butz-type scheme, here in the transposed
 *                                 form published by J. Skilling, "Programming
 *                                 the Hilbert curve", AIP Conf. Proc. 707, 2004)
 *   hco_zorder_encode / _decode   the Z-order key, a comparison curve: the
 *                                 coordinates' bits intercalated (Sec. 2.2.1)
 *   hco_keys, hco_keys_ex         Alg. 1 / Alg. 2 projection + key
 *   hco_build                     Alg. 1 (sorted <key, id> list per curve)
 *   hco_lower_bound, hco_positions  binary search of the query key
 *   hco_candidates                Alg. 2 union of the per-curve windows
 *   hco_search                    Alg. 2 (k closest of the candidates)
 *   hco_brute_force               Eq. (3) exact kNN
 *   hco_labels                    smallest per-side window recovering Eq. (3)
 *   hco_features, hco_mlp_*       learned probe depth (not in the paper)
 *
 * Readings of the paper where it is silent (all fixed here, normative for the
 * GPU library):
 *   - key bit layout: transposed form, most significant bit first, for bit
 *     level b = m-1 .. 0 and for dim i = 0 .. d-1 emit bit b of X[i];
 *   - the probe-depth entries nearest the key in Alg. 2 are a positional window:
 *     w list entries with key < qkey and w entries with key >= qkey (the
 *     half-list model of Sec. 4.2), each half clamped to the list ends;
 *   - lists are ordered by (key, id); the union is a set; the result is
 *     ordered by (squared distance, id) and padded with 0xFFFFFFFF.
 *
 * Parity status: every routine here is pinned by tests/ (Hilbert invariants,
 * library routines, brute force on tiny inputs, finite differences).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef unsigned __int128 u128;

#define PAD 0xFFFFFFFFu

/* Threads of the parallel loops over queries (timing of the CPU baseline):
 * hco_set_threads(t) for t >= 1; hco_threads() is the count in use. */
void hco_set_threads(int t)
{
    if (t >= 1) omp_set_num_threads(t);
}

int hco_threads(void)
{
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Hilbert extended key (Sec. 2.2.1)                                         */
/* ------------------------------------------------------------------------ */

/* Skilling's forward transform: axes -> transposed Hilbert index, in place.
 * n coordinates of `bits` bits each. */
static void axes_to_transposed(uint32_t *x, int n, int bits)
{
    uint32_t top = 1u << (bits - 1);
    /* undo the excess work of the recursive construction, level by level */
    for (uint32_t q = top; q > 1; q >>= 1) {
        uint32_t low = q - 1;
        for (int i = 0; i < n; i++) {
            if (x[i] & q) {
                x[0] ^= low;                          /* invert */
            } else {
                uint32_t t = (x[0] ^ x[i]) & low;     /* exchange */
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
    /* Gray encode */
    for (int i = 1; i < n; i++)
        x[i] ^= x[i - 1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (x[n - 1] & q)
            t ^= q - 1;
    for (int i = 0; i < n; i++)
        x[i] ^= t;
}

/* Skilling's inverse transform: transposed Hilbert index -> axes, in place. */
static void transposed_to_axes(uint32_t *x, int n, int bits)
{
    /* Gray decode */
    uint32_t t = x[n - 1] >> 1;
    for (int i = n - 1; i > 0; i--)
        x[i] ^= x[i - 1];
    x[0] ^= t;
    /* redo the excess work, lowest level first */
    for (int b = 1; b < bits; b++) {
        uint32_t q = 1u << b;
        uint32_t low = q - 1;
        for (int i = n - 1; i >= 0; i--) {
            if (x[i] & q) {
                x[0] ^= low;
            } else {
                uint32_t s = (x[0] ^ x[i]) & low;
                x[0] ^= s;
                x[i] ^= s;
            }
        }
    }
}

/* Transposed form -> integer key: level b from the top, dim i = 0..n-1. */
static u128 transposed_to_key(const uint32_t *x, int n, int bits)
{
    u128 key = 0;
    for (int b = bits - 1; b >= 0; b--)
        for (int i = 0; i < n; i++)
            key = (key << 1) | ((x[i] >> b) & 1u);
    return key;
}

static void key_to_transposed(u128 key, uint32_t *x, int n, int bits)
{
    for (int i = 0; i < n; i++)
        x[i] = 0;
    for (int b = 0; b < bits; b++)
        for (int i = 0; i < n; i++) {
            int pos = b * n + (n - 1 - i);   /* bit position from the LSB */
            x[i] |= (uint32_t)((key >> pos) & 1u) << b;
        }
}

/* Returns 0 on success, -1 when n*bits does not fit a 128-bit key. */
int hco_hilbert_encode(const uint32_t *coords, int64_t npts, int n, int bits,
                       uint64_t *hi, uint64_t *lo)
{
    if (n < 1 || n > 128 || bits < 1 || bits > 32 || n * bits > 128)
        return -1;
    uint32_t x[128];
    for (int64_t p = 0; p < npts; p++) {
        memcpy(x, coords + p * n, sizeof(uint32_t) * (size_t)n);
        axes_to_transposed(x, n, bits);
        u128 key = transposed_to_key(x, n, bits);
        hi[p] = (uint64_t)(key >> 64);
        lo[p] = (uint64_t)key;
    }
    return 0;
}

int hco_hilbert_decode(const uint64_t *hi, const uint64_t *lo, int64_t npts,
                       int n, int bits, uint32_t *coords)
{
    if (n < 1 || n > 128 || bits < 1 || bits > 32 || n * bits > 128)
        return -1;
    uint32_t x[128];
    for (int64_t p = 0; p < npts; p++) {
        u128 key = ((u128)hi[p] << 64) | lo[p];
        key_to_transposed(key, x, n, bits);
        transposed_to_axes(x, n, bits);
        memcpy(coords + p * n, x, sizeof(uint32_t) * (size_t)n);
    }
    return 0;
}

/* Z-order key: the coordinates' bits intercalated (Sec. 2.2.1; G. M. Morton,
 * 1966), in the same bit layout as the Hilbert key: most significant level
 * first, dim 0 first within a level.  Both curves visit every cell once
 * (Sec. 2.2.1), but only the Hilbert curve moves between adjacent cells. */
int hco_zorder_encode(const uint32_t *coords, int64_t npts, int n, int bits,
                      uint64_t *hi, uint64_t *lo)
{
    if (n < 1 || n > 128 || bits < 1 || bits > 32 || n * bits > 128)
        return -1;
    for (int64_t p = 0; p < npts; p++) {
        u128 key = transposed_to_key(coords + p * n, n, bits);
        hi[p] = (uint64_t)(key >> 64);
        lo[p] = (uint64_t)key;
    }
    return 0;
}

int hco_zorder_decode(const uint64_t *hi, const uint64_t *lo, int64_t npts,
                      int n, int bits, uint32_t *coords)
{
    if (n < 1 || n > 128 || bits < 1 || bits > 32 || n * bits > 128)
        return -1;
    for (int64_t p = 0; p < npts; p++) {
        u128 key = ((u128)hi[p] << 64) | lo[p];
        key_to_transposed(key, coords + p * n, n, bits);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection + key of every row, every curve (Alg. 1 / Alg. 2)             */
/* ------------------------------------------------------------------------ */

/* Keys of one row, curve c taking dims perm[c*dpc + j], j < dpc.  The data
 * are 8-bit, so the curve is of order 8 (m-bit coordinates need an order-m
 * curve, Sec. 2.2.1) and a key holds dpc*8 bits. */
static void row_keys(const uint8_t *row, const uint16_t *perm, int curves,
                     int dpc, int curve, uint64_t *hi, uint64_t *lo)
{
    uint32_t proj[16];
    for (int c = 0; c < curves; c++) {
        for (int j = 0; j < dpc; j++)
            proj[j] = row[perm[c * dpc + j]];
        if (curve == 1)
            hco_zorder_encode(proj, 1, dpc, 8, &hi[c], &lo[c]);
        else
            hco_hilbert_encode(proj, 1, dpc, 8, &hi[c], &lo[c]);
    }
}

/* Output keys are laid out [row][curve].  curve: 0 Hilbert, 1 Z-order. */
int hco_keys_ex(const uint8_t *rows, int64_t nrows, int dim, const uint16_t *perm,
                int curves, int dpc, int bits, int curve, uint64_t *hi, uint64_t *lo)
{
    if (bits != 8 || dpc < 1 || dpc > 16 || curves * dpc > dim || curve < 0 || curve > 1)
        return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; r++)
        row_keys(rows + r * dim, perm, curves, dpc, curve, hi + r * curves, lo + r * curves);
    return 0;
}

int hco_keys(const uint8_t *rows, int64_t nrows, int dim, const uint16_t *perm,
             int curves, int dpc, int bits, uint64_t *hi, uint64_t *lo)
{
    return hco_keys_ex(rows, nrows, dim, perm, curves, dpc, bits, 0, hi, lo);
}

/* ------------------------------------------------------------------------ */
/* Index build (Alg. 1): per curve, <key, id> sorted by (key, id)           */
/* ------------------------------------------------------------------------ */

typedef struct { u128 key; uint32_t id; } entry;

static int cmp_entry(const void *a, const void *b)
{
    const entry *x = (const entry *)a, *y = (const entry *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Output lists laid out [curve][n].  curve: 0 Hilbert, 1 Z-order. */
int hco_build_ex(const uint8_t *db, int64_t n, int dim, const uint16_t *perm,
                 int curves, int dpc, int bits, int curve,
                 uint64_t *shi, uint64_t *slo, uint32_t *sids)
{
    if (bits != 8 || dpc < 1 || dpc > 16 || curves * dpc > dim || curve < 0 || curve > 1)
        return -1;
    uint64_t *khi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n * curves + 1));
    uint64_t *klo = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n * curves + 1));
    if (!khi || !klo) { free(khi); free(klo); return -2; }
    hco_keys_ex(db, n, dim, perm, curves, dpc, bits, curve, khi, klo);
    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < curves; c++) {
        entry *e = (entry *)malloc(sizeof(entry) * (size_t)(n + 1));
        if (!e) { fail = 1; continue; }
        for (int64_t i = 0; i < n; i++) {
            e[i].key = ((u128)khi[i * curves + c] << 64) | klo[i * curves + c];
            e[i].id = (uint32_t)i;
        }
        qsort(e, (size_t)n, sizeof(entry), cmp_entry);
        for (int64_t i = 0; i < n; i++) {
            shi[c * n + i] = (uint64_t)(e[i].key >> 64);
            slo[c * n + i] = (uint64_t)e[i].key;
            sids[c * n + i] = e[i].id;
        }
        free(e);
    }
    free(khi);
    free(klo);
    return fail ? -2 : 0;
}

int hco_build(const uint8_t *db, int64_t n, int dim, const uint16_t *perm,
              int curves, int dpc, int bits,
              uint64_t *shi, uint64_t *slo, uint32_t *sids)
{
    return hco_build_ex(db, n, dim, perm, curves, dpc, bits, 0, shi, slo, sids);
}

/* ------------------------------------------------------------------------ */
/* Binary search: number of list entries whose key is < qkey                */
/* ------------------------------------------------------------------------ */

int64_t hco_lower_bound(const uint64_t *hi, const uint64_t *lo, int64_t n,
                        uint64_t qhi, uint64_t qlo)
{
    u128 q = ((u128)qhi << 64) | qlo;
    int64_t a = 0, b = n;
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        u128 k = ((u128)hi[mid] << 64) | lo[mid];
        if (k < q)
            a = mid + 1;
        else
            b = mid;
    }
    return a;
}

/* Index description shared by the query-side routines. */
typedef struct {
    const uint64_t *shi, *slo;   /* [curve][n] */
    const uint32_t *sids;        /* [curve][n] */
    const uint8_t *db;           /* [n][dim]   */
    int64_t n;
    int dim, curves, dpc, bits;
    const uint16_t *perm;
    int curve;                   /* 0 Hilbert, 1 Z-order */
} oindex;

static void query_positions(const oindex *ix, const uint8_t *q,
                            u128 *qkey, int64_t *pos)
{
    uint64_t hi[64], lo[64];
    row_keys(q, ix->perm, ix->curves, ix->dpc, ix->curve, hi, lo);
    for (int c = 0; c < ix->curves; c++) {
        qkey[c] = ((u128)hi[c] << 64) | lo[c];
        pos[c] = hco_lower_bound(ix->shi + c * ix->n, ix->slo + c * ix->n,
                                 ix->n, hi[c], lo[c]);
    }
}

int hco_positions(const uint64_t *shi, const uint64_t *slo, int64_t n,
                  int dim, const uint16_t *perm, int curves, int dpc, int bits, int curve,
                  const uint8_t *queries, int64_t nq, int64_t *pos_out)
{
    if (curves > 64) return -1;
    oindex ix = { shi, slo, NULL, NULL, n, dim, curves, dpc, bits, perm, curve };
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < nq; qi++) {
        u128 qkey[64];
        query_positions(&ix, queries + qi * dim, qkey, pos_out + qi * curves);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Candidates (Alg. 2): union over curves of the positional windows          */
/* ------------------------------------------------------------------------ */

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Collects the window ids of every curve, sorts them and drops repeats.
 * Returns the number of distinct ids written to `out` (capacity >= 2*w*curves). */
static int64_t candidate_set(const oindex *ix, const int64_t *pos, int64_t w,
                             uint32_t *out)
{
    int64_t m = 0;
    for (int c = 0; c < ix->curves; c++) {
        int64_t a = pos[c] - w < 0 ? 0 : pos[c] - w;           /* side < qkey  */
        int64_t b = pos[c] + w > ix->n ? ix->n : pos[c] + w;    /* side >= qkey */
        for (int64_t r = a; r < b; r++)
            out[m++] = ix->sids[c * ix->n + r];
    }
    qsort(out, (size_t)m, sizeof(uint32_t), cmp_u32);
    int64_t u = 0;
    for (int64_t i = 0; i < m; i++)
        if (u == 0 || out[u - 1] != out[i])
            out[u++] = out[i];
    return u;
}

/* counts[q] = |C_q|; ids[q*stride ...] = C_q ascending (stride >= 2*w_q*curves). */
int hco_candidates(const uint64_t *shi, const uint64_t *slo, const uint32_t *sids,
                   int64_t n, int dim, const uint16_t *perm, int curves, int dpc,
                   int bits, int curve, const uint8_t *queries, int64_t nq, const uint32_t *w,
                   uint32_t *counts, uint32_t *ids, int64_t stride)
{
    if (curves > 64) return -1;
    oindex ix = { shi, slo, sids, NULL, n, dim, curves, dpc, bits, perm, curve };
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; qi++) {
        u128 qkey[64];
        int64_t pos[64];
        query_positions(&ix, queries + qi * dim, qkey, pos);
        int64_t cap = 2 * (int64_t)w[qi] * curves;
        if (cap > stride) { bad = 1; counts[qi] = 0; continue; }
        uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
        int64_t u = candidate_set(&ix, pos, w[qi], buf);
        counts[qi] = (uint32_t)u;
        memcpy(ids + qi * stride, buf, sizeof(uint32_t) * (size_t)u);
        free(buf);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Distances (Eq. 2, squared) and ordered results                           */
/* ------------------------------------------------------------------------ */

static uint32_t sqdist(const uint8_t *a, const uint8_t *b, int dim)
{
    uint32_t s = 0;
    for (int j = 0; j < dim; j++) {
        int32_t d = (int32_t)a[j] - (int32_t)b[j];
        s += (uint32_t)(d * d);
    }
    return s;
}

typedef struct { uint32_t d, id; } hit;

static int cmp_hit(const void *a, const void *b)
{
    const hit *x = (const hit *)a, *y = (const hit *)b;
    if (x->d != y->d) return (x->d > y->d) - (x->d < y->d);
    return (x->id > y->id) - (x->id < y->id);
}

/* Alg. 2: the k candidates closest to q, by (distance, id). */
int hco_search(const uint64_t *shi, const uint64_t *slo, const uint32_t *sids,
               const uint8_t *db, int64_t n, int dim, const uint16_t *perm,
               int curves, int dpc, int bits, int curve, const uint8_t *queries,
               int64_t nq, int k, const uint32_t *w, uint32_t *out_ids,
               uint32_t *out_dists)
{
    if (curves > 64 || k < 1) return -1;
    oindex ix = { shi, slo, sids, db, n, dim, curves, dpc, bits, perm, curve };
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; qi++) {
        const uint8_t *q = queries + qi * dim;
        u128 qkey[64];
        int64_t pos[64];
        query_positions(&ix, q, qkey, pos);
        int64_t cap = 2 * (int64_t)w[qi] * curves;
        uint32_t *cand = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
        int64_t u = candidate_set(&ix, pos, w[qi], cand);
        hit *h = (hit *)malloc(sizeof(hit) * (size_t)(u + 1));
        for (int64_t i = 0; i < u; i++) {
            h[i].id = cand[i];
            h[i].d = sqdist(q, db + (int64_t)cand[i] * dim, dim);
        }
        qsort(h, (size_t)u, sizeof(hit), cmp_hit);
        for (int j = 0; j < k; j++) {
            out_ids[qi * k + j] = j < u ? h[j].id : PAD;
            out_dists[qi * k + j] = j < u ? h[j].d : PAD;
        }
        free(h);
        free(cand);
    }
    return 0;
}

/* Eq. (3): exact k nearest over the whole database, ties broken by id. */
int hco_brute_force(const uint8_t *db, int64_t n, int dim, const uint8_t *queries,
                    int64_t nq, int k, uint32_t *out_ids, uint32_t *out_dists)
{
    if (k < 1) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; qi++) {
        const uint8_t *q = queries + qi * dim;
        hit *best = (hit *)malloc(sizeof(hit) * (size_t)k);
        for (int j = 0; j < k; j++) { best[j].d = PAD; best[j].id = PAD; }
        for (int64_t i = 0; i < n; i++) {
            hit h = { sqdist(q, db + i * dim, dim), (uint32_t)i };
            if (cmp_hit(&h, &best[k - 1]) >= 0)
                continue;
            int j = k - 1;                       /* insertion into sorted list */
            while (j > 0 && cmp_hit(&h, &best[j - 1]) < 0) {
                best[j] = best[j - 1];
                j--;
            }
            best[j] = h;
        }
        for (int j = 0; j < k; j++) {
            out_ids[qi * k + j] = best[j].id;
            out_dists[qi * k + j] = best[j].d;
        }
        free(best);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Labels: the smallest per-side window w whose candidates hold the exact    */
/* top-k.  j is in curve c's window iff r_c(j) <= w, with                   */
/*   r_c(j) = pos_c - rank_c(j)      if rank_c(j) <  pos_c                   */
/*          = rank_c(j) - pos_c + 1  otherwise,                              */
/* so the label is max over j in the exact top-k of min over c of r_c(j).   */
/* ------------------------------------------------------------------------ */

int hco_labels(const uint64_t *shi, const uint64_t *slo, const uint32_t *sids,
               int64_t n, int dim, const uint16_t *perm, int curves, int dpc,
               int bits, int curve, const uint8_t *queries, int64_t nq, int k,
               const uint32_t *truth_ids, uint32_t *labels)
{
    if (curves > 64) return -1;
    uint32_t *rank = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n * curves + 1));
    if (!rank) return -2;
    for (int c = 0; c < curves; c++)
        for (int64_t r = 0; r < n; r++)
            rank[c * n + sids[c * n + r]] = (uint32_t)r;
    oindex ix = { shi, slo, sids, NULL, n, dim, curves, dpc, bits, perm, curve };
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < nq; qi++) {
        u128 qkey[64];
        int64_t pos[64];
        query_positions(&ix, queries + qi * dim, qkey, pos);
        int64_t need = 0;
        for (int j = 0; j < k; j++) {
            uint32_t id = truth_ids[qi * k + j];
            if (id == PAD) continue;
            int64_t best = INT64_MAX;
            for (int c = 0; c < curves; c++) {
                int64_t rk = rank[c * n + id];
                int64_t r = rk < pos[c] ? pos[c] - rk : rk - pos[c] + 1;
                if (r < best) best = r;
            }
            if (best > need) need = best;
        }
        labels[qi] = (uint32_t)need;
    }
    free(rank);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Features of the learned probe depth (24 per query, FP64)                  */
/*   [0..5]   min over curves of log2(1+|key_c[pos_c+o'] - qkey_c|),         */
/*            o in {-64,-8,-1,+1,+8,+64}, o' = o (o<0) or o-1 (o>0)          */
/*   [6..11]  mean over curves of the same                                   */
/*   [12..19] log2(1 + squared distance to the entry at pos_c), per curve    */
/*   [20]     log2(k)                                                        */
/*   [21..23] max over curves of log2(1 + key_c[pos_c+s-1] - key_c[pos_c-s]), */
/*            s in {1, 8, 64}                                                */
/* Every list index is clamped to [0, n-1].                                  */
/* ------------------------------------------------------------------------ */

static int64_t clampi(int64_t v, int64_t n)
{
    return v < 0 ? 0 : (v > n - 1 ? n - 1 : v);
}

static double lg1p128(u128 g)
{
    return log2(1.0 + (double)g);
}

int hco_features(const uint64_t *shi, const uint64_t *slo, const uint32_t *sids,
                 const uint8_t *db, int64_t n, int dim, const uint16_t *perm,
                 int curves, int dpc, int bits, int curve, const uint8_t *queries,
                 int64_t nq, const uint32_t *k, double *feat)
{
    if (curves != 8 || n < 1) return -1;
    static const int offs[6] = { -64, -8, -1, 1, 8, 64 };
    static const int spans[3] = { 1, 8, 64 };
    oindex ix = { shi, slo, sids, db, n, dim, curves, dpc, bits, perm, curve };
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < nq; qi++) {
        const uint8_t *q = queries + qi * dim;
        double *f = feat + qi * 24;
        u128 qkey[64];
        int64_t pos[64];
        query_positions(&ix, q, qkey, pos);
        for (int o = 0; o < 6; o++) {
            double mn = INFINITY, sum = 0.0;
            for (int c = 0; c < curves; c++) {
                int64_t at = clampi(pos[c] + (offs[o] < 0 ? offs[o] : offs[o] - 1), n);
                u128 kk = ((u128)shi[c * n + at] << 64) | slo[c * n + at];
                u128 g = kk > qkey[c] ? kk - qkey[c] : qkey[c] - kk;
                double v = lg1p128(g);
                if (v < mn) mn = v;
                sum += v;
            }
            f[o] = mn;
            f[6 + o] = sum / curves;
        }
        for (int c = 0; c < curves; c++) {
            uint32_t id = sids[c * n + clampi(pos[c], n)];
            f[12 + c] = log2(1.0 + (double)sqdist(q, db + (int64_t)id * dim, dim));
        }
        f[20] = log2((double)k[qi]);
        for (int s = 0; s < 3; s++) {
            double mx = -INFINITY;
            for (int c = 0; c < curves; c++) {
                int64_t a = clampi(pos[c] - spans[s], n);
                int64_t b = clampi(pos[c] + spans[s] - 1, n);
                u128 ka = ((u128)shi[c * n + a] << 64) | slo[c * n + a];
                u128 kb = ((u128)shi[c * n + b] << 64) | slo[c * n + b];
                double v = lg1p128(kb - ka);
                if (v > mx) mx = v;
            }
            f[21 + s] = mx;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* MLP for the probe depth: in -> h1 -> h2 -> 1, ReLU, FP64.                 */
/* Parameter vector: W1[h1][in], b1[h1], W2[h2][h1], b2[h2], W3[h2], b3.    */
/* ------------------------------------------------------------------------ */

int64_t hco_mlp_nparams(int in, int h1, int h2)
{
    return (int64_t)h1 * in + h1 + (int64_t)h2 * h1 + h2 + h2 + 1;
}

static void mlp_one(const double *p, const double *x, int in, int h1, int h2,
                    double *a1, double *a2, double *y)
{
    const double *W1 = p, *b1 = W1 + h1 * in;
    const double *W2 = b1 + h1, *b2 = W2 + h2 * h1;
    const double *W3 = b2 + h2, *b3 = W3 + h2;
    for (int o = 0; o < h1; o++) {
        double s = b1[o];
        for (int i = 0; i < in; i++) s += W1[o * in + i] * x[i];
        a1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < h2; o++) {
        double s = b2[o];
        for (int i = 0; i < h1; i++) s += W2[o * h1 + i] * a1[i];
        a2[o] = s > 0.0 ? s : 0.0;
    }
    double s = b3[0];
    for (int i = 0; i < h2; i++) s += W3[i] * a2[i];
    *y = s;
}

int hco_mlp_forward(const double *params, const double *x, int64_t batch,
                    int in, int h1, int h2, double *y)
{
    if (h1 > 1024 || h2 > 1024) return -1;
    for (int64_t b = 0; b < batch; b++) {
        double a1[1024], a2[1024];
        mlp_one(params, x + b * in, in, h1, h2, a1, a2, &y[b]);
    }
    return 0;
}

/* Loss = mean over the batch of (y_hat - y)^2; grad has hco_mlp_nparams entries. */
int hco_mlp_loss_grad(const double *params, const double *x, const double *y,
                      int64_t batch, int in, int h1, int h2,
                      double *grad, double *loss)
{
    if (h1 > 1024 || h2 > 1024 || batch < 1) return -1;
    int64_t np = hco_mlp_nparams(in, h1, h2);
    memset(grad, 0, sizeof(double) * (size_t)np);
    double *gW1 = grad, *gb1 = gW1 + h1 * in;
    double *gW2 = gb1 + h1, *gb2 = gW2 + h2 * h1;
    double *gW3 = gb2 + h2, *gb3 = gW3 + h2;
    const double *W2 = params + h1 * in + h1;
    const double *W3 = W2 + h2 * h1 + h2;
    double total = 0.0;
    for (int64_t b = 0; b < batch; b++) {
        const double *xb = x + b * in;
        double a1[1024], a2[1024], d1[1024], d2[1024], out;
        mlp_one(params, xb, in, h1, h2, a1, a2, &out);
        double e = out - y[b];
        total += e * e;
        double dy = 2.0 * e / (double)batch;            /* dL/dy_hat */
        gb3[0] += dy;
        for (int i = 0; i < h2; i++) {
            gW3[i] += dy * a2[i];
            d2[i] = a2[i] > 0.0 ? dy * W3[i] : 0.0;      /* through ReLU */
        }
        for (int o = 0; o < h2; o++) {
            gb2[o] += d2[o];
            for (int i = 0; i < h1; i++) gW2[o * h1 + i] += d2[o] * a1[i];
        }
        for (int i = 0; i < h1; i++) {
            double s = 0.0;
            for (int o = 0; o < h2; o++) s += W2[o * h1 + i] * d2[o];
            d1[i] = a1[i] > 0.0 ? s : 0.0;
        }
        for (int o = 0; o < h1; o++) {
            gb1[o] += d1[o];
            for (int i = 0; i < in; i++) gW1[o * in + i] += d1[o] * xb[i];
        }
    }
    *loss = total / (double)batch;
    return 0;
}

/* One Adam step (Kingma & Ba, 2015) with bias correction at step t >= 1. */
int hco_adam_step(double *theta, double *m, double *v, const double *g,
                  int64_t np, int64_t t, double lr, double beta1, double beta2,
                  double eps)
{
    if (t < 1) return -1;
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < np; i++) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}
