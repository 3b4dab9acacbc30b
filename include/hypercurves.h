/*
 * hypercurves.h -- C ABI of the MI355X (gfx950) Multicurves search library.
 *
 * The method is the per-node local search of Hypercurves (Teodoro et al.,
 * arXiv 1209.0410): the Multicurves index of Sec. 3.1.  Each database vector
 * is projected onto `curves` subspaces; each projection gets a Hilbert
 * extended key (Sec. 2.2.1); each curve keeps its <key, id> list sorted
 * (Alg. 1).  A query is projected and keyed the same way, located in every
 * list by binary search, the probe-depth entries nearest its key are taken
 * from every list, and the k candidates closest to the query in Euclidean
 * distance are returned (Alg. 2, Eq. 2, Eq. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory: the library allocates no device memory.  Every `d_` pointer is
 *    device memory owned by the caller (e.g. a torch tensor's data_ptr()),
 *    which must stay alive until the work enqueued on `stream` has finished.
 *    `hc_index` is a small host object holding device pointers into the
 *    caller's index buffer and the caller's database buffer.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = null
 *    stream).  Calls only enqueue work; results are valid once the stream
 *    has been synchronised.  An index may be searched from several streams
 *    at once, each call with its own scratch buffer.
 *  - Errors: arguments are validated before anything is launched; a bad
 *    argument returns HC_ERR_INVALID, a buffer that is too small returns
 *    HC_ERR_SIZE, an unsupported shape HC_ERR_UNSUPPORTED, and a failed HIP
 *    launch or copy HC_ERR_HIP.  No C++ exception crosses the ABI.  Calls on
 *    distinct handles and scratch buffers are thread-safe.
 *  - Shapes: vectors are 128 uint8 dims, rows 128 B apart (the database and
 *    query buffers must be 16-byte aligned).  A curve covers 16 dims at 8
 *    bits each, so its key has 128 bits (order-8 curve of 16 dims,
 *    Sec. 2.2.1: d coordinates of m bits give a d*m-bit key); 1..8 curves.
 *    Ids are database row numbers; n < 2^32 - 1.
 *  - Keys: 128-bit unsigned, stored as two uint64 words {hi, lo} (16 B per
 *    key).  Bit layout (Hilbert index in Skilling's transposed form): most
 *    significant first, for bit level b = 7..0 and for dim i = 0..15 of the
 *    curve, bit b of the transformed coordinate X[i].
 *  - Results: squared Euclidean distance (uint32, exact: 128*255^2 < 2^24)
 *    and id, each query's row ordered by (distance, id) ascending; slots
 *    beyond the number of candidates hold 0xFFFFFFFF in both arrays.
 */
#ifndef HYPERCURVES_H
#define HYPERCURVES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_ERR_INVALID = -1,
    HC_ERR_SIZE = -2,
    HC_ERR_HIP = -3,
    HC_ERR_UNSUPPORTED = -4
} hc_status;

/* hipStream_t, passed opaquely; NULL is the null stream. */
typedef void *hc_stream;

/* Index parameters (Alg. 1 inputs `curves`, `dims[]`, `a`). */
typedef struct {
    uint32_t dim;             /* vector dimension; must be 128 */
    uint32_t curves;          /* number of curves / subindexes, 1..8 */
    uint32_t dims_per_curve;  /* dims of each curve; must be 16 */
    uint32_t bits;            /* bits per coordinate; must be 8 */
    const uint16_t *perm;     /* host array of curves*16 dims: curve c takes
                                 dims perm[16c .. 16c+15] in that order (the
                                 attribution a[c, j] of Alg. 1); each < dim.
                                 NULL = identity (curve c takes dims
                                 16c .. 16c+15).  Copied by the library. */
} hc_params;

typedef struct hc_index hc_index;   /* opaque host handle */

/* Largest k accepted by the search entry points. */
#define HC_K_MAX 256u

const char *hc_status_str(hc_status s);

/* ---------------------------------------------------------------------- */
/* Index build (Alg. 1)                                                    */
/* ---------------------------------------------------------------------- */

/* Bytes of the index buffer for n vectors, and of the scratch buffer that
 * hc_build_index needs.  The index holds, per curve, n keys (16 B), n ids
 * (4 B) and a 64-ary table of sampled keys (about n/63 keys) that the search
 * uses to locate a key in a few coalesced probes. */
hc_status hc_index_bytes(const hc_params *p, uint64_t n, size_t *index_bytes,
                         size_t *build_scratch_bytes);

/* Alg. 1: for every curve c and every row i of d_db (n x 128 uint8), key =
 * C^-1(projection of row i onto curve c); the <key, i> pairs are sorted by
 * (key, i) into d_index (a stable LSD radix sort of the keys, ids ascending
 * on entry).  On success *out receives a new handle, which keeps d_db and
 * d_index (both must outlive it).  Enqueued on `stream`; the call itself
 * synchronises the stream once per curve (to read the digit histograms). */
hc_status hc_build_index(const hc_params *p, const uint8_t *d_db, uint64_t n,
                         void *d_index, size_t index_bytes, void *d_scratch,
                         size_t scratch_bytes, hc_stream stream, hc_index **out);

/* A handle over an index buffer already built by hc_build_index with the same
 * parameters, n and database (e.g. one restored from a file).  Nothing is
 * launched. */
hc_status hc_index_attach(const hc_params *p, const uint8_t *d_db, uint64_t n,
                          void *d_index, size_t index_bytes, hc_index **out);

/* Frees the host handle only (the caller owns every device buffer). */
hc_status hc_index_destroy(hc_index *idx);

/* Device pointers of curve c's sorted list: keys[n] as {hi, lo} uint64 pairs
 * (16 B each) and ids[n]. */
hc_status hc_index_curve(const hc_index *idx, uint32_t c, const uint64_t **d_keys,
                         const uint32_t **d_ids);

/* Number of vectors and curves of the index. */
hc_status hc_index_info(const hc_index *idx, uint64_t *n, uint32_t *curves);

/* ---------------------------------------------------------------------- */
/* Search (Alg. 2)                                                         */
/* ---------------------------------------------------------------------- */

/* Scratch bytes hc_search_batch needs for nq queries (also valid for
 * hc_positions and hc_candidates). */
hc_status hc_search_scratch_bytes(const hc_index *idx, uint32_t nq, size_t *bytes);

/* Alg. 2 for a batch of queries (d_queries: nq x 128 uint8).  Per query and
 * curve c: key = C^-1(projection onto c); pos_c = number of list entries whose
 * key is < the query key; the window is list entries
 * [max(0, pos_c - w), min(n, pos_c + w)) -- w entries on each side of the
 * query's place, the probe-depth 2w split evenly as in the half-list model of
 * Sec. 4.2; the candidates are the union (as a set) of the windows' ids;
 * the k candidates nearest the query (squared Eq. 2, ties by id) are written
 * to d_out_ids / d_out_dists (nq x k, uint32, row-major).
 * w: d_w[q] when d_w != NULL (device, nq entries, any value >= 0), else
 * w_fixed for every query.  When d_w != NULL, w_fixed is a hint of the
 * typical w used to size the work of a block (0 = default).
 * 1 <= k <= HC_K_MAX. */
hc_status hc_search_batch(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                          uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                          uint32_t *d_out_ids, uint32_t *d_out_dists,
                          void *d_scratch, size_t scratch_bytes, hc_stream stream);

/* The two launches of hc_search_batch, for callers that time or overlap them:
 * hc_encode_queries writes the query keys into d_scratch (the keys step of
 * Alg. 2); hc_search_encoded runs the rest of Alg. 2 with the keys already in
 * d_scratch (same queries, same scratch, same stream order).  Arguments as in
 * hc_search_batch. */
hc_status hc_encode_queries(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            void *d_scratch, size_t scratch_bytes, hc_stream stream);
hc_status hc_search_encoded(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                            uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                            uint32_t *d_out_ids, uint32_t *d_out_dists,
                            void *d_scratch, size_t scratch_bytes, hc_stream stream);

/* ---------------------------------------------------------------------- */
/* Parity / inspection exports: the same kernels, stopping early           */
/* ---------------------------------------------------------------------- */

/* Keys of every row and curve (Sec. 2.2.1, Alg. 1 lines 4-9): d_keys receives
 * nrows x curves keys as {hi, lo} pairs, laid out [row][curve]. */
hc_status hc_encode_keys(const hc_params *p, const uint8_t *d_rows, uint64_t nrows,
                         uint64_t *d_keys, hc_stream stream);

/* pos_c of every query and curve (nq x curves uint32, [query][curve]). */
hc_status hc_positions(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                       uint32_t *d_pos, void *d_scratch, size_t scratch_bytes,
                       hc_stream stream);

/* Candidate set of every query (the union of Alg. 2), unordered: d_counts[q]
 * = its size, d_ids[q*stride ...] its ids.  Requires stride >= 16*w for every
 * query's w (HC_ERR_SIZE otherwise when d_w == NULL) and 16*w <= 65536. */
hc_status hc_candidates(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                        uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_counts,
                        uint32_t *d_ids, uint32_t stride, void *d_scratch,
                        size_t scratch_bytes, hc_stream stream);

/* Exact kNN (Eq. 3, ties broken by id) over all n rows, for recall truth and
 * training labels; not on the search path.  Output as hc_search_batch. */
hc_status hc_brute_force_scratch_bytes(uint64_t n, uint32_t nq, uint32_t k,
                                       size_t *bytes);
hc_status hc_brute_force(const uint8_t *d_db, uint64_t n, const uint8_t *d_queries,
                         uint32_t nq, uint32_t k, uint32_t *d_out_ids,
                         uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                         hc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* HYPERCURVES_H */
