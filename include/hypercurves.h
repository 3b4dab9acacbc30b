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
/* hipEvent_t, passed opaquely. */
typedef void *hc_event;

/* Kinds of space-filling curve: the Hilbert curve of the method and, as a
 * comparison, the Z-order curve, whose key intercalates the coordinates' bits
 * (Sec. 2.2.1); both keys have the bit layout below. */
#define HC_CURVE_HILBERT 0u
#define HC_CURVE_ZORDER 1u

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
    uint32_t curve;           /* HC_CURVE_HILBERT (0, the method's) or
                                 HC_CURVE_ZORDER; keys of both kinds share the
                                 bit layout below */
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
 * (4 B), a 64-ary table of sampled keys (about n/63 keys), every 8th key and
 * every 512th key (n/8 + n/512 keys) that the search uses to locate a key in
 * a few coalesced probes. */
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

/* Rows appended to the database, inserted without a rebuild (Alg. 1 may run
 * incrementally, Sec. 3.1, and the index builder/updater pipeline adds
 * arriving vectors to a live index, Sec. 4.1; Alg. 1 defines the lists that
 * result).  d_db holds n + m rows whose first n are the
 * rows idx was built over (the buffer may be a new one); rows n .. n + m - 1
 * are inserted.  The new index goes to d_index (hc_insert_bytes: at least
 * index_bytes, 256-byte aligned, not overlapping idx's buffer); idx and its
 * buffer are only read and stay valid.  Per curve, the appended rows' keys are
 * sorted by (key, id) and merged with the old list (every appended id is
 * larger than every old one, so at an equal key the old entry comes first),
 * then the sampled-key table is rebuilt: the result equals hc_build_index
 * over all n + m rows, bit for bit.  Scratch: hc_insert_bytes' scratch_bytes,
 * 256-byte aligned.  Synchronises the stream once per curve.  Errors: null
 * or misaligned pointers, m = 0, overlapping buffers -> HC_ERR_INVALID;
 * n + m >= 2^32 - 1 -> HC_ERR_UNSUPPORTED; small buffers -> HC_ERR_SIZE. */
hc_status hc_insert_bytes(const hc_index *idx, uint64_t m, size_t *index_bytes,
                          size_t *scratch_bytes);
hc_status hc_insert_rows(const hc_index *idx, const uint8_t *d_db, uint64_t m, void *d_index,
                         size_t index_bytes, void *d_scratch, size_t scratch_bytes,
                         hc_stream stream, hc_index **out);

/* ---------------------------------------------------------------------- */
/* Host-core search (the CPU side of the cooperative scheduler, Sec. 6)    */
/* ---------------------------------------------------------------------- */

/* The paper's scheduler (Alg. 3) answers a request on a CPU core when the
 * ready requests are few enough for the cores, and batches it for the GPU
 * otherwise.  These calls give the CPU side: host copies of the curve lists
 * and Alg. 2 over them.  They never replace the GPU search: the caller chooses
 * the host path per request.
 *
 * hc_host_index_bytes: bytes of the host copy (per curve n keys of 16 B, then
 * per curve n ids).  hc_host_index_copy: copies the lists of idx into h_index
 * (caller-owned host memory, at least those bytes) and waits for the copy;
 * HC_ERR_SIZE if too small. */
hc_status hc_host_index_bytes(const hc_index *idx, size_t *bytes);
hc_status hc_host_index_copy(const hc_index *idx, void *h_index, size_t bytes,
                             hc_stream stream);

/* Alg. 2 on the calling thread for nq queries in host memory (nq x 128 uint8)
 * against h_index (from hc_host_index_copy of idx) and h_db (the n x 128
 * database in host memory): w = h_w[q] (or w_fixed), k = h_k[q] (or k_fixed;
 * h_k entries are clamped to [1, k_stride]).  Row q of h_out_ids /
 * h_out_dists (nq x k_stride) holds the k results, then 0xFFFFFFFF: the same
 * rows hc_search_uneven writes, bit for bit.  Calls on distinct output
 * buffers may run on concurrent threads.  Errors: null pointers, k_stride
 * outside [1, HC_K_MAX], k_fixed outside [1, k_stride] (without h_k) ->
 * HC_ERR_INVALID. */
hc_status hc_host_search(const hc_index *idx, const void *h_index, const uint8_t *h_db,
                         const uint8_t *h_queries, uint32_t nq, uint32_t w_fixed,
                         const uint32_t *h_w, uint32_t k_fixed, const uint32_t *h_k,
                         uint32_t k_stride, uint32_t *h_out_ids, uint32_t *h_out_dists);

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

/* Scratch bytes hc_search_batch needs for nq queries on either path with
 * k <= 16 (also valid for hc_positions, hc_candidates and the learned-depth
 * entry points).  A smaller buffer of at least nq * curves * 16 bytes
 * restricts the search to the gather path.
 * hc_search_scratch_bytes_k: the same for k up to k_max (1..HC_K_MAX): with
 * 16 < k_max the banded path's two-pass buffers are included (k up to
 * HC_BAND_K_MAX, row store attached; about 8 KiB + 512 B x curves per query).
 * Up to 4,096 queries it also holds the work items of a small batch's gather
 * search (256 B x k_max per query; see HC_PATH_AUTO).
 * Errors: null pointers, k_max outside [1, HC_K_MAX] -> HC_ERR_INVALID. */
hc_status hc_search_scratch_bytes(const hc_index *idx, uint32_t nq, size_t *bytes);
hc_status hc_search_scratch_bytes_k(const hc_index *idx, uint32_t nq, uint32_t k_max,
                                    size_t *bytes);

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

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as hc_search_batch on the gather path (HC_PATH_GATHER, identical
 * results), with the query keys kept in a scratch array the library owns, so
 * the caller passes only the queries and the outputs.  The array,
 * HC_NOALLOC_SCRATCH_BYTES (4 MiB), is a static device array: each GPU the
 * library runs on holds its own copy until the process ends.  Its address on
 * the current device is looked up on the first call on that device (the
 * index's buffers must be on the current device).  Nothing is allocated:
 * no hipMalloc or hipFree, and no library routine that allocates.  Limit:
 * nq * curves * 16 <= HC_NOALLOC_SCRATCH_BYTES (32,768 queries with 8
 * curves), else HC_ERR_SIZE.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller.  Other arguments and errors as in
 * hc_search_batch; a failed symbol lookup returns HC_ERR_HIP. */
#define HC_NOALLOC_SCRATCH_BYTES (4u << 20)
hc_status hc_search_batch_noalloc(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                                  uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                                  uint32_t *d_out_ids, uint32_t *d_out_dists,
                                  hc_stream stream);

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

/* Execution paths of the search; both give identical results.
 *  HC_PATH_GATHER: one wavefront per query gathers its candidates' rows.
 *  HC_PATH_BAND:   per curve, the batch ordered by place in the list; one
 *                  block per 128 or 256 neighbouring queries streams the union of
 *                  their windows once, the distances of every query to every
 *                  streamed row come from the int8 matrix cores, and each
 *                  query keeps the entries inside its own window (for large
 *                  batches with large windows, where one list entry lies in
 *                  many windows).  k <= 16 in one pass.  With the row store
 *                  attached, 16 < k <= HC_BAND_K_MAX in two passes: the
 *                  first keeps the 16 nearest of each half of every window's
 *                  rows, whose k-th nearest distinct key bounds the result;
 *                  the second collects every pair of the windows at or below
 *                  that bound (up to 1,024 per query), whose k nearest
 *                  distinct keys are the result.  A query left without a
 *                  bound or with more pairs is answered by the gather kernel.
 *  HC_PATH_AUTO:   banded when 2 w nq >= 3.5 n (w = w_fixed or the hint), the
 *                  batch makes at least 512 blocks (nq / 128 or nq / 256 per
 *                  curve, times curves; with the row store at least 256,
 *                  counting the blocks a small batch's groups are dealt out
 *                  over, up to 4 each), k <= 16 (or
 *                  k <= HC_BAND_K_MAX with the row store) and the scratch holds
 *                  hc_search_scratch_bytes_k for that k; else gather.  A
 *                  gather search of a batch under a third of the device's
 *                  resident gather wavefronts (and at most 4,096 queries),
 *                  with 2 w curves >= 32,768 window slots per query and a
 *                  scratch of hc_search_scratch_bytes_k for that k, runs as
 *                  the work items of hc_search_uneven instead (each query's
 *                  windows cut into pieces that many wavefronts stream at
 *                  once, then merged); the results are the same.
 * hc_search_encoded is hc_search_encoded_ex with HC_PATH_AUTO. */
#define HC_BAND_K_MAX 128u
#define HC_PATH_AUTO 0u
#define HC_PATH_GATHER 1u
#define HC_PATH_BAND 2u
hc_status hc_search_choose_path(const hc_index *idx, uint32_t nq, uint32_t k, uint32_t w,
                                size_t scratch_bytes, uint32_t *path);
hc_status hc_search_encoded_ex(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                               uint32_t k, uint32_t w_fixed, const uint32_t *d_w,
                               uint32_t *d_out_ids, uint32_t *d_out_dists, void *d_scratch,
                               size_t scratch_bytes, uint32_t path, hc_stream stream);

/* Timing aid for the search's main kernel (the distance and top-k work of
 * Alg. 2; its helpers are left out).  With begin and end set (hipEvent_t
 * handles created by the caller), every later hc_search_encoded(_ex) and
 * hc_search_batch call on idx records begin on its stream just before that
 * kernel (the gather kernel, or the banded kernel on the banded path) and end
 * just after it, so hipEventElapsedTime(begin, end) is the kernel's duration.
 * Both NULL turns it off.  The events stay the caller's and must outlive the
 * calls that record them.  A measurement aid: it makes the handle stateful
 * and is not thread-safe per handle (searches on several streams or threads
 * at once would record the same pair), so leave it off outside timing runs.  HC_ERR_INVALID if idx is NULL or only one event is given;
 * a failed record returns HC_ERR_HIP from the search. */
hc_status hc_index_set_kernel_events(hc_index *idx, hc_event begin, hc_event end);

/* Row store: for the banded path, each curve's rows copied in list order
 * (stored as 127 - x, the form the matrix products take) with floor(crow / 2)
 * and crow mod 2 for crow = sum x (x - 256), and the list's ids, each curve
 * padded to a multiple of 256 entries.  The banded search then copies its
 * tiles from contiguous memory straight into LDS instead of gathering rows by
 * id.  It trades memory for locality: about curves * n * 137 B (11.0 GB at
 * n = 10^7).  Results are unchanged.
 *
 * hc_rowstore_bytes: bytes of the store.  hc_rowstore_build: fills d_rows
 * (caller-owned device memory, 256-byte aligned, at least those bytes) from
 * the index and its database on `stream`, and attaches it to idx: searches
 * enqueued after it on the same stream use it (on other streams, after the
 * stream has been synchronised).  The caller keeps d_rows alive while
 * attached.  hc_rowstore_detach: the banded path gathers rows by id again.
 * An index made by hc_insert_rows starts without a store.  Errors: null or
 * misaligned pointers -> HC_ERR_INVALID; too small -> HC_ERR_SIZE. */
hc_status hc_rowstore_bytes(const hc_index *idx, size_t *bytes);
hc_status hc_rowstore_build(hc_index *idx, void *d_rows, size_t bytes, hc_stream stream);
hc_status hc_rowstore_detach(hc_index *idx);

/* Uneven batches: every query has its own w and its own k.  A query's window
 * slots (up to 16 w) are cut into work items of at most chunk_slots slots
 * (at most max_split items per query; the chunk grows beyond that); a
 * persistent grid of wavefronts takes items from a counter in scratch, and a
 * merge kernel combines the items of a query, dropping repeated ids.  Nothing
 * waits on the host, so the call may be captured in a HIP graph.
 * Fields set to 0 take defaults: chunk_slots 8192, max_split 32,
 * blocks_per_cu = the occupancy limit of the work kernel. */
typedef struct {
    uint32_t chunk_slots;
    uint32_t max_split;
    uint32_t blocks_per_cu;
} hc_uneven_cfg;

hc_status hc_uneven_scratch_bytes(const hc_index *idx, uint32_t nq, uint32_t k_stride,
                                  const hc_uneven_cfg *cfg, size_t *bytes);

/* Alg. 2 per query with w = d_w[q] (or w_fixed) and k = d_k[q] (or k_fixed;
 * device entries are clamped to [1, k_stride]).  Row q of d_out_ids /
 * d_out_dists (nq x k_stride) holds the query's k results then 0xFFFFFFFF up
 * to k_stride.  1 <= k_stride <= HC_K_MAX.  d_scratch must be 256-byte aligned
 * and hc_uneven_scratch_bytes long (it holds the query keys, positions, item
 * offsets, the work counter and nq * max_split * k_stride partial results). */
hc_status hc_search_uneven(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                           uint32_t w_fixed, const uint32_t *d_w, uint32_t k_fixed,
                           const uint32_t *d_k, uint32_t k_stride, uint32_t *d_out_ids,
                           uint32_t *d_out_dists, void *d_scratch, size_t scratch_bytes,
                           const hc_uneven_cfg *cfg, hc_stream stream);

/* ---------------------------------------------------------------------- */
/* Parity / inspection exports: the same kernels, stopping early           */
/* ---------------------------------------------------------------------- */

/* Keys of every row and curve (Sec. 2.2.1, the keys of Alg. 1): d_keys receives
 * nrows x curves keys as {hi, lo} pairs, laid out [row][curve]. */
hc_status hc_encode_keys(const hc_params *p, const uint8_t *d_rows, uint64_t nrows,
                         uint64_t *d_keys, hc_stream stream);

/* pos_c of every query and curve (nq x curves uint32, [query][curve]). */
hc_status hc_positions(const hc_index *idx, const uint8_t *d_queries, uint32_t nq,
                       uint32_t *d_pos, void *d_scratch, size_t scratch_bytes,
                       hc_stream stream);

/* Candidate set of every query (the union of Alg. 2), unordered: d_counts[q]
 * = its size, d_ids[q*stride ...] its ids.  1 <= stride <= 4096 (the union is
 * built in one LDS table; HC_ERR_UNSUPPORTED beyond).  With d_w == NULL,
 * stride < 16 * w_fixed -> HC_ERR_SIZE.  With d_w, a query whose window slots
 * (the sum over curves of its clamped window lengths, at most 16 w) exceed
 * stride gets d_counts[q] = 0xFFFFFFFF and its row is left unwritten. */
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

/* ---------------------------------------------------------------------- */
/* Learned probe depth                                                     */
/*                                                                        */
/* The paper's probe depth is one value for every query.  These entry     */
/* points predict a window w per query with a small MLP over cheap        */
/* features of the query's neighbourhood in the curves, and produce the   */
/* labels it is trained on.  Search stays exact given the w array.        */
/* ---------------------------------------------------------------------- */

#define HC_FEATURES 24u
#define HC_MLP_PARAMS 5825u   /* 24 -> 64 -> 64 -> 1 */

/* Place of every id in every list: d_rank[id * curves + c] = r such that curve
 * c's list holds id at r (n * curves uint32). */
hc_status hc_index_ranks(const hc_index *idx, uint32_t *d_rank, hc_stream stream);

/* Label of each query: the smallest w whose candidate union holds all of its
 * exact top-k (d_truth_ids, nq x k, from hc_brute_force; 0xFFFFFFFF = none).
 * Curve c's window of w holds id j iff r_c(j) <= w, with r_c(j) =
 * pos_c - rank_c(j) when rank_c(j) < pos_c and rank_c(j) - pos_c + 1
 * otherwise; so label = max over j of min over c of r_c(j).  A search with w
 * >= label returns exactly the truth (the union then contains it, and the
 * top-k of a superset of it is itself). */
hc_status hc_labels(const hc_index *idx, const uint32_t *d_rank, const uint8_t *d_queries,
                    uint32_t nq, uint32_t k, const uint32_t *d_truth_ids, uint32_t *d_labels,
                    void *d_scratch, size_t scratch_bytes, hc_stream stream);

/* Size of every query's candidate set (the union of Alg. 2) for any w: a
 * window slot of curve c counts unless its id lies in the window of a curve
 * c' < c.  w as in hc_search_batch. */
hc_status hc_union_sizes(const hc_index *idx, const uint32_t *d_rank, const uint8_t *d_queries,
                         uint32_t nq, uint32_t w_fixed, const uint32_t *d_w, uint32_t *d_counts,
                         void *d_scratch, size_t scratch_bytes, hc_stream stream);

/* HC_FEATURES floats per query (d_feat, nq x 24), FP32; every list place is
 * clamped to [0, n-1]:
 *  [0..5]   min over curves of log2(1 + |key_c[pos_c + o'] - qkey_c|) for
 *           o = -64, -8, -1, +1, +8, +64 (o' = o if o < 0, else o - 1)
 *  [6..11]  the mean over curves of the same
 *  [12..19] log2(1 + squared distance to the entry at pos_c), curve c
 *  [20]     log2(k) (d_k[q] if d_k != NULL, else k)
 *  [21..23] max over curves of log2(1 + key_c[pos_c + s - 1] - key_c[pos_c - s])
 *           for s = 1, 8, 64. */
hc_status hc_features(const hc_index *idx, const uint8_t *d_queries, uint32_t nq, uint32_t k,
                      const uint32_t *d_k, float *d_feat, void *d_scratch, size_t scratch_bytes,
                      hc_stream stream);

/* MLP inference.  Parameters (BF16, HC_MLP_PARAMS): W1[64][24], b1[64],
 * W2[64][64], b2[64], W3[64], b3; ReLU after both hidden layers; FP32
 * arithmetic.  Inputs are standardised as (f - mean) / std with d_norm =
 * {mean[24], std[24]} (NULL = raw).  y = MLP(x) estimates log2 of the label;
 * w = clamp(ceil(2^(y + delta)), w_min, w_max), or w_fallback when a
 * standardised feature or y + delta is not finite (y is then NaN).  d_w_out (nq uint32) and/or d_y_out (nq float) may be NULL. */
hc_status hc_mlp_infer(const uint16_t *d_params_bf16, const float *d_norm, const float *d_feat,
                       uint32_t nq, float delta, uint32_t w_min, uint32_t w_max,
                       uint32_t w_fallback, uint32_t *d_w_out, float *d_y_out, hc_stream stream);

/* Training.  A batch is rows d_idx[0..batch) of d_x (NULL = rows 0..batch-1),
 * standardised with d_norm.  hc_mlp_forward writes y (batch floats).
 * hc_mlp_backward computes the gradient of loss = mean over the batch of
 * (y - d_target[row])^2 into d_grad (HC_MLP_PARAMS floats, layout of the
 * parameters) and the loss into *d_loss (device, may be NULL); the sums over
 * the batch run in sample order, so the result is deterministic. */
hc_status hc_mlp_train_scratch_bytes(uint32_t batch, size_t *bytes);
hc_status hc_mlp_forward(const uint16_t *d_params_bf16, const float *d_norm, const float *d_x,
                         const uint32_t *d_idx, uint32_t batch, float *d_y, hc_stream stream);
hc_status hc_mlp_backward(const uint16_t *d_params_bf16, const float *d_norm, const float *d_x,
                          const float *d_target, const uint32_t *d_idx, uint32_t batch,
                          float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes,
                          hc_stream stream);

/* One Adam step (Kingma & Ba) at step t >= 1 on FP32 master weights, with bias
 * correction; also writes the BF16 copy the kernels compute with (d_params_bf16,
 * may be NULL; round to nearest even). */
hc_status hc_adam_step(float *d_master, float *d_m, float *d_v, const float *d_grad, uint32_t np,
                       uint32_t t, float lr, float beta1, float beta2, float eps,
                       uint16_t *d_params_bf16, hc_stream stream);

/* Preparation of the training set (caller-side steps of training, run on
 * the device).  hc_mlp_targets: d_y[i] = log2(clamp(d_labels[i], w_min, w_max))
 * (FP64 log2 rounded to FP32), the regression target of the MLP.
 * hc_feature_norm: the standardisation {mean[24], std[24]} of d_feat (rows x
 * 24) into d_norm, FP64 sums in a fixed order (deterministic), std with
 * divisor rows - 1; a std below 1e-3 (a feature constant over the training
 * set) becomes 1.  Errors: null pointers, rows = 0, w_min = 0 or
 * w_min > w_max -> HC_ERR_INVALID. */
hc_status hc_mlp_targets(const uint32_t *d_labels, uint32_t nq, uint32_t w_min, uint32_t w_max,
                         float *d_y, hc_stream stream);
hc_status hc_feature_norm(const float *d_feat, uint32_t rows, float *d_norm, hc_stream stream);

/* FP32 -> BF16, round to nearest even. */
hc_status hc_to_bf16(const float *d_src, uint32_t n, uint16_t *d_dst, hc_stream stream);

/* ---------------------------------------------------------------------- */
/* Measurement aid (not a step of the method)                               */
/* ---------------------------------------------------------------------- */

/* Reads `bytes` of device memory at d_buf once (16-byte aligned, bytes a
 * multiple of 16) with coalesced 16-byte loads from `blocks` blocks of 256
 * threads (1..65536; a few per compute unit fill the device), and writes one
 * word per block to d_sink[0 .. blocks) (the XOR of what the block read), so
 * that no load is dropped.  Timing it gives the streaming-read bandwidth the
 * device achieves.  Errors: null or misaligned pointers, bytes not a multiple
 * of 16, blocks out of range -> HC_ERR_INVALID. */
hc_status hc_read_probe(const void *d_buf, size_t bytes, uint32_t *d_sink, uint32_t blocks,
                        hc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* HYPERCURVES_H */
