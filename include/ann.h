/*
 * ann.h — C ABI of the MI355X filtering stage of a multi-tiered IVF-PQ index.
 *
 * The library implements the GPU-side online search of the paper's
 * multi-tiered index (Sec. 3, steps 1-8), with the PQ codes, the posting-list
 * metadata and the raw vectors all resident in HBM:
 *   step 1  per-query PQ distance table                         (Sec. 2.2)
 *   step 2  top-m nearest posting lists (exact over centroids)  (Sec. 2.1)
 *   step 3  gather the vector IDs of those lists                (Sec. 4.1)
 *   step 5  remove the duplicate IDs replication creates        (Eq. 2, Sec. 5)
 *   step 6  approximate distances by table lookups              (Eq. 1)
 *   step 7  keep the n best (rerank_n, the paper's top-n)
 *   step 8  re-rank those n by exact squared L2, keep the top-k
 *
 * Conventions shared by every entry point:
 *  - Every pointer named d_* is device memory on the index's device; every
 *    other pointer is host memory.  Device arrays are row-major and densely
 *    packed.  `stream` is a hipStream_t (NULL = the null stream).  Work is
 *    enqueued on `stream` and the call returns without synchronising;
 *    outputs are valid once the stream reaches that point.  The library
 *    keeps no caller pointer after the call returns.
 *  - Vector IDs are external IDs: row numbers of the vectors in the index
 *    file.  List IDs are 0..nlist-1.
 *  - Distances are squared Euclidean distances (float32).  Every selection
 *    orders by (distance, id): ties go to the lower ID.
 *  - Queries are float32 [nq, dim].  For uint8 / int8 indexes each query
 *    value is first rounded half to even and saturated to the data type.
 *  - Outputs are padded with id -1 and distance +inf where fewer than the
 *    requested results exist.
 *  - Errors: a non-zero ann_status; ann_last_error() then returns a message
 *    (thread-local, valid until the next call on the same thread).  No
 *    argument is modified on error except that partially enqueued work may
 *    have written outputs.
 */
#ifndef ANN_H
#define ANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ANN_OK = 0,
  ANN_EINVAL = 1,      /* bad argument: shape, k, rerank_n, nprobe, NULL pointer */
  ANN_ENOMEM = 2,      /* device or host allocation failed */
  ANN_EIO = 3,         /* index file cannot be read */
  ANN_EFORMAT = 4,     /* bad magic, version, sizes or checksum */
  ANN_EDEVICE = 5,     /* a HIP runtime call failed */
  ANN_EUNSUPPORTED = 6 /* valid but not supported by this build (e.g. ksub != 256) */
} ann_status;

typedef struct ann_index ann_index; /* opaque */

typedef struct {
  int64_t n;               /* vectors */
  int32_t dim;             /* dimension D */
  int32_t dtype;           /* 0 float32, 1 uint8, 2 int8 */
  int32_t nlist;           /* posting lists */
  int32_t m;               /* PQ subspaces */
  int32_t ksub;            /* codewords per subspace (256) */
  int32_t dsub;            /* D / m */
  int32_t r;               /* max lists per vector (Eq. 2 cap) */
  int32_t int_grid;        /* 1: integer arithmetic is exact on this index */
  int64_t entries;         /* posting-list entries, duplicates included */
  int64_t replica_entries; /* entries that are not a vector's first list */
  int64_t max_list;        /* longest posting list (entries) */
  int64_t hbm_bytes;       /* device memory held by the index */
  int32_t device;
  int32_t max_rerank_n;    /* largest rerank_n accepted */
  int32_t raw_tier;        /* 0: raw vectors in HBM; 1: on pages in pinned host memory */
  int32_t page_bytes;      /* raw tier 1: bytes per page */
  int64_t pages;           /* raw tier 1: pages */
  int64_t host_bytes;      /* raw tier 1: pinned host memory held by the index */
} ann_index_desc;

/*
 * Load options.  raw_tier 0 (default): raw vectors in HBM, by external ID.
 * raw_tier 1: the raw vectors stay in pinned host memory (hipHostMalloc) on
 * pages of page_bytes (0: 4096), laid out by ann_page_layout with each
 * vector's nearest list as its bucket (Sec. 4.3); only their page and slot
 * numbers go to HBM.  Re-ranking then reads whole pages over PCIe (see
 * ann_search_pages); rerank_n is limited to 2048 and ann_rerank is not
 * available.
 */
typedef struct {
  int32_t raw_tier;
  int32_t page_bytes;  /* multiple of 16 in [16, 65536], at least one vector */
} ann_load_cfg;

/*
 * Load an index file (format: the paper's offline output, Sec. 3 / Sec. 4.1:
 * centroids, PQ codebooks, one M-byte code per vector, raw vectors, posting
 * lists of external IDs and each vector's list assignment) onto `device`.
 * The file is validated (magic, version, sizes, CRC32 of every section,
 * list / assignment consistency) and copied to HBM, the code rows reordered
 * by first list, the raw vectors kept in external-ID order.  *out receives an index owned by the
 * caller, freed with ann_free_index.  Errors: ANN_EIO, ANN_EFORMAT,
 * ANN_EUNSUPPORTED (ksub != 256, R > 15, N >= 2^28), ANN_ENOMEM, ANN_EDEVICE.
 */
ann_status ann_load_index(const char* path, int device, ann_index** out);

/* ann_load_index with options (cfg NULL: the defaults).  Errors as
 * ann_load_index; ANN_EINVAL for a bad option, ANN_ENOMEM also when the host
 * pages cannot be allocated. */
ann_status ann_load_index_ex(const char* path, int device, const ann_load_cfg* cfg,
                             ann_index** out);

/* Describe a loaded index.  Errors: ANN_EINVAL (NULL). */
ann_status ann_index_info(const ann_index* ix, ann_index_desc* out);

/* Release every device and host resource of the index (NULL is a no-op).
 * The caller must ensure no enqueued work still uses it. */
void ann_free_index(ann_index* ix);

/* Message of the last error on this thread ("" if none). */
const char* ann_last_error(void);

/*
 * Layout of raw vectors on pages (Sec. 4.3, optimized storage layout), as the
 * host-memory raw tier uses it: vectors are bucketed by bucket_of[v] (the
 * nearest list), ascending ID inside a bucket; a page of page_bytes holds
 * floor(page_bytes / row_bytes) whole vectors.  Every bucket's whole pages
 * come first, bucket by bucket; the leftover tails are then packed onto
 * shared pages -- each new page takes the largest remaining tail, then keeps
 * adding the largest remaining tail that still fits (equal sizes: lower
 * bucket first) -- so no tail is split over two pages.
 *   bucket_of  host int32 [n], values in [0, nbuckets)
 *   page, slot host int32 [n] outputs: page of each vector, position on it
 * Returns the number of pages, or -1 on bad arguments (ann_last_error says
 * which).  Host-only; touches no device.
 */
int64_t ann_page_layout(const int32_t* bucket_of, int64_t n, int32_t nbuckets, int32_t row_bytes,
                        int32_t page_bytes, int32_t* page, int32_t* slot);

/*
 * Steps 1-8 (plain form): search nq queries.
 *   d_queries   float32 [nq, dim]
 *   d_nprobe    int32 [nq] lists to probe per query, or NULL: every query
 *               probes nprobe_max lists.  Values are clamped to
 *               [0, min(nprobe_max, nlist)].
 *   nprobe_max  >= 1, upper bound of the per-query values
 *   k           >= 1 results per query
 *   rerank_n    k <= rerank_n <= max_rerank_n: candidates re-ranked (top-n)
 *   d_out_ids   int64 [nq, k], d_out_dists float32 [nq, k]
 * nq = 0 is a no-op.  Errors: ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE.
 */
ann_status ann_search(ann_index* ix, const float* d_queries, int64_t nq, const int32_t* d_nprobe,
                      int32_t nprobe_max, int32_t k, int32_t rerank_n, int64_t* d_out_ids,
                      float* d_out_dists, void* stream);

/*
 * ann_search for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same steps, arguments, results and errors as ann_search, but the working
 * buffers come from one fixed device array of ann_noalloc_scratch_bytes()
 * bytes (128 MiB) per device, set up when an index is first loaded on that
 * device and held until the process ends.  The call allocates and frees
 * nothing and records no timing events; a batch whose working buffers exceed
 * the array is searched in chunks that fit, one after another on `stream`.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, or threads without ordering) race and may
 * return wrong results; calls ordered on one stream are safe.  The array
 * keeps the last call's contents; nothing in it needs to start at zero.
 * Errors: as ann_search; ANN_EINVAL also when a single query needs more
 * working memory than the array holds.
 */
ann_status ann_search_noalloc(ann_index* ix, const float* d_queries, int64_t nq,
                              const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                              int32_t rerank_n, int64_t* d_out_ids, float* d_out_dists,
                              void* stream);

/* Size in bytes of the per-device array ann_search_noalloc works in. */
size_t ann_noalloc_scratch_bytes(void);

/*
 * Steps 1-8 with step 8 by the heuristic re-ranking of Alg. 1 (change rate
 * of Eq. 3) instead of a fixed number of exact distances.  The rerank_n
 * candidates of step 7 are taken in ascending (ADC distance, id) order in
 * mini-batches of batch_size.  After each mini-batch the current best k
 * (exact distance, id) pairs are those of all candidates re-ranked so far;
 * the change rate is the number of their IDs that were not among the best k
 * before the mini-batch, divided by k.  Re-ranking stops once the change rate
 * has been <= eps for beta consecutive mini-batches (or when the candidates
 * run out).  The result is the exact top-k of the candidates re-ranked.
 *   1 <= k <= 64, k <= rerank_n <= max_rerank_n, batch_size >= 1, beta >= 1,
 *   eps >= 0
 *   d_out_reranked optional int32 [nq]: candidates re-ranked per query
 * Other arguments and errors as ann_search.
 */
ann_status ann_search_heuristic(ann_index* ix, const float* d_queries, int64_t nq,
                                const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                                int32_t rerank_n, int32_t batch_size, double eps, int32_t beta,
                                int64_t* d_out_ids, float* d_out_dists, int32_t* d_out_reranked,
                                void* stream);

/*
 * Steps 1-7: like ann_search but returns the rerank_n best approximate
 * candidates (ascending by (ADC distance, id)) instead of re-ranking them.
 *   d_out_ids int32 [nq, rerank_n] (-1 padded), d_out_adc float32 [nq, rerank_n]
 *   d_out_ncand optional int64 [nq]: distinct candidates scored per query.
 *   d_out_nwalk optional int64 [nq]: list entries the scan walked per query
 *     (every first-list member of each probed list, plus the replica entries
 *     it did not skip as a group because their first list is also probed);
 *     a measure of work, not of results: it depends on the index layout.
 */
ann_status ann_search_topn(ann_index* ix, const float* d_queries, int64_t nq,
                           const int32_t* d_nprobe, int32_t nprobe_max, int32_t rerank_n,
                           int32_t* d_out_ids, float* d_out_adc, int64_t* d_out_ncand,
                           int64_t* d_out_nwalk, void* stream);

/*
 * Steps 1-8 on an index loaded with the host-memory raw tier (raw_tier 1),
 * reporting the I/O of step 8 (Sec. 4.3, redundancy-aware I/O
 * de-duplication).  Step 8 is the fixed re-rank of all rerank_n candidates
 * (batch_size 0) or the heuristic re-ranking of Alg. 1 (batch_size >= 1,
 * eps, beta as for ann_search_heuristic).  The candidates' raw vectors are
 * read a whole page at a time from host memory: a page is read in the first
 * mini-batch that re-ranks a candidate on it, and that one read serves every
 * candidate of the query on the page -- requests for one page within a
 * mini-batch are merged, and later mini-batches find their candidates on it
 * already read (the page buffer across mini-batches).  Results equal
 * ann_search / ann_search_heuristic on the same index kept in HBM.
 *   d_out_reranked    optional int32 [nq]: candidates re-ranked
 *   d_out_page_reads  optional int32 [nq]: pages read = distinct pages of
 *                     the re-ranked candidates
 * k <= rerank_n <= 2048 (and k <= 64 with batch_size >= 1).  Errors as
 * ann_search_heuristic; ANN_EUNSUPPORTED on an index whose raw vectors are
 * in HBM.
 */
ann_status ann_search_pages(ann_index* ix, const float* d_queries, int64_t nq,
                            const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                            int32_t rerank_n, int32_t batch_size, double eps, int32_t beta,
                            int64_t* d_out_ids, float* d_out_dists, int32_t* d_out_reranked,
                            int32_t* d_out_page_reads, void* stream);

/*
 * Step 2 alone: the nearest lists of each query, ascending by
 * (centroid distance, list id).
 *   d_out_lists int32 [nq, nprobe_max] (-1 padded)
 *   d_out_dists optional float32 [nq, nprobe_max] (+inf padded)
 */
ann_status ann_probe(ann_index* ix, const float* d_queries, int64_t nq, const int32_t* d_nprobe,
                     int32_t nprobe_max, int32_t* d_out_lists, float* d_out_dists, void* stream);

/*
 * Step 1 alone: d_out_lut float32 [nq, m, ksub], entry [q][s][j] = squared
 * distance between subvector s of query q and codeword j of subspace s.
 */
ann_status ann_lut(ann_index* ix, const float* d_queries, int64_t nq, float* d_out_lut,
                   void* stream);

/*
 * Steps 3, 5 and 6 for given lists and tables (trace form, for testing):
 * every distinct candidate of each query with its Eq. 1 distance.
 *   d_lists     int32 [nq, nprobe_max], -1 entries ignored (as ann_probe writes)
 *   d_lut       float32 [nq, m, ksub]
 *   capacity    slots per query in the outputs
 *   d_out_ids   int32 [nq, capacity] external IDs, in no particular order
 *   d_out_adc   float32 [nq, capacity]
 *   d_out_count int64 [nq]: candidates found (may exceed capacity; only the
 *               first `capacity` are written)
 */
ann_status ann_scan_trace(ann_index* ix, const int32_t* d_lists, int64_t nq, int32_t nprobe_max,
                          const float* d_lut, int64_t capacity, int32_t* d_out_ids,
                          float* d_out_adc, int64_t* d_out_count, void* stream);

/*
 * Step 8 alone: exact re-rank of given candidates.
 *   d_cand_ids  int32 [nq, n] external IDs (-1 = empty slot)
 *   d_out_ids   int64 [nq, k], d_out_dists float32 [nq, k]
 * Requires 1 <= k <= n <= max_rerank_n.
 */
ann_status ann_rerank(ann_index* ix, const float* d_queries, int64_t nq, const int32_t* d_cand_ids,
                      int32_t n, int32_t k, int64_t* d_out_ids, float* d_out_dists, void* stream);

/*
 * Stage timing (measurement support, not part of the paper's method).
 * When enabled, every kernel stage launched by the search entry points on
 * this index is bracketed by a pair of HIP events recorded on the caller's
 * stream.  ann_get_profile waits for the recorded events, returns the summed
 * elapsed times and launch counts, and (reset != 0) clears them.
 * Stages: 0 probe (distances + selection), 1 distance table, 2 per-query
 * scan (planning + fused gather/dedup/Eq. 1/top-n), 3 merge + exact re-rank,
 * 4 the list-major launch (ANN_OPT_LIST_MAJOR), 5 the list-major pass's
 * bookkeeping (split, work list, per-query selection, overflow fallback).
 */
typedef struct {
  double ms[6];
  int64_t launches[6];
} ann_profile;

ann_status ann_set_profiling(ann_index* ix, int enable);
ann_status ann_get_profile(ann_index* ix, ann_profile* out, int reset);

/*
 * Options of an index.
 * Tuning knobs of the scan work split (no effect on any result: the top-n of
 * a query is the same however its gathered entries are split into items):
 *   ANN_OPT_SCAN_TILE   target entries per work item, in [64, 2^30]; 0 (default):
 *                       65536 for launches of 1024 queries or more, and
 *                       65536 * queries / 1024 but at least 4096 below, so a
 *                       small launch still has work items enough to fill the GPU
 *   ANN_OPT_SCAN_SPLIT  most work items per query, in [1, 16] (default 16;
 *                       the kernel also caps it at max(1, 4096 / rerank_n))
 *   ANN_OPT_SCAN_ORDER  1: queries are scanned in order of their
 *                       nearest list, each of the GPU's 8 L2 domains taking a
 *                       contiguous share, so queries that probe the same lists
 *                       run side by side and share cached code rows; 0
 *                       (default): input order.  Measured on the uint8 10M
 *                       workload the ordered scan was slower (2.32 vs 2.11
 *                       ms), so it stays off unless chosen.
 * Batched form, list-major (no effect on any result):
 *   ANN_OPT_LIST_MAJOR  1: searches run list-major -- the (query, probed
 *                       list) pairs of a chunk are inverted into per-list
 *                       groups of queries, and one persistent launch reads
 *                       each probed list's code rows once per group.  On
 *                       integer-grid indexes a group is up to 16 queries: the
 *                       rows are decoded and scored on the int8 matrix cores
 *                       (Eq. 1 equals ||q - decoded||^2 exactly there); on
 *                       float indexes it is 4 queries (8 with
 *                       ANN_OPT_LUT_F16) whose distance tables sit in LDS
 *                       side by side.  The replica entries, a few leading
 *                       lists per query and lists shorter than
 *                       ANN_OPT_LM_MIN_ROWS stay with the per-query scan,
 *                       which also bounds each query's top-n.  0 (default):
 *                       per-query scan only.  Applies to ann_search,
 *                       ann_search_heuristic, ann_search_topn and graphs
 *                       created while it is set; ignored where the index
 *                       is not supported (float indexes with more than 36
 *                       subspaces).
 *   ANN_OPT_LM_ALPHA    the per-query part walks the first-list rows of the
 *                       leading probed lists until alpha * rerank_n rows, in
 *                       [1, 64] (default 2)
 *   ANN_OPT_LM_TILE     rows of a list per work item, in [64, 2^24] (default 4096)
 *   ANN_OPT_LM_BLOCKS   blocks of the persistent launch, in [0, 65536]
 *                       (default 0: as many as the device holds at once)
 *   ANN_OPT_LM_CAP      list-major keys kept per query before it falls back
 *                       to the per-query scan, in [0, 2^20] (default 0:
 *                       min(32768, max(4096, 16 * rerank_n)))
 *   ANN_OPT_LM_MIN_ROWS lists with fewer first-list rows are scanned per
 *                       query, in [0, 2^30] (default 0)
 * Numeric variant (changes results, deterministically):
 *   ANN_OPT_LUT_F16     1: the distance table of Eq. 1 is held in binary16 --
 *                       each float32 entry rounded to the nearest binary16,
 *                       ties to even, widened exactly before the float32 sum
 *                       over subspaces; 0 (default): float32 entries.  Meant
 *                       for data whose table entries stay below 65504 (larger
 *                       entries become +inf).  ann_search / ann_search_topn
 *                       and the forms built on them; ann_lut and
 *                       ann_scan_trace stay float32.
 * Probe variant (changes which lists are probed):
 *   ANN_OPT_PROBE_BEAM  > 0: step 2 walks the navigation graph given by
 *                       ann_set_nav_graph with this beam width, in [1, 1024]
 *                       (raised to a query's nprobe when smaller); nprobe_max
 *                       is then at most 1024.  0 (default): exact probe over
 *                       all centroids.  Applies to every search entry point,
 *                       ann_probe, the server, and graphs created while it is
 *                       set.
 * Errors: ANN_EINVAL for an unknown option or an out-of-range value.
 */
enum {
  ANN_OPT_SCAN_TILE = 1,
  ANN_OPT_SCAN_SPLIT = 2,
  ANN_OPT_LUT_F16 = 3,
  ANN_OPT_SCAN_ORDER = 4,
  ANN_OPT_LIST_MAJOR = 5,
  ANN_OPT_LM_ALPHA = 6,
  ANN_OPT_LM_TILE = 7,
  ANN_OPT_LM_BLOCKS = 8,
  ANN_OPT_LM_CAP = 9,
  ANN_OPT_LM_MIN_ROWS = 10,
  ANN_OPT_PROBE_BEAM = 11
};
ann_status ann_set_option(ann_index* ix, int option, int64_t value);
ann_status ann_get_option(ann_index* ix, int option, int64_t* value);

/*
 * Navigation graph over the list centroids (Sec. 4.1: the top-m lists are
 * found by walking an in-memory graph whose vertices are the posting lists'
 * centroids, each joined to its nearest neighbours).  With
 * ANN_OPT_PROBE_BEAM = B > 0 step 2 becomes a best-first beam walk of it, per
 * query (B raised to the query's nprobe when smaller):
 *   - the candidate set holds the B nearest (centroid distance, list) pairs
 *     found so far, each expanded or not; it starts with the entry vertices;
 *   - the nearest candidate not yet expanded is expanded: each neighbour whose
 *     distance was not computed before is computed and offered to the set,
 *     which keeps its B nearest;
 *   - the walk ends when every candidate has been expanded; the first nprobe
 *     candidates are the probed lists, ascending.
 * Distances are those of the exact probe, ties to the lower list id.
 *   adj      host int32 [nlist, deg]: neighbours of each list (-1 pads a row;
 *            no list twice in a row), deg in [1, 1024]
 *   entry    host int32 [n_entry]: distinct entry lists, 1 <= n_entry <= nlist
 * The arrays are copied to the device (the caller keeps ownership).  A NULL
 * adj removes the graph and sets the beam to 0.  The call waits for the
 * device, and must not run concurrently with searches on this index.
 * Errors: ANN_EINVAL (ranges, duplicates), ANN_ENOMEM, ANN_EDEVICE.
 */
ann_status ann_set_nav_graph(ann_index* ix, const int32_t* adj, int32_t deg, const int32_t* entry,
                             int32_t n_entry);

/*
 * Batched form: the search of one query batch captured into a HIP graph.
 * ann_graph_create records ann_search(ix, d_queries, nq, d_nprobe, nprobe_max,
 * k, rerank_n, d_out_ids, d_out_dists) -- probe, scan and merge of every
 * chunk -- into a graph with its own working memory (allocated here, held
 * until ann_graph_free).  Each ann_graph_launch replays the whole search with
 * one launch call and allocates nothing; it reads whatever d_queries and
 * d_nprobe hold when it runs (same shapes), and writes the same results
 * ann_search would.  Launches of one graph are ordered after each other even
 * on different streams (they share its working memory).  The scan's work
 * split (ann_set_option) is fixed at capture time.  The buffers must stay
 * valid while the graph exists.  Errors: as ann_search (nq >= 1 here).
 */
typedef struct ann_graph ann_graph; /* opaque */
ann_status ann_graph_create(ann_index* ix, const float* d_queries, int64_t nq,
                            const int32_t* d_nprobe, int32_t nprobe_max, int32_t k,
                            int32_t rerank_n, int64_t* d_out_ids, float* d_out_dists,
                            ann_graph** out);
ann_status ann_graph_launch(ann_graph* g, void* stream);
void ann_graph_free(ann_graph* g); /* waits for its last launch; NULL is a no-op */

/*
 * Autotuner of the batched form for a batch: runs ann_search on the given
 * queries for each candidate, `reps` timed runs each after one warm-up, and
 * keeps the one with the lowest median time, setting its options on the
 * index.  Candidates: first the per-query scan's work split (tile in {4096 ..
 * 131072, 2^30}, split in {1, 2, 4, 8, 16}, ANN_OPT_LIST_MAJOR 0); then the
 * list-major form with the best split: on integer-grid indexes alpha in
 * {1, 2, 4, 8}, rows per work item in {1024, 4096, 16384}, persistent blocks
 * in {2, 4, 8} per compute unit; on float indexes alpha in {1, 2, 8},
 * shortest list taken in {0, 2048, 16384} rows, rows per item 16384 or
 * whole lists, one block per compute unit.  No option changes results.  Synchronous;
 * allocates temporary outputs.  Errors: as ann_search, ANN_EINVAL for reps
 * outside [1, 100].
 */
typedef struct {
  int64_t tile;        /* chosen ANN_OPT_SCAN_TILE */
  int32_t split;       /* chosen ANN_OPT_SCAN_SPLIT */
  int32_t tried;       /* candidates timed */
  double ms;           /* median search time of the chosen candidate */
  int32_t list_major;  /* chosen ANN_OPT_LIST_MAJOR; when 1, the three below */
  int32_t lm_alpha;    /* ANN_OPT_LM_ALPHA */
  int32_t lm_tile;     /* ANN_OPT_LM_TILE */
  int32_t lm_blocks;   /* ANN_OPT_LM_BLOCKS */
  int32_t lm_min_rows; /* ANN_OPT_LM_MIN_ROWS */
} ann_tune_result;
ann_status ann_autotune(ann_index* ix, const float* d_queries, int64_t nq, const int32_t* d_nprobe,
                        int32_t nprobe_max, int32_t k, int32_t rerank_n, int32_t reps,
                        ann_tune_result* out);

/*
 * Served form: continuous batching of small search requests on one GPU.
 *
 * The paper serves concurrent queries with one CPU thread per query and gives
 * each in-flight query its own block of working memory (Sec. 5).  Here a
 * server owns an HBM arena of hbm_budget_bytes and max_slots streams.  Its
 * scheduler thread coalesces consecutive waiting requests that share
 * (k, rerank_n) into one launch of at most max_batch queries and starts it as
 * soon as a stream is free and the launch's device footprint (queries,
 * outputs, working buffers) fits in the arena's free bytes.  A finished launch
 * frees its stream and bytes immediately, so requests that arrive while others
 * run are admitted without waiting for a batch boundary, and launches on
 * different streams overlap on the device.  No device memory is allocated
 * while serving.  Every query is searched exactly as by ann_search with the
 * same nprobe, k and rerank_n, so results do not depend on the mix.
 */
typedef struct ann_server ann_server; /* opaque */

typedef struct {
  int64_t hbm_budget_bytes; /* device bytes for in-flight launches (0: 2 GiB); must hold
                               one launch of max_batch queries at the max_* limits */
  int32_t max_slots;        /* launches in flight at once, 1..16 (0: 4) */
  int32_t max_batch;        /* most queries per launch and per request (0: 1024) */
  int32_t max_nprobe;       /* largest nprobe_max accepted, 1..4096 (0: 256) */
  int32_t max_k;            /* largest k accepted (0: 64) */
  int32_t max_rerank_n;     /* largest rerank_n accepted (0: max_rerank_n of the index) */
} ann_server_cfg;

typedef struct {
  int64_t requests_done;    /* requests completed (since start or the last reset) */
  int64_t queries_done;
  int64_t launches;         /* device launches started */
  int64_t max_in_flight;    /* most launches on the device at once */
  int64_t peak_bytes;       /* most arena bytes held by in-flight launches */
  int64_t budget_bytes;
  double latency_p50_ms;    /* submit -> results available, per request */
  double latency_p99_ms;
  double latency_max_ms;
} ann_server_stats;

/* Start a server on a loaded index (cfg NULL: all defaults).  The index must
 * outlive the server.  Errors: ANN_EINVAL (limits; a budget too small for one
 * launch of max_batch queries; max_nprobe with max_rerank_n needing more
 * scan LDS than a block has; max_rerank_n above 2048 on the host-memory raw
 * tier), ANN_ENOMEM, ANN_EDEVICE.  A launch that fails with a device error
 * stops the server (later submits fail); any other failure fails only the
 * requests of that launch. */
ann_status ann_server_start(ann_index* ix, const ann_server_cfg* cfg, ann_server** out);

/* Queue a request of nq (1..max_batch) float32 queries in HOST memory
 * (copied; the caller may reuse the buffer at once).  nprobe: host int32 [nq]
 * or NULL (every query probes nprobe_max lists); same limits as ann_search.
 * *ticket identifies the request for ann_server_poll.  Thread-safe.
 * Errors: ANN_EINVAL (limits, server stopping), or the status of an earlier
 * failed launch. */
ann_status ann_server_submit(ann_server* s, const float* queries, int32_t nq,
                             const int32_t* nprobe, int32_t nprobe_max, int32_t k,
                             int32_t rerank_n, uint64_t* ticket);

/* *done = 1 once the request has finished; then its results are copied to
 * ids (host int64 [nq, k]) and dists (host float32 [nq, k]) when non-NULL and
 * the ticket is forgotten (a later poll of it fails with ANN_EINVAL).  wait != 0
 * blocks until the request has finished.  Thread-safe. */
ann_status ann_server_poll(ann_server* s, uint64_t ticket, int64_t* ids, float* dists,
                           int32_t* done, int32_t wait);

/* Counters and latency percentiles; reset != 0 clears them afterwards. */
ann_status ann_server_get_stats(ann_server* s, ann_server_stats* out, int reset);

/* Finish every submitted request, stop the scheduler and free the server's
 * resources.  No other call on `s` may run concurrently or follow. */
ann_status ann_server_stop(ann_server* s);

/*
 * Differentiable PQ distance with fixed codes (codebook fine-tuning).
 * Eq. 1 with dist = squared L2 of sub-vectors, as a function of the queries
 * and the codebooks:  Dhat[b][c] = sum_m ||q_b,m - CB[m][code[c][m]]||^2.
 *   d_queries   float32 [B, M*dsub]
 *   d_codebooks float32 [M, 256, dsub]   (dsub <= 16, M*256*4 <= 64 KiB)
 *   d_codes     uint8   [C, M]
 *   d_out       float32 [B, C]
 * Index-free: works on any caller tensors.  float32 arithmetic.
 */
ann_status ann_adc_forward(const float* d_queries, int64_t B, const float* d_codebooks, int32_t M,
                           int32_t dsub, const uint8_t* d_codes, int64_t C, float* d_out,
                           void* stream);

/*
 * Exact squared distances of a query batch to a vector batch, the reference
 * term of the fine-tuning loss: d_out[b][c] = sum_t (q[b][t] - x[c][t])^2,
 * summed in float64 over t in order and rounded once to float32 (direct
 * form: no expansion into norms and a product).
 *   d_queries float32 [B, D], d_vectors float32 [C, D], d_out float32 [B, C]
 * B <= 1048560.  Index-free.
 */
ann_status ann_exact_sq(const float* d_queries, int64_t B, const float* d_vectors, int64_t C,
                        int32_t D, float* d_out, void* stream);

/* Bytes of device workspace ann_adc_backward needs for these sizes. */
size_t ann_adc_backward_workspace(int64_t B, int64_t C, int32_t M, int32_t dsub);

/*
 * Backward of ann_adc_forward given d_grad = dL/dDhat float32 [B, C]:
 *   d_dq  float32 [B, M*dsub] (may be NULL):
 *         dQ[b] = 2 (sum_c G[b][c]) q_b - 2 sum_c G[b][c] dec(c)
 *   d_dcb float32 [M, 256, dsub] (may be NULL):
 *         dCB[m][j] = -2 sum_{c: code[c][m]=j} sum_b G[b][c] (q_b,m - CB[m][j])
 * Codewords no candidate uses get exactly zero gradient; results do not depend
 * on thread timing (no floating-point atomics).  d_workspace: caller-owned
 * device memory of at least ann_adc_backward_workspace(...) bytes (the call
 * allocates nothing).
 */
ann_status ann_adc_backward(const float* d_queries, int64_t B, const float* d_codebooks,
                            int32_t M, int32_t dsub, const uint8_t* d_codes, int64_t C,
                            const float* d_grad, float* d_dq, float* d_dcb, void* d_workspace,
                            size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ANN_H */
