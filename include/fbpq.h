/*
 * fbpq.h -- C ABI of the FBPQ query-time search on AMD Instinct MI355X (gfx950).
 *
 * The library answers approximate nearest-neighbour queries over a second-order
 * inverted multi-index whose points are stored as PQ codes of their
 * displacement from the cell centroid (Babenko & Lempitsky, "Improving Bilayer
 * Product Quantization for Billion-Scale Approximate Nearest Neighbors in High
 * Dimensions"). Given a query q in R^D it forms the candidate list of the
 * multi-sequence traversal (Section 2.3.3: cells in ascending distance until
 * L points are collected) and reranks the candidates with the FBPQ distance of
 * Section 3.1, equations (distance) and (decomposition): work linear in the
 * code length M per candidate, using query-independent tables of
 * centroid-by-codeword dot products and squared norms.
 *
 * Conventions shared by every entry point
 *  - Return value: FBPQ_OK (0) or a negative FBPQ_E_* code; no exception and no
 *    abort crosses the ABI. fbpq_last_error() gives a message for the calling
 *    thread.
 *  - Index geometry: D (even), T centroids per half, M PQ subspaces (even,
 *    D % M == 0), Kc = 256 codewords per subspace. Cell id = i*T + j for the
 *    half-centroid pair (i, j); subspace k covers coordinates
 *    [k*D/M, (k+1)*D/M); the first M/2 subspaces lie in the first half.
 *  - Candidate list: exactly min(L, N) points. Cells are visited in ascending
 *    (d1[i] + d2[j], a, b), where the half distances are FP64 and a, b are the
 *    ranks of i, j in the (distance, index) sorted half lists; the last cell
 *    is cut in storage order. Empty cells are visited and add nothing.
 *  - Results: row-major [nq][k_max]; row r holds the k[r] smallest candidates
 *    by (FP32 FBPQ distance, id), ascending; positions past min(k[r], L_eff)
 *    hold id -1 and distance +inf.
 *  - Ownership: the caller owns query and result buffers; the library owns
 *    all device memory behind an index handle. A handle may be used by one
 *    host thread at a time.
 *  - Errors on the device (a failed HIP call) poison the handle: later calls
 *    on it return FBPQ_E_DEVICE.
 */
#ifndef FBPQ_H
#define FBPQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FBPQ_OK 0
#define FBPQ_E_INVALID (-1)  /* bad argument (null pointer, nq < 0, L < 1, k < 1, k > k_max ...) */
#define FBPQ_E_IO (-2)       /* index file cannot be opened or read */
#define FBPQ_E_FORMAT (-3)   /* index file or descriptor is malformed (magic, sizes, CRC, offsets) */
#define FBPQ_E_OOM (-4)      /* host or device allocation failed */
#define FBPQ_E_DEVICE (-5)   /* a HIP call failed, or the handle was poisoned by one */
#define FBPQ_E_STATE (-6)    /* call out of order (e.g. search before fbpq_build_tables) */
#define FBPQ_E_CAPACITY (-7) /* a query needs more traversal depth than the library supports, or a
                                server's admission limits refuse a request */
#define FBPQ_E_TIMEOUT (-8)   /* served request still queued at its deadline (not searched) */
#define FBPQ_E_CANCELLED (-9) /* served request taken out of the queue by fbpq_server_cancel */

#define FBPQ_KC 256
#define FBPQ_K_MAX 1024 /* largest k per query */

typedef struct fbpq_index fbpq_index;

/* Host-side description of an index, all pointers to host memory that the
 * library copies during fbpq_index_create (the caller keeps ownership).
 *   C1, C2   float  [T][D/2]       half codebooks (Section 2.3.1)
 *   R        float  [M][Kc][D/M]   displacement codebooks R_1..R_M
 *   offsets  int64  [T*T + 1]      start of each cell in storage order (Section 2.3.2)
 *   codes    uint8  [N][M]         PQ code of each stored point
 *   ids      uint32 [N]            point id of each stored point
 *   QL, SL   float  [T][M/2][Kc][D/M] each, or both NULL: local codebooks
 *            (HBPQ, Section 3.2). QL[i] codes the first half of the
 *            displacements in the cells (i, *), SL[j] the second half in the
 *            cells (*, j) (equation residual); R is then not used. With them
 *            the search returns the kNN of the reconstructions through the
 *            local codebooks; without them, the FBPQ / Multi-D-ADC result.
 *   Rot      float  [D][D] row-major, or NULL: the orthogonal rotation of
 *            optimized product quantization (OPQ, Section 2.1; the optimized
 *            variants of Sections 3.1-3.2). The index lives in the rotated
 *            space and every search first maps its queries there: coordinate
 *            a of q' = Rot q is the FP64 sum over b = 0..D-1 in that order (one
 *            fused multiply-add per term) rounded once to FP32. Queries and
 *            results are otherwise unchanged. */
typedef struct {
    int32_t D, T, M, Kc;
    int64_t N;
    const float *C1;
    const float *C2;
    const float *R;
    const int64_t *offsets;
    const uint8_t *codes;
    const uint32_t *ids;
    const float *QL;
    const float *SL;
    const float *Rot;
} fbpq_index_desc;

typedef struct {
    int32_t D, T, M, Kc;
    int64_t N;
    int64_t table_bytes;  /* centroid-by-codeword dot products: T*M*Kc floats (Section 3.3) */
    int64_t norm_bytes;   /* squared norms: (2T + M*Kc) floats (Section 3.3) */
    int64_t device_bytes; /* all device memory currently held by the handle */
    int32_t tables_ready; /* fbpq_build_tables has run */
    int32_t device;       /* HIP device ordinal */
} fbpq_info_t;

/* Upload an index described by host arrays to device `device`. Validates
 * geometry and offsets (offsets[0] == 0, non-decreasing, offsets[T*T] == N).
 * On success *out owns the device copy. Errors: INVALID, FORMAT, OOM, DEVICE. */
int fbpq_index_create(const fbpq_index_desc *desc, int device, fbpq_index **out);

/* Read an index file (layout: 64-byte header "FBPQIDX1", six to nine section
 * records with CRC-32, then the payloads: C1, C2, R, offsets, codes, ids,
 * required once each, and optionally QL and SL (local codebooks, both or
 * neither) and Rot (OPQ rotation), as in fbpq_index_desc), validate it and
 * upload it. Errors: INVALID, IO, FORMAT (magic, version, section set, sizes,
 * CRC, offsets), OOM, DEVICE. */
int fbpq_load_index(const char *path, int device, fbpq_index **out);

/* Validate an index file on the host only (no device work). Same checks and
 * error codes as fbpq_load_index; writes the geometry to *info if non-null. */
int fbpq_index_file_check(const char *path, fbpq_info_t *info);

/* Build the query-independent tables of equation (decomposition), Section 3.1:
 *   CR1[i][k][r] = 2 <c1_i|k, R_k(r)>        k <  M/2
 *   CR2[j][k][r] = 2 <c2_j|k, R_{M/2+k}(r)>  k <  M/2
 *   nR[k][r]     = ||R_k(r)||^2, nC1[i] = ||c1_i||^2, nC2[j] = ||c2_j||^2
 * accumulated in FP64 and stored in FP32 (c|k is the k-th D/M slice of the
 * half centroid). Idempotent. Errors: INVALID, DEVICE. */
int fbpq_build_tables(fbpq_index *ix);

/* Search nq queries (host memory, float [nq][D]) with one budget L >= 1 and
 * 1 <= k <= FBPQ_K_MAX; writes host ids [nq][k] and dists [nq][k].
 * nq == 0 is a no-op. Errors: INVALID, STATE, CAPACITY, OOM, DEVICE.
 * CAPACITY (for every search entry point): some queries need more than the
 * traversal supports (min(T, prefix_cap) ranks of a half list, at most 16384,
 * or 2^26 visited cells);
 * their rows hold id -2 and NaN distances, every other row is complete. */
int fbpq_search(fbpq_index *ix, const float *q, int64_t nq, int64_t L, int32_t k,
                int64_t *ids, float *dists);

/* Same with per-query budgets L[nq] and k[nq] (host arrays), outputs
 * [nq][k_max] with k[r] <= k_max <= FBPQ_K_MAX. */
int fbpq_search_uneven(fbpq_index *ix, const float *q, int64_t nq, const int64_t *L,
                       const int32_t *k, int32_t k_max, int64_t *ids, float *dists);

/* Device-resident form: d_q, d_ids, d_dists are device pointers on the index's
 * device ([nq][D], [nq][k_max], [nq][k_max]); L and k are HOST arrays of nq
 * entries. Work is queued on `hip_stream` (a hipStream_t, or null for the
 * default stream). The call returns after the search has completed on the
 * stream (it reads a per-query status word back to decide whether deeper
 * traversal is needed). */
int fbpq_search_device(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L,
                       const int32_t *k, int32_t k_max, int64_t *d_ids, float *d_dists,
                       void *hip_stream);

/* Device-resident form that does not wait for the device (the survey's
 * fbpq_search_device contract): queries d_q [nq][D], budgets d_L [nq] (int64)
 * and d_k [nq] (int32), results d_ids / d_dists [nq][k_max] are all device
 * pointers on the index's device; the call queues the search on hip_stream
 * and returns without synchronizing. L_max is a host upper bound on the
 * budgets (it sizes the distance rows); an entry of d_L outside [1, L_max] or
 * of d_k outside [1, k_max] is clamped into range and counted. d_pending
 * [2] (device, written on the stream): [0] = the queries whose traversal
 * needs a longer sorted prefix or more visited cells than the first round
 * provided (their rows are not final yet), [1] = the clamped entries. When
 * [0] is not zero, fbpq_search_device_finish (or the next search on the
 * handle, which calls it first) runs the deeper rounds on the same stream and
 * synchronizes; when it is zero, the results are complete once the stream
 * reaches them. The first round replays a captured HIP graph when option
 * "graph" is on and a search of the same shape was captured. Inputs and
 * outputs must stay valid until the stream has passed the search (and its
 * finish, when [0] is not zero). Errors: INVALID, STATE, DEVICE, OOM; from
 * finish, also CAPACITY (rows (-2, NaN) as for the other entries). */
int fbpq_search_device_async(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *d_L,
                             const int32_t *d_k, int64_t L_max, int32_t k_max, int64_t *d_ids,
                             float *d_dists, int32_t *d_pending, void *hip_stream);
int fbpq_search_device_finish(fbpq_index *ix);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * search as fbpq_search_device, same arguments and results, but every
 * workspace buffer (both traversal rounds included) is carved from a static
 * scratch array of 128 MiB that the library holds on each device it runs on
 * until the process ends, and host staging uses pageable memory. It calls no
 * hipMalloc, hipFree, hipHostMalloc or other allocating routine; graph replay
 * and profiling are off for it. A search whose workspace exceeds the 128 MiB
 * returns FBPQ_E_CAPACITY, its result rows undefined (about 230 KB per query at
 * T = 4096, M = 16, L = 10^4; workspace grows with nq, T, L and the visited
 * cells). Every call on a device shares that device's array: calls that
 * overlap on one device (two host threads, or two handles) race and must be
 * serialized by the caller. Errors: as fbpq_search_device, plus CAPACITY for
 * the scratch limit. */
int fbpq_search_device_noalloc(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L,
                               const int32_t *k, int32_t k_max, int64_t *d_ids, float *d_dists,
                               void *hip_stream);

/* Parity/debug: the visited cells and candidate positions of each query, in
 * traversal order, produced by the GPU traversal. Host buffers:
 *   cells [nq][cells_cap][2]  (cell id, points taken from it)
 *   ncells [nq]
 *   pos   [nq][pos_cap]       storage positions of the candidates
 *   npos  [nq]
 * Errors: INVALID, STATE, CAPACITY (a cap too small), OOM, DEVICE. */
int fbpq_debug_visit(fbpq_index *ix, const float *q, int64_t nq, int64_t L,
                     int64_t *cells, int64_t cells_cap, int64_t *ncells,
                     int64_t *pos, int64_t pos_cap, int64_t *npos);

/* Parity/debug: FP32 FBPQ distance of every candidate of each query, as
 * (storage position, distance) pairs in an unspecified order. Host buffers
 * pos [nq][cap], dist [nq][cap], n [nq]. Errors as fbpq_debug_visit. */
int fbpq_debug_dists(fbpq_index *ix, const float *q, int64_t nq, int64_t L,
                     int64_t *pos, float *dist, int64_t cap, int64_t *n);

/* Parity/debug: copy the tables of fbpq_build_tables to host buffers
 * CR1 [T][M/2][Kc], CR2 [T][M/2][Kc], nR [M][Kc], nC1 [T], nC2 [T] (any may be
 * null). Errors: INVALID, STATE, DEVICE. */
int fbpq_debug_tables(fbpq_index *ix, float *CR1, float *CR2, float *nR, float *nC1, float *nC2);

/* Parity/debug: the first P entries of both sorted half lists of each query:
 * keys FP64 [nq][2][P] and centroid indices int32 [nq][2][P]. P <= T. */
int fbpq_debug_rank(fbpq_index *ix, const float *q, int64_t nq, int32_t P, double *keys,
                    int32_t *idx);

/* Geometry and memory of an index. Errors: INVALID. */
int fbpq_info(const fbpq_index *ix, fbpq_info_t *out);

/* Table and norm sizes in bytes for a geometry (host arithmetic only):
 * T*M*Kc and (2T + M*Kc) FP32 values (Section 3.3). Errors: INVALID. */
int fbpq_table_bytes(int64_t T, int64_t M, int64_t Kc, int64_t *table_bytes, int64_t *norm_bytes);

/* Tuning knobs (autotuner and tests). Keys: "prefix" (initial sorted-list
 * length P, 1..16384), "prefix_cap" (longest sorted-list length a retry round
 * may take, 1..16384, default 16384; a query whose traversal needs more ranks
 * of a half list than min(T, prefix_cap) ends with its row (-2, NaN) and the
 * search returns FBPQ_E_CAPACITY, the other rows being complete), "max_cells"
 * (initial per-query visited-cell capacity), "chunk"
 * (candidates per scan chunk), "hint_first" (0/1, default 1: with graph
 * replay off, a batch whose queries' budget classes (floor(log2(min(L, N))))
 * all needed deeper traversal rounds before starts its first round at the
 * prefix length and cell capacity those rounds reached; same results),
 * "block_min" (0 off, 1 on, 2 = default: on
 * when T >= 4096; the first layer's key kernel also writes the smallest key
 * of each block of 16 centroids, and the prefix select draws its samples from
 * them and reads only the blocks that can hold survivors; same prefixes
 * either way), "persist" (0/1: the cell scan as a persistent kernel over a
 * device queue of (query, cell range) work items of at least "tile"
 * candidates, 64..2^30, default 8192, largest queries first, in workgroups of
 * "pwaves" (2, 4 or 8) wavefronts; same distances and results), "items" (0/1: use the cell scan for
 * queries whose visited cells hold many points; 0 sends every query to the
 * two-pass scan), "profile" (0/1: time kernel launches with HIP events,
 * read with fbpq_profile_read), "profile_mask" (bit s set: stage s is timed
 * while profiling is on; default all), "stats" (0/1: path counters, read
 * with fbpq_stats_read), "pop_budget" (cells the traversal visits one at a
 * time before it switches to threshold steps, which load the point counts of
 * many cells at once; 0 switches at once; default 512; the visited cells are
 * the same either way), "adc_od" (0/1: score every candidate by explicit
 * reconstruction, O(D) per candidate -- the Multi-D-ADC rerank of Section
 * 2.3.3 -- instead of the FBPQ tables; same visited cells and, up to FP32
 * rounding, the same distances; a baseline for comparison), "graph" (0/1: the first traversal round of a search
 * is captured once into a HIP graph and replayed on later searches with the
 * same queries buffer, result buffers, nq, k_max, min(L, N) and options;
 * retry rounds and profiled or debug searches run eagerly), "split_keys"
 * (0/1, default 1: at D/2 = 64 the first layer's approximate keys come from
 * two-part FP16 half-centroids on the FP16 matrix cores, with the error
 * bound of that form; 0 uses FP32 products; the same prefixes either way),
 * "inject_device_error" (n >= 1, for tests of error handling: the n-th
 * checked HIP call after this one reports a failure instead of being made,
 * which poisons the handle like a real device error; 0 clears it).
 * Errors: INVALID, DEVICE. */
int fbpq_set_option(fbpq_index *ix, const char *key, int64_t value);

/* Kernel stages timed by the library's profiler (one kernel each, except
 * SCAN2, which launches one kernel per table placement). */
#define FBPQ_STAGE_HALF_KEYS 0 /* first layer: approximate half distances on the matrix cores */
#define FBPQ_STAGE_PREFIX 1    /* sorted prefix of each half list: one wavefront per half */
#define FBPQ_STAGE_PREFIX_FB 2 /* sorted prefix: workgroup select for the halves left over */
#define FBPQ_STAGE_TRAVERSE 3  /* multi-sequence traversal */
#define FBPQ_STAGE_LAYOUT 4    /* row-major layout of the visited cells */
#define FBPQ_STAGE_LQ 5        /* per-query tables LQ of the cell scan */
#define FBPQ_STAGE_SCORE 6     /* cell scan: FP32 distance of every candidate */
#define FBPQ_STAGE_SELECT 7    /* per-query k smallest of the scored candidates */
#define FBPQ_STAGE_SCAN2 8     /* two-pass scan (queries whose cells hold few points) */
#define FBPQ_STAGE_TRAVERSE_WIDE 9 /* threshold-stepping traversal (queries with many visited cells) */
#define FBPQ_STAGE_SCAN_WIDE 10 /* two-pass scan with sums in HBM (many candidates in sparse cells) */
#define FBPQ_STAGE_ROTATE 11 /* OPQ rotation of the queries (indexes with Rot) */
#define FBPQ_NUM_STAGES 12

/* ---- served form: continuous batching (Section 4 measures per-query time;
 * a server keeps the GPU busy with overlapping batches of arriving queries) --
 *
 * fbpq_server_create2: a server over a handle whose tables are built. It owns
 *   cfg->nlanes (1..16) lanes, each with its own HIP stream and workspace over
 *   the handle's index arrays, and one host worker thread per lane. A lane
 *   that is free takes the oldest queued request and, in arrival order, the
 *   queued requests of the same candidate-budget class (floor(log2(min(L, N))))
 *   up to cfg->max_batch, and searches them as one batch; the lanes' batches
 *   overlap on the GPU. Results have cfg->k_max columns.
 *   Admission: each request reserves an estimate of its search workspace
 *   (bytes per query plus bytes per candidate); one lane's batch reserves at
 *   most cfg->ws_budget / nlanes (ws_budget 0: 16 GiB), so the lanes'
 *   workspace stays within ws_budget. A request whose own reservation exceeds
 *   a lane's share, or that arrives while cfg->max_pending requests are queued
 *   (0: 2^20), is refused by fbpq_server_submit with FBPQ_E_CAPACITY. A
 *   request still queued cfg->timeout_s seconds after its submission (0: no
 *   limit) completes with status FBPQ_E_TIMEOUT without being searched.
 *   Test backend: with ix NULL, cfg->D > 0 and cfg->fake_ns_per_cand > 0 the
 *   lanes run on the host instead: a batch sleeps fake_ns_per_cand per
 *   candidate (sum of L) and answers request (q, k) with ids
 *   j + 1000 * round(q[0]) and distances q[1] + j for j < k. The scheduler
 *   (batching, admission, timeouts, cancellation) is the same.
 *   The handle must outlive the server and must not be searched directly while
 *   the server runs. Errors: INVALID, STATE, DEVICE.
 * fbpq_server_create: fbpq_server_create2 with max_batch, nlanes and k_max
 *   given and every other field 0 (the defaults).
 * fbpq_server_submit: queues one query (host, D floats, copied), its L >= 1 and
 *   1 <= k <= k_max, under a caller tag. Thread-safe. Errors: INVALID, STATE
 *   (server stopping), CAPACITY (refused by admission; nothing is queued).
 * fbpq_server_cancel: completes the queued request of that tag with status
 *   FBPQ_E_CANCELLED. Errors: STATE (no such request is queued: it runs,
 *   finished or never existed), INVALID.
 * fbpq_server_poll: moves up to max_n finished requests out, waiting up to
 *   wait_s seconds for the first: tags[n], ids/dists [n][k_max] (padded with
 *   -1 / +inf past k), times[n][3] = submit, batch start, batch end (seconds on
 *   the host steady clock), status[n] = FBPQ_OK, the batch's error code,
 *   FBPQ_E_CAPACITY for a row the traversal could not serve (ids -2),
 *   FBPQ_E_TIMEOUT or FBPQ_E_CANCELLED. Writes the count to *n_out. Errors:
 *   INVALID.
 * fbpq_server_counts: requests still queued, batches run, requests batched.
 * fbpq_server_stats: copies min(n, FBPQ_SERVER_NUM_STATS) counters to out[].
 * fbpq_server_first_error: message of the first failed batch ("" if none).
 * fbpq_server_destroy: finishes every queued request, then frees the lanes;
 *   results not polled are dropped. */
typedef struct fbpq_server fbpq_server;
typedef struct {
    int32_t max_batch;       /* requests per batch, >= 1 */
    int32_t nlanes;          /* concurrent batches, 1..16 */
    int32_t k_max;           /* result columns, 1..FBPQ_K_MAX */
    int32_t D;               /* query dimension: test backend only (taken from the index otherwise) */
    int64_t ws_budget;       /* workspace bytes all lanes together may reserve (0: 16 GiB) */
    int64_t max_pending;     /* queued requests above which submit refuses (0: 2^20) */
    double timeout_s;        /* queueing deadline per request in seconds (0: none) */
    double fake_ns_per_cand; /* > 0 with a NULL index: host test backend */
} fbpq_server_config;
#define FBPQ_SERVER_STAT_SUBMITTED 0   /* requests queued */
#define FBPQ_SERVER_STAT_COMPLETED 1   /* ... finished with FBPQ_OK */
#define FBPQ_SERVER_STAT_FAILED 2      /* ... finished by a batch with an error (CAPACITY rows included) */
#define FBPQ_SERVER_STAT_TIMEOUT 3     /* ... completed with FBPQ_E_TIMEOUT */
#define FBPQ_SERVER_STAT_CANCELLED 4   /* ... completed with FBPQ_E_CANCELLED */
#define FBPQ_SERVER_STAT_REJECTED 5    /* submissions refused with FBPQ_E_CAPACITY */
#define FBPQ_SERVER_STAT_BATCHES 6     /* batches run */
#define FBPQ_SERVER_STAT_BATCHED 7     /* requests in them */
#define FBPQ_SERVER_STAT_PEAK_RESERVED 8 /* largest workspace reserved at once by running batches */
#define FBPQ_SERVER_STAT_PEAK_BATCH_RESERVED 9 /* largest reservation of one batch */
#define FBPQ_SERVER_STAT_BUDGET 10     /* ws_budget in effect */
#define FBPQ_SERVER_STAT_LANE_BUDGET 11 /* a lane's share of it */
#define FBPQ_SERVER_STAT_PENDING 12    /* requests queued now */
#define FBPQ_SERVER_NUM_STATS 13
int fbpq_server_create2(fbpq_index *ix, const fbpq_server_config *cfg, fbpq_server **out);
int fbpq_server_create(fbpq_index *ix, int32_t max_batch, int32_t nlanes, int32_t k_max, fbpq_server **out);
int fbpq_server_submit(fbpq_server *s, const float *q, int64_t L, int32_t k, int64_t tag);
int fbpq_server_cancel(fbpq_server *s, int64_t tag);
int fbpq_server_poll(fbpq_server *s, int32_t max_n, double wait_s, int64_t *tags, int64_t *ids, float *dists,
                     double *times, int32_t *status, int32_t *n_out);
int fbpq_server_counts(fbpq_server *s, int64_t *pending, int64_t *batches, int64_t *batched);
int fbpq_server_stats(fbpq_server *s, int64_t *out, int32_t n);
const char *fbpq_server_first_error(fbpq_server *s);
void fbpq_server_destroy(fbpq_server *s);

/* Autotuner. Times fbpq_search_device on the caller's batch (device queries
 * d_q [nq][D], per-query host L and k, device results as in
 * fbpq_search_device, on hip_stream): one warm search, then `reps` searches
 * timed with HIP events, median kept, for each candidate setting, in two
 * stages: the options "prefix" (16, 32, 64, 128, 256, 512, capped at T) x "items"
 * (1, 0), each timed in two round-robin passes with its faster median kept;
 * then, if the cell scan won, "persist" 1 with "tile" (2048, 8192,
 * 32768, 2^30 candidates per work item) x "pwaves" (2, 4, 8 wavefronts per
 * workgroup, where the kernel has that shape) against the per-query launch.
 * The fastest setting stays set on the handle. chosen [6]: prefix, items,
 * median microseconds per search, persist, tile, pwaves. Synchronizes the
 * stream. Profiling and graph replay are off while it runs. Errors: INVALID,
 * STATE, DEVICE, CAPACITY, OOM (then the handle keeps its previous options). */
int fbpq_autotune(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                  int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream, int32_t reps, int64_t *chosen);

/* The same with a cache: cache_path names a file of JSON lines, one record
 * per tuned setting, keyed by the index geometry (D, T, M, N, local
 * codebooks), the batch (floor(log2(nq)), floor(log2 of the mean min(L, N)),
 * floor(log2(k_max))) and the device (architecture name and compute unit
 * count). A key present in the file is applied without timing anything
 * (*from_cache = 1); otherwise the batch is tuned as fbpq_autotune does and a
 * record is appended (*from_cache = 0). Errors: as fbpq_autotune, IO. */
int fbpq_autotune_cached(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                         int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream, int32_t reps,
                         const char *cache_path, int64_t *chosen, int32_t *from_cache);

/* Path counters, accumulated on the device while option "stats" is 1 (setting
 * it to 1 clears them). fbpq_stats_read copies min(n, FBPQ_NUM_STATS) of them
 * to out[] and, if reset != 0, clears them. The counters say which kernels
 * served each query, for tests and tuning. Errors: INVALID, DEVICE, STATE
 * (stats not enabled). */
#define FBPQ_STAT_CELL_SCAN 0   /* queries scored by the query-major cell scan */
#define FBPQ_STAT_FUSED_TOPK 1  /* ... of which the top-k was selected inside the scan */
#define FBPQ_STAT_TWO_PASS 2    /* queries scored by the two-pass scan */
#define FBPQ_STAT_PREFIX_WAVE 3 /* (query, half) prefixes finished by the wavefront select */
#define FBPQ_STAT_PREFIX_WG 4   /* (query, half) prefixes finished by the workgroup select */
#define FBPQ_STAT_RETRIED 5     /* queries traversed again with a longer prefix or more cells */
#define FBPQ_STAT_GRAPH_REPLAYS 6 /* searches whose first round was a replayed graph */
#define FBPQ_STAT_WIDE 7        /* queries traversed by threshold steps */
#define FBPQ_STAT_WIDE_BANDS 8  /* ... bands of cells they took (dropped ones included) */
#define FBPQ_STAT_WIDE_EVALS 9  /* ... row widths evaluated at a threshold (per query) */
#define FBPQ_STAT_WIDE_LOADS 10 /* ... cell point counts they loaded */
#define FBPQ_STAT_CAND_CELL_SCAN 11 /* candidates scored by the cell scan */
#define FBPQ_STAT_CAND_TWO_PASS 12  /* candidates scored by the two-pass scan in LDS */
#define FBPQ_STAT_CAND_WIDE 13      /* candidates scored by the two-pass scan with sums in HBM
                                       (once per pass group with adc_od) */
#define FBPQ_STAT_FUSED_RESCAN 14   /* cell-scan queries scored again with streamed distances
                                       because their candidate window overflowed */
#define FBPQ_STAT_WIN_ADMITTED 15   /* candidates the running bound admitted to those windows */
#define FBPQ_STAT_WIN_LOST 16       /* windows that overflowed during the scan (before the
                                       final bound) */
#define FBPQ_NUM_STATS 17
int fbpq_stats_read(fbpq_index *ix, int64_t *out, int32_t n, int32_t reset);

/* Device time per kernel stage, measured with HIP events recorded on the
 * search stream around every launch while profiling is on (option "profile"
 * = 1). Writes the accumulated milliseconds and launch count of `stage` and,
 * if reset != 0, clears that stage's counters. Errors: INVALID. */
int fbpq_profile_read(fbpq_index *ix, int32_t stage, int32_t reset, double *ms, int64_t *launches);

/* Measurement probe (no index needed): the chip-wide rate of random 4-byte
 * LDS reads from 256-entry tables, the access pattern of the scans' table
 * lookups (16 tables, random code bytes, 8 workgroups of 256 threads per
 * compute unit), in lookups per second. A denominator for the scans' LDS
 * roof. Errors: INVALID, DEVICE. */
int fbpq_probe_lds_gather(int device, double *lookups_per_s);

/* Release the handle and all device memory it holds. Null is a no-op. */
void fbpq_free_index(fbpq_index *ix);

/* Message of the last error on the calling thread ("" if none). */
const char *fbpq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FBPQ_H */
