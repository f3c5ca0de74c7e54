/*
 * swdb — score-only Smith-Waterman / Gotoh protein database search on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Section 2.2, equations for H, E and F): for a query Q
 * (m residues, rows i) and each database subject D (n residues, columns j),
 *
 *   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
 *   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)
 *   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)
 *
 * with H = E = F = 0 on row 0 and column 0; the subject's score is the
 * largest H of its matrix (the optimal local alignment score), returned as
 * int32.  A gap of L residues therefore costs Go + (L-1)*Ge.  Scores are exact
 * integers: every mode of this library returns bit-identical results.
 *
 * Conventions for every call:
 *   - "device" pointers are HIP device memory of the current device (for
 *     example torch tensors' data_ptr()); "host" pointers are ordinary memory;
 *   - the caller owns every device buffer: inputs, outputs, the prepared
 *     database's layout (sw_db_prepare) and every search workspace; a
 *     database handle owns only host memory (its sorted lengths, plan cache
 *     and pinned plan-upload buffers).  The one-shot sw_db_search and the
 *     autotuner are the only calls that take device memory of their own, as
 *     stream-ordered allocations released before they return;
 *   - the substitution matrix is read from HOST memory by every call: the
 *     library picks the kernel variant from its values (8- or 16-bit profile
 *     entries) and passes it to the profile kernel by value, so a search needs
 *     no device-to-host copy and stays capturable in a graph;
 *   - searches are asynchronous on `stream` (a hipStream_t, NULL = default
 *     stream); results are valid once the stream has been synchronised;
 *   - every call returns SW_OK (0) or a negative SW_E* code and validates its
 *     arguments before any HIP call; sw_last_error() gives detail text.
 *
 * Residues are uint8 codes 0..31; the substitution matrix is 32x32 int32,
 * row-major, indexed [query residue][subject residue], entries in
 * [-128, 127].  Gap penalties are non-negative magnitudes (subtracted as in
 * the E and F equations), each at most SW_MAX_GAP.
 */
#ifndef SWDB_H
#define SWDB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_ALPHA 32
#define SW_MAX_GAP 32000
#define SW_MAX_QLEN (1 << 24)

#define SW_OK 0
#define SW_EINVAL (-1)     /* bad argument (null, negative, out of range)        */
#define SW_ENOMEM (-2)     /* workspace too small, or an allocation failed        */
#define SW_EHIP (-3)       /* a HIP runtime call failed; see sw_last_error()      */
#define SW_EUNSUP (-4)     /* the current device is not gfx950                    */
#define SW_EBADRES (-5)    /* a residue code is >= SW_ALPHA (database: from
                              sw_db_prepare; query: from the search status)      */
#define SW_ERESCORE (-6)   /* the exact int32 rescore gave up on a subject (its
                              score is stored as -1); from the search status      */
#define SW_EINTERNAL (-7)  /* a search skipped a work item inconsistent with its
                              launch (a library bug); from the search status      */

/* Arithmetic mode of a search.  All modes give identical scores. */
#define SW_MODE_AUTO 0     /* packed 16-bit lanes + exact int32 rescore           */
#define SW_MODE_I32 1      /* int32 lanes (the paper's 32-bit formulation)        */
#define SW_MODE_I16 2      /* packed 2x16-bit saturating lanes; subjects whose
                              16-bit score reaches 32767 are rescored in int32    */
#define SW_MODE_TUNED 3    /* per query length, the schedule sw_autotune chose or
                              sw_tune_set installed on the handle (AUTO if none);
                              a batch runs one persistent launch per schedule      */

typedef struct sw_db_s* sw_db_t;

/* Tuning knobs.  Zero-initialise and set what you need; 0 = library default. */
typedef struct sw_options {
    int32_t mode;          /* SW_MODE_*                                            */
    int32_t waves;         /* wavefronts per workgroup (1..8)                      */
    int32_t lane_cells;    /* target cells per lane per work item (load balance)  */
    int32_t max_lanes;     /* largest lane group per subject (1..64)               */
    int32_t lds_limit;     /* largest query profile staged in LDS, bytes           */
    int32_t grid_limit;    /* cap on persistent workgroups (0 = fill the device);
                              the pipelined pair pass then runs its bands in
                              rounds on 4 * grid_limit wavefronts               */
    int32_t wide_profile;  /* 1: 16-bit profile entries even where 8 bits hold
                              every s + Go (measurement and testing)             */
    int32_t pair_cols;     /* sw_pair_score: subject columns per tile (multiple
                              of 16, <= 2^20; 0 = planner); max_lanes sets the
                              lanes per band there (a power of two)              */
    int32_t pair_rows;     /* sw_pair_score: query rows per lane, 8 or 16
                              (0 = planner)                                      */
    int32_t align_block;   /* sw_align_pair: 0 = direction codes for the whole
                              matrix up to 2^35 cells, blocks of 65536 x 65536
                              beyond; > 0 = always blocks of this side (rounded
                              up to 512 rows and to the chunk width), <= 2^24  */
    int32_t slice_mcells;  /* searches: > 0 cuts each launch group's work queue,
                              in queue order, into persistent launches of at most
                              this many million lane cells each (at least one
                              work item per launch), enqueued one after another
                              on the stream, so that work on other streams gets
                              the device between them (serving); 0 = one launch */
    int32_t pair_mode;     /* sw_pair_score: 0 = planner, 1 = anti-diagonal tile
                              launches, 2 = one pipelined launch (bands hand rows
                              to the band below through memory; needs the largest
                              score below 2^24); pair_rows then picks R from
                              4, 6, 8, 10, 12, 16 (sw_align_pair: the code pass
                              runs there with 4 or 8 only, the tiles else)     */
    int32_t pair_sm_max;   /* sw_pair_plan: the largest substitution-matrix entry
                              the pair will be scored with (0 = 127); scoring
                              calls take it from the matrix                    */
    int32_t slice_begin;   /* searches with slice_mcells > 0: run only launches
                              slice_begin .. slice_begin + slice_count - 1 of the
                              sliced search (slice_count 0 = through the last;
                              sw_plan_info counts the launches), so a caller can
                              enqueue a long search launch by launch and put
                              other work between them.  Calls that cover
                              0 .. launches - 1 in order, on one workspace and
                              stream, equal one call: launch 0 zeroes the status
                              words, later launches add to them.  A begin at or
                              past the launch count is SW_EINVAL.              */
    int32_t slice_count;
    int32_t pair_entry_bytes; /* sw_pair_plan: profile entry bytes the pair will
                              be scored with, 1 (every s + Go in [-128, 127]) or
                              2 (0 = 2); scoring calls take it from the matrix  */
    int32_t strict_groups; /* searches: 1 = each subject's lane group is the
                              cheapest whose per-lane work fits the item target;
                              0 = also take a group of up to twice the target
                              when it sweeps 10% fewer cells (the default)     */
    int32_t pair_group_waves; /* sw_pair_score, pipelined pass: waves per
                              workgroup, 1, 2, 4, 8 or 16 (0 = planner)       */
    /* Optional timing events (created by the caller, may be NULL): recorded on
       the search stream immediately before the search kernel, immediately
       after it, and after the int32 rescore (16-bit modes).                   */
    hipEvent_t ev_search_begin;
    hipEvent_t ev_search_end;
    hipEvent_t ev_rescore_end;
} sw_options;

/* One autotuner result: the schedule for queries of length <= qlen. */
typedef struct sw_tune_entry {
    int32_t qlen;
    int32_t pad;
    double gcups;          /* measured with the chosen schedule                     */
    sw_options opt;        /* mode, waves, lane_cells (events unused)               */
} sw_tune_entry;

/* Plan summary (for measurement; all counts are per search call). */
typedef struct sw_plan_stats {
    int64_t cells;         /* sum over queries of m * (sum of subject lengths)     */
    int64_t lane_cells;    /* cells the lanes sweep including padding              */
    int64_t items;         /* wavefront work items                                 */
    int64_t launches;      /* search launches (launch groups of SW_MODE_TUNED)     */
    int64_t grid;          /* persistent workgroups launched                       */
    int64_t slot_bytes;    /* per-wavefront pass-boundary scratch                  */
    int64_t workspace;     /* bytes sw_workspace_bytes() returns                   */
    int32_t variant;       /* kernel variant (0: int32 lanes, 8-bit profile; 1:
                              int32 lanes, 16-bit profile; 2: packed 16-bit lanes,
                              16-bit profile; 3: packed 16-bit lanes, 8-bit
                              profile)                                           */
    int32_t rows;          /* query rows per lane                                  */
} sw_plan_stats;

/*
 * One-shot search (paper Section 2.2 problem statement; the database search
 * workload of Section 4.1).
 *   query        device, uint8[qlen]
 *   db_residues  device, uint8[sum of lengths], subject i at db_offsets[i]
 *   db_offsets   device, int64[nseq]
 *   db_lengths   device, int32[nseq], each >= 0
 *   subst_matrix HOST, int32[32*32], [query residue][subject residue]
 *   scores_out   device, int32[nseq], in the caller's subject order
 * Prepares a temporary database and a workspace in stream-ordered device
 * memory of its own (hipMallocAsync on `stream`, freed before returning),
 * searches in SW_MODE_AUTO, checks the search status and synchronises
 * `stream` (this call is blocking: the length sort runs on the host).
 * qlen = 0, nseq = 0 and empty subjects are legal (score 0).  Returns
 * SW_EBADRES for a residue code >= 32 in the query or the database.
 */
int sw_db_search(const uint8_t* query, int32_t qlen,
                 const uint8_t* db_residues, const int64_t* db_offsets,
                 const int32_t* db_lengths, int32_t nseq,
                 const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                 int32_t* scores_out, hipStream_t stream);

/*
 * Device bytes sw_db_prepare needs for a database of nseq subjects holding
 * total_residues residues, the longest of them max_len residues (host only,
 * no HIP call; 0 on invalid or inconsistent input).  An upper bound of the
 * layout: residues padded per 64-subject chunk to its longest member, plus
 * 12 bytes per subject; monotone in each argument.  (The padded size depends
 * on the longest subject, hence max_len beside the total and the count.)
 */
size_t sw_db_prepare_bytes(int64_t total_residues, int32_t nseq, int32_t max_len);

/*
 * Resident database (paper Section 3.1: the database is split by length; here
 * it is sorted by length, descending, and lane-interleaved 64 subjects to a
 * chunk).
 *   db_residues, db_offsets, db_lengths, nseq   as for sw_db_search (device)
 *   workspace   device, 256-byte aligned, at least
 *               sw_db_prepare_bytes(sum of lengths, nseq, longest length)
 *               bytes; owned by the caller, holds the database layout for
 *               the handle's lifetime (do not free or reuse it before
 *               sw_db_release)
 * Blocking: copies the lengths to the host, sorts, then builds the layout in
 * `workspace` on `stream` and waits for it.  Returns SW_ENOMEM if the
 * workspace is too small (checked before any HIP call against the layout's
 * metadata, then against the exact layout once the lengths are read),
 * SW_EBADRES if a residue code is >= 32, SW_EUNSUP off gfx950.  A handle may
 * be used by several streams at once if each call has its own workspace.
 */
int sw_db_prepare(const uint8_t* db_residues, const int64_t* db_offsets,
                  const int32_t* db_lengths, int32_t nseq, void* workspace, size_t ws_bytes,
                  hipStream_t stream, sw_db_t* out);

/*
 * Host-only handle for planning (no device memory, no HIP call): subject
 * lengths in HOST memory, and the device's compute-unit count and per-workgroup
 * LDS bytes (0 = MI355X values: 256 and 160 KiB).  Valid for
 * sw_workspace_bytes, sw_plan_info, sw_plan_items and sw_db_release; searches
 * with it return SW_EINVAL.
 */
int sw_db_describe(const int32_t* lengths_host, int32_t nseq, int32_t cu_count, int32_t lds_bytes,
                   sw_db_t* out);

/* Frees the handle (host memory).  No search may still be in flight; the
   caller's database workspace may be reused afterwards. */
int sw_db_release(sw_db_t db);

/* nseq, residues, and the bytes of the caller's database workspace the
   handle keeps using (any pointer may be NULL). */
int sw_db_info(sw_db_t db, int64_t* nseq, int64_t* residues, int64_t* device_bytes);

/*
 * Workspace bytes a search of nq queries with HOST lengths q_lens[nq] needs
 * under `opt` (NULL = defaults).  Returns 0 on invalid arguments.
 */
size_t sw_workspace_bytes(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt);

/*
 * Kernel variant (the numbering of sw_plan_stats.variant) a search runs with
 * the HOST 32x32 matrix `sm`, gap-open penalty `go` and options `opt` (NULL =
 * defaults; SW_MODE_TUNED answers for SW_MODE_AUTO): 8-bit profile entries
 * wherever every s + Go fits (int32 lanes: [-128, 127]; packed lanes: [0, 127]),
 * else 16-bit.  sw_plan_info, which does not see the matrix, reports the
 * 16-bit variant its workspace sizing assumes.  Negative code on invalid input.
 */
int sw_select_variant(const int32_t* sm, int32_t go, const sw_options* opt);

/* Plan summary for the same arguments (host only; no HIP call). */
int sw_plan_info(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt,
                 sw_plan_stats* out);

/*
 * The work queues a search would run: for each wavefront item four int32
 * (first sorted subject, columns swept, query index in the call, subjects |
 * lanes-per-subject << 16 | critical-path flag << 24).  Each query's items are
 * contiguous, largest per-lane work first; queries follow in queue order
 * (largest query first) within each launch group.  Writes at most `cap` items
 * to `out` (HOST) and returns the total count, or a negative code.
 */
int64_t sw_plan_items(sw_db_t db, int32_t nq, const int32_t* q_lens, const sw_options* opt,
                      int32_t* out, int64_t cap);

/* Sorted subject lengths (descending) of the handle, into HOST out[nseq]. */
int sw_db_sorted_lengths(sw_db_t db, int32_t* out);

/*
 * One query against a resident database.
 *   query       device, uint8[qlen]
 *   workspace   device, at least sw_workspace_bytes(db, 1, &qlen, opt) bytes,
 *               256-byte aligned; must not be shared by concurrent calls
 *   scores_out  device, int32[nseq], caller's subject order
 * Asynchronous on `stream`; the host returns once the work is enqueued.
 * Errors found on the device (a query residue code >= 32, an incomplete
 * rescore) are reported by sw_search_status on the workspace afterwards.
 */
int sw_db_search_ex(sw_db_t db, const uint8_t* query, int32_t qlen,
                    const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                    const sw_options* opt, void* workspace, size_t ws_bytes,
                    int32_t* scores_out, hipStream_t stream);

/*
 * nq queries against a resident database in one persistent launch (paper
 * Section 4.1: 20 queries per search; length-binned work items served
 * longest first).
 *   queries     device, uint8, query k at q_offsets[k]
 *   q_offsets   HOST, int64[nq]
 *   q_lens      HOST, int32[nq], each in [0, SW_MAX_QLEN]
 *   scores_out  device, int32[nq][nseq] (row k = query k, caller's order)
 * Workspace as for sw_db_search_ex with all nq lengths.  Asynchronous.
 */
int sw_db_search_batch(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets,
                       const int32_t* q_lens, int32_t nq,
                       const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                       const sw_options* opt, void* workspace, size_t ws_bytes,
                       int32_t* scores_out, hipStream_t stream);

/*
 * Graph form of a batched search (the batched launch of paper Section 4.1's
 * multi-query workload, replayed without per-launch host work): captures
 * exactly what sw_db_search_batch would enqueue -- plan upload, profile,
 * search and rescore kernels -- into a HIP graph.  The graph owns a pinned
 * copy of the plan; it reads `queries` and writes `scores_out` and
 * `workspace` (all device, fixed at capture) each time it is launched, so new
 * query residues of the same lengths may be written into `queries` between
 * launches.  The database handle and those buffers must outlive the graph.
 * Launches are asynchronous on `stream`; concurrent launches of one graph
 * race on its workspace.  Timing events in `opt` are ignored.
 */
typedef struct sw_graph_s* sw_graph_t;
int sw_graph_create(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets,
                    const int32_t* q_lens, int32_t nq,
                    const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                    const sw_options* opt, void* workspace, size_t ws_bytes,
                    int32_t* scores_out, sw_graph_t* out);
int sw_graph_launch(sw_graph_t graph, hipStream_t stream);
int sw_graph_destroy(sw_graph_t graph);

/*
 * Autotuner (schedule choice for the batched and single-query searches).  For
 * each length qlens[b] (HOST, ascending), times candidate schedules -- arithmetic
 * mode (packed 16-bit + rescore, or int32) x per-item work target x waves per
 * workgroup -- on this database with a query of that length drawn from the
 * database's own residue composition, and keeps the fastest (the default
 * schedule is the first candidate, and another replaces it only when more than
 * 0.5% faster).  Results go to out[nbins] (HOST) and are installed on the
 * handle for SW_MODE_TUNED.
 * Blocking (synchronises `stream`); allocates and frees its own device memory.
 */
int sw_autotune(sw_db_t db, const int32_t* qlens, int32_t nbins, const int32_t* subst_matrix,
                int32_t gap_open, int32_t gap_extend, hipStream_t stream, sw_tune_entry* out);

/*
 * Autotuner for one batch as a unit (the work distribution that paper
 * Sections 4.3 and 6 find decisive, here over the CUs of one device): starting
 * from the default schedule, varies one choice at a time -- arithmetic mode,
 * waves per workgroup, the per-item work target, the lane-group rule
 * (strict_groups) -- timing each on this batch itself (fastest of two runs
 * after a warm-up), and keeps a change only when it is more than 1% faster
 * in two timings of both; variations that resolve to the schedule already
 * kept are skipped.
 *   queries     device, uint8, query k at q_offsets[k]
 *   q_offsets   HOST, int64[nq];  q_lens HOST, int32[nq]
 *   subst_matrix HOST, int32[32*32]
 *   out         HOST: out->opt the schedule to pass to sw_db_search_batch or
 *               sw_graph_create for this batch (events unset), out->gcups its
 *               rate, out->qlen the longest query
 * Installs nothing on the handle.  Allocates its workspace and a score buffer
 * in stream-ordered memory on `stream` (freed before returning) and
 * synchronises `stream`; a search status error is returned as such.
 */
int sw_autotune_batch(sw_db_t db, const uint8_t* queries, const int64_t* q_offsets,
                      const int32_t* q_lens, int32_t nq, const int32_t* subst_matrix,
                      int32_t gap_open, int32_t gap_extend, hipStream_t stream,
                      sw_tune_entry* out);

/* Install (n > 0) or clear (n == 0) the handle's tuned schedules, e.g. from a
   cache of an earlier sw_autotune on the same database and device. */
int sw_tune_set(sw_db_t db, const sw_tune_entry* entries, int32_t n);

/* Copy up to cap installed entries to out (HOST); returns how many exist. */
int32_t sw_tune_get(sw_db_t db, sw_tune_entry* out, int32_t cap);

/*
 * Status of the last search that used `workspace` (the first 16 bytes of the
 * workspace; cleared at the start of every search call, graph launches
 * included, and accumulated over a call's launch groups).  A search call
 * returns once its work is enqueued, so errors found on the device are
 * reported here:
 *   bad_query       nonzero if a query residue code was >= 32 (the search read
 *                   it modulo 32; its scores are meaningless)
 *   rescore_failed  subjects the exact int32 rescore gave up on (a bounded
 *                   wait timed out, or the subject exceeded the rescore
 *                   buffers); their score is stored as -1
 *   flagged         subjects the 16-bit pass sent to the int32 rescore
 *   bad_items       work items skipped as inconsistent with the launch (a
 *                   library bug; their subjects keep no score)
 */
typedef struct sw_status {
    int32_t bad_query;
    int32_t rescore_failed;
    int32_t flagged;
    int32_t bad_items;
} sw_status;

/* Enqueue on `stream` a copy of the status words into `out` (HOST memory,
   pinned for an asynchronous copy); read it once the stream has passed the
   copy.  Ordered after the search when enqueued on the search's stream. */
int sw_search_status_async(const void* workspace, sw_status* out, hipStream_t stream);

/* Error code of a status: SW_EBADRES (bad query code), else SW_ERESCORE
   (rescore incomplete), else SW_EINTERNAL (skipped items), else SW_OK. */
int sw_status_code(const sw_status* status);

/* Blocking form: copy the status words, synchronise `stream`, fill `out`
   (may be NULL) and return sw_status_code of it (or SW_EHIP). */
int sw_search_status(const void* workspace, hipStream_t stream, sw_status* out);

/*
 * Number of subjects the last search that used `workspace` sent to the int32
 * rescore (16-bit modes; the status's `flagged`).  Synchronises `stream`.
 * Negative on error.
 */
int64_t sw_flagged_count(const void* workspace, hipStream_t stream);

const char* sw_strerror(int code);
const char* sw_last_error(void);   /* thread-local detail of the last failure */
const char* sw_version(void);

/* ------------------------------------------------------------------ one long pair
 *
 * Intra-task alignment (paper Section 2.2, Fig. 1; the pairwise DNA workload
 * of Section 4.1): the score of ONE pair, query `query[m]` along the rows and
 * subject `subject[n]` along the columns, with the whole device working on the
 * single matrix.  The matrix is cut into bands of K*R query rows (R = 8 or 16
 * rows per lane, K lanes pipelined per band, int32 lanes) and each band into
 * chunks of `cols` subject columns, every lane's chunk starting one column
 * after the row block above it (skewed tiles: lane g of band b covers columns
 * [c*cols - b*kr - g, +cols) in chunk c, kr = K rounded up to 16); the tiles of
 * each anti-diagonal b + c run in one launch and pass their boundary rows and
 * columns to the next launch through the workspace.  Same recurrence, borders
 * and result as sw_db_search; int32 score.
 */
typedef struct sw_pair_stats {
    int32_t rows;          /* R: query rows per lane                              */
    int32_t lanes;         /* K: lanes per band (band = R*K query rows)           */
    int32_t cols;          /* subject columns per tile (0 for the pipelined pass) */
    int32_t flow;          /* 1: one pipelined launch; 0: anti-diagonal tiles     */
    int64_t bands;         /* ceil(m / (R*K))                                     */
    int64_t chunks;        /* ceil(n / cols)                                      */
    int64_t launches;      /* anti-diagonals holding tiles (one launch each)      */
    double est_ms;         /* the planner's time model                            */
    int64_t workspace;     /* sw_pair_workspace_bytes                             */
    int32_t groups;        /* pipelined pass: workgroups (one per CU)             */
    int32_t group_waves;   /* pipelined pass: waves per workgroup, one band each
                              at a time (group_waves / 4 per SIMD)               */
} sw_pair_stats;

/* Workspace bytes sw_pair_score needs for lengths m, n (0 on invalid input);
   independent of the matrix and the device. */
size_t sw_pair_workspace_bytes(int64_t m, int64_t n, const sw_options* opt);

/* The schedule sw_pair_score would run on a device with `cu_count` compute
   units (0 = 256); host only.  opt->pair_rows fixes R, opt->max_lanes (a
   power of two) K, opt->pair_cols the chunk width. */
int sw_pair_plan(int64_t m, int64_t n, const sw_options* opt, int32_t cu_count, sw_pair_stats* out);

/*
 * Score of one pair.
 *   query, subject  device, uint8[m], uint8[n]; codes are read modulo 32
 *                   (m, n in [0, SW_MAX_QLEN])
 *   subst_matrix    HOST, int32[32*32], row = query residue, entries in [-128, 127]
 *   gap_open/extend as in sw_db_search
 *   opt             NULL or options (pair_rows, max_lanes, pair_cols,
 *                   ev_search_begin/end around the tile launches)
 *   workspace       device, >= sw_pair_workspace_bytes(m, n, opt), 256-byte aligned
 *   score_out       device, int32[1]
 * Asynchronous on `stream`; enqueues one preparation kernel, the profile
 * kernel and one tile launch per anti-diagonal (sw_pair_stats.launches).
 * Returns SW_EINVAL, SW_ENOMEM (workspace too small) or SW_EHIP.
 */
int sw_pair_score(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n,
                  const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                  const sw_options* opt, void* workspace, size_t ws_bytes, int32_t* score_out,
                  hipStream_t stream);

/*
 * Score of one pair without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): sw_pair_score with its workspace taken from a
 * static device array of SW_STATIC_SCRATCH_BYTES (64 MiB) that the library
 * holds on every GPU it runs on until the process ends.  Arguments as for
 * sw_pair_score, minus the workspace.  Returns SW_ENOMEM, with nothing
 * enqueued, if the pair needs more scratch than that
 * (sw_pair_workspace_bytes(m, n, opt) > SW_STATIC_SCRATCH_BYTES: the
 * paper's smallest DNA pair, 162,000 x 172,000, needs 25 MiB; m = n =
 * 400,000 needs 61 MiB).
 * All calls on one GPU share its array: calls that overlap in time on one
 * GPU (different streams, or threads) race and give wrong scores; serialise
 * them on one stream.  Calls no hipMalloc or hipFree.
 */
#define SW_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int sw_pair_score_static(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n,
                         const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                         const sw_options* opt, int32_t* score_out, hipStream_t stream);

/* ------------------------------------------------------------------ alignment of one pair
 *
 * The optional traceback after the score (paper Section 2.2: the alignment
 * itself can be recovered from the matrix when it is wanted): the optimal
 * local alignment of one pair, not only its score.  Two passes: the score (with whole-matrix
 * codes from the pipelined pass when the planner picks it, else the pair
 * tiles), then the pair tiles (8 query rows per lane, 64 lanes per band)
 * writing a 4-bit direction code per cell and finding the end cell; one
 * wavefront then walks the codes back.  With whole-matrix codes the tile
 * passes run skewed tiles; the passes of a blocked alignment run rectangular
 * tiles (lane g on column step - g of its chunk), whose checkpoint columns
 * and blocks follow columns.  Beyond 2^35 cells (or with options.align_block)
 * the score pass also keeps checkpoint rows and columns at block edges, and
 * the codes are recomputed block by block along the walk (the blocks above,
 * to the left and above-left of the walk's block on three more streams beside
 * it, where the walk usually goes next); the alignment is the same.
 * Tie-breaks (the paper gives none): the end is the first
 * cell holding the score in column-major order (smallest subject position,
 * then smallest query position); walking back, the diagonal is taken before E
 * before F, a gap is opened (from H) rather than extended when both give its
 * value, and the alignment begins at the first residue pair whose
 * predecessor holds H = 0 or lies on the border.
 */
typedef struct sw_alignment {
    int32_t score;
    int32_t q_begin, s_begin;  /* 1-based, inclusive (0 when score = 0)        */
    int32_t q_end, s_end;
    int32_t n_ops;             /* operations written (-1: inconsistent codes)  */
} sw_alignment;

/* Workspace bytes sw_align_pair needs (0 on invalid input).  Whole-matrix
   direction codes (m * n <= 2^35 and options.align_block = 0) take half a
   byte per cell: about m * n / 2 bytes (14.6 GB for 162K x 172K).  Blocks of
   side B take about 16 * m * n / B + 2 B^2 bytes (10.8 GB for 1M x 1M with
   B = 65536). */
size_t sw_align_workspace_bytes(int64_t m, int64_t n, const sw_options* opt);

/*
 * Optimal local alignment of query[m] (rows) against subject[n] (columns).
 *   query, subject  device, uint8 codes (read modulo 32)
 *   subst_matrix    HOST, int32[32*32]; gap_open/extend as in sw_db_search
 *   opt             NULL or options (pair_cols; align_block; ev_search_begin
 *                   / end around the tile passes)
 *   workspace       device, >= sw_align_workspace_bytes(m, n, opt), 256-byte aligned
 *   out             device, one sw_alignment
 *   ops             device, char[m + n]: 'M' (query residue paired with a
 *                   subject residue), 'I' (query residue against a gap), 'D'
 *                   (subject residue against a gap), begin to end; out->n_ops
 *                   of them are written
 * Asynchronous on `stream` with whole-matrix codes; with blocks the call
 * reads the walk's position after each block and returns with the stream
 * drained.  With whole-matrix codes either pass may run on the pipelined
 * pass (as in sw_pair_score); out->score = -1 (and no operations) then means
 * that a wait of that pass gave up, an error.  Returns SW_EINVAL, SW_ENOMEM
 * or SW_EHIP.
 */
int sw_align_pair(const uint8_t* query, int64_t m, const uint8_t* subject, int64_t n,
                  const int32_t* subst_matrix, int32_t gap_open, int32_t gap_extend,
                  const sw_options* opt, void* workspace, size_t ws_bytes, sw_alignment* out,
                  char* ops, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SWDB_H */
