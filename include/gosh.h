/*
 * gosh.h -- C ABI of the MI355X (gfx950) GOSH hot path.
 *
 * Method: "Boosting Graph Embedding on a Single GPU" (arXiv 2110.10049).
 * A graph G_0 is coarsened level by level (MultiEdgeCollapse, Algorithm 4,
 * Section 4); the levels are trained coarsest first (TrainInGPU,
 * Algorithm 3, Section 3.1, built on UpdateEmbed, Algorithm 1) and each
 * trained level is expanded onto the next finer one (ExpandEmbedding of
 * Algorithm 2, Section 3).
 *
 * Conventions
 *  - Every function returns gosh_status; none throws or aborts.  After a
 *    failure, gosh_last_error(ctx) returns a message (valid until the next
 *    call on that context).
 *  - Pointers named `*_dev` or documented as device pointers are HIP device
 *    memory owned by the caller unless stated otherwise; host pointers are
 *    named `*_host`.
 *  - All device work of a context is ordered on the context's stream
 *    (gosh_ctx_create / gosh_set_stream).  Calls marked "asynchronous" only
 *    enqueue; gosh_sync waits for them.
 *  - A graph is a simple undirected graph stored as CSR with both
 *    directions present: offsets[n+1] (int32 or int64, offsets[0] = 0,
 *    non-decreasing, offsets[n] = nnz), indices[nnz] int32 in [0, n), rows
 *    strictly ascending, no self-loops, symmetric.
 *  - Embeddings are row-major [n, d] arrays of float32 or bfloat16.
 *  - Random numbers come from Philox4x32-10 (Salmon et al., SC'11) keyed by
 *    the context seed, with counter (src, epoch, level | tag << 8,
 *    kind << 24 | slot << 16 | block): kind 0 draws the samples of a source,
 *    kind 1 gives stochastic-rounding bits (slot t = update t of the visit,
 *    slot 255 = the source row's write-back; element e of a d-wide row is in
 *    32-bit word w = e/2, which draws block w mod (d/8) and uses its 16-bit
 *    half 2*(w div (d/8)) + e mod 2, low half of each output word first).
 */
#ifndef GOSH_H
#define GOSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GOSH_OK = 0,
    GOSH_E_INVALID_ARG = 1,   /* bad argument (null pointer, size, d, k, lr ...) */
    GOSH_E_BAD_GRAPH = 2,     /* CSR violates the graph convention above        */
    GOSH_E_OOM = 3,           /* device allocation failed                       */
    GOSH_E_CAP_EXCEEDED = 4,  /* the context's memory cap would be exceeded     */
    GOSH_E_UNSUPPORTED = 5,   /* valid request this build does not implement    */
    GOSH_E_DEVICE = 6         /* HIP runtime error                              */
} gosh_status;

typedef enum { GOSH_F32 = 0, GOSH_BF16 = 1 } gosh_dtype;

typedef struct gosh_ctx gosh_ctx;
typedef struct gosh_levels gosh_levels;
typedef struct gosh_mlp gosh_mlp;

/* Borrowed device view of a CSR graph (see conventions). */
typedef struct {
    int64_t n;                /* |V|                                         */
    int64_t nnz;              /* stored directed entries = 2 |E|             */
    const void* offsets;      /* device, n+1 entries of int32 or int64       */
    int32_t offsets_is_i64;   /* 0: int32 offsets, 1: int64 offsets          */
    const int32_t* indices;   /* device, nnz entries                         */
} gosh_csr;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  `seed` keys every Philox
 * stream.  `hip_stream` is the hipStream_t to order work on (NULL: the
 * device's null stream).  `mem_cap_bytes` caps the device memory the
 * library allocates for this context (0 = no cap); allocations beyond it
 * fail with GOSH_E_CAP_EXCEEDED.  On success *out owns the context. */
gosh_status gosh_ctx_create(int device, uint64_t seed, void* hip_stream,
                            uint64_t mem_cap_bytes, gosh_ctx** out);
/* Frees the context and all device memory it allocated, including that of
 * level hierarchies still alive; those can then only be destroyed. */
gosh_status gosh_ctx_destroy(gosh_ctx* ctx);
/* Orders subsequent work on `hip_stream` (NULL: the null stream).  Waits
 * for the work already queued on the previous stream first, since temporary
 * blocks of asynchronous calls return to the context's cache when the call
 * returns and may be handed out again on the new stream. */
gosh_status gosh_set_stream(gosh_ctx* ctx, void* hip_stream);
/* Blocks until all work enqueued by the context has finished; returns
 * GOSH_E_DEVICE if a resident launch's barrier expired since the last call
 * (see gosh_set_resident_epochs). */
gosh_status gosh_sync(gosh_ctx* ctx);
const char* gosh_last_error(const gosh_ctx* ctx);
/* Bytes currently allocated by the library for this context. */
gosh_status gosh_mem_in_use(const gosh_ctx* ctx, uint64_t* bytes);
/* Releases the device blocks the context keeps cached for reuse (every
 * temporary of the library returns to this cache, and later calls take
 * blocks of a fitting size from it before allocating).  Waits for the
 * context stream.  Live levels, networks and the caller's buffers are not
 * affected. */
gosh_status gosh_trim(gosh_ctx* ctx);

/* Debug mode: when on, gosh_train visits sources strictly one after another
 * in ascending id order (the sequential semantics of Algorithm 3 with its
 * parallel loop run in order), so results are reproducible.  Default off:
 * sources of an epoch run concurrently without locks (Section 3.1). */
gosh_status gosh_set_deterministic(gosh_ctx* ctx, int on);

/* Mapping step of MultiEdgeCollapse used by gosh_coarsen. */
typedef enum {
    GOSH_COARSEN_EXACT = 0,      /* Algorithm 4's result exactly (default)                    */
    GOSH_COARSEN_LOCK_SKIP = 1   /* the paper's parallel lock-and-skip mapping (Section 4)    */
} gosh_coarsen_mode;

/* Selects the mapping step of gosh_coarsen.  GOSH_COARSEN_EXACT computes the
 * clusters of sequential Algorithm 4 (bit-exact, deterministic).
 * GOSH_COARSEN_LOCK_SKIP runs the parallel scheme of Section 4: vertices are
 * taken in Algorithm 4's order by concurrent threads, `batch` of them per
 * launch (0: max(64, n/64) per level); an unmarked vertex is claimed as a
 * hub and marks its unmarked neighbours over eligible edges, each mark a
 * compare-and-swap, and a vertex already marked by another thread is
 * skipped.  Every cluster is still a hub with eligible neighbours, cluster
 * ids count hubs in Algorithm 4's order, but the clusters depend on thread
 * timing (more, smaller clusters than the exact mapping when many vertices
 * run at once).  In deterministic mode one wave takes all vertices in
 * order, which is Algorithm 4 exactly.  batch >= 0. */
gosh_status gosh_set_coarsen_mode(gosh_ctx* ctx, gosh_coarsen_mode mode, int64_t batch);

/* Concurrent epochs on large levels (the extension the paper suggests in
 * Section 6.3: overlapping epochs on the upper levels, full synchronisation
 * elsewhere): gosh_train runs `epochs_in_flight` consecutive epochs in one
 * launch, with no barrier between them, on levels of at least
 * `min_vertices` vertices; smaller levels keep one epoch per launch.  Each
 * visit keeps its own epoch's samples and lr.  1 (the default) restores
 * Algorithm 3's barriers everywhere.  Ignored in deterministic mode.
 * epochs_in_flight in [1, 64], min_vertices >= 0. */
gosh_status gosh_set_epoch_overlap(gosh_ctx* ctx, int32_t epochs_in_flight, int64_t min_vertices);

/* Small levels: gosh_train runs all epochs of a call on a level of at most
 * `max_vertices` vertices in one cooperative launch, with a device-wide
 * barrier between epochs instead of a launch boundary (Algorithm 3's epochs
 * still never overlap; every visit draws the same samples and uses the same
 * lr and rounding bits as with one launch per epoch).  Levels where negatives
 * are stored plainly (gosh_set_plain_negatives) keep one launch per epoch.
 * The barrier's wait is bounded (a few seconds); if one ever expires the
 * rows are invalid and the next gosh_sync returns GOSH_E_DEVICE.  0 turns it
 * off; ignored in deterministic mode and with overlapping epochs.  Default:
 * 0 (off): measured on MI355X, a level's epochs run faster as separate
 * launches, since after every barrier the rows must be read coherently
 * across the dies.  max_vertices >= 0. */
gosh_status gosh_set_resident_epochs(gosh_ctx* ctx, int64_t max_vertices);

/* Hot coarse levels in LDS: gosh_train trains a level of at most
 * `max_vertices` vertices whose rows and one epoch's samples fit in the
 * 160 KiB LDS of one compute unit (n d b + 4 n (1 + k) bytes, b = 4 for
 * FP32, 2 for BF16) inside a single workgroup of 16 waves: the rows are read
 * from HBM once, every epoch draws the samples of all sources into an LDS
 * table (the same Philox draws as the per-epoch launch) and then visits the
 * sources with the rows in LDS, a workgroup barrier between epochs (Section
 * 3.1's shared-memory staging applied to the whole level), and the rows are
 * written back once.  The sources of an epoch run concurrently over the 16
 * waves; BF16 words are committed by LDS compare-and-swap (exactly the
 * stochastically rounded pair when uncontended, the change added to the
 * current value and rounded again otherwise).  Levels where negatives are
 * stored plainly keep one launch per epoch; ignored in deterministic mode
 * and with overlapping epochs.  gosh_train_batched applies the same to every
 * job of at most max_vertices vertices that fits: such jobs run first, one
 * workgroup each in one launch, the others as before (not
 * gosh_train_batched_noalloc).  Default 0 (off): measured on MI355X, one
 * launch per epoch over the whole device is faster for single levels (a
 * workgroup serialises an epoch into rounds of 64 visits).
 * max_vertices >= 0. */
gosh_status gosh_set_lds_levels(gosh_ctx* ctx, int64_t max_vertices);

/* Write discipline of negative samples (Section 3.1 lets the sources of an
 * epoch race on rows without locks).  By default every row change is applied
 * with atomic adds, so no concurrent update is lost.  With min_vertices > 0,
 * gosh_train and gosh_train_walks write the rows of negative samples with
 * plain stores of the new value (the paper's lock-free discipline) on levels
 * of at least min_vertices vertices: a negative is a uniform draw, so on a
 * large level two visits rarely hold the same negative row at once, while
 * the positive and source rows, which concentrate on high-degree vertices,
 * keep their atomic adds.  A store may overwrite an update that another
 * visit applied to the same row in the meantime (which the paper's kernel
 * accepts for every row).  0 (the default) turns it off; ignored in
 * deterministic mode.  min_vertices >= 0. */
gosh_status gosh_set_plain_negatives(gosh_ctx* ctx, int64_t min_vertices);

/* Write discipline by degree (Section 3.1's lock-free sources; Section 4.1's
 * hub definition).  With min_vertices > 0, gosh_train and gosh_train_walks
 * write every row of
 * degree at most the level's average (deg * n <= nnz: not a hub) with plain
 * stores of the new value -- the source, the positive and the negatives
 * alike -- on levels of at least min_vertices vertices, and keeps the atomic
 * commits for hub rows.  A light row is touched a few times per epoch, so a
 * store rarely overwrites a concurrent update, while hub rows, which take
 * most positive updates, lose none.  The atomic units bound the training
 * kernel, and most rows are light.  Also applied in deterministic mode,
 * where it changes no bit (one visit at a time).  Levels it applies to keep
 * one launch per epoch.  0 (the default) turns it off.  min_vertices >= 0. */
gosh_status gosh_set_plain_light_rows(gosh_ctx* ctx, int64_t min_vertices);

/* Grouped visits of hot positives (a schedule of Algorithm 3's concurrent
 * sources; Section 3.1): on levels with min_vertices <= n <= max_vertices,
 * each epoch of gosh_train first draws every source's samples (the same
 * draws) and files the visits whose positive is a hub of degree at least
 * hot_factor times the level's average (the first 4,096 such ids) into one
 * bucket per hub; one launch then runs the other visits and, per chunk of
 * the bucketed visits of one hub (as many as a workgroup has lane groups),
 * a workgroup that reads the hub row once, runs the chunk's visits against
 * that copy with their changes to it summed in FP32, and commits the sum
 * once (BF16: stochastically rounded once per chunk, exact commit).  No
 * change is lost; a chunk's visits read the hub row as it was when the chunk
 * started.  The draws of up to 16 epochs are made in one launch, into
 * device memory of 4 (n (1+k) + the hubs' degree sum) bytes per epoch of the
 * batch (batches kept within 256 MiB, at least one epoch), allocated per
 * call.  Not used in deterministic mode, with overlapping epochs or on
 * levels where light rows are stored plainly.  The result is one of the
 * interleavings Algorithm 3's concurrent sources allow, but not the one the
 * per-epoch launch takes: on the scale-20 R-MAT workload (level 1 grouped,
 * hot_factor 64) the level after it ends with a last-epoch loss 1.5-2% above
 * the ungrouped run's.  max_vertices = 0 (the default) turns it off;
 * hot_factor defaults to 64.  min_vertices, max_vertices >= 0,
 * hot_factor >= 1. */
gosh_status gosh_set_grouped_positives(gosh_ctx* ctx, int64_t min_vertices, int64_t max_vertices, double hot_factor);

/* Running loss of training (the objective of Section 2, the logistic loss of
 * the classifier sigma(M[v].M[u]) on the positive and negative samples).
 * When loss_dev is not NULL, every later gosh_train call adds to
 * loss_dev[j] the running loss of its epoch j: the sum over the epoch's
 * executed UpdateEmbed calls of -log sigma(x) (positive) or
 * -log(1 - sigma(x)) (negative), x the dot product the update reads before
 * it changes the rows; gosh_update_batch adds its batch's sum to loss_dev[0].
 * Terms are FP32, summed in FP32 within a wave and in FP64 across waves
 * (atomic adds, so the last bits depend on timing; in deterministic mode
 * every visit's terms are summed in FP64 in source order).  The caller
 * zeroes the buffer.  A gosh_train call with more epochs than `capacity`
 * returns GOSH_E_INVALID_ARG.  loss_dev: device, caller-owned, `capacity`
 * doubles; NULL (the default) turns recording off.  Recording adds a few
 * instructions and one atomic per wave to every visit. */
gosh_status gosh_set_loss_record(gosh_ctx* ctx, double* loss_dev, int64_t capacity);

/* Test hook: when samples_dev is not NULL, gosh_train writes the samples
 * each visit draws inside the training kernel to samples_dev[src * (1+k) +
 * t] (t = 0 the positive, -1 for a source without neighbours; t >= 1 the
 * negatives), overwriting them every epoch (with overlapping epochs, the
 * entries of one of the launch's epochs remain).  A gosh_train call on a
 * level with n * (1 + k) > capacity returns GOSH_E_INVALID_ARG.
 * samples_dev: device, caller-owned int32; NULL (the default) turns it off. */
gosh_status gosh_set_draw_record(gosh_ctx* ctx, int32_t* samples_dev, int64_t capacity);

/* ---------------------------------------------------------------- graphs */

/* Checks `g` against the graph convention (Section 4.1: the method works on
 * CSR).  check_symmetry != 0 also verifies that every (v,u) has (u,v).
 * Synchronous.  GOSH_E_BAD_GRAPH names the first violated rule. */
gosh_status gosh_validate_csr(gosh_ctx* ctx, const gosh_csr* g, int check_symmetry);

/* MultiEdgeCollapse (Algorithm 4, Section 4).  Coarsens `g0` level by
 * level: vertices are visited by decreasing degree (ties: ascending id); an
 * unmarked vertex opens the next cluster id and takes every unmarked
 * neighbour reached over an edge allowed by the hub^2 restriction
 * (deg(v) <= nnz/n or deg(u) <= nnz/n); the coarse graph keeps one edge per
 * pair of distinct clusters.  A level is appended, then coarsening stops
 * when |V_{i+1}| < threshold or |V_{i+1}| > max_ratio * |V_i|.  The result
 * equals the sequential algorithm exactly.
 * `g0` is borrowed and must outlive *out.  Synchronous (level sizes drive
 * allocation).  *out owns levels 1..D-1 (device CSR with the offset width
 * of g0), the maps map_0..map_{D-2} and the cluster sizes. */
gosh_status gosh_coarsen(gosh_ctx* ctx, const gosh_csr* g0, int64_t threshold,
                         double max_ratio, gosh_levels** out);
/* Wraps `g0` as a single-level hierarchy (no coarsening, D = 1). */
gosh_status gosh_levels_single(gosh_ctx* ctx, const gosh_csr* g0, gosh_levels** out);
gosh_status gosh_levels_destroy(gosh_levels* lv);
gosh_status gosh_levels_count(const gosh_levels* lv, int32_t* D);
gosh_status gosh_level_shape(const gosh_levels* lv, int32_t level, int64_t* n, int64_t* nnz);
/* Device view of level `level` (valid while lv lives). */
gosh_status gosh_level_csr(const gosh_levels* lv, int32_t level, gosh_csr* out);
/* Device pointer to map_level (|V_level| int32 entries, values in
 * [0, |V_{level+1}|)) and to the sizes of level+1's clusters (|V_{level+1}|
 * int32; computed on the context stream at the first request). */
gosh_status gosh_level_map(const gosh_levels* lv, int32_t level, const int32_t** map_dev,
                           const int32_t** clsz_dev);
/* Copies a level to host memory; any of the pointers may be NULL.
 * offsets_host receives n+1 int64 values whatever the device width;
 * map_host receives map_level and clsz_host the |V_{level+1}| cluster sizes
 * (both invalid for the coarsest level).  Synchronous. */
gosh_status gosh_level_copy_out(gosh_ctx* ctx, const gosh_levels* lv, int32_t level,
                                int64_t* offsets_host, int32_t* indices_host,
                                int32_t* map_host, int32_t* clsz_host);

/* ---------------------------------------------------------------- training */

/* Epoch distribution (Section 3): a share p of the e epochs is spread evenly
 * over the D levels and the rest geometrically, each coarser level getting
 * twice the finer one's share; integer epochs by floor, the remainder one
 * each to the largest fractional parts (ties to the coarser level).
 * e_out[i] for level i (0 = finest).  Host function. */
gosh_status gosh_epoch_schedule(int32_t e, double p, int32_t D, int32_t* e_out);

/* TrainInGPU (Algorithm 3) on level `level` of `lv`: `epochs` epochs run
 * one after another; in epoch j every source vertex draws one positive
 * (uniform neighbour; none if it has no neighbour) and k negatives (uniform
 * over the level's vertices; one equal to the source is skipped) and
 * applies UpdateEmbed (Algorithm 1) to each in turn with
 * lr' = lr * max(1 - j/epochs, 1e-4): x = M[src].M[u],
 * score = (b - sigmoid(x)) * lr', M[src] += score M[u], then
 * M[u] += score M[src] with the updated source row.
 * `emb` is a caller-owned device array [n_level, d] of `dt`, updated in
 * place.  Sources of an epoch run concurrently; every row change is applied
 * atomically by default (FP32: atomic adds per element; BF16, per 2-element
 * word: the packed atomic add of the difference to the rounded value when
 * that difference is a BF16 value, else two exact packed adds through zero,
 * -cur then +rounded), so concurrent updates of a shared row are all kept
 * and an uncontended word holds exactly its rounded value
 * (gosh_set_plain_negatives and gosh_set_plain_light_rows store some rows
 * plainly instead).  BF16 rows are widened to FP32 for
 * the arithmetic and every written row is stochastically rounded back
 * (sample rows once per update, the source row once per visit).  d in {8,16,32,64,128,256}, 0 <= k <= 15,
 * lr finite and >= 0.  `tag` (24 bits) separates independent random
 * streams.  If `updates_dev` is not NULL, the number of UpdateEmbed calls
 * executed is added to *updates_dev (device uint64).  An epoch is one
 * launch with up to 16 lanes per source (32 at d = 256): a level whose
 * vertices times lanes reach 2^32 - 4096 (268M vertices at d = 128)
 * returns GOSH_E_UNSUPPORTED outside deterministic mode.  Asynchronous. */
gosh_status gosh_train(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, void* emb,
                       gosh_dtype dt, int32_t d, int32_t epochs, float lr, int32_t k,
                       uint32_t tag, uint64_t* updates_dev);

/* Random-walk positive sampling (Section 3.2) on level `level` of `lv`, in
 * place of the one-neighbour positives of gosh_train: epoch j starts one
 * walk of `walk_len` steps at every vertex v (w_0 = v; step i picks the
 * neighbour floor(r deg / 2^32) of the current vertex with r = word i mod 4
 * of the stream (v, j, kind 4, block i div 4); a walk stops early at a
 * vertex without neighbours).  Every pair (w_a, w_b) with
 * 0 < b - a <= window is a positive sample with source w_a.  With P the
 * number of offsets (a, b), 0 <= a < b <= walk_len, b - a <= window, taken in
 * order of a then b, pair q = v P + l is offset l of walk v; the epoch visits
 * the n P pairs sorted by the key word 0 of stream (q, j, kind 5), ties by q
 * (a shuffle of the epoch's samples).  The pair at rank r draws k negatives
 * uniformly over the level's vertices from words 1..k of stream (r, j,
 * kind 6) and applies UpdateEmbed (Algorithm 1) as gosh_train does, with
 * lr' = lr * max(1 - j/epochs, 1e-4), a sample equal to its source skipped
 * and BF16 rounding bits from stream (r, j, kind 7, slot, block) laid out as
 * for kind 1.  Pairs past the end of a shortened walk are skipped.  Pairs of
 * an epoch run concurrently with atomic row updates (as gosh_train); in
 * deterministic mode they run one at a time in rank order.
 * 0 <= walk_len <= 1024, window >= 0; n * P must be below 2^32
 * (GOSH_E_UNSUPPORTED otherwise).  Device memory: 4 n (walk_len + 1) +
 * 16 n P bytes of scratch for the walks and the shuffle, taken from the
 * context (GOSH_E_CAP_EXCEEDED under its cap).  Other arguments and errors
 * as gosh_train.  Asynchronous when timing_host is NULL; otherwise the call
 * waits for its work and fills *timing_host. */
typedef struct {
    double sample_ms;   /* device time of the walks, shuffle keys and sort, all epochs */
    double train_ms;    /* device time of the update launches, all epochs             */
    int32_t epochs;     /* epochs run                                                 */
} gosh_walk_timing;

gosh_status gosh_train_walks(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, void* emb,
                             gosh_dtype dt, int32_t d, int32_t epochs, float lr, int32_t k,
                             int32_t walk_len, int32_t window, uint32_t tag, uint64_t* updates_dev,
                             gosh_walk_timing* timing_host);

/* The positive pairs of epoch `epoch` of gosh_train_walks in visiting order:
 * src_dev[r], pos_dev[r] for the pair at rank r (both -1 for a pair past the
 * end of its walk).  *count receives n P.  With src_dev and pos_dev both NULL
 * only *count is set; otherwise both must hold `capacity` >= n P entries
 * (GOSH_E_INVALID_ARG).  Asynchronous. */
gosh_status gosh_walk_pairs(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, int32_t epoch,
                            int32_t walk_len, int32_t window, uint32_t tag, int32_t* src_dev,
                            int32_t* pos_dev, int64_t capacity, int64_t* count);

/* One independent training job of gosh_train_batched. */
typedef struct {
    gosh_csr g;          /* the job's graph (device, borrowed; must satisfy the graph
                            convention, e.g. a level of gosh_coarsen or a graph accepted
                            by gosh_validate_csr)                                      */
    void* emb;           /* device [g.n, d] rows of the call's dtype, updated in place */
    int32_t epochs;      /* epochs of this job (its lr decays over these)              */
    float lr;            /* initial learning rate                                      */
    int32_t level;       /* level field of the job's Philox counters (0..255)          */
    uint32_t tag;        /* tag field of the job's Philox counters (24 bits)           */
} gosh_job;

typedef enum {
    GOSH_BATCH_AUTO = 0,        /* autotuned per (dtype, d, k, size class), cached  */
    GOSH_BATCH_PERSISTENT = 1,  /* one persistent launch, per-job epoch barriers    */
    GOSH_BATCH_EPOCH_GRAPH = 2  /* one launch per epoch round, chained in a hipGraph */
} gosh_batch_mode;

/* Trains `njobs` independent jobs (Algorithm 3 on each job's graph, Section
 * 3.1): every job gets exactly the semantics of gosh_train on its own graph
 * with its own epochs, lr, level and tag (its epochs never overlap; jobs do
 * not wait for one another).  d, k and dtype are shared.  Meant for many
 * small graphs and for small coarse levels, where one launch per epoch and
 * graph would leave the device mostly idle.  GOSH_BATCH_AUTO times the
 * executions on a dry run of up to 8 epochs over scratch copies of the rows the
 * first time a (dtype, d, k, size class) is seen and caches the winner (also
 * appended to the file named by the GOSH_TUNE_CACHE environment variable).
 * chosen_out (may be NULL) receives {mode, blocks per CU, chunk length} of
 * the execution used.  In deterministic mode (gosh_set_deterministic) the
 * persistent launch is used with each job epoch as one task whose sources
 * are visited one at a time in ascending id order: every job then gets
 * exactly the result of gosh_train in deterministic mode (sequential
 * Algorithm 3), independent of timing; chosen_out reports chunk length 0.
 * Synchronous.  Errors as gosh_train; a scheduling failure inside the
 * persistent launch returns GOSH_E_DEVICE. */
gosh_status gosh_train_batched(gosh_ctx* ctx, const gosh_job* jobs_host, int32_t njobs,
                               gosh_dtype dt, int32_t d, int32_t k, gosh_batch_mode mode,
                               uint64_t* updates_dev, int32_t* chosen_out);

/* gosh_train_batched for callers that cannot allocate device memory (code
 * recorded into a HIP graph by stream capture, tight serving loops, hosts
 * that forbid allocation during a run): the same persistent execution, with
 * no hipMalloc, hipFree or other allocating call.  Its device tables (job
 * table, per-round task starts, per-job done counters, task counter, error
 * word) live in a static device array of 524,800 bytes that every GPU the library
 * runs on holds until the process ends, set up by gosh_ctx_create.  Limits:
 * at most 4096 jobs with work and at most 16384 epochs per job
 * (GOSH_E_INVALID_ARG beyond).  Every call on a GPU shares that GPU's
 * array: calls that overlap in time on one GPU (from several contexts or
 * streams) race and must not be issued; each call clears the counters it
 * uses.  Jobs, rows, dtype, d, k and the update counter as
 * gosh_train_batched; the execution is GOSH_BATCH_PERSISTENT (2 blocks per
 * CU, tasks of 4 waves' sources), or in deterministic mode each job epoch
 * one task visited in source order (then every job equals gosh_train in
 * deterministic mode).  Synchronous (it waits for the stream to read the
 * error word); a scheduling failure returns GOSH_E_DEVICE. */
gosh_status gosh_train_batched_noalloc(gosh_ctx* ctx, const gosh_job* jobs_host, int32_t njobs, gosh_dtype dt,
                                       int32_t d, int32_t k, uint64_t* updates_dev);

/* ExpandEmbedding (Algorithm 2): every vertex v of level fine_level starts
 * from the trained row of its super vertex.  mlp == NULL: copy,
 * fine[v] = coarse[map_{fine_level}[v]] (bit-exact).  Otherwise the learned
 * prolongation (an addition, not in the paper): with c = coarse[map v],
 * y = c + W2 GELU(W1 [c, log1p(deg v), log(clsz(map v))] + b1) + b2, where
 * deg is v's degree in level fine_level and clsz the size of its cluster;
 * products in BF16 with FP32 accumulation, c, the biases and the sum in
 * FP32, BF16 rows rounded to nearest even.  W2 = 0, b2 = 0 reproduces the
 * copy exactly.  coarse_emb: [n_{fine_level+1}, d], fine_emb:
 * [n_{fine_level}, d], both device, same dtype, not overlapping; the
 * network's d must equal d.  Asynchronous. */
gosh_status gosh_prolong(gosh_ctx* ctx, const gosh_levels* lv, int32_t fine_level,
                         const void* coarse_emb, void* fine_emb, gosh_dtype dt, int32_t d,
                         const gosh_mlp* mlp);

/* ---------------------------------------------------------------- partitioned embedding */

/* Parameters of the partitioned embedding of Section 5. */
typedef struct {
    int32_t parts;      /* K, the number of vertex parts (1..255); 0: the smallest K > sub_bins
                           whose device working set fits the budget (memory cap of the context,
                           else 90% of the free device memory)                            */
    int32_t sub_bins;   /* P_GPU: parts resident on the device at a time (2..16; 3)        */
    int32_t pool_bins;  /* S_GPU: sample pools resident on the device (1..16; 2)          */
    int32_t B;          /* positives per vertex and part pair in a round (1..31; 5)        */
    int32_t threads;    /* host sampler threads; 0: all hardware threads (at most 64)      */
} gosh_part_params;

typedef struct {
    int32_t parts;          /* K used                                                     */
    int32_t rounds;         /* ceil(epochs / B)                                           */
    int64_t positives;      /* positive visits run (at most epochs * n)                   */
    int64_t pool_entries;   /* pool entries copied to the device (= positives)            */
    int64_t part_loads;     /* host-to-device part copies                                 */
    int64_t part_stores;    /* device-to-host part copies                                 */
    int64_t kernels;        /* pair kernels launched                                      */
    double h2d_bytes;       /* bytes copied host to device (parts and pools)              */
    double d2h_bytes;       /* bytes copied device to host                                */
    double seconds;         /* wall time of the call                                      */
    double sample_seconds;  /* producer time spent building pools                         */
    double kernel_seconds;  /* sum of pair-kernel durations (kernels may overlap)         */
    uint64_t device_bytes;  /* device memory held by the context during the run           */
} gosh_part_stats;

/* Section 5: embeds a graph whose rows and adjacency stay in host memory.
 * The ids are split into K contiguous parts (part p = [floor(p n/K),
 * floor((p+1) n/K))).  Each of ceil(epochs/B) rounds runs a kernel K_{i,j}
 * for every part pair in inside-out order ((0,0), then (a, b+1) while a > b,
 * else (a+1, 0)); K_{i,j} visits, for every vertex u of part i with c > 0
 * neighbours in part j, B positives drawn uniformly among them on the host
 * (Philox: epoch round*B + b, slot j), and for i != j the same for part j
 * towards part i; each visit applies UpdateEmbed to its positive and to k
 * negatives drawn on the device uniformly from the opposite part, with
 * lr' = lr * max(1 - round/rounds, 1e-4).  Positive visits stop after
 * epochs * n (the pool sequence is cut in order).  With K = 1 and B = 1 this
 * is gosh_train's Algorithm 3 (for a graph without isolated vertices).
 * g_host: HOST arrays (offsets n+1 entries, int32 or int64; indices nnz
 * int32; symmetric, sorted rows, no self-loops; borrowed).  emb_host: HOST
 * rows [n, d] of dt, updated in place (pinned memory lets the copies run
 * asynchronously).  Rows move between host and device part by part, at most
 * sub_bins at a time; pools are built by host threads and copied while
 * kernels run.  Deterministic mode (gosh_set_deterministic) runs every
 * kernel on one wave in pool order.  updates_dev (device, may be NULL)
 * accumulates executed UpdateEmbed calls; stats (host, may be NULL).
 * Synchronous.  Errors: E_INVALID_ARG, E_CAP_EXCEEDED (no K fits),
 * E_UNSUPPORTED (a part above 2^27 rows), E_OOM (pinned host buffers). */
gosh_status gosh_train_partitioned(gosh_ctx* ctx, const gosh_csr* g_host, void* emb_host, gosh_dtype dt,
                                   int32_t d, int32_t epochs, float lr, int32_t k, int32_t level,
                                   uint32_t tag, const gosh_part_params* params, uint64_t* updates_dev,
                                   gosh_part_stats* stats);

/* K chosen by gosh_train_partitioned for n rows under `budget` device bytes
 * (params->parts > 0 is returned as is), and the device bytes it needs.
 * Host only. */
gosh_status gosh_partition_plan(int64_t n, int32_t d, gosh_dtype dt, uint64_t budget,
                                const gosh_part_params* params, int32_t* parts_out, uint64_t* bytes_out);

/* The K(K+1)/2 part pairs in inside-out order: pairs_out[2q], pairs_out[2q+1].
 * Host only. */
gosh_status gosh_inside_out(int32_t K, int32_t* pairs_out);

/* Test hook (host only): pool S_{i,j} of `round` as gosh_train_partitioned
 * builds it with Philox key `seed`: *count entries (source id, positive id,
 * b), side i first.  Output arrays (host, may be NULL to count) need
 * `capacity` entries. */
gosh_status gosh_partition_pool(const gosh_csr* g_host, int32_t K, int32_t i, int32_t j, int32_t B,
                                uint64_t seed, int32_t level, uint32_t tag, int32_t round, int32_t threads,
                                int64_t* count, int32_t* src_out, int32_t* pos_out, int32_t* b_out,
                                int64_t capacity);

/* ---------------------------------------------------------------- learned prolongation */

/* Creates the prolongation network for rows of width d (32, 64, 128 or 256)
 * with `hidden` GELU units (64, 128 or 256).  The library owns its FP32
 * master weights, Adam moments and BF16 operand copies (device memory
 * charged to the context).  W1 is drawn uniformly from +-1/sqrt(d+2) with
 * the context's Philox key, b1, W2 and b2 start at 0 (so the network starts
 * as copy prolongation).  Destroy before or after the context (a network
 * whose context is gone only accepts gosh_mlp_destroy). */
gosh_status gosh_mlp_create(gosh_ctx* ctx, int32_t d, int32_t hidden, gosh_mlp** out);
gosh_status gosh_mlp_destroy(gosh_mlp* mlp);
/* Number of parameters P = hidden*(d+2) + hidden + d*hidden + d. */
gosh_status gosh_mlp_num_params(const gosh_mlp* mlp, int64_t* n);
/* Host FP32 parameter vector of P floats, in order W1 [hidden][d+2]
 * (row-major; column d is log1p(deg), column d+1 is log(clsz)), b1 [hidden],
 * W2 [d][hidden], b2 [d].  set also clears the Adam state.  Both
 * synchronous. */
gosh_status gosh_mlp_set_weights(gosh_ctx* ctx, gosh_mlp* mlp, const float* params_host);
gosh_status gosh_mlp_get_weights(gosh_ctx* ctx, const gosh_mlp* mlp, float* params_host);

/* An explicit batch of training rows (all device arrays of `rows` entries):
 * coarse rows [rows, d], fine degrees, cluster sizes (>= 1) and target rows
 * [rows, d]; rows of the call's dtype. */
typedef struct {
    int64_t rows;
    const void* coarse;
    const int32_t* deg;
    const int32_t* clsz;
    const void* target;
} gosh_mlp_batch;

/* Gradient of the mean squared error mean((y - target)^2) over all
 * rows*d entries with respect to the parameters, written to grads_dev
 * (device, P floats, parameter order as above); loss_dev (device float,
 * may be NULL) receives the loss.  Products in BF16 with FP32 accumulation
 * (inputs, hidden activations and output gradients rounded to BF16).
 * 1 <= rows <= 2^24.  Synchronous. */
gosh_status gosh_mlp_grad(gosh_ctx* ctx, gosh_mlp* mlp, gosh_dtype dt, const gosh_mlp_batch* batch,
                          float* grads_dev, float* loss_dev);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the
 * FP32 master weights with the given gradient (device, P floats).
 * Asynchronous. */
gosh_status gosh_mlp_adam_step(gosh_ctx* ctx, gosh_mlp* mlp, const float* grads_dev, float lr);

/* Training pairs: every vertex v of level `level` of lv (which must have a
 * coarser level) with input coarse[map v] (trained rows of level+1) and
 * target fine[v] (trained rows of level). */
typedef struct {
    const gosh_levels* lv;
    int32_t level;
    const void* coarse;
    const void* fine;
} gosh_mlp_source;

/* `steps` Adam steps (learning rate lr) on minibatches of `batch` pairs drawn
 * uniformly with replacement over the union of the sources' pairs (Philox
 * with the context key; `tag` separates runs).  loss_dev (device, `steps`
 * floats, may be NULL) receives each step's minibatch loss before its
 * update.  Synchronous. */
gosh_status gosh_mlp_train(gosh_ctx* ctx, gosh_mlp* mlp, gosh_dtype dt, const gosh_mlp_source* srcs_host,
                           int32_t nsrc, int32_t steps, int32_t batch, float lr, uint32_t tag,
                           float* loss_dev);

/* ---------------------------------------------------------------- test hooks */

/* Writes the samples of every source of level `level` for epoch `epoch`:
 * out_dev[src * (1+k) + 0] = positive (-1 if deg(src) = 0), [.. + t] =
 * negative t.  Asynchronous. */
gosh_status gosh_draw_samples(gosh_ctx* ctx, const gosh_levels* lv, int32_t level,
                              int32_t epoch, int32_t k, uint32_t tag, int32_t* out_dev);

/* UpdateEmbed over explicit samples: one source per entry of src_dev
 * (nsrc entries), samples_dev[i * (1+k) + t] as in gosh_draw_samples (-1 =
 * skip).  Rows are visited concurrently, so the result equals the
 * sequential one only when no row is touched by two listed sources.
 * Stochastic-rounding bits use (level, tag, epoch) and the source id.
 * emb_dev holds n_rows rows; every index must be < n_rows.  The write
 * discipline is gosh_train's for a level of n_rows vertices: with
 * gosh_set_plain_negatives(ctx, m), m > 0 and n_rows >= m (and not in
 * deterministic mode), negative rows are written with plain stores, so this
 * call runs the timed kernel's store path on chosen samples.  Asynchronous. */
gosh_status gosh_update_batch(gosh_ctx* ctx, void* emb_dev, gosh_dtype dt, int32_t d,
                              int64_t n_rows, int32_t nsrc, const int32_t* src_dev,
                              const int32_t* samples_dev, int32_t k, float lr,
                              int32_t level, uint32_t tag, int32_t epoch);

#ifdef __cplusplus
}
#endif
#endif
