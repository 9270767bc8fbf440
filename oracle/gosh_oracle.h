/*
 * GOSH CPU oracle (test infrastructure only).
 *
 * Plain, slow, single-threaded C11, FP64 for every real quantity.  It is the
 * reference that the HIP path is checked against and shares no code with it.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never does.
 *
 * Paper: "Boosting Graph Embedding on a Single GPU" (arXiv 2110.10049;
 * GOSH).  Algorithms are numbered in the paper's order:
 *   - UpdateEmbed .......... Algorithm 1 (Section 2)
 *   - TrainInGPU ........... Algorithm 3 (Section 3.1), lr decay (Section 3)
 *   - MultiEdgeCollapse .... Algorithm 4 (Section 4), CSR build (Section 4.1)
 *   - epoch distribution ... Section 3 (calculateEpochs of Algorithm 2)
 *   - partitioned embedding  Section 5 (parts, inside-out order, sample pools)
 *   - random-walk sampling . Section 3.2
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers:
 * As Easy as 1, 2, 3", SC'11.
 */
#ifndef GOSH_ORACLE_H
#define GOSH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32 with 10 rounds: out = philox(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* m blocks at once: ctr and out hold m consecutive 4-word groups. */
void orc_philox_many(const uint32_t *ctr, int64_t m, const uint32_t key[2], uint32_t *out);

/* One 128-bit block of the method's random stream.  Counter layout:
 *   ctr = (src, epoch, (level & 0xFF) | tag << 8, kind << 24 | slot << 16 | block)
 *   key = (seed low 32 bits, seed high 32 bits)
 * kind 0 = sample draws, kind 1 = stochastic-rounding bits. */
void orc_stream_block(uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                      int64_t src, uint32_t kind, uint32_t slot, uint32_t block,
                      uint32_t out[4]);

/* Samples of one source (Algorithm 3): out[0] = positive (uniform neighbour,
 * -1 when deg(src) = 0), out[1..k] = uniform negatives over [0, n). */
void orc_draw_samples(const int64_t* offsets, const int32_t* indices, int64_t n,
                      uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                      int64_t src, int32_t k, int32_t* out);

/* 16 stochastic-rounding bits for element e (row dimension d) of update
 * slot `slot`: element e sits in 32-bit word w = e/2; with L = d/8 the word
 * draws from block w mod L and takes half 2*(w div L) + e mod 2. */
uint32_t orc_sr_bits(uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                     int64_t src, uint32_t slot, int32_t e, int32_t d);

/* FP32 -> BF16 with stochastic rounding by 16 random bits. */
uint16_t orc_bf16_sr(float x, uint32_t r16);
/* FP32 -> BF16 round to nearest even. */
uint16_t orc_bf16_rne(float x);
double   orc_bf16_to_f64(uint16_t h);

double orc_sigmoid(double x);
/* -[b log s(x) + (1-b) log(1-s(x))], stable. */
double orc_loss(double x, int b);

/* Embedding storage.  bf16 == 0: rows are double[n*d]; bf16 != 0: rows are
 * uint16_t[n*d] BF16 bit patterns, updated with stochastic rounding. */
typedef struct {
    void*   rows;
    int32_t bf16;
    int32_t d;
} orc_emb;

/* Applies the updates of one source visit with explicit samples (slot 0 is
 * the positive, slots 1..k negatives; -1 or src itself = skipped).  Returns
 * the number of UpdateEmbed calls executed. */
int32_t orc_visit(orc_emb* M, int64_t src, const int32_t* samples, int32_t k,
                  double lr, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch);

/* Visits the listed sources in list order with explicit samples. */
int64_t orc_update_batch(orc_emb* M, int64_t nsrc, const int32_t* src,
                         const int32_t* samples, int32_t k, double lr,
                         uint64_t seed, int32_t level, uint32_t tag, int32_t epoch);

/* Sequential Algorithm 3: `epochs` passes, every source in [src_lo, src_hi)
 * in ascending id order, lr' = lr * max(1 - j/epochs, 1e-4) at epoch j.
 * Returns the number of executed UpdateEmbed calls. */
int64_t orc_train(const int64_t* offsets, const int32_t* indices, int64_t n,
                  orc_emb* M, int32_t epochs, double lr, int32_t k,
                  uint64_t seed, int32_t level, uint32_t tag,
                  int64_t src_lo, int64_t src_hi);

/* orc_train over all sources with loss_out[j] = sum over epoch j's executed
 * updates of the Section 2 objective at each update (running loss, FP64). */
int64_t orc_train_loss(const int64_t* offsets, const int32_t* indices, int64_t n,
                       orc_emb* M, int32_t epochs, double lr, int32_t k,
                       uint64_t seed, int32_t level, uint32_t tag, double* loss_out);

/* orc_train over all sources with each epoch's sources spread over `threads`
 * OpenMP threads without locks (Hogwild; timing only, results depend on
 * thread timing). */
int64_t orc_train_hogwild(const int64_t* offsets, const int32_t* indices, int64_t n,
                          orc_emb* M, int32_t epochs, double lr, int32_t k,
                          uint64_t seed, int32_t level, uint32_t tag, int32_t threads);

/* orc_draw_samples for every source of one epoch: out[src * (1 + k) + t]. */
void orc_draw_all(const int64_t* offsets, const int32_t* indices, int64_t n, uint64_t seed,
                  int32_t level, uint32_t tag, int32_t epoch, int32_t k, int32_t* out);

/* One level of Algorithm 4 (MultiEdgeCollapse): fills map[n] and the
 * processing order order[n] (may be NULL); returns |V_{i+1}|. */
int64_t orc_coarsen_map(const int64_t* offsets, const int32_t* indices, int64_t n,
                        int32_t* map, int32_t* order);

/* Coarse graph of Section 4.1: deduplicated {(map v, map u) : map v != map u},
 * rows ascending.  off_out has n_next+1 entries; idx_out must hold
 * offsets[n] entries.  Returns nnz of the coarse graph, or -1 on OOM. */
int64_t orc_coarse_graph(const int64_t* offsets, const int32_t* indices, int64_t n,
                         const int32_t* map, int64_t n_next,
                         int64_t* off_out, int32_t* idx_out);

/* Epoch distribution over D levels (Section 3): e_out[i], i = 0 finest. */
int32_t orc_epoch_schedule(int32_t e, double p, int32_t D, int32_t* e_out);

/* ---- Embedding with the matrix split into K parts (Section 5) ----------
 * Part p holds the ids [starts[p], starts[p+1]), starts[p] = floor(p n / K).
 * Kernel pairs follow the inside-out order: (0,0), then from (a,b) the next
 * pair is (a, b+1) while a > b and (a+1, 0) once a = b; K(K+1)/2 pairs.
 * Pool S_{i,j} of round r: for every u in part i with c > 0 neighbours in
 * part j, B entries (u, pos, b), b = 0..B-1; then (if i != j) the same for
 * every v in part j towards part i.  The positive of entry b is neighbour
 * floor(w c / 2^32) of u's neighbours in the opposite part o (in row order),
 * w = word 0 of the stream block at epoch r*B + b, kind 0, slot o, block 0.
 * A visit's k negatives are words 1..k of the same stream, mapped onto
 * part o; its stochastic-rounding bits carry o in bits 8.. of the block
 * field.  With K = 1 and B = 1 this is Algorithm 3 exactly. */
void    orc_part_starts(int64_t n, int32_t K, int64_t* starts);
/* pairs[2j], pairs[2j+1] = (a_j, b_j); returns K(K+1)/2. */
int64_t orc_inside_out(int32_t K, int32_t* pairs);
/* Entries of pool S_{i,j} (arrays may be NULL to count only). */
int64_t orc_pool(const int64_t* offsets, const int32_t* indices, int64_t n, int32_t K,
                 int32_t i, int32_t j, int32_t B, uint64_t seed, int32_t level, uint32_t tag,
                 int32_t round, int32_t* src_out, int32_t* pos_out, int32_t* b_out);
/* ceil(epochs / B) rounds over all pairs in inside-out order, every pool
 * entry visited in pool order with lr * max(1 - round/rounds, 1e-4); at most
 * epochs * n positive visits run (later entries are skipped).  Returns the
 * executed UpdateEmbed calls; *positives_out (may be NULL) the positive
 * visits. */
int64_t orc_train_partitioned(const int64_t* offsets, const int32_t* indices, int64_t n,
                              orc_emb* M, int32_t K, int32_t B, int32_t epochs, double lr,
                              int32_t k, uint64_t seed, int32_t level, uint32_t tag,
                              int64_t* positives_out);

/* ---- Random-walk sampling (Section 3.2) ---------------------------------
 * Epoch j starts one walk of `len` steps at every vertex v: w_0 = v and
 * w_{i+1} = neighbour floor(r deg / 2^32) of w_i, r = word i mod 4 of the
 * stream (v, j, kind 4, block i div 4); a walk stops at a vertex without
 * neighbours.  Every pair (w_a, w_b) with 0 < b - a <= window is a positive
 * sample with source w_a.  The P pair offsets (a, b), 0 <= a < b <= len,
 * b - a <= window, are numbered by a, then b; pair q = v P + l is offset l
 * of walk v and is void when b is past the end of walk v.  The epoch visits
 * the n P pairs in the order of the key word 0 of (q, j, kind 5), ties by q.
 * The pair at rank r (void ones keep their rank and are not visited) draws
 * its k negatives uniformly over [0, n) from words 1..k of (r, j, kind 6)
 * and is visited like a source of Algorithm 3, with lr' = lr max(1 - j/e,
 * 1e-4), a positive or negative equal to the source skipped, and BF16
 * rounding bits from (r, j, kind 7, slot, block) laid out as for kind 1. */
int32_t orc_walk(const int64_t* offsets, const int32_t* indices, uint64_t seed, int32_t level,
                 uint32_t tag, int32_t epoch, int64_t v, int32_t len, int32_t* out);
/* P, and the offsets (a in i_out, b in j_out; may be NULL). */
int32_t orc_walk_offsets(int32_t len, int32_t window, int32_t* i_out, int32_t* j_out);
/* The shuffle keys of pair numbers 0..m-1. */
void orc_walk_keys(int64_t m, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch, uint32_t* keys_out);
/* The visiting order of the epoch's n P pair indices. */
int64_t orc_walk_order(int64_t n, int32_t P, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                       int64_t* order_out);
/* The epoch's pairs in visiting order (src_out/pos_out[n P]; -1 for void). */
int64_t orc_walk_pairs(const int64_t* offsets, const int32_t* indices, int64_t n, uint64_t seed,
                       int32_t level, uint32_t tag, int32_t epoch, int32_t len, int32_t window,
                       int32_t* src_out, int32_t* pos_out);
/* `epochs` epochs of walk-sampled training; returns the executed UpdateEmbed
 * calls. */
int64_t orc_train_walks(const int64_t* offsets, const int32_t* indices, int64_t n, orc_emb* M,
                        int32_t epochs, double lr, int32_t k, int32_t len, int32_t window,
                        uint64_t seed, int32_t level, uint32_t tag);

#ifdef __cplusplus
}
#endif
#endif
