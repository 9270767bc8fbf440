/*
 * GOSH CPU oracle (test infrastructure only) -- see gosh_oracle.h.
 *
 * Readings of the paper that this file fixes (each applied identically by
 * the tests and the HIP path):
 *  - UpdateEmbed (Algorithm 1): score = (b - sigma(M[v].M[s])) * lr; the
 *    source row is updated first and the sample row then uses the updated
 *    source row (literal statement order).
 *  - sigma(x) = 1 / (1 + exp(-x)), no clamp or table.
 *  - Positive sample: uniform over the neighbours of src; a source with no
 *    neighbour skips its positive but still does its negatives.  Negatives
 *    are uniform over V_i; a negative equal to src is skipped.  A sample that
 *    repeats within one source sees that source's earlier update of it.
 *  - hub^2 restriction with delta = |E_i|/|V_i| read as nnz/n (average CSR
 *    degree), tested exactly as deg * n <= nnz.
 *  - Ordering: counting sort by degree, larger degree first, ties in
 *    ascending vertex id.  Cluster ids are handed out in processing order.
 *  - Coarse graph: intra-cluster edges dropped, duplicates merged, rows
 *    sorted, unweighted.
 */
#include "gosh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 bit     */
/* multiplies mixing the four counter words, with a Weyl-sequence key        */
/* schedule.                                                                 */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_stream_block(uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                      int64_t src, uint32_t kind, uint32_t slot, uint32_t block,
                      uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)src;
    ctr[1] = (uint32_t)epoch;
    ctr[2] = ((uint32_t)level & 0xFFu) | (tag << 8);
    ctr[3] = (kind << 24) | ((slot & 0xFFu) << 16) | (block & 0xFFFFu);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, out);
}

/* m independent Philox blocks: out[4i..4i+3] = philox(ctr[4i..4i+3], key). */
void orc_philox_many(const uint32_t *ctr, int64_t m, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < m; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* floor(r * N / 2^32): maps a uniform 32-bit word onto [0, N). */
static int64_t scale_word(uint32_t r, int64_t N)
{
    return (int64_t)(((uint64_t)r * (uint64_t)N) >> 32);
}

void orc_draw_samples(const int64_t* offsets, const int32_t* indices, int64_t n,
                      uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                      int64_t src, int32_t k, int32_t* out)
{
    uint32_t w[64];
    int32_t nwords = 1 + k;
    for (int32_t b = 0; 4 * b < nwords; ++b)
        orc_stream_block(seed, level, tag, epoch, src, 0u, 0u, (uint32_t)b, w + 4 * b);
    int64_t deg = offsets[src + 1] - offsets[src];
    out[0] = deg > 0 ? indices[offsets[src] + scale_word(w[0], deg)] : -1;
    for (int32_t t = 1; t <= k; ++t)
        out[t] = (int32_t)scale_word(w[t], n);
}

uint32_t orc_sr_bits(uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                     int64_t src, uint32_t slot, int32_t e, int32_t d)
{
    /* Element e lies in 32-bit word w = e / 2 of the row.  With L = d / 8,
     * word w draws from block w mod L, and inside that block's 8 halves it
     * takes half 2 * (w div L) + (e mod 2) (low half of a 32-bit output
     * word first). */
    const int32_t L = d >= 8 ? d / 8 : 1;
    const int32_t w = e / 2;
    uint32_t out[4];
    orc_stream_block(seed, level, tag, epoch, src, 1u, slot, (uint32_t)(w % L), out);
    const int32_t h = 2 * (w / L) + (e % 2);
    const uint32_t word = out[h / 2];
    return (h & 1) ? (word >> 16) : (word & 0xFFFFu);
}

/* ------------------------------------------------------------------------ */
/* BF16 storage                                                              */
/* ------------------------------------------------------------------------ */
static uint32_t f32_bits(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    return u;
}

uint16_t orc_bf16_sr(float x, uint32_t r16)
{
    uint32_t u = f32_bits(x);
    if ((u & 0x7F800000u) == 0x7F800000u) {          /* Inf or NaN */
        if (u & 0x007FFFFFu)
            return (uint16_t)((u >> 16) | 0x0040u);   /* quiet NaN */
        return (uint16_t)(u >> 16);
    }
    /* Adding r16 to the 16 dropped bits carries into the kept half with
     * probability (dropped bits)/2^16: unbiased rounding of the magnitude. */
    return (uint16_t)((u + (r16 & 0xFFFFu)) >> 16);
}

uint16_t orc_bf16_rne(float x)
{
    uint32_t u = f32_bits(x);
    if ((u & 0x7F800000u) == 0x7F800000u) {
        if (u & 0x007FFFFFu)
            return (uint16_t)((u >> 16) | 0x0040u);
        return (uint16_t)(u >> 16);
    }
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

double orc_bf16_to_f64(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* ------------------------------------------------------------------------ */
/* Objective (Section 2): logistic classifier on M[v].M[u]                  */
/* ------------------------------------------------------------------------ */
double orc_sigmoid(double x)
{
    return 1.0 / (1.0 + exp(-x));
}

/* log(sigma(x)) without overflow. */
static double log_sigmoid(double x)
{
    return x >= 0.0 ? -log1p(exp(-x)) : x - log1p(exp(x));
}

double orc_loss(double x, int b)
{
    return b ? -log_sigmoid(x) : -log_sigmoid(-x);
}

/* ------------------------------------------------------------------------ */
/* UpdateEmbed (Algorithm 1) over the samples of one source                 */
/* ------------------------------------------------------------------------ */
static double row_get(const orc_emb* M, int64_t v, int32_t e)
{
    if (M->bf16)
        return orc_bf16_to_f64(((const uint16_t*)M->rows)[v * M->d + e]);
    return ((const double*)M->rows)[v * M->d + e];
}

/* Stochastic-rounding bits as orc_sr_bits, with `hi` in bits 8.. of the
 * counter's block field (0 for Algorithm 3; the opposite part of a
 * partitioned visit). */
static uint32_t sr_bits_hi(uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                           int64_t src, uint32_t kind, uint32_t slot, int32_t e, int32_t d, uint32_t hi)
{
    const int32_t L = d >= 8 ? d / 8 : 1;
    const int32_t w = e / 2;
    uint32_t out[4];
    orc_stream_block(seed, level, tag, epoch, src, kind, slot, (hi << 8) | (uint32_t)(w % L), out);
    const int32_t h = 2 * (w / L) + (e % 2);
    const uint32_t word = out[h / 2];
    return (h & 1) ? (word >> 16) : (word & 0xFFFFu);
}

/* One visit (Algorithm 1 on each sample in turn).  BF16 rounding bits come
 * from the stream (sid, epoch, kind sr_kind, slot, block hi << 8 | ...).
 * loss (may be NULL) accumulates the objective of Section 2 at each executed
 * update, evaluated on the rows the update reads (before it changes them):
 * -log sigma(x) for the positive, -log(1 - sigma(x)) for a negative. */
static int32_t visit_stream_loss(orc_emb* M, int64_t src, const int32_t* samples, int32_t k,
                                 double lr, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                                 int64_t sid, uint32_t sr_kind, uint32_t hi, double* loss)
{
    const int32_t d = M->d;
    double* s = (double*)malloc(sizeof(double) * (size_t)d);
    double* m = (double*)malloc(sizeof(double) * (size_t)d);
    int32_t done = 0;
    for (int32_t e = 0; e < d; ++e)
        s[e] = row_get(M, src, e);
    for (int32_t t = 0; t <= k; ++t) {
        int64_t u = samples[t];
        if (u < 0 || u == src)
            continue;
        const double b = (t == 0) ? 1.0 : 0.0;
        for (int32_t e = 0; e < d; ++e)
            m[e] = row_get(M, u, e);
        double x = 0.0;
        for (int32_t e = 0; e < d; ++e)
            x += s[e] * m[e];
        const double score = (b - orc_sigmoid(x)) * lr;
        if (loss)
            *loss += orc_loss(x, t == 0);
        for (int32_t e = 0; e < d; ++e)
            s[e] += m[e] * score;
        for (int32_t e = 0; e < d; ++e) {
            double val = m[e] + s[e] * score;
            if (M->bf16) {
                uint32_t r = sr_bits_hi(seed, level, tag, epoch, sid, sr_kind, (uint32_t)t, e, d, hi);
                ((uint16_t*)M->rows)[u * d + e] = orc_bf16_sr((float)val, r);
            } else {
                ((double*)M->rows)[u * d + e] = val;
            }
        }
        ++done;
    }
    for (int32_t e = 0; e < d; ++e) {
        if (M->bf16) {
            uint32_t r = sr_bits_hi(seed, level, tag, epoch, sid, sr_kind, 0xFFu, e, d, hi);
            ((uint16_t*)M->rows)[src * d + e] = orc_bf16_sr((float)s[e], r);
        } else {
            ((double*)M->rows)[src * d + e] = s[e];
        }
    }
    free(s);
    free(m);
    return done;
}

static int32_t visit_stream(orc_emb* M, int64_t src, const int32_t* samples, int32_t k,
                            double lr, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                            int64_t sid, uint32_t sr_kind, uint32_t hi)
{
    return visit_stream_loss(M, src, samples, k, lr, seed, level, tag, epoch, sid, sr_kind, hi, NULL);
}

static int32_t visit_hi(orc_emb* M, int64_t src, const int32_t* samples, int32_t k,
                        double lr, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                        uint32_t hi)
{
    return visit_stream(M, src, samples, k, lr, seed, level, tag, epoch, src, 1u, hi);
}

int32_t orc_visit(orc_emb* M, int64_t src, const int32_t* samples, int32_t k,
                  double lr, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch)
{
    return visit_hi(M, src, samples, k, lr, seed, level, tag, epoch, 0u);
}

int64_t orc_update_batch(orc_emb* M, int64_t nsrc, const int32_t* src,
                         const int32_t* samples, int32_t k, double lr,
                         uint64_t seed, int32_t level, uint32_t tag, int32_t epoch)
{
    int64_t done = 0;
    for (int64_t i = 0; i < nsrc; ++i)
        done += orc_visit(M, src[i], samples + i * (1 + k), k, lr, seed, level, tag, epoch);
    return done;
}

/* ------------------------------------------------------------------------ */
/* TrainInGPU (Algorithm 3), run sequentially                               */
/* ------------------------------------------------------------------------ */
int64_t orc_train(const int64_t* offsets, const int32_t* indices, int64_t n,
                  orc_emb* M, int32_t epochs, double lr, int32_t k,
                  uint64_t seed, int32_t level, uint32_t tag,
                  int64_t src_lo, int64_t src_hi)
{
    int32_t samples[64];
    int64_t done = 0;
    for (int32_t j = 0; j < epochs; ++j) {
        double f = 1.0 - (double)j / (double)epochs;
        double lrj = lr * (f > 1e-4 ? f : 1e-4);
        for (int64_t src = src_lo; src < src_hi; ++src) {
            orc_draw_samples(offsets, indices, n, seed, level, tag, j, src, k, samples);
            done += orc_visit(M, src, samples, k, lrj, seed, level, tag, j);
        }
    }
    return done;
}

/* Algorithm 3 run sequentially as orc_train, with loss_out[j] (epochs
 * entries) receiving the sum over epoch j's executed updates of the
 * objective of Section 2 at the moment of each update (the running loss). */
int64_t orc_train_loss(const int64_t* offsets, const int32_t* indices, int64_t n,
                       orc_emb* M, int32_t epochs, double lr, int32_t k,
                       uint64_t seed, int32_t level, uint32_t tag, double* loss_out)
{
    int32_t samples[64];
    int64_t done = 0;
    for (int32_t j = 0; j < epochs; ++j) {
        double f = 1.0 - (double)j / (double)epochs;
        double lrj = lr * (f > 1e-4 ? f : 1e-4);
        double acc = 0.0;
        for (int64_t src = 0; src < n; ++src) {
            orc_draw_samples(offsets, indices, n, seed, level, tag, j, src, k, samples);
            done += visit_stream_loss(M, src, samples, k, lrj, seed, level, tag, j, src, 1u, 0u, &acc);
        }
        loss_out[j] = acc;
    }
    return done;
}

/* Algorithm 3 as orc_train (FP64 rows, same samples and lr schedule), with
 * the sources of each epoch spread over `threads` OpenMP threads without
 * locks (Hogwild, as the paper's parallel loop): rows shared by concurrent
 * visits race, so the result depends on thread timing.  For timing the
 * oracle on all host cores; returns the executed updates. */
int64_t orc_train_hogwild(const int64_t* offsets, const int32_t* indices, int64_t n,
                          orc_emb* M, int32_t epochs, double lr, int32_t k,
                          uint64_t seed, int32_t level, uint32_t tag, int32_t threads)
{
    int64_t done = 0;
    for (int32_t j = 0; j < epochs; ++j) {
        double f = 1.0 - (double)j / (double)epochs;
        double lrj = lr * (f > 1e-4 ? f : 1e-4);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1024) reduction(+ : done)
        for (int64_t src = 0; src < n; ++src) {
            int32_t samples[64];
            orc_draw_samples(offsets, indices, n, seed, level, tag, j, src, k, samples);
            done += orc_visit(M, src, samples, k, lrj, seed, level, tag, j);
        }
    }
    return done;
}

/* Samples of every source of one epoch (orc_draw_samples for src = 0..n-1):
 * out[src * (1 + k) + t]. */
void orc_draw_all(const int64_t* offsets, const int32_t* indices, int64_t n, uint64_t seed,
                  int32_t level, uint32_t tag, int32_t epoch, int32_t k, int32_t* out)
{
    for (int64_t src = 0; src < n; ++src)
        orc_draw_samples(offsets, indices, n, seed, level, tag, epoch, src, k, out + src * (1 + k));
}

/* ------------------------------------------------------------------------ */
/* MultiEdgeCollapse (Algorithm 4), one level                               */
/* ------------------------------------------------------------------------ */
int64_t orc_coarsen_map(const int64_t* offsets, const int32_t* indices, int64_t n,
                        int32_t* map, int32_t* order_out)
{
    const int64_t nnz = offsets[n];
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t dv = offsets[v + 1] - offsets[v];
        if (dv > maxdeg)
            maxdeg = dv;
    }
    /* Counting sort on degree, larger first; equal degrees keep id order. */
    int64_t* start = (int64_t*)calloc((size_t)maxdeg + 2, sizeof(int64_t));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; ++v)
        start[maxdeg - (offsets[v + 1] - offsets[v])]++;
    int64_t acc = 0;
    for (int64_t b = 0; b <= maxdeg; ++b) {
        int64_t c = start[b];
        start[b] = acc;
        acc += c;
    }
    for (int64_t v = 0; v < n; ++v)
        order[start[maxdeg - (offsets[v + 1] - offsets[v])]++] = (int32_t)v;
    free(start);

    for (int64_t v = 0; v < n; ++v)
        map[v] = -1;
    int64_t cluster = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = order[i];
        if (map[v] != -1)
            continue;
        map[v] = (int32_t)cluster++;
        const int64_t dv = offsets[v + 1] - offsets[v];
        for (int64_t p = offsets[v]; p < offsets[v + 1]; ++p) {
            const int64_t u = indices[p];
            const int64_t du = offsets[u + 1] - offsets[u];
            /* hub^2 restriction: deg <= |E|/|V| written as deg * |V| <= |E| */
            if (dv * n <= nnz || du * n <= nnz) {
                if (map[u] == -1)
                    map[u] = map[v];
            }
        }
    }
    if (order_out)
        memcpy(order_out, order, sizeof(int32_t) * (size_t)n);
    free(order);
    return cluster;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

int64_t orc_coarse_graph(const int64_t* offsets, const int32_t* indices, int64_t n,
                         const int32_t* map, int64_t n_next,
                         int64_t* off_out, int32_t* idx_out)
{
    const int64_t nnz = offsets[n];
    uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!pairs)
        return -1;
    int64_t m = 0;
    for (int64_t v = 0; v < n; ++v)
        for (int64_t p = offsets[v]; p < offsets[v + 1]; ++p) {
            uint32_t a = (uint32_t)map[v], b = (uint32_t)map[indices[p]];
            if (a != b)
                pairs[m++] = ((uint64_t)a << 32) | b;
        }
    qsort(pairs, (size_t)m, sizeof(uint64_t), cmp_u64);
    for (int64_t c = 0; c <= n_next; ++c)
        off_out[c] = 0;
    int64_t w = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i > 0 && pairs[i] == pairs[i - 1])
            continue;
        off_out[(pairs[i] >> 32) + 1]++;
        idx_out[w++] = (int32_t)(pairs[i] & 0xFFFFFFFFu);
    }
    for (int64_t c = 0; c < n_next; ++c)
        off_out[c + 1] += off_out[c];
    free(pairs);
    return w;
}

/* ------------------------------------------------------------------------ */
/* Epoch distribution (Section 3): a share p spread evenly over the D       */
/* levels, the rest geometrically with each coarser level getting twice    */
/* the finer one's share.  Integer epochs: floors, then the remainder one   */
/* each to the largest fractional parts (ties to the coarser level).        */
/* ------------------------------------------------------------------------ */
int32_t orc_epoch_schedule(int32_t e, double p, int32_t D, int32_t* e_out)
{
    if (D <= 0 || e < 0 || !(p >= 0.0 && p <= 1.0))
        return -1;
    double* real = (double*)malloc(sizeof(double) * (size_t)D);
    double denom = ldexp(1.0, D) - 1.0;
    int64_t sum = 0;
    for (int32_t i = 0; i < D; ++i) {
        real[i] = p * (double)e / (double)D + (1.0 - p) * (double)e * ldexp(1.0, i) / denom;
        e_out[i] = (int32_t)floor(real[i]);
        sum += e_out[i];
    }
    int64_t rem = (int64_t)e - sum;
    while (rem > 0) {
        int32_t best = -1;
        double bf = -1.0;
        for (int32_t i = D - 1; i >= 0; --i) {
            double f = real[i] - floor(real[i]);
            if (f > bf) {
                bf = f;
                best = i;
            }
        }
        e_out[best] += 1;
        real[best] = floor(real[best]);   /* fractional part consumed */
        --rem;
    }
    free(real);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Embedding with the matrix split into K parts (Section 5)                 */
/* ------------------------------------------------------------------------ */
void orc_part_starts(int64_t n, int32_t K, int64_t* starts)
{
    for (int32_t p = 0; p <= K; ++p)
        starts[p] = (int64_t)(((__int128)p * n) / K);
}

int64_t orc_inside_out(int32_t K, int32_t* pairs)
{
    /* (0,0) first; from (a,b): (a, b+1) while a > b, else (a+1, 0). */
    const int64_t len = (int64_t)K * (K + 1) / 2;
    int32_t a = 0, b = 0;
    for (int64_t j = 0; j < len; ++j) {
        if (j > 0) {
            if (a > b) {
                b += 1;
            } else {
                a += 1;
                b = 0;
            }
        }
        pairs[2 * j] = a;
        pairs[2 * j + 1] = b;
    }
    return len;
}

/* First position in the sorted row of u whose neighbour is >= x. */
static int64_t row_lower(const int64_t* offsets, const int32_t* indices, int64_t u, int64_t x)
{
    int64_t lo = offsets[u], hi = offsets[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (indices[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* Neighbours of u inside part o: positions [*lo, *lo + return value). */
static int64_t part_neighbours(const int64_t* offsets, const int32_t* indices, const int64_t* starts,
                               int64_t u, int32_t o, int64_t* lo)
{
    *lo = row_lower(offsets, indices, u, starts[o]);
    return row_lower(offsets, indices, u, starts[o + 1]) - *lo;
}

/* Positive of the b-th visit of u towards part o in round `round`: word 0 of
 * block 0 of the stream at epoch round*B + b with the part in the slot field
 * (c = neighbours of u in part o, > 0). */
static int32_t part_positive(const int32_t* indices, int64_t lo, int64_t c, uint64_t seed, int32_t level,
                             uint32_t tag, int32_t eps, int64_t u, int32_t o)
{
    uint32_t w[4];
    orc_stream_block(seed, level, tag, eps, u, 0u, (uint32_t)o, 0u, w);
    return indices[lo + scale_word(w[0], c)];
}

static int64_t pool_side(const int64_t* offsets, const int32_t* indices, const int64_t* starts,
                         int32_t s, int32_t o, int32_t B, uint64_t seed, int32_t level, uint32_t tag,
                         int32_t round, int32_t* src, int32_t* pos, int32_t* bb, int64_t at)
{
    for (int64_t u = starts[s]; u < starts[s + 1]; ++u) {
        int64_t lo;
        const int64_t c = part_neighbours(offsets, indices, starts, u, o, &lo);
        if (c == 0)
            continue;
        for (int32_t b = 0; b < B; ++b) {
            if (src) {
                src[at] = (int32_t)u;
                pos[at] = part_positive(indices, lo, c, seed, level, tag, round * B + b, u, o);
                bb[at] = b;
            }
            ++at;
        }
    }
    return at;
}

int64_t orc_pool(const int64_t* offsets, const int32_t* indices, int64_t n, int32_t K,
                 int32_t i, int32_t j, int32_t B, uint64_t seed, int32_t level, uint32_t tag,
                 int32_t round, int32_t* src_out, int32_t* pos_out, int32_t* b_out)
{
    int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K + 1));
    orc_part_starts(n, K, starts);
    int64_t at = pool_side(offsets, indices, starts, i, j, B, seed, level, tag, round,
                           src_out, pos_out, b_out, 0);
    if (i != j)
        at = pool_side(offsets, indices, starts, j, i, B, seed, level, tag, round,
                       src_out, pos_out, b_out, at);
    free(starts);
    return at;
}

int64_t orc_train_partitioned(const int64_t* offsets, const int32_t* indices, int64_t n,
                              orc_emb* M, int32_t K, int32_t B, int32_t epochs, double lr,
                              int32_t k, uint64_t seed, int32_t level, uint32_t tag,
                              int64_t* positives_out)
{
    int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K + 1));
    int32_t* pairs = (int32_t*)malloc(sizeof(int32_t) * (size_t)K * (size_t)(K + 1));
    orc_part_starts(n, K, starts);
    const int64_t npairs = orc_inside_out(K, pairs);
    const int32_t rounds = (epochs + B - 1) / B;
    const int64_t cap = (int64_t)epochs * n;      /* positive samples of `epochs` passes */
    int64_t positives = 0, updates = 0;
    int32_t samples[64];
    uint32_t w[64];
    for (int32_t rho = 0; rho < rounds; ++rho) {
        const double f = 1.0 - (double)rho / (double)rounds;
        const double lrr = lr * (f > 1e-4 ? f : 1e-4);
        for (int64_t q = 0; q < npairs; ++q) {
            const int32_t a = pairs[2 * q], b2 = pairs[2 * q + 1];
            for (int32_t side = 0; side < (a != b2 ? 2 : 1); ++side) {
                const int32_t s = side == 0 ? a : b2, o = side == 0 ? b2 : a;
                const int64_t size_o = starts[o + 1] - starts[o];
                for (int64_t u = starts[s]; u < starts[s + 1]; ++u) {
                    int64_t lo;
                    const int64_t c = part_neighbours(offsets, indices, starts, u, o, &lo);
                    if (c == 0)
                        continue;
                    for (int32_t b = 0; b < B; ++b) {
                        if (positives >= cap)
                            continue;
                        ++positives;
                        const int32_t eps = rho * B + b;
                        for (int32_t blk = 0; 4 * blk <= k; ++blk)
                            orc_stream_block(seed, level, tag, eps, u, 0u, (uint32_t)o, (uint32_t)blk,
                                             w + 4 * blk);
                        samples[0] = indices[lo + scale_word(w[0], c)];
                        for (int32_t t = 1; t <= k; ++t)
                            samples[t] = (int32_t)(starts[o] + scale_word(w[t], size_o));
                        updates += visit_hi(M, u, samples, k, lrr, seed, level, tag, eps, (uint32_t)o);
                    }
                }
            }
        }
    }
    if (positives_out)
        *positives_out = positives;
    free(starts);
    free(pairs);
    return updates;
}

/* ------------------------------------------------------------------------ */
/* Random-walk sampling (Section 3.2)                                       */
/* ------------------------------------------------------------------------ */
int32_t orc_walk(const int64_t* offsets, const int32_t* indices, uint64_t seed, int32_t level,
                 uint32_t tag, int32_t epoch, int64_t v, int32_t len, int32_t* out)
{
    uint32_t w[4];
    int64_t cur = v;
    out[0] = (int32_t)v;
    int32_t m = 1;
    for (int32_t i = 0; i < len; ++i) {
        if (i % 4 == 0)
            orc_stream_block(seed, level, tag, epoch, v, 4u, 0u, (uint32_t)(i / 4), w);
        const int64_t deg = offsets[cur + 1] - offsets[cur];
        if (deg == 0)
            break;
        cur = indices[offsets[cur] + scale_word(w[i % 4], deg)];
        out[m++] = (int32_t)cur;
    }
    return m;
}

int32_t orc_walk_offsets(int32_t len, int32_t window, int32_t* i_out, int32_t* j_out)
{
    int32_t P = 0;
    for (int32_t i = 0; i < len; ++i)
        for (int32_t j = i + 1; j <= len && j - i <= window; ++j) {
            if (i_out) {
                i_out[P] = i;
                j_out[P] = j;
            }
            ++P;
        }
    return P;
}

typedef struct {
    uint32_t key;
    int64_t idx;
} key_idx;

static int cmp_key_idx(const void* a, const void* b)
{
    const key_idx* x = (const key_idx*)a;
    const key_idx* y = (const key_idx*)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

void orc_walk_keys(int64_t m, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch, uint32_t* keys_out)
{
    for (int64_t q = 0; q < m; ++q) {
        uint32_t w[4];
        orc_stream_block(seed, level, tag, epoch, q, 5u, 0u, 0u, w);
        keys_out[q] = w[0];
    }
}

int64_t orc_walk_order(int64_t n, int32_t P, uint64_t seed, int32_t level, uint32_t tag, int32_t epoch,
                       int64_t* order_out)
{
    const int64_t m = n * (int64_t)P;
    key_idx* kv = (key_idx*)malloc(sizeof(key_idx) * (size_t)(m > 0 ? m : 1));
    for (int64_t q = 0; q < m; ++q) {
        uint32_t w[4];
        orc_stream_block(seed, level, tag, epoch, q, 5u, 0u, 0u, w);
        kv[q].key = w[0];
        kv[q].idx = q;
    }
    qsort(kv, (size_t)m, sizeof(key_idx), cmp_key_idx);
    for (int64_t r = 0; r < m; ++r)
        order_out[r] = kv[r].idx;
    free(kv);
    return m;
}

int64_t orc_walk_pairs(const int64_t* offsets, const int32_t* indices, int64_t n, uint64_t seed,
                       int32_t level, uint32_t tag, int32_t epoch, int32_t len, int32_t window,
                       int32_t* src_out, int32_t* pos_out)
{
    const int32_t P = orc_walk_offsets(len, window, NULL, NULL);
    const int64_t m = n * (int64_t)P;
    int32_t* ti = (int32_t*)malloc(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
    int32_t* tj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
    orc_walk_offsets(len, window, ti, tj);
    /* every walk of the epoch, walk v in row v */
    int32_t* walks = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)(len + 1));
    int32_t* wlen = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; ++v)
        wlen[v] = orc_walk(offsets, indices, seed, level, tag, epoch, v, len, walks + v * (len + 1));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    orc_walk_order(n, P, seed, level, tag, epoch, order);
    for (int64_t r = 0; r < m; ++r) {
        const int64_t v = order[r] / P;
        const int32_t l = (int32_t)(order[r] % P);
        const int void_pair = tj[l] >= wlen[v];
        src_out[r] = void_pair ? -1 : walks[v * (len + 1) + ti[l]];
        pos_out[r] = void_pair ? -1 : walks[v * (len + 1) + tj[l]];
    }
    free(order);
    free(wlen);
    free(walks);
    free(tj);
    free(ti);
    return m;
}

int64_t orc_train_walks(const int64_t* offsets, const int32_t* indices, int64_t n, orc_emb* M,
                        int32_t epochs, double lr, int32_t k, int32_t len, int32_t window,
                        uint64_t seed, int32_t level, uint32_t tag)
{
    const int64_t m = n * (int64_t)orc_walk_offsets(len, window, NULL, NULL);
    int32_t* src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t done = 0;
    int32_t samples[64];
    uint32_t w[64];
    for (int32_t j = 0; j < epochs; ++j) {
        const double f = 1.0 - (double)j / (double)epochs;
        const double lrj = lr * (f > 1e-4 ? f : 1e-4);
        orc_walk_pairs(offsets, indices, n, seed, level, tag, j, len, window, src, pos);
        for (int64_t r = 0; r < m; ++r) {
            if (src[r] < 0)
                continue;
            for (int32_t b = 0; 4 * b <= k; ++b)
                orc_stream_block(seed, level, tag, j, r, 6u, 0u, (uint32_t)b, w + 4 * b);
            samples[0] = pos[r];
            for (int32_t t = 1; t <= k; ++t)
                samples[t] = (int32_t)scale_word(w[t], n);
            done += visit_stream(M, src[r], samples, k, lrj, seed, level, tag, j, r, 7u, 0u);
        }
    }
    free(src);
    free(pos);
    return done;
}
