// Internal declarations of the gfx950 GOSH library: context, device memory
// accounting, level store and the device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <array>
#include <map>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "gosh.h"

namespace gosh {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    gosh_status code;
    Error(gosh_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define GOSH_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::gosh::Error(GOSH_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GOSH_REQUIRE(cond, code, msg)                                                      \
    do {                                                                                   \
        if (!(cond)) throw ::gosh::Error(code, msg);                                       \
    } while (0)

// ---------------------------------------------------------------- context
struct Ctx {
    int device = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;   // nullptr = the device's null stream
    uint64_t cap = 0;          // 0 = unlimited
    uint64_t in_use = 0;       // bytes held by live allocations and the cache
    bool deterministic = false;
    int overlap = 1;           // epochs per launch on large levels (1: Algorithm 3's barriers)
    int64_t overlap_min = 0;   // levels with at least this many vertices overlap
    int64_t plain_neg_min = 0; // levels with at least this many vertices store negatives plainly (0: never)
    int64_t plain_light_min = 0; // levels with at least this many vertices store light rows plainly (0: never)
    // levels with group_min <= n <= group_max train with the visits of hot
    // positives grouped (hubs of degree >= group_factor x the average)
    int64_t group_min = 0, group_max = 0;
    double group_factor = 64.0;
    int64_t resident_max = 0;  // levels with at most this many vertices run all epochs in one launch (0: never)
    int64_t lds_max = 0;       // levels with at most this many vertices (and rows fitting in LDS) train in one workgroup
    int32_t* record = nullptr; // test hook: samples drawn inside gosh_train (device, caller-owned)
    int64_t record_cap = 0;
    double* loss = nullptr;    // running loss per epoch of gosh_train (device, caller-owned)
    int64_t loss_cap = 0;
    int coarsen_mode = GOSH_COARSEN_EXACT;
    int coarse_build = 0;      // coarse graph: 0 by cluster segments (one sort of all pair keys where they do not fit), 1 always the sort
    int64_t claim_batch = 0;   // lock-and-skip ranks per launch (0: max(64, n/64))
    std::string err;
    // Size-bucketed cache of freed device blocks, reused before hipMalloc.
    std::multimap<size_t, void*> cache;
    std::map<void*, size_t> live;
    // small device scratch for counters and flags
    void* scratch = nullptr;   // 4 KiB
    // pinned host slots for single values read back from the device (a copy
    // into pageable memory would block the host on its own)
    int64_t* pinned = nullptr; // kPinnedSlots slots
    int64_t* pinned_dev = nullptr; // the same slots as kernels address them (they write scan totals there)
    // coarse-build launch facts queried once: compute units, the LDS limits
    // of the segment kernels, and the dedup kernel's workgroups per CU by LDS size
    int cus = 0;
    bool seg_lds_set = false;
    std::map<size_t, int> dedup_per_cu;
    static constexpr int kPinnedSlots = 64;
    // batched-training autotune cache: key -> (mode, blocks per CU, chunk iterations)
    std::map<std::string, std::array<int, 3>> tune;
    bool tune_loaded = false;

    void* alloc(size_t bytes);
    void free(void* p);
    void trim();               // releases cached blocks
};

// Size a device block of `bytes` occupies in the context's allocator.
size_t alloc_bucket(size_t bytes);

// RAII device buffer tied to a context
template <class T>
struct DevBuf {
    Ctx* ctx = nullptr;
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(Ctx* c, size_t count) : ctx(c), n(count) {
        p = static_cast<T*>(c->alloc(count * sizeof(T)));
    }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : ctx(o.ctx), p(o.p), n(o.n) { o.p = nullptr; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        reset();
        ctx = o.ctx; p = o.p; n = o.n; o.p = nullptr;
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p && ctx) ctx->free(p);
        p = nullptr;
        n = 0;
    }
    T* release() { T* q = p; p = nullptr; n = 0; return q; }
};

// ---------------------------------------------------------------- levels
struct Level {
    int64_t n = 0, nnz = 0;
    bool off64 = false;
    const void* offsets = nullptr;     // device
    const int32_t* indices = nullptr;  // device
    void* own_offsets = nullptr;       // owned storage (levels >= 1)
    int32_t* own_indices = nullptr;
    int32_t* map = nullptr;            // map to level+1 (owned), null on the coarsest
    int32_t* clsz = nullptr;           // sizes of level+1's clusters (owned)
    uint32_t* hub_bits = nullptr;      // bit v set: deg(v) * n > nnz (owned, built on first use)
    int64_t n_deg0 = -1;               // vertices without neighbours (-1: not yet counted)
};

}  // namespace gosh

struct gosh_levels;
struct gosh_mlp;

struct gosh_ctx {
    gosh::Ctx c;
    std::set<gosh_levels*> levels;   // live hierarchies built on this context
    std::set<gosh_mlp*> mlps;        // live prolongation networks
};

struct gosh_levels {
    gosh_ctx* owner = nullptr;       // cleared when the context is destroyed first
    gosh::Ctx* ctx = nullptr;
    std::vector<gosh::Level> lv;
};

// Learned-prolongation network: FP32 master weights, Adam moments and the
// BF16 operand fragments of the products (see mlp.hip).
struct gosh_mlp {
    gosh_ctx* owner = nullptr;       // cleared when the context is destroyed first
    gosh::Ctx* ctx = nullptr;
    int d = 0, hidden = 0;
    int64_t nparams = 0;
    float* master = nullptr;   // W1[H][d+2], b1[H], W2[d][H], b2[d]
    float* m1 = nullptr;       // Adam first moments
    float* m2 = nullptr;       // Adam second moments
    int64_t t = 0;             // Adam steps taken
    uint16_t* w1f = nullptr;   // BF16 fragments of W1 (layer-1 A operand)
    uint16_t* w2f = nullptr;   // BF16 fragments of W2 (layer-2 A operand, permuted K)
    uint16_t* w2tf = nullptr;  // BF16 fragments of W2^T (backward-data A operand)
};

namespace gosh {

// One source of (coarse row, fine row) training pairs: every vertex of a
// fine level with its super vertex in the next level.
struct PairSrcHost {
    const Level* L;
    int64_t n_coarse;
    const void* coarse;
    const void* fine;
};

// ---------------------------------------------------------------- host entry points
// (implemented in coarsen.hip / train.hip / prolong.hip)
void validate_csr(Ctx* c, const gosh_csr* g, bool symmetry);
void coarsen(Ctx* c, const gosh_csr* g0, int64_t threshold, double ratio, gosh_levels* out);
int64_t count_isolated(Ctx* c, const Level& L);           // cached in L
const int32_t* cluster_sizes(Ctx* c, const Level& L, int64_t n_next);  // computed on first use
// bit v set iff deg(v) >= light_below (built on first use, kept with the level)
const uint32_t* hub_bits(Ctx* c, const Level& L, int64_t light_below);
void train_level(Ctx* c, const Level& L, int32_t level, void* emb, gosh_dtype dt, int d,
                 int epochs, float lr, int k, uint32_t tag, uint64_t* updates_dev);
void draw_samples(Ctx* c, const Level& L, int32_t level, int32_t epoch, int k, uint32_t tag,
                  int32_t* out);
void update_batch(Ctx* c, void* emb, gosh_dtype dt, int d, int64_t n_rows, int nsrc,
                  const int32_t* src, const int32_t* samples, int k, float lr, int32_t level,
                  uint32_t tag, int32_t epoch);
void prolong_copy(Ctx* c, const Level& fine, const void* coarse, void* fine_emb, gosh_dtype dt,
                  int d);
void train_batched(Ctx* c, const gosh_job* jobs, int njobs, gosh_dtype dt, int d, int k, int mode,
                   uint64_t* updates_dev, int32_t* chosen);
// the no-allocation variant: tables in a static device array set up per device
void batched_noalloc_init(int device);
void train_batched_noalloc(Ctx* c, const gosh_job* jobs, int njobs, gosh_dtype dt, int d, int k,
                           uint64_t* updates_dev);
unsigned int batched_noalloc_error(Ctx* c);   // waits for the stream
void free_level(Ctx* c, Level& L);
// (partition.hip)
void train_partitioned(Ctx* c, const gosh_csr* g_host, void* emb_host, gosh_dtype dt, int d, int epochs,
                       float lr, int k, int32_t level, uint32_t tag, const gosh_part_params& p,
                       uint64_t* updates_dev, gosh_part_stats* stats);
int partition_parts(int64_t n, int d, gosh_dtype dt, uint64_t budget, const gosh_part_params& p,
                    uint64_t* bytes);
int64_t partition_pool(const gosh_csr* g, int K, int i, int j, int B, uint64_t seed, int32_t level,
                       uint32_t tag, int32_t round, int threads, int32_t* src, int32_t* pos, int32_t* b,
                       int64_t capacity);
void inside_out_pairs(int K, int32_t* out);
// (walk.hip)
int64_t walk_pair_count(int32_t len, int32_t window);
void train_walks(Ctx* c, const Level& L, int32_t level, void* emb, gosh_dtype dt, int d, int epochs, float lr,
                 int k, int32_t len, int32_t window, uint32_t tag, uint64_t* updates_dev,
                 gosh_walk_timing* timing);
int64_t walk_pairs(Ctx* c, const Level& L, int32_t level, int32_t epoch, int32_t len, int32_t window, uint32_t tag,
                   int32_t* src, int32_t* pos, int64_t capacity);
// (mlp.hip)
gosh_mlp* mlp_create(gosh_ctx* owner, int d, int hidden);
void mlp_free(gosh_mlp* M);
void mlp_set_weights(Ctx* c, gosh_mlp* M, const float* host);
void mlp_get_weights(Ctx* c, const gosh_mlp* M, float* host);
void mlp_prolong(Ctx* c, const gosh_mlp* M, const Level& fine, int64_t n_coarse, const void* coarse,
                 void* fine_emb, gosh_dtype dt, int d);
void mlp_grad(Ctx* c, gosh_mlp* M, gosh_dtype dt, const gosh_mlp_batch* b, float* grads, float* loss);
void mlp_adam_step(Ctx* c, gosh_mlp* M, const float* grads, float lr);
void mlp_train(Ctx* c, gosh_mlp* M, gosh_dtype dt, const std::vector<PairSrcHost>& srcs, int steps,
               int batch, float lr, uint32_t tag, float* loss_dev);

}  // namespace gosh
