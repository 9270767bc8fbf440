// C ABI of the library (declared in include/gosh.h): argument checks, the
// context with its capped caching allocator, and the level store.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "gosh_internal.hpp"

namespace gosh {

// ---------------------------------------------------------------- allocator
size_t alloc_bucket(size_t bytes) {
    // 256 B granularity below 1 MiB, then 1/8 power-of-two steps
    if (bytes < (1u << 20)) return (bytes + 255) & ~size_t(255);
    size_t p = 1;
    while (p < bytes) p <<= 1;
    const size_t step = p >> 3;
    return (bytes + step - 1) / step * step;
}

void* Ctx::alloc(size_t bytes) {
    const size_t b = alloc_bucket(bytes == 0 ? 1 : bytes);
    auto it = cache.lower_bound(b);
    if (it != cache.end() && it->first <= b + b / 4) {
        void* p = it->second;
        live[p] = it->first;
        cache.erase(it);
        return p;
    }
    if (cap && in_use + b > cap) {
        trim();
        if (in_use + b > cap)
            throw Error(GOSH_E_CAP_EXCEEDED, "device memory cap of " + std::to_string(cap) +
                                                 " bytes would be exceeded");
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim();
        e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(GOSH_E_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
    }
    in_use += b;
    live[p] = b;
    return p;
}

void Ctx::free(void* p) {
    if (!p) return;
    auto it = live.find(p);
    if (it == live.end()) return;
    cache.emplace(it->second, p);
    live.erase(it);
}

void Ctx::trim() {
    if (cache.empty()) return;
    // blocks may still be in use by queued kernels of this stream
    (void)hipStreamSynchronize(stream);
    for (auto& kv : cache) {
        (void)hipFree(kv.second);
        in_use -= kv.first;
    }
    cache.clear();
}

}  // namespace gosh

using gosh::Ctx;
using gosh::Error;

namespace {

template <class F>
gosh_status guarded(gosh_ctx* ctx, F&& f) {
    try {
        f();
        if (ctx) ctx->c.err.clear();
        return GOSH_OK;
    } catch (const Error& e) {
        if (ctx) ctx->c.err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->c.err = "host allocation failed";
        return GOSH_E_OOM;
    } catch (const std::exception& e) {
        if (ctx) ctx->c.err = e.what();
        return GOSH_E_DEVICE;
    } catch (...) {
        if (ctx) ctx->c.err = "unknown failure";
        return GOSH_E_DEVICE;
    }
}

// Host-only entry points report their status without a context.
template <class F>
gosh_status host_guarded(F&& f) {
    try {
        f();
        return GOSH_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return GOSH_E_OOM;
    } catch (...) {
        return GOSH_E_DEVICE;
    }
}

void set_device(Ctx* c) { GOSH_HIP(hipSetDevice(c->device)); }

const gosh::Level& level_of(const gosh_levels* lv, int32_t i) {
    GOSH_REQUIRE(lv, GOSH_E_INVALID_ARG, "null levels");
    GOSH_REQUIRE(lv->ctx, GOSH_E_INVALID_ARG, "levels outlived their context");
    GOSH_REQUIRE(i >= 0 && i < static_cast<int32_t>(lv->lv.size()), GOSH_E_INVALID_ARG,
                 "level out of range");
    return lv->lv[i];
}

void check_csr_view(const gosh_csr* g) {
    GOSH_REQUIRE(g, GOSH_E_INVALID_ARG, "null csr");
    GOSH_REQUIRE(g->n >= 0 && g->nnz >= 0, GOSH_E_INVALID_ARG, "negative csr size");
    GOSH_REQUIRE(g->offsets, GOSH_E_INVALID_ARG, "null offsets");
    GOSH_REQUIRE(g->nnz == 0 || g->indices, GOSH_E_INVALID_ARG, "null indices");
    GOSH_REQUIRE(g->offsets_is_i64 || g->nnz <= INT32_MAX, GOSH_E_INVALID_ARG,
                 "nnz beyond int32 needs int64 offsets");
    GOSH_REQUIRE(g->n < INT32_MAX, GOSH_E_UNSUPPORTED, "vertex ids are int32");
}

}  // namespace

extern "C" {

gosh_status gosh_ctx_create(int device, uint64_t seed, void* hip_stream, uint64_t mem_cap_bytes,
                            gosh_ctx** out) {
    if (!out) return GOSH_E_INVALID_ARG;
    *out = nullptr;
    gosh_ctx* ctx = nullptr;
    try {
        ctx = new gosh_ctx();
    } catch (...) {
        return GOSH_E_OOM;
    }
    gosh_status st = guarded(ctx, [&] {
        int count = 0;
        GOSH_HIP(hipGetDeviceCount(&count));
        GOSH_REQUIRE(device >= 0 && device < count, GOSH_E_INVALID_ARG, "no such HIP device");
        Ctx* c = &ctx->c;
        c->device = device;
        c->seed = seed;
        c->cap = mem_cap_bytes;
        set_device(c);
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->scratch = c->alloc(4096);
        GOSH_HIP(hipMemsetAsync(c->scratch, 0, 4096, c->stream));
        GOSH_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->pinned), sizeof(int64_t) * Ctx::kPinnedSlots,
                               hipHostMallocDefault));
        GOSH_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->pinned_dev), c->pinned, 0));
        gosh::batched_noalloc_init(device);
    });
    if (st != GOSH_OK) {
        gosh_ctx_destroy(ctx);
        return st;
    }
    *out = ctx;
    return GOSH_OK;
}

gosh_status gosh_ctx_destroy(gosh_ctx* ctx) {
    if (!ctx) return GOSH_OK;
    Ctx* c = &ctx->c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    // hierarchies that outlive the context lose their storage with it
    for (gosh_levels* lv : ctx->levels) {
        lv->owner = nullptr;
        lv->ctx = nullptr;
    }
    for (gosh_mlp* m : ctx->mlps) {
        m->owner = nullptr;
        m->ctx = nullptr;
    }
    for (auto& kv : c->live) (void)hipFree(kv.first);
    for (auto& kv : c->cache) (void)hipFree(kv.second);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete ctx;
    return GOSH_OK;
}

gosh_status gosh_set_stream(gosh_ctx* ctx, void* hip_stream) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (s == ctx->c.stream) return GOSH_OK;
    return guarded(ctx, [&] {
        // blocks freed to the context's cache may still be read by work queued
        // on the old stream; the new stream reuses them only after that work
        set_device(&ctx->c);
        GOSH_HIP(hipStreamSynchronize(ctx->c.stream));
        ctx->c.stream = s;
    });
}

gosh_status gosh_sync(gosh_ctx* ctx) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        set_device(&ctx->c);
        GOSH_HIP(hipStreamSynchronize(ctx->c.stream));
        // a device-wide barrier of a resident launch that waited beyond its limit
        unsigned int err = 0;
        char* flag = static_cast<char*>(ctx->c.scratch) + 516;
        GOSH_HIP(hipMemcpy(&err, flag, 4, hipMemcpyDeviceToHost));
        if (err) {
            GOSH_HIP(hipMemset(flag, 0, 4));
            throw gosh::Error(GOSH_E_DEVICE, "resident epochs: a device-wide barrier waited beyond its spin limit");
        }
    });
}

const char* gosh_last_error(const gosh_ctx* ctx) {
    if (!ctx) return "null context";
    return ctx->c.err.c_str();
}

gosh_status gosh_mem_in_use(const gosh_ctx* ctx, uint64_t* bytes) {
    if (!ctx || !bytes) return GOSH_E_INVALID_ARG;
    *bytes = ctx->c.in_use;
    return GOSH_OK;
}

gosh_status gosh_trim(gosh_ctx* ctx) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        set_device(&ctx->c);
        ctx->c.trim();
    });
}

gosh_status gosh_set_deterministic(gosh_ctx* ctx, int on) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    ctx->c.deterministic = on != 0;
    return GOSH_OK;
}

gosh_status gosh_set_epoch_overlap(gosh_ctx* ctx, int32_t epochs_in_flight, int64_t min_vertices) {
    if (!ctx || epochs_in_flight < 1 || epochs_in_flight > 64 || min_vertices < 0) return GOSH_E_INVALID_ARG;
    ctx->c.overlap = epochs_in_flight;
    ctx->c.overlap_min = min_vertices;
    return GOSH_OK;
}

gosh_status gosh_set_coarsen_mode(gosh_ctx* ctx, gosh_coarsen_mode mode, int64_t batch) {
    if (!ctx || batch < 0 || (mode != GOSH_COARSEN_EXACT && mode != GOSH_COARSEN_LOCK_SKIP))
        return GOSH_E_INVALID_ARG;
    ctx->c.coarsen_mode = mode;
    ctx->c.claim_batch = batch;
    return GOSH_OK;
}

gosh_status gosh_set_plain_negatives(gosh_ctx* ctx, int64_t min_vertices) {
    if (!ctx || min_vertices < 0) return GOSH_E_INVALID_ARG;
    ctx->c.plain_neg_min = min_vertices;
    return GOSH_OK;
}

gosh_status gosh_set_plain_light_rows(gosh_ctx* ctx, int64_t min_vertices) {
    if (!ctx || min_vertices < 0) return GOSH_E_INVALID_ARG;
    ctx->c.plain_light_min = min_vertices;
    return GOSH_OK;
}

gosh_status gosh_set_grouped_positives(gosh_ctx* ctx, int64_t min_vertices, int64_t max_vertices, double hot_factor) {
    if (!ctx || min_vertices < 0 || max_vertices < 0 || !(hot_factor >= 1.0) || !std::isfinite(hot_factor))
        return GOSH_E_INVALID_ARG;
    ctx->c.group_min = min_vertices;
    ctx->c.group_max = max_vertices;
    ctx->c.group_factor = hot_factor;
    return GOSH_OK;
}

gosh_status gosh_set_resident_epochs(gosh_ctx* ctx, int64_t max_vertices) {
    if (!ctx || max_vertices < 0) return GOSH_E_INVALID_ARG;
    ctx->c.resident_max = max_vertices;
    return GOSH_OK;
}

gosh_status gosh_set_lds_levels(gosh_ctx* ctx, int64_t max_vertices) {
    if (!ctx || max_vertices < 0) return GOSH_E_INVALID_ARG;
    ctx->c.lds_max = max_vertices;
    return GOSH_OK;
}

gosh_status gosh_set_draw_record(gosh_ctx* ctx, int32_t* samples_dev, int64_t capacity) {
    if (!ctx || capacity < 0 || (samples_dev && capacity == 0)) return GOSH_E_INVALID_ARG;
    ctx->c.record = samples_dev;
    ctx->c.record_cap = samples_dev ? capacity : 0;
    return GOSH_OK;
}

gosh_status gosh_set_loss_record(gosh_ctx* ctx, double* loss_dev, int64_t capacity) {
    if (!ctx || capacity < 0 || (loss_dev && capacity == 0)) return GOSH_E_INVALID_ARG;
    ctx->c.loss = loss_dev;
    ctx->c.loss_cap = loss_dev ? capacity : 0;
    return GOSH_OK;
}

gosh_status gosh_validate_csr(gosh_ctx* ctx, const gosh_csr* g, int check_symmetry) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        check_csr_view(g);
        set_device(&ctx->c);
        gosh::validate_csr(&ctx->c, g, check_symmetry != 0);
    });
}

gosh_status gosh_coarsen(gosh_ctx* ctx, const gosh_csr* g0, int64_t threshold, double max_ratio,
                         gosh_levels** out) {
    if (!ctx || !out) return GOSH_E_INVALID_ARG;
    *out = nullptr;
    gosh_levels* lv = nullptr;
    gosh_status st = guarded(ctx, [&] {
        check_csr_view(g0);
        GOSH_REQUIRE(threshold >= 0, GOSH_E_INVALID_ARG, "threshold must be >= 0");
        GOSH_REQUIRE(std::isfinite(max_ratio) && max_ratio > 0.0 && max_ratio <= 1.0, GOSH_E_INVALID_ARG,
                     "max_ratio must be in (0, 1]");
        set_device(&ctx->c);
        gosh::validate_csr(&ctx->c, g0, false);
        lv = new gosh_levels();
        lv->owner = ctx;
        lv->ctx = &ctx->c;
        ctx->levels.insert(lv);
        gosh::coarsen(&ctx->c, g0, threshold, max_ratio, lv);
        GOSH_HIP(hipStreamSynchronize(ctx->c.stream));
    });
    if (st != GOSH_OK) {
        if (lv) gosh_levels_destroy(lv);
        return st;
    }
    *out = lv;
    return GOSH_OK;
}

gosh_status gosh_levels_single(gosh_ctx* ctx, const gosh_csr* g0, gosh_levels** out) {
    if (!ctx || !out) return GOSH_E_INVALID_ARG;
    *out = nullptr;
    gosh_levels* lv = nullptr;
    gosh_status st = guarded(ctx, [&] {
        check_csr_view(g0);
        set_device(&ctx->c);
        gosh::validate_csr(&ctx->c, g0, false);
        lv = new gosh_levels();
        lv->owner = ctx;
        lv->ctx = &ctx->c;
        ctx->levels.insert(lv);
        gosh::Level L;
        L.n = g0->n;
        L.nnz = g0->nnz;
        L.off64 = g0->offsets_is_i64 != 0;
        L.offsets = g0->offsets;
        L.indices = g0->indices;
        lv->lv.push_back(L);
    });
    if (st != GOSH_OK) {
        if (lv) gosh_levels_destroy(lv);
        return st;
    }
    *out = lv;
    return GOSH_OK;
}

gosh_status gosh_levels_destroy(gosh_levels* lv) {
    if (!lv) return GOSH_OK;
    if (lv->ctx) {
        (void)hipSetDevice(lv->ctx->device);
        for (auto& L : lv->lv) gosh::free_level(lv->ctx, L);
    }
    if (lv->owner) lv->owner->levels.erase(lv);
    delete lv;
    return GOSH_OK;
}

gosh_status gosh_levels_count(const gosh_levels* lv, int32_t* D) {
    if (!lv || !D) return GOSH_E_INVALID_ARG;
    *D = static_cast<int32_t>(lv->lv.size());
    return GOSH_OK;
}

gosh_status gosh_level_shape(const gosh_levels* lv, int32_t level, int64_t* n, int64_t* nnz) {
    if (!lv || level < 0 || level >= static_cast<int32_t>(lv->lv.size())) return GOSH_E_INVALID_ARG;
    if (n) *n = lv->lv[level].n;
    if (nnz) *nnz = lv->lv[level].nnz;
    return GOSH_OK;
}

gosh_status gosh_level_csr(const gosh_levels* lv, int32_t level, gosh_csr* out) {
    if (!lv || !out || level < 0 || level >= static_cast<int32_t>(lv->lv.size())) return GOSH_E_INVALID_ARG;
    const gosh::Level& L = lv->lv[level];
    out->n = L.n;
    out->nnz = L.nnz;
    out->offsets = L.offsets;
    out->offsets_is_i64 = L.off64 ? 1 : 0;
    out->indices = L.indices;
    return GOSH_OK;
}

gosh_status gosh_level_map(const gosh_levels* lv, int32_t level, const int32_t** map_dev,
                           const int32_t** clsz_dev) {
    if (!lv || !lv->ctx || level < 0 || level + 1 >= static_cast<int32_t>(lv->lv.size())) return GOSH_E_INVALID_ARG;
    if (map_dev) *map_dev = lv->lv[level].map;
    if (clsz_dev) {
        gosh::Ctx* c = lv->ctx;
        try {
            GOSH_HIP(hipSetDevice(c->device));
            *clsz_dev = gosh::cluster_sizes(c, lv->lv[level], lv->lv[level + 1].n);
        } catch (const gosh::Error& e) {
            c->err = e.what();
            return e.code;
        }
    }
    return GOSH_OK;
}

gosh_status gosh_level_copy_out(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, int64_t* offsets_host,
                                int32_t* indices_host, int32_t* map_host, int32_t* clsz_host) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        const gosh::Level& L = level_of(lv, level);
        Ctx* c = &ctx->c;
        set_device(c);
        if (offsets_host) {
            if (L.off64) {
                GOSH_HIP(hipMemcpyAsync(offsets_host, L.offsets, 8 * (L.n + 1), hipMemcpyDeviceToHost, c->stream));
            } else {
                std::vector<int32_t> tmp(L.n + 1);
                GOSH_HIP(hipMemcpyAsync(tmp.data(), L.offsets, 4 * (L.n + 1), hipMemcpyDeviceToHost, c->stream));
                GOSH_HIP(hipStreamSynchronize(c->stream));
                for (int64_t i = 0; i <= L.n; ++i) offsets_host[i] = tmp[i];
            }
        }
        if (indices_host && L.nnz > 0)
            GOSH_HIP(hipMemcpyAsync(indices_host, L.indices, 4 * L.nnz, hipMemcpyDeviceToHost, c->stream));
        if (map_host) {
            GOSH_REQUIRE(L.map, GOSH_E_INVALID_ARG, "the coarsest level has no map");
            if (L.n > 0)
                GOSH_HIP(hipMemcpyAsync(map_host, L.map, 4 * L.n, hipMemcpyDeviceToHost, c->stream));
        }
        if (clsz_host) {
            GOSH_REQUIRE(L.map, GOSH_E_INVALID_ARG, "the coarsest level has no clusters");
            const int64_t nn = lv->lv[level + 1].n;
            const int32_t* cs = gosh::cluster_sizes(c, L, nn);
            if (nn > 0)
                GOSH_HIP(hipMemcpyAsync(clsz_host, cs, 4 * nn, hipMemcpyDeviceToHost, c->stream));
        }
        GOSH_HIP(hipStreamSynchronize(c->stream));
    });
}

gosh_status gosh_epoch_schedule(int32_t e, double p, int32_t D, int32_t* e_out) {
    if (!e_out || D <= 0 || e < 0 || !(p >= 0.0 && p <= 1.0)) return GOSH_E_INVALID_ARG;
    std::vector<double> real(D);
    const double denom = std::ldexp(1.0, D) - 1.0;
    int64_t sum = 0;
    for (int32_t i = 0; i < D; ++i) {
        real[i] = p * e / D + (1.0 - p) * e * std::ldexp(1.0, i) / denom;
        e_out[i] = static_cast<int32_t>(std::floor(real[i]));
        sum += e_out[i];
    }
    for (int64_t rem = static_cast<int64_t>(e) - sum; rem > 0; --rem) {
        int32_t best = D - 1;
        double bf = -1.0;
        for (int32_t i = D - 1; i >= 0; --i) {
            const double f = real[i] - std::floor(real[i]);
            if (f > bf) {
                bf = f;
                best = i;
            }
        }
        e_out[best] += 1;
        real[best] = std::floor(real[best]);
    }
    return GOSH_OK;
}

gosh_status gosh_train(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, void* emb, gosh_dtype dt,
                       int32_t d, int32_t epochs, float lr, int32_t k, uint32_t tag, uint64_t* updates_dev) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        const gosh::Level& L = level_of(lv, level);
        set_device(&ctx->c);
        gosh::train_level(&ctx->c, L, level, emb, dt, d, epochs, lr, k, tag, updates_dev);
    });
}

gosh_status gosh_train_walks(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, void* emb, gosh_dtype dt,
                             int32_t d, int32_t epochs, float lr, int32_t k, int32_t walk_len, int32_t window,
                             uint32_t tag, uint64_t* updates_dev, gosh_walk_timing* timing_host) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        const gosh::Level& L = level_of(lv, level);
        set_device(&ctx->c);
        gosh::train_walks(&ctx->c, L, level, emb, dt, d, epochs, lr, k, walk_len, window, tag, updates_dev,
                          timing_host);
    });
}

gosh_status gosh_walk_pairs(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, int32_t epoch, int32_t walk_len,
                            int32_t window, uint32_t tag, int32_t* src_dev, int32_t* pos_dev, int64_t capacity,
                            int64_t* count) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        GOSH_REQUIRE(count, GOSH_E_INVALID_ARG, "null count");
        const gosh::Level& L = level_of(lv, level);
        set_device(&ctx->c);
        *count = gosh::walk_pairs(&ctx->c, L, level, epoch, walk_len, window, tag, src_dev, pos_dev, capacity);
    });
}

gosh_status gosh_train_batched(gosh_ctx* ctx, const gosh_job* jobs_host, int32_t njobs, gosh_dtype dt, int32_t d,
                               int32_t k, gosh_batch_mode mode, uint64_t* updates_dev, int32_t* chosen_out) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        Ctx* c = &ctx->c;
        set_device(c);
        gosh::train_batched(c, jobs_host, njobs, dt, d, k, static_cast<int>(mode), updates_dev, chosen_out);
        GOSH_HIP(hipStreamSynchronize(c->stream));
        unsigned int err = 0;
        GOSH_HIP(hipMemcpy(&err, static_cast<char*>(c->scratch) + 256, 4, hipMemcpyDeviceToHost));
        GOSH_REQUIRE(err == 0, GOSH_E_DEVICE, "batched training: a task waited beyond the spin limit");
    });
}

gosh_status gosh_train_batched_noalloc(gosh_ctx* ctx, const gosh_job* jobs_host, int32_t njobs, gosh_dtype dt,
                                       int32_t d, int32_t k, uint64_t* updates_dev) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        Ctx* c = &ctx->c;
        set_device(c);
        gosh::train_batched_noalloc(c, jobs_host, njobs, dt, d, k, updates_dev);
        GOSH_REQUIRE(gosh::batched_noalloc_error(c) == 0, GOSH_E_DEVICE,
                     "batched training: a task waited beyond the spin limit");
    });
}

gosh_status gosh_prolong(gosh_ctx* ctx, const gosh_levels* lv, int32_t fine_level, const void* coarse_emb,
                         void* fine_emb, gosh_dtype dt, int32_t d, const gosh_mlp* mlp) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        const gosh::Level& L = level_of(lv, fine_level);
        GOSH_REQUIRE(fine_level + 1 < static_cast<int32_t>(lv->lv.size()), GOSH_E_INVALID_ARG,
                     "fine_level must have a coarser level");
        set_device(&ctx->c);
        if (mlp) {
            GOSH_REQUIRE(mlp->owner == ctx, GOSH_E_INVALID_ARG, "network belongs to another context");
            gosh::mlp_prolong(&ctx->c, mlp, L, lv->lv[fine_level + 1].n, coarse_emb, fine_emb, dt, d);
        } else {
            gosh::prolong_copy(&ctx->c, L, coarse_emb, fine_emb, dt, d);
        }
    });
}

namespace {
gosh_mlp* mlp_of(gosh_ctx* ctx, const gosh_mlp* m) {
    GOSH_REQUIRE(m, GOSH_E_INVALID_ARG, "null network");
    GOSH_REQUIRE(m->owner == ctx, GOSH_E_INVALID_ARG, "network belongs to another context");
    return const_cast<gosh_mlp*>(m);
}
}  // namespace

gosh_status gosh_mlp_create(gosh_ctx* ctx, int32_t d, int32_t hidden, gosh_mlp** out) {
    if (!ctx || !out) return GOSH_E_INVALID_ARG;
    *out = nullptr;
    return guarded(ctx, [&] {
        set_device(&ctx->c);
        gosh_mlp* m = gosh::mlp_create(ctx, d, hidden);
        ctx->mlps.insert(m);
        *out = m;
    });
}

gosh_status gosh_mlp_destroy(gosh_mlp* mlp) {
    if (!mlp) return GOSH_OK;
    if (mlp->owner) {
        (void)hipSetDevice(mlp->ctx->device);
        (void)hipStreamSynchronize(mlp->ctx->stream);
        gosh::mlp_free(mlp);
        mlp->owner->mlps.erase(mlp);
    }
    delete mlp;
    return GOSH_OK;
}

gosh_status gosh_mlp_num_params(const gosh_mlp* mlp, int64_t* n) {
    if (!mlp || !n) return GOSH_E_INVALID_ARG;
    *n = mlp->nparams;
    return GOSH_OK;
}

gosh_status gosh_mlp_set_weights(gosh_ctx* ctx, gosh_mlp* mlp, const float* params_host) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        gosh_mlp* m = mlp_of(ctx, mlp);
        set_device(&ctx->c);
        gosh::mlp_set_weights(&ctx->c, m, params_host);
    });
}

gosh_status gosh_mlp_get_weights(gosh_ctx* ctx, const gosh_mlp* mlp, float* params_host) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        gosh_mlp* m = mlp_of(ctx, mlp);
        set_device(&ctx->c);
        gosh::mlp_get_weights(&ctx->c, m, params_host);
    });
}

gosh_status gosh_mlp_grad(gosh_ctx* ctx, gosh_mlp* mlp, gosh_dtype dt, const gosh_mlp_batch* batch,
                          float* grads_dev, float* loss_dev) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        gosh_mlp* m = mlp_of(ctx, mlp);
        set_device(&ctx->c);
        gosh::mlp_grad(&ctx->c, m, dt, batch, grads_dev, loss_dev);
    });
}

gosh_status gosh_mlp_adam_step(gosh_ctx* ctx, gosh_mlp* mlp, const float* grads_dev, float lr) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        gosh_mlp* m = mlp_of(ctx, mlp);
        set_device(&ctx->c);
        gosh::mlp_adam_step(&ctx->c, m, grads_dev, lr);
    });
}

gosh_status gosh_mlp_train(gosh_ctx* ctx, gosh_mlp* mlp, gosh_dtype dt, const gosh_mlp_source* srcs_host,
                           int32_t nsrc, int32_t steps, int32_t batch, float lr, uint32_t tag, float* loss_dev) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        gosh_mlp* m = mlp_of(ctx, mlp);
        GOSH_REQUIRE(nsrc >= 1 && srcs_host, GOSH_E_INVALID_ARG, "no pair sources");
        std::vector<gosh::PairSrcHost> v;
        for (int32_t i = 0; i < nsrc; ++i) {
            const gosh_mlp_source& s = srcs_host[i];
            const gosh::Level& L = level_of(s.lv, s.level);
            GOSH_REQUIRE(s.lv->owner == ctx, GOSH_E_INVALID_ARG, "levels belong to another context");
            GOSH_REQUIRE(s.level + 1 < static_cast<int32_t>(s.lv->lv.size()), GOSH_E_INVALID_ARG,
                         "source level must have a coarser level");
            v.push_back(gosh::PairSrcHost{&L, s.lv->lv[s.level + 1].n, s.coarse, s.fine});
        }
        set_device(&ctx->c);
        gosh::mlp_train(&ctx->c, m, dt, v, steps, batch, lr, tag, loss_dev);
    });
}

// ---------------------------------------------------------------- partitioned embedding

gosh_status gosh_train_partitioned(gosh_ctx* ctx, const gosh_csr* g_host, void* emb_host, gosh_dtype dt,
                                   int32_t d, int32_t epochs, float lr, int32_t k, int32_t level, uint32_t tag,
                                   const gosh_part_params* params, uint64_t* updates_dev, gosh_part_stats* stats) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        GOSH_REQUIRE(params, GOSH_E_INVALID_ARG, "null parameters");
        set_device(&ctx->c);
        gosh::train_partitioned(&ctx->c, g_host, emb_host, dt, d, epochs, lr, k, level, tag, *params, updates_dev,
                                stats);
    });
}

gosh_status gosh_partition_plan(int64_t n, int32_t d, gosh_dtype dt, uint64_t budget, const gosh_part_params* params,
                                int32_t* parts_out, uint64_t* bytes_out) {
    if (!params || !parts_out || n < 0) return GOSH_E_INVALID_ARG;
    return host_guarded([&] { *parts_out = gosh::partition_parts(n, d, dt, budget, *params, bytes_out); });
}

gosh_status gosh_inside_out(int32_t K, int32_t* pairs_out) {
    if (!pairs_out) return GOSH_E_INVALID_ARG;
    return host_guarded([&] { gosh::inside_out_pairs(K, pairs_out); });
}

gosh_status gosh_partition_pool(const gosh_csr* g_host, int32_t K, int32_t i, int32_t j, int32_t B, uint64_t seed,
                                int32_t level, uint32_t tag, int32_t round, int32_t threads, int64_t* count,
                                int32_t* src_out, int32_t* pos_out, int32_t* b_out, int64_t capacity) {
    if (!count) return GOSH_E_INVALID_ARG;
    if ((src_out || pos_out || b_out) && !(src_out && pos_out && b_out)) return GOSH_E_INVALID_ARG;
    return host_guarded([&] {
        *count = gosh::partition_pool(g_host, K, i, j, B, seed, level, tag, round, threads, src_out, pos_out, b_out,
                                      capacity);
    });
}

gosh_status gosh_draw_samples(gosh_ctx* ctx, const gosh_levels* lv, int32_t level, int32_t epoch, int32_t k,
                              uint32_t tag, int32_t* out_dev) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        const gosh::Level& L = level_of(lv, level);
        GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
        set_device(&ctx->c);
        gosh::draw_samples(&ctx->c, L, level, epoch, k, tag, out_dev);
    });
}

gosh_status gosh_update_batch(gosh_ctx* ctx, void* emb_dev, gosh_dtype dt, int32_t d, int64_t n_rows,
                              int32_t nsrc, const int32_t* src_dev, const int32_t* samples_dev, int32_t k,
                              float lr, int32_t level, uint32_t tag, int32_t epoch) {
    if (!ctx) return GOSH_E_INVALID_ARG;
    return guarded(ctx, [&] {
        set_device(&ctx->c);
        gosh::update_batch(&ctx->c, emb_dev, dt, d, n_rows, nsrc, src_dev, samples_dev, k, lr, level, tag,
                           epoch);
    });
}

}  // extern "C"
