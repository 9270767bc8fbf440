// MultiEdgeCollapse (Algorithm 4, Section 4) on gfx950, bit-exact with the
// sequential algorithm.
//
// The sequential loop visits vertices in the order pi = (degree descending,
// id ascending); a visited unmarked vertex becomes a hub with the next
// cluster id and marks every unmarked neighbour reached over an eligible
// edge (hub^2 restriction: deg(v) <= nnz/n or deg(u) <= nnz/n).  A vertex is
// therefore a hub exactly when no hub precedes it among its eligible
// neighbours: the hubs are the lexicographically-first maximal independent
// set of the eligible graph in pi order, and a marked vertex belongs to the
// earliest hub among its eligible neighbours.  Cluster ids count hubs in pi
// order.  This file computes that set with synchronous rounds (a vertex is
// decided IN once all earlier eligible neighbours are OUT, OUT as soon as
// one is IN), which needs as many rounds as the longest dependency chain
// (2-4 on the R-MAT levels measured), then builds the coarse CSR of Section
// 4.1 with a radix sort of the mapped edge pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_util.hpp"
#include "gosh_internal.hpp"
#include "primitives.hpp"

namespace gosh {
namespace {

constexpr int kThreads = 256;
constexpr uint8_t kUndecided = 0, kIn = 1, kOut = 2;

inline dim3 grid_for(int64_t items, int64_t per_block = kThreads) {
    int64_t b = ceil_div(std::max<int64_t>(items, 1), per_block);
    return dim3(static_cast<unsigned>(std::min<int64_t>(b, int64_t(1) << 20)));
}

#define GRID_STRIDE(i, N) \
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (N); \
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// ---------------------------------------------------------------- degrees, order
template <class Off>
__global__ void k_degree(const Off* off, int64_t n, int64_t nnz, uint8_t* light,
                         int64_t* deg_out, unsigned long long* maxdeg, unsigned long long* isolated) {
    unsigned long long mx = 0, iso = 0;
    GRID_STRIDE(v, n) {
        const int64_t d = static_cast<int64_t>(off[v + 1]) - static_cast<int64_t>(off[v]);
        if (light) light[v] = (d * n <= nnz) ? 1 : 0;
        if (deg_out) deg_out[v] = d;
        mx = mx > static_cast<unsigned long long>(d) ? mx : static_cast<unsigned long long>(d);
        iso += (d == 0);
    }
    // wave-level reduction, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(mx, o, 64);
        mx = mx > t ? mx : t;
        iso += __shfl_xor(iso, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (maxdeg) atomicMax(maxdeg, mx);
        if (isolated) atomicAdd(isolated, iso);
    }
}

__global__ void k_sort_keys(const int64_t* deg, int64_t n, uint64_t maxdeg, uint32_t* key, uint32_t* val) {
    GRID_STRIDE(v, n) {
        key[v] = static_cast<uint32_t>(maxdeg - static_cast<uint64_t>(deg[v]));
        val[v] = static_cast<uint32_t>(v);
    }
}

__global__ void k_rank_from_perm(const uint32_t* perm, int64_t n, int32_t* rank) {
    GRID_STRIDE(r, n) rank[perm[r]] = static_cast<int32_t>(r);
}

// src[p] = row of entry p: one wave per vertex streams its row.
template <class Off>
__global__ void k_expand_rows(const Off* off, int64_t n, int32_t* src) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x / 64;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6); v < n;
         v += static_cast<int64_t>(gridDim.x) * wpb) {
        const int64_t b = off[v], e = off[v + 1];
        for (int64_t p = b + lane; p < e; p += 64) src[p] = static_cast<int32_t>(v);
    }
}

// ---------------------------------------------------------------- eligible edges to earlier vertices
__global__ void k_flag_lower(const int32_t* src, const int32_t* idx, int64_t nnz, const uint8_t* light,
                             const int32_t* rank, int32_t* flag) {
    GRID_STRIDE(p, nnz) {
        const int32_t v = src[p], u = idx[p];
        flag[p] = ((light[v] | light[u]) && rank[u] < rank[v]) ? 1 : 0;
    }
}

__global__ void k_write_lower(const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* flag,
                              const int64_t* pos, int2* low) {
    GRID_STRIDE(p, nnz) {
        if (flag[p]) low[pos[p]] = make_int2(src[p], idx[p]);
    }
}

// ---------------------------------------------------------------- hub selection rounds
__global__ void k_round_edges(const int2* low, int64_t m, const uint8_t* state, uint8_t* saw_in,
                              uint8_t* saw_pending) {
    GRID_STRIDE(i, m) {
        const int2 e = low[i];
        if (state[e.x] != kUndecided) continue;
        const uint8_t su = state[e.y];
        if (su == kIn) saw_in[e.x] = 1;
        else if (su == kUndecided) saw_pending[e.x] = 1;
    }
}

__global__ void k_round_vertices(int64_t n, uint8_t* state, uint8_t* saw_in, uint8_t* saw_pending,
                                 unsigned long long* undecided) {
    unsigned long long cnt = 0;
    GRID_STRIDE(v, n) {
        if (state[v] == kUndecided) {
            if (saw_in[v]) state[v] = kOut;
            else if (!saw_pending[v]) state[v] = kIn;
            else ++cnt;
            saw_pending[v] = 0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(undecided, cnt);
}

// earliest hub among the eligible earlier neighbours of each marked vertex
__global__ void k_best_hub(const int2* low, int64_t m, const uint8_t* state, const int32_t* rank,
                           int32_t* best) {
    GRID_STRIDE(i, m) {
        const int2 e = low[i];
        if (state[e.x] == kOut && state[e.y] == kIn) atomicMin(&best[e.x], rank[e.y]);
    }
}

__global__ void k_hub_flags_by_rank(const uint32_t* perm, int64_t n, const uint8_t* state, int32_t* hf) {
    GRID_STRIDE(r, n) hf[r] = state[perm[r]] == kIn ? 1 : 0;
}

__global__ void k_assign(int64_t n, const uint8_t* state, const int32_t* rank, const int32_t* best,
                         const int64_t* cid_by_rank, int32_t* map, int32_t* clsz, unsigned int* bad) {
    GRID_STRIDE(v, n) {
        const int32_t r = state[v] == kIn ? rank[v] : best[v];
        if (state[v] == kUndecided || r < 0 || r >= n) {   // cannot happen for a valid CSR
            map[v] = 0;
            atomicOr(bad, 1u);
            continue;
        }
        const int32_t c = static_cast<int32_t>(cid_by_rank[r]);
        map[v] = c;
        atomicAdd(&clsz[c], 1);
    }
}

// ---------------------------------------------------------------- coarse graph
__global__ void k_flag_cross(const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* map,
                             int32_t* flag) {
    GRID_STRIDE(p, nnz) flag[p] = map[src[p]] != map[idx[p]] ? 1 : 0;
}

template <class K>
__global__ void k_write_pairs(const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* map,
                              const int32_t* flag, const int64_t* pos, int bb, K* keys) {
    GRID_STRIDE(p, nnz) {
        if (flag[p]) {
            const K a = static_cast<K>(static_cast<uint32_t>(map[src[p]]));
            const K b = static_cast<K>(static_cast<uint32_t>(map[idx[p]]));
            keys[pos[p]] = (a << bb) | b;
        }
    }
}

template <class K>
__global__ void k_flag_unique(const K* keys, int64_t m, int32_t* flag) {
    GRID_STRIDE(i, m) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

template <class K>
__global__ void k_write_unique(const K* keys, int64_t m, const int32_t* flag, const int64_t* pos, int bb,
                               K* ukeys, int32_t* indices) {
    GRID_STRIDE(i, m) {
        if (flag[i]) {
            const K k = keys[i];
            ukeys[pos[i]] = k;
            indices[pos[i]] = static_cast<int32_t>(k & ((K(1) << bb) - 1));
        }
    }
}

// offsets[a] = first position of a key >= a << bb (lower bound)
template <class K, class Off>
__global__ void k_offsets_lb(const K* ukeys, int64_t m, int64_t n_next, int bb, Off* offsets) {
    GRID_STRIDE(a, n_next + 1) {
        const K target = static_cast<K>(a) << bb;
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ukeys[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        offsets[a] = static_cast<Off>(lo);
    }
}

// ---------------------------------------------------------------- validation
// Offsets must be non-decreasing before any kernel may read a row.
template <class Off>
__global__ void k_check_offsets(const Off* off, int64_t n, int64_t nnz, unsigned int* bad) {
    GRID_STRIDE(v, n) {
        const int64_t b = off[v], e = off[v + 1];
        if (e < b || b < 0 || e > nnz) atomicOr(bad, 1u);
    }
}

template <class Off>
__global__ void k_validate(const Off* off, const int32_t* idx, int64_t n, int check_sym,
                           unsigned int* bad) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x / 64;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6); v < n;
         v += static_cast<int64_t>(gridDim.x) * wpb) {
        const int64_t b = off[v], e = off[v + 1];
        unsigned int f = 0;
        if (e < b) f |= 1u;
        for (int64_t p = b + lane; p < e; p += 64) {
            const int32_t u = idx[p];
            if (u < 0 || u >= n) { f |= 2u; continue; }
            if (u == v) f |= 4u;
            if (p > b && idx[p - 1] >= u) f |= 8u;
            if (check_sym) {
                int64_t lo = off[u], hi = off[u + 1];
                bool found = false;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    const int32_t w = idx[mid];
                    if (w == v) { found = true; break; }
                    if (w < v) lo = mid + 1;
                    else hi = mid;
                }
                if (!found) f |= 16u;
            }
        }
        if (f) atomicOr(bad, f);
    }
}

// ---------------------------------------------------------------- host helpers
inline int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

template <class T>
void fill(Ctx* c, T* p, int64_t count, int byte) {
    if (count > 0) GOSH_HIP(hipMemsetAsync(p, byte, sizeof(T) * count, c->stream));
}

unsigned long long* scratch_u64(Ctx* c, int slot) {
    return static_cast<unsigned long long*>(c->scratch) + slot;
}

uint64_t read_u64(Ctx* c, const unsigned long long* p) {
    unsigned long long h = 0;
    GOSH_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
    return h;
}

template <class K>
int64_t build_coarse(Ctx* c, const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* map,
                     int64_t n_next, bool off64, void** off_out, int32_t** idx_out) {
    const int bb = std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(n_next - 1, 0))));
    DevBuf<int32_t> flag(c, std::max<int64_t>(nnz, 1));
    DevBuf<int64_t> pos(c, std::max<int64_t>(nnz, 1));
    int64_t m = 0;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_flag_cross, grid_for(nnz), dim3(kThreads), 0, c->stream, src, idx, nnz,
                           map, flag.p);
        GOSH_HIP(hipGetLastError());
        scan_i32_to_i64(c, flag.p, pos.p, nnz, &m);
    }
    DevBuf<K> keys(c, std::max<int64_t>(m, 1)), tmp(c, std::max<int64_t>(m, 1));
    int64_t nnz_next = 0;
    if (m > 0) {
        hipLaunchKernelGGL((k_write_pairs<K>), grid_for(nnz), dim3(kThreads), 0, c->stream, src, idx,
                           nnz, map, flag.p, pos.p, bb, keys.p);
        GOSH_HIP(hipGetLastError());
        if constexpr (sizeof(K) == 4)
            radix_sort_u32(c, reinterpret_cast<uint32_t*>(keys.p), reinterpret_cast<uint32_t*>(tmp.p),
                           nullptr, nullptr, m, 2 * bb);
        else
            radix_sort_u64(c, reinterpret_cast<uint64_t*>(keys.p), reinterpret_cast<uint64_t*>(tmp.p), m,
                           2 * bb);
        hipLaunchKernelGGL((k_flag_unique<K>), grid_for(m), dim3(kThreads), 0, c->stream, keys.p, m,
                           flag.p);
        GOSH_HIP(hipGetLastError());
        scan_i32_to_i64(c, flag.p, pos.p, m, &nnz_next);
    }
    int32_t* indices = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * std::max<int64_t>(nnz_next, 1)));
    void* offsets = c->alloc((off64 ? 8 : 4) * (n_next + 1));
    if (m > 0) {
        // tmp receives the unique keys (the sorted keys stay in `keys`)
        hipLaunchKernelGGL((k_write_unique<K>), grid_for(m), dim3(kThreads), 0, c->stream, keys.p, m,
                           flag.p, pos.p, bb, tmp.p, indices);
        GOSH_HIP(hipGetLastError());
    }
    if (off64)
        hipLaunchKernelGGL((k_offsets_lb<K, int64_t>), grid_for(n_next + 1), dim3(kThreads), 0,
                           c->stream, tmp.p, nnz_next, n_next, bb, static_cast<int64_t*>(offsets));
    else
        hipLaunchKernelGGL((k_offsets_lb<K, int32_t>), grid_for(n_next + 1), dim3(kThreads), 0,
                           c->stream, tmp.p, nnz_next, n_next, bb, static_cast<int32_t*>(offsets));
    GOSH_HIP(hipGetLastError());
    *off_out = offsets;
    *idx_out = indices;
    return nnz_next;
}

template <class Off>
void coarsen_one(Ctx* c, Level& L, Level& next) {
    const int64_t n = L.n, nnz = L.nnz;
    const Off* off = static_cast<const Off*>(L.offsets);
    const int32_t* idx = L.indices;

    // degrees, eligibility and the processing order pi
    DevBuf<uint8_t> light(c, n);
    DevBuf<int64_t> deg(c, n);
    GOSH_HIP(hipMemsetAsync(c->scratch, 0, 64, c->stream));
    hipLaunchKernelGGL((k_degree<Off>), grid_for(n), dim3(kThreads), 0, c->stream, off, n, nnz,
                       light.p, deg.p, scratch_u64(c, 0), nullptr);
    GOSH_HIP(hipGetLastError());
    const uint64_t maxdeg = read_u64(c, scratch_u64(c, 0));
    DevBuf<uint32_t> key(c, n), key_tmp(c, n), perm(c, n), perm_tmp(c, n);
    hipLaunchKernelGGL(k_sort_keys, grid_for(n), dim3(kThreads), 0, c->stream, deg.p, n, maxdeg, key.p,
                       perm.p);
    GOSH_HIP(hipGetLastError());
    radix_sort_u32(c, key.p, key_tmp.p, perm.p, perm_tmp.p, n, bits_for(maxdeg));
    key_tmp.reset();
    perm_tmp.reset();
    key.reset();
    deg.reset();
    DevBuf<int32_t> rank(c, n);
    hipLaunchKernelGGL(k_rank_from_perm, grid_for(n), dim3(kThreads), 0, c->stream, perm.p, n, rank.p);
    GOSH_HIP(hipGetLastError());

    // row of every entry, and the eligible entries towards earlier vertices
    DevBuf<int32_t> src(c, std::max<int64_t>(nnz, 1));
    if (nnz > 0) {
        hipLaunchKernelGGL((k_expand_rows<Off>), grid_for(n, kThreads / 64), dim3(kThreads), 0, c->stream,
                           off, n, src.p);
        GOSH_HIP(hipGetLastError());
    }
    int64_t m = 0;
    DevBuf<int2> low;
    {
        DevBuf<int32_t> flag(c, std::max<int64_t>(nnz, 1));
        DevBuf<int64_t> pos(c, std::max<int64_t>(nnz, 1));
        if (nnz > 0) {
            hipLaunchKernelGGL(k_flag_lower, grid_for(nnz), dim3(kThreads), 0, c->stream, src.p, idx, nnz,
                               light.p, rank.p, flag.p);
            GOSH_HIP(hipGetLastError());
            scan_i32_to_i64(c, flag.p, pos.p, nnz, &m);
        }
        low = DevBuf<int2>(c, std::max<int64_t>(m, 1));
        if (m > 0) {
            hipLaunchKernelGGL(k_write_lower, grid_for(nnz), dim3(kThreads), 0, c->stream, src.p, idx, nnz,
                               flag.p, pos.p, low.p);
            GOSH_HIP(hipGetLastError());
        }
    }

    // hub selection rounds
    DevBuf<uint8_t> state(c, n), saw_in(c, n), saw_pending(c, n);
    fill(c, state.p, n, 0);
    fill(c, saw_in.p, n, 0);
    fill(c, saw_pending.p, n, 0);
    for (int64_t round = 0;; ++round) {
        GOSH_REQUIRE(round <= n + 1, GOSH_E_DEVICE, "coarsening rounds did not converge");
        if (m > 0) {
            hipLaunchKernelGGL(k_round_edges, grid_for(m), dim3(kThreads), 0, c->stream, low.p, m, state.p,
                               saw_in.p, saw_pending.p);
            GOSH_HIP(hipGetLastError());
        }
        GOSH_HIP(hipMemsetAsync(scratch_u64(c, 1), 0, 8, c->stream));
        hipLaunchKernelGGL(k_round_vertices, grid_for(n), dim3(kThreads), 0, c->stream, n, state.p, saw_in.p,
                           saw_pending.p, scratch_u64(c, 1));
        GOSH_HIP(hipGetLastError());
        if (read_u64(c, scratch_u64(c, 1)) == 0) break;
    }
    saw_in.reset();
    saw_pending.reset();

    // each marked vertex joins the earliest hub among its eligible earlier neighbours
    DevBuf<int32_t> best(c, n);
    fill(c, best.p, n, 0x7F);
    if (m > 0) {
        hipLaunchKernelGGL(k_best_hub, grid_for(m), dim3(kThreads), 0, c->stream, low.p, m, state.p, rank.p,
                           best.p);
        GOSH_HIP(hipGetLastError());
    }
    low.reset();
    DevBuf<int32_t> hf(c, n);
    DevBuf<int64_t> cid(c, n);
    hipLaunchKernelGGL(k_hub_flags_by_rank, grid_for(n), dim3(kThreads), 0, c->stream, perm.p, n, state.p,
                       hf.p);
    GOSH_HIP(hipGetLastError());
    int64_t n_next = 0;
    scan_i32_to_i64(c, hf.p, cid.p, n, &n_next);
    hf.reset();
    L.map = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * n));
    L.clsz = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * std::max<int64_t>(n_next, 1)));
    fill(c, L.clsz, n_next, 0);
    unsigned int* bad = reinterpret_cast<unsigned int*>(scratch_u64(c, 4));
    GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    hipLaunchKernelGGL(k_assign, grid_for(n), dim3(kThreads), 0, c->stream, n, state.p, rank.p, best.p,
                       cid.p, L.map, L.clsz, bad);
    GOSH_HIP(hipGetLastError());
    GOSH_REQUIRE(read_u64(c, scratch_u64(c, 4)) == 0, GOSH_E_BAD_GRAPH,
                 "coarsening found a vertex without a cluster (graph not symmetric?)");
    cid.reset();
    best.reset();
    state.reset();
    rank.reset();
    perm.reset();
    light.reset();

    // coarse graph: distinct pairs (map v, map u), map v != map u, rows ascending
    void* noff = nullptr;
    int32_t* nidx = nullptr;
    int64_t nnz_next;
    if (2 * std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(n_next - 1, 0)))) <= 32)
        nnz_next = build_coarse<uint32_t>(c, src.p, idx, nnz, L.map, n_next, L.off64, &noff, &nidx);
    else
        nnz_next = build_coarse<uint64_t>(c, src.p, idx, nnz, L.map, n_next, L.off64, &noff, &nidx);
    next.n = n_next;
    next.nnz = nnz_next;
    next.off64 = L.off64;
    next.offsets = next.own_offsets = noff;
    next.indices = next.own_indices = nidx;
    next.n_deg0 = count_isolated(c, next);
}

}  // namespace

int64_t count_isolated(Ctx* c, const Level& L) {
    if (L.n == 0) return 0;
    GOSH_HIP(hipMemsetAsync(scratch_u64(c, 2), 0, 8, c->stream));
    if (L.off64)
        hipLaunchKernelGGL((k_degree<int64_t>), grid_for(L.n), dim3(kThreads), 0, c->stream,
                           static_cast<const int64_t*>(L.offsets), L.n, L.nnz, nullptr, nullptr, nullptr,
                           scratch_u64(c, 2));
    else
        hipLaunchKernelGGL((k_degree<int32_t>), grid_for(L.n), dim3(kThreads), 0, c->stream,
                           static_cast<const int32_t*>(L.offsets), L.n, L.nnz, nullptr, nullptr, nullptr,
                           scratch_u64(c, 2));
    GOSH_HIP(hipGetLastError());
    return static_cast<int64_t>(read_u64(c, scratch_u64(c, 2)));
}

void validate_csr(Ctx* c, const gosh_csr* g, bool symmetry) {
    GOSH_REQUIRE(g && g->n >= 0 && g->nnz >= 0, GOSH_E_INVALID_ARG, "bad csr shape");
    GOSH_REQUIRE(g->offsets && (g->nnz == 0 || g->indices), GOSH_E_INVALID_ARG, "null csr pointer");
    GOSH_REQUIRE(g->offsets_is_i64 || g->nnz <= INT32_MAX, GOSH_E_INVALID_ARG,
                 "nnz needs int64 offsets");
    GOSH_REQUIRE(g->n < INT32_MAX, GOSH_E_UNSUPPORTED, "vertex ids are int32");
    int64_t first = 0, last = 0;
    if (g->offsets_is_i64) {
        const int64_t* o = static_cast<const int64_t*>(g->offsets);
        GOSH_HIP(hipMemcpyAsync(&first, o, 8, hipMemcpyDeviceToHost, c->stream));
        GOSH_HIP(hipMemcpyAsync(&last, o + g->n, 8, hipMemcpyDeviceToHost, c->stream));
    } else {
        int32_t f32 = 0, l32 = 0;
        const int32_t* o = static_cast<const int32_t*>(g->offsets);
        GOSH_HIP(hipMemcpyAsync(&f32, o, 4, hipMemcpyDeviceToHost, c->stream));
        GOSH_HIP(hipMemcpyAsync(&l32, o + g->n, 4, hipMemcpyDeviceToHost, c->stream));
        GOSH_HIP(hipStreamSynchronize(c->stream));
        first = f32;
        last = l32;
    }
    GOSH_HIP(hipStreamSynchronize(c->stream));
    GOSH_REQUIRE(first == 0 && last == g->nnz, GOSH_E_BAD_GRAPH, "offsets must run from 0 to nnz");
    if (g->n == 0) return;
    unsigned int* bad = reinterpret_cast<unsigned int*>(scratch_u64(c, 3));
    unsigned int h = 0;
    GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    if (g->offsets_is_i64)
        hipLaunchKernelGGL((k_check_offsets<int64_t>), grid_for(g->n), dim3(kThreads), 0, c->stream,
                           static_cast<const int64_t*>(g->offsets), g->n, g->nnz, bad);
    else
        hipLaunchKernelGGL((k_check_offsets<int32_t>), grid_for(g->n), dim3(kThreads), 0, c->stream,
                           static_cast<const int32_t*>(g->offsets), g->n, g->nnz, bad);
    GOSH_HIP(hipGetLastError());
    GOSH_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
    GOSH_REQUIRE(h == 0, GOSH_E_BAD_GRAPH, "offsets decrease or leave [0, nnz]");
    GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    if (g->offsets_is_i64)
        hipLaunchKernelGGL((k_validate<int64_t>), grid_for(g->n, kThreads / 64), dim3(kThreads), 0,
                           c->stream, static_cast<const int64_t*>(g->offsets), g->indices, g->n,
                           0, bad);
    else
        hipLaunchKernelGGL((k_validate<int32_t>), grid_for(g->n, kThreads / 64), dim3(kThreads), 0,
                           c->stream, static_cast<const int32_t*>(g->offsets), g->indices, g->n,
                           0, bad);
    GOSH_HIP(hipGetLastError());
    GOSH_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
    GOSH_REQUIRE(!(h & 1u), GOSH_E_BAD_GRAPH, "offsets decrease");
    GOSH_REQUIRE(!(h & 2u), GOSH_E_BAD_GRAPH, "neighbour index out of range");
    GOSH_REQUIRE(!(h & 4u), GOSH_E_BAD_GRAPH, "self-loop");
    GOSH_REQUIRE(!(h & 8u), GOSH_E_BAD_GRAPH, "row not strictly ascending (unsorted or duplicate)");
    if (symmetry) {
        // only run once the structure is known to be in range
        GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
        if (g->offsets_is_i64)
            hipLaunchKernelGGL((k_validate<int64_t>), grid_for(g->n, kThreads / 64), dim3(kThreads), 0,
                               c->stream, static_cast<const int64_t*>(g->offsets), g->indices, g->n, 1,
                               bad);
        else
            hipLaunchKernelGGL((k_validate<int32_t>), grid_for(g->n, kThreads / 64), dim3(kThreads), 0,
                               c->stream, static_cast<const int32_t*>(g->offsets), g->indices, g->n, 1,
                               bad);
        GOSH_HIP(hipGetLastError());
        GOSH_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, c->stream));
        GOSH_HIP(hipStreamSynchronize(c->stream));
        GOSH_REQUIRE(!(h & 16u), GOSH_E_BAD_GRAPH, "graph is not symmetric");
    }
}

void coarsen(Ctx* c, const gosh_csr* g0, int64_t threshold, double ratio, gosh_levels* out) {
    Level L0;
    L0.n = g0->n;
    L0.nnz = g0->nnz;
    L0.off64 = g0->offsets_is_i64 != 0;
    L0.offsets = g0->offsets;
    L0.indices = g0->indices;
    L0.n_deg0 = count_isolated(c, L0);
    out->lv.push_back(L0);
    if (L0.n == 0) return;
    constexpr int kMaxLevels = 128;
    while (static_cast<int>(out->lv.size()) < kMaxLevels) {
        Level next;
        Level& cur = out->lv.back();
        if (cur.off64) coarsen_one<int64_t>(c, cur, next);
        else coarsen_one<int32_t>(c, cur, next);
        const int64_t n_prev = cur.n;
        out->lv.push_back(next);
        if (!(next.n >= threshold && static_cast<double>(next.n) <= ratio * static_cast<double>(n_prev)))
            break;
    }
}

void free_level(Ctx* c, Level& L) {
    if (L.own_offsets) c->free(L.own_offsets);
    if (L.own_indices) c->free(L.own_indices);
    if (L.map) c->free(L.map);
    if (L.clsz) c->free(L.clsz);
    L.own_offsets = nullptr;
    L.own_indices = nullptr;
    L.map = nullptr;
    L.clsz = nullptr;
}

}  // namespace gosh
