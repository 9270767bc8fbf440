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
#include <utility>
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

// Kernels that fold into one global counter: at most this many blocks, and
// one atomic per block (same-address atomics serialise at one L2 channel,
// one per wave cost ~80 us on a 93k-vertex level)
constexpr int64_t kReduceBlocks = 2048;
inline dim3 grid_reduce(int64_t items, int64_t per_block = kThreads) {
    return dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div(std::max<int64_t>(items, 1), per_block),
                                                        kReduceBlocks)));
}

// Block sum (op 0) or maximum (op 1) of v, added / maxed into *dst by thread
// 0; every thread of the block calls it (blocks of at most kThreads).
template <int OP>
__device__ __forceinline__ void block_fold(unsigned long long* dst, unsigned long long v) {
    __shared__ unsigned long long part[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(v, o, 64);
        v = OP == 0 ? v + t : (v > t ? v : t);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = part[0];
        for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) r = OP == 0 ? r + part[w] : (r > part[w] ? r : part[w]);
        if (OP == 0 && r) atomicAdd(dst, r);
        if (OP == 1) atomicMax(dst, r);
    }
}

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
    // block-level reductions, one atomic per block (pointer tests are uniform)
    if (maxdeg) block_fold<1>(maxdeg, mx);
    if (isolated) {
        __syncthreads();
        block_fold<0>(isolated, iso);
    }
}

__global__ void k_sort_keys(const int64_t* deg, int64_t n, const unsigned long long* maxdeg_dev, uint32_t* key,
                            uint32_t* val) {
    const uint64_t maxdeg = *maxdeg_dev;
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
// Entry p = (v, u) is kept when one end is light and u comes earlier in pi.
// The kept entries are compacted in CSR order, so vertex v's eligible
// earlier neighbours form the segment [lstart[v], lstart[v+1]) of `lower`.
// The keep decisions (two random lookups per entry) are taken once, into a
// bit per entry (word w holds entries 64 w .. 64 w + 63), with each word's
// count of kept entries before it in its tile of kLowerTile entries and
// each tile's count; an exclusive sum over the tiles then places every
// entry and every row start without a second pass over the lookups.
constexpr int kLowerItems = 16;
constexpr int64_t kLowerTile = int64_t(kThreads) * kLowerItems;
constexpr int kLowerWords = static_cast<int>(kLowerTile / 64);   // 64 words per tile

// rl[v] = rank of v in pi, with bit 31 set when v is light: the keep test
// then takes one random lookup per entry instead of two.  Also starts every
// vertex of the hub rounds undecided.
__global__ void k_pack_rank_light(const int32_t* rank, const uint8_t* light, int64_t n, uint32_t* rl,
                                  uint8_t* state) {
    GRID_STRIDE(v, n) {
        rl[v] = static_cast<uint32_t>(rank[v]) | (light[v] ? 0x80000000u : 0u);
        state[v] = kUndecided;
    }
}

__global__ __launch_bounds__(kThreads) void k_lower_bits(const int32_t* src, const int32_t* idx, int64_t nnz,
                                                         const uint32_t* rl, unsigned long long* bits,
                                                         uint16_t* wpre, int64_t* tile_cnt) {
    __shared__ int wc[kLowerWords];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kLowerTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) tile_cnt[gridDim.x] = 0;   // the total's slot of the scan
#pragma unroll 4
    for (int r = 0; r < kLowerItems; ++r) {
        const int64_t p = base + r * kThreads + threadIdx.x;
        bool keep = false;
        if (p < nnz) {
            const uint32_t kv = rl[src[p]], ku = rl[idx[p]];
            keep = ((kv | ku) >> 31) != 0u && (ku & 0x7FFFFFFFu) < (kv & 0x7FFFFFFFu);
        }
        const unsigned long long m = __ballot(keep);
        const int word = r * (kThreads / 64) + w;   // entries base + 64 word .. + 63
        if (lane == 0) {
            wc[word] = __popcll(m);
            if (base + 64 * word < nnz) bits[(base >> 6) + word] = m;
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {   // exclusive prefix of the 64 word counts, one wave
        const int c = wc[lane];
        int inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (base + 64 * lane < nnz) wpre[(base >> 6) + lane] = static_cast<uint16_t>(inc - c);
        if (lane == 63) tile_cnt[blockIdx.x] = inc;
    }
}

// Kept entry p goes to tile_base[p / kLowerTile] + wpre[p / 64] + (kept
// entries before p in its word).
__global__ void k_lower_write(const int32_t* idx, int64_t nnz, const unsigned long long* bits,
                              const uint16_t* wpre, const int64_t* tile_base, int32_t* lower) {
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    GRID_STRIDE(p, nnz) {
        const int64_t word = p >> 6;
        const unsigned long long m = bits[word];
        if ((m >> lane) & 1ull)
            lower[tile_base[p / kLowerTile] + wpre[word] + __popcll(m & lt)] = idx[p];
    }
}

// lstart[v] = kept entries before off[v] (v = 0..n); tile_base has tiles + 1
// entries, the last the total.
template <class Off>
__global__ void k_lower_starts(const Off* off, int64_t n, int64_t nnz, const unsigned long long* bits,
                               const uint16_t* wpre, const int64_t* tile_base, int64_t tiles, int64_t* lstart) {
    GRID_STRIDE(v, n + 1) {
        const int64_t e = off[v];
        if (e >= nnz) {
            lstart[v] = tile_base[tiles];
        } else {
            const int64_t word = e >> 6;
            const int b = static_cast<int>(e & 63);
            const unsigned long long below = b == 0 ? 0ull : (bits[word] & (~0ull >> (64 - b)));
            lstart[v] = tile_base[e / kLowerTile] + wpre[word] + __popcll(below);
        }
    }
}

// ---------------------------------------------------------------- hub selection rounds
constexpr int kSparseGroup = 8;   // lanes per vertex in the rounds and the assignment of sparse levels
// In place: a decision only uses states that are final (IN, OUT), so reading
// a neighbour before or after its own decision in the same round is safe.
// The round's decision with GL lanes per vertex (GL = 64 on dense levels
// whose segments run to hundreds of entries, 8 on the others): lanes split
// the segment and OR their findings across the group (reading every entry
// instead of stopping at the first IN gives the same decision); a vertex's
// lanes share its loop iterations, so the group's shuffles see them all.
// *undecided is set to 1 (one plain store per workgroup that left a vertex
// undecided), so the grid needs no cap for a shared counter; *next_flag, the
// next round's, is cleared here (it is nobody else's in this launch).
template <int GL>
__global__ void k_round_group(int64_t n, const int64_t* lstart, const int32_t* lower, uint8_t* state,
                              unsigned long long* undecided, unsigned long long* next_flag) {
    __shared__ int left;
    if (threadIdx.x == 0) left = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_flag = 0ull;
    __syncthreads();
    const int sub = threadIdx.x % GL;
    const int64_t gpb = blockDim.x / GL;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * gpb + threadIdx.x / GL; v < n;
         v += static_cast<int64_t>(gridDim.x) * gpb) {
        const uint8_t sv = state[v];
        if (sv != kUndecided) continue;   // one address: the same value in every lane of the group
        int any_in = 0, pending = 0;
        const int64_t e = lstart[v + 1];
        for (int64_t i = lstart[v] + sub; i < e; i += GL) {
            const uint8_t su = state[lower[i]];
            any_in |= (su == kIn);
            pending |= (su == kUndecided);
        }
#pragma unroll
        for (int o = GL / 2; o > 0; o >>= 1) {
            any_in |= __shfl_xor(any_in, o, 64);
            pending |= __shfl_xor(pending, o, 64);
        }
        if (sub == 0) {
            if (any_in) state[v] = kOut;
            else if (!pending) state[v] = kIn;
            else left = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && left) *undecided = 1ull;
}

__global__ void k_hub_flags_by_rank(const uint32_t* perm, int64_t n, const uint8_t* state, int32_t* hf) {
    GRID_STRIDE(r, n) hf[r] = state[perm[r]] == kIn ? 1 : 0;
}

// A hub keeps its own cluster; a marked vertex joins the earliest hub among
// its eligible earlier neighbours (GL lanes per vertex take the minimum hub
// rank over their part of the segment, then the group reduces it).  Cluster
// id = hubs before it in pi order.
template <int GL>
__global__ void k_assign_group(int64_t n, const int64_t* lstart, const int32_t* lower, const uint8_t* state,
                               const int32_t* rank, const int64_t* cid_by_rank, int32_t* map, unsigned int* bad) {
    const int sub = threadIdx.x % GL;
    const int64_t gpb = blockDim.x / GL;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * gpb + threadIdx.x / GL; v < n;
         v += static_cast<int64_t>(gridDim.x) * gpb) {
        const uint8_t sv = state[v];
        int32_t best = INT32_MAX;
        if (sv == kIn) {
            best = rank[v];
        } else if (sv == kOut) {
            const int64_t e = lstart[v + 1];
            for (int64_t i = lstart[v] + sub; i < e; i += GL) {
                const int32_t u = lower[i];
                if (state[u] == kIn) best = min(best, rank[u]);
            }
#pragma unroll
            for (int o = GL / 2; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
        }
        if (sub == 0) {
            if (best < 0 || best >= n) {   // cannot happen once every vertex is decided
                map[v] = 0;
                atomicOr(bad, 1u);
            } else {
                map[v] = static_cast<int32_t>(cid_by_rank[best]);
            }
        }
    }
}

// ---------------------------------------------------------------- lock-and-skip mapping
// The paper's parallel coarsening (Section 4, parallelisation): vertices are
// taken in pi order by concurrent threads; a thread that finds its vertex v
// unmarked claims it as a hub (owner[v] = v) and then marks every unmarked
// neighbour u over an eligible edge (owner[u] = v).  Each claim is one
// compare-and-swap from -1, so a mark is never overwritten, and a vertex
// that another thread marked first is skipped (the paper's lock that fails).
// Vertices of ranks [r0, r1) run concurrently; ranks in later launches see
// all earlier claims.  One wave over all ranks is Algorithm 4 exactly.
// One wave per vertex (a thread per vertex would leave a hub's whole
// neighbour list to one lane): lane 0 claims, the wave marks the neighbours.
// With one wave in the grid the ranks run strictly in order.
template <class Off>
__global__ void k_claim(const Off* off, const int32_t* idx, const uint32_t* perm, int64_t r0, int64_t r1,
                             const uint8_t* light, int32_t* owner) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x >> 6;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6); i < r1 - r0;
         i += static_cast<int64_t>(gridDim.x) * wpb) {
        const int64_t v = perm[r0 + i];
        int won = 0;
        if (lane == 0 && __hip_atomic_load(owner + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1)
            won = atomicCAS(owner + v, -1, static_cast<int32_t>(v)) == -1 ? 1 : 0;
        if (__shfl(won, 0, 64) == 0) continue;
        const bool lv = light[v] != 0;
        for (int64_t e = off[v] + lane, end = off[v + 1]; e < end; e += 64) {
            const int32_t u = idx[e];
            if (!(lv || light[u])) continue;
            if (__hip_atomic_load(owner + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1)
                atomicCAS(owner + u, -1, static_cast<int32_t>(v));
        }
    }
}

__global__ void k_owner_hub_flags(const uint32_t* perm, int64_t n, const int32_t* owner, int32_t* hf) {
    GRID_STRIDE(r, n) hf[r] = owner[perm[r]] == static_cast<int32_t>(perm[r]) ? 1 : 0;
}

// Cluster id of v = number of hubs before its hub in pi order.
__global__ void k_owner_assign(int64_t n, const int32_t* owner, const int32_t* rank, const int64_t* cid_by_rank,
                               int32_t* map, unsigned int* bad) {
    GRID_STRIDE(v, n) {
        const int32_t h = owner[v];
        if (h < 0 || h >= n) {   // cannot happen once every rank was processed
            map[v] = 0;
            atomicOr(bad, 1u);
            continue;
        }
        map[v] = static_cast<int32_t>(cid_by_rank[rank[h]]);
    }
}

__global__ void k_cluster_sizes(const int32_t* map, int64_t n, int32_t* clsz) {
    GRID_STRIDE(v, n) atomicAdd(&clsz[map[v]], 1);
}

// ---------------------------------------------------------------- coarse graph
// Key of every entry: (map v) << bb | (map u) for an entry between two
// clusters, `sent` (above every such key in the low 2 bb bits) inside one.
template <class K>
__global__ void k_write_pairs(const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* map, int bb,
                              K sent, K* keys) {
    GRID_STRIDE(p, nnz) {
        const uint32_t a = static_cast<uint32_t>(map[src[p]]);
        const uint32_t b = static_cast<uint32_t>(map[idx[p]]);
        keys[p] = a != b ? (static_cast<K>(a) << bb) | static_cast<K>(b) : sent;
    }
}

template <class K>
__global__ void k_flag_unique(const K* keys, int64_t m, K sent, int32_t* flag) {
    GRID_STRIDE(i, m) flag[i] = (keys[i] != sent && (i == 0 || keys[i] != keys[i - 1])) ? 1 : 0;
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

// ---------------------------------------------------------------- coarse graph by cluster segments
// The coarse row of cluster c is the sorted set of clusters adjacent to its
// members.  Members are grouped by cluster (a sort of the n vertices by map),
// so the entries of one cluster form one contiguous segment of the level's
// entries in member order; each entry is replaced by its neighbour's cluster
// (or kSegSent inside c).  A segment's distinct clusters are collected in a
// bitmap over the next level's vertex ids and read back in bit order, which
// is ascending: one wave with an LDS bitmap per segment of at most kSegSmall
// entries; longer segments (hub clusters) are cut into chunks of kGiantChunk
// entries, one workgroup each, whose LDS bitmaps are OR-ed into one global
// bitmap per cluster.
constexpr int kSegSmall = 4096;     // entries of a segment deduplicated by one wave
constexpr int kGiantChunk = 16384;  // entries of a long segment per workgroup
constexpr int kSegWaves = 4;
constexpr int kSegBatch = 8;        // entries per lane loaded before their bitmap updates
constexpr int kSegDenseWords = 256; // bitmap words (ids < 8192: the hub clusters) read back densely
constexpr int64_t kSegMaxWords = 8192;   // bitmap words per wave (next level of at most 262,144 vertices)
constexpr uint32_t kSegSent = 0xFFFFFFFFu;

template <class Off>
__global__ void k_member_deg(const Off* off, const uint32_t* mem, int64_t n, int32_t* mdeg) {
    GRID_STRIDE(i, n) {
        const int64_t v = mem[i];
        mdeg[i] = static_cast<int32_t>(static_cast<int64_t>(off[v + 1]) - static_cast<int64_t>(off[v]));
    }
}

// cstart[c] = first member position of cluster c (lower bound in the sorted
// cluster keys), segstart[c] = its first entry; both for c in [0, n_next]
__global__ void k_seg_starts(const uint32_t* ckey, int64_t n, int64_t n_next, const int64_t* E, int64_t nnz,
                             int64_t* segstart) {
    GRID_STRIDE(c, n_next + 1) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (static_cast<int64_t>(ckey[mid]) < c) lo = mid + 1;
            else hi = mid;
        }
        segstart[c] = lo < n ? E[lo] : nnz;
    }
}

// dbase[v] = E[position of v among the members] - off[v], so that entry p of
// row v goes to raw[dbase[v] + p]
template <class Off>
__global__ void k_dest_base(const Off* off, const uint32_t* mem, const int64_t* E, int64_t n, int64_t* dbase) {
    GRID_STRIDE(i, n) {
        const int64_t v = mem[i];
        dbase[v] = E[i] - static_cast<int64_t>(off[v]);
    }
}

// raw[dbase[v] + p] = cluster of entry p's neighbour (kSegSent inside v's cluster)
__global__ void k_gather_raw(const int32_t* src, const int32_t* idx, int64_t nnz, const int64_t* dbase,
                             const int32_t* map, uint32_t* raw) {
    GRID_STRIDE(p, nnz) {
        const int32_t v = src[p];
        const uint32_t m = static_cast<uint32_t>(map[idx[p]]);
        raw[dbase[v] + p] = m != static_cast<uint32_t>(map[v]) ? m : kSegSent;
    }
}

// orders the wave's LDS writes before its later LDS reads
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per small segment: its clusters OR-ed into the wave's bitmap over
// the next level's vertex ids (W 32-bit words of dynamic LDS, cleared once
// per wave), then the distinct ids written back in place, ascending (bit
// order), and exactly the words that were set cleared again; cnt[c] = their
// number.  A segment with at least W / 2 entries (dense coarse levels) reads
// all W words back 64 at a time, each lane placing its word's ids after a
// wave prefix sum of the popcounts.  A shorter one (level 0: a few hundred
// entries against thousands of words) also marks a summary with one bit per
// bitmap word (S = ceil(W / 32) words after the bitmap).  Its first
// kSegDenseWords words -- the ids of the level's hub clusters, which most
// segments reach (71% of a level-0 segment's ids) -- are read back by all
// lanes 64 at a time; past them lane l reads back only the marked words of
// its summary words, so the segment costs its entries, not the words of the
// bitmap, and no lane is left with most of them.
__global__ __launch_bounds__(64 * kSegWaves) void k_dedup_small(const int64_t* segstart, int64_t n_next, int W,
                                                                uint32_t* raw, int32_t* cnt) {
    extern __shared__ uint32_t seg_bitmaps[];
    const int lane = threadIdx.x & 63;
    const int S = (W + 31) >> 5;
    uint32_t* bm = seg_bitmaps + static_cast<int64_t>(threadIdx.x >> 6) * (W + S);
    uint32_t* sm = bm + W;
    for (int w = lane; w < W + S; w += 64) bm[w] = 0u;
    wave_lds_sync();
    const int64_t nw = static_cast<int64_t>(gridDim.x) * kSegWaves;
    int64_t c = static_cast<int64_t>(blockIdx.x) * kSegWaves + (threadIdx.x >> 6);
    // the bounds of the wave's next segment are loaded while it works on the
    // current one, and a segment's entries kSegBatch per lane at a time: a
    // level-0 segment (about 270 entries) then costs one dependent round trip
    // to memory instead of six
    int64_t nb0 = c < n_next ? segstart[c] : 0, nb1 = c < n_next ? segstart[c + 1] : 0;
    for (; c < n_next; c += nw) {
        const int64_t s0 = nb0;
        const int64_t len = nb1 - s0;
        if (c + nw < n_next) {
            nb0 = segstart[c + nw];
            nb1 = segstart[c + nw + 1];
        }
        if (len > kSegSmall) continue;   // a hub cluster: chunked with the others
        const bool sparse = static_cast<int64_t>(W) > 2 * len;   // wave-uniform
        for (int64_t i0 = 0; i0 < len; i0 += 64 * kSegBatch) {
            uint32_t x[kSegBatch];
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u) {
                const int64_t i = i0 + u * 64 + lane;
                x[u] = i < len ? raw[s0 + i] : kSegSent;
            }
#pragma unroll
            for (int u = 0; u < kSegBatch; ++u) {
                if (x[u] != kSegSent) {
                    atomicOr(&bm[x[u] >> 5], 1u << (x[u] & 31u));
                    if (sparse) atomicOr(&sm[x[u] >> 10], 1u << ((x[u] >> 5) & 31u));
                }
            }
        }
        wave_lds_sync();
        int total = 0;
        // words [0, P) read back by all lanes, 64 at a time, in order
        const int P = sparse ? min(W, kSegDenseWords) : W;
        for (int base = 0; base < P; base += 64) {
            const int w = base + lane;
            uint32_t word = w < P ? bm[w] : 0u;
            const int pc = __popc(word);
            int incl = pc;
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            int64_t pos = s0 + total + (incl - pc);
            if (w < P) bm[w] = 0u;
            while (word) {
                const int bit = __ffs(word) - 1;
                raw[pos++] = (static_cast<uint32_t>(w) << 5) | static_cast<uint32_t>(bit);
                word &= word - 1u;
            }
            total += __shfl(incl, 63, 64);
        }
        if (sparse) {
            // the rest through the summary: each lane takes qq summary words
            // (32 bitmap words each) past the s_lo that cover [0, P)
            const int s_lo = P == W ? S : (P >> 5);
            for (int i = lane; i < s_lo; i += 64) sm[i] = 0u;
            const int qq = (S - s_lo + 63) >> 6;
            int pc = 0;
            for (int j = 0; j < qq; ++j) {
                const int sidx = s_lo + lane * qq + j;
                if (sidx < S) {
                    uint32_t sw = sm[sidx];
                    while (sw) {
                        const int b = __ffs(sw) - 1;
                        pc += __popc(bm[(sidx << 5) + b]);
                        sw &= sw - 1u;
                    }
                }
            }
            int incl = pc;
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            int64_t pos = s0 + total + (incl - pc);
            total += __shfl(incl, 63, 64);
            for (int j = 0; j < qq; ++j) {
                const int sidx = s_lo + lane * qq + j;
                if (sidx < S) {
                    uint32_t sw = sm[sidx];
                    while (sw) {
                        const int w = (sidx << 5) + __ffs(sw) - 1;
                        uint32_t word = bm[w];
                        while (word) {
                            const int bit = __ffs(word) - 1;
                            raw[pos++] = (static_cast<uint32_t>(w) << 5) | static_cast<uint32_t>(bit);
                            word &= word - 1u;
                        }
                        bm[w] = 0u;
                        sw &= sw - 1u;
                    }
                    sm[sidx] = 0u;
                }
            }
        }
        if (lane == 0) cnt[c] = total;
        wave_lds_sync();
    }
}

// Segments longer than kSegSmall ("giant": hub clusters) are cut into chunks
// of kGiantChunk entries.  pk[c] = gf + (chunks << 32), gf = 1 for a giant
// and chunks its chunk count (0 if not giant): one exclusive scan of pk gives
// a giant's index among the giants in the low half (at most n_next < 2^31, so
// it never carries) and its first chunk in the high half.
__global__ void k_giant_flags(const int64_t* segstart, int64_t n_next, int64_t* pk) {
    GRID_STRIDE(c, n_next + 1) {   // pk[n_next] = 0: the scan leaves the packed total there
        const int64_t len = c < n_next ? segstart[c + 1] - segstart[c] : 0;
        pk[c] = len > kSegSmall ? 1 + (ceil_div(len, kGiantChunk) << 32) : 0;
    }
}
__device__ __forceinline__ int64_t giant_index(int64_t pre) { return pre & 0xFFFFFFFFll; }
__device__ __forceinline__ int64_t first_chunk(int64_t pre) { return pre >> 32; }

constexpr int kGiantThreads = 1024;
constexpr int64_t kGiantBlocks = 1024;        // workgroups of the giant zero / emit launches, at most
constexpr int64_t kGiantChunkBlocks = 4096;   // workgroups of the chunk launch, at most
constexpr int64_t kGiantBoundWords = int64_t(256) << 20;   // bitmap words sized by the bound, at most (1 GiB)

// One workgroup per chunk of a giant segment: the chunk's clusters OR-ed
// into the workgroup's LDS bitmap, then its non-zero words OR-ed into the
// giant's global bitmap (row giant_index(pre[c]) of gbm, W words).  Chunk t
// belongs to the last cluster c whose first chunk is <= t (clusters without
// chunks share their first chunk with the next cluster, so the last one is a
// giant).
// The chunk count is read from the device (pre[n_next], the packed total),
// so the host need not wait for it; the grid is an upper bound.
__global__ __launch_bounds__(kGiantThreads) void k_giant_chunks(const int64_t* segstart, int64_t n_next,
                                                                const int64_t* pre, int W, const uint32_t* raw,
                                                                uint32_t* gbm) {
    extern __shared__ uint32_t seg_bitmaps[];
    __shared__ uint32_t red[2][kGiantThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t chunks = first_chunk(pre[n_next]);
    for (int64_t t = blockIdx.x; t < chunks; t += gridDim.x) {
        int64_t lo = 0, hi = n_next;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (first_chunk(pre[mid]) <= t) lo = mid;
            else hi = mid;
        }
        const int64_t cl = lo;
        const int64_t s0 = segstart[cl] + (t - first_chunk(pre[cl])) * kGiantChunk;
        const int64_t len = min(static_cast<int64_t>(kGiantChunk), segstart[cl + 1] - s0);
        uint32_t kmin = kSegSent, kmax = 0;
        for (int64_t i = threadIdx.x; i < len; i += kGiantThreads) {
            const uint32_t x = raw[s0 + i];
            if (x != kSegSent) {
                kmin = min(kmin, x);
                kmax = max(kmax, x);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            kmin = min(kmin, static_cast<uint32_t>(__shfl_xor(static_cast<int>(kmin), o, 64)));
            kmax = max(kmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(kmax), o, 64)));
        }
        if (lane == 0) {
            red[0][wv] = kmin;
            red[1][wv] = kmax;
        }
        __syncthreads();
        kmin = kSegSent;
        kmax = 0;
        for (int i = 0; i < kGiantThreads / 64; ++i) {
            kmin = min(kmin, red[0][i]);
            kmax = max(kmax, red[1][i]);
        }
        if (kmin <= kmax) {   // block-uniform
            const int w0 = static_cast<int>(kmin >> 5), w1 = static_cast<int>(kmax >> 5);
            for (int w = w0 + static_cast<int>(threadIdx.x); w <= w1; w += kGiantThreads) seg_bitmaps[w] = 0u;
            __syncthreads();
            for (int64_t i = threadIdx.x; i < len; i += kGiantThreads) {
                const uint32_t x = raw[s0 + i];
                if (x != kSegSent) atomicOr(&seg_bitmaps[x >> 5], 1u << (x & 31u));
            }
            __syncthreads();
            uint32_t* g = gbm + giant_index(pre[cl]) * static_cast<int64_t>(W);
            for (int w = w0 + static_cast<int>(threadIdx.x); w <= w1; w += kGiantThreads) {
                const uint32_t word = seg_bitmaps[w];
                if (word) atomicOr(&g[w], word);
            }
        }
        __syncthreads();
    }
}

// Block-wide exclusive prefix of v (blocks of kGiantThreads); *total gets the sum.
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[kGiantThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < kGiantThreads / 64; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// One block per giant (cluster gc[g]): count of its global bitmap (out ==
// nullptr) or its ids written ascending from indices[offs[c]].  The giant
// count is read from the device (*packed, the total of the giant scan).
__global__ __launch_bounds__(kGiantThreads) void k_giant_emit(const int32_t* gc, const int64_t* packed, int W,
                                                              const uint32_t* gbm, int32_t* cnt, const int64_t* offs,
                                                              int32_t* indices) {
    const int64_t G = giant_index(*packed);
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        const int64_t cl = gc[g];
        const uint32_t* bm = gbm + g * static_cast<int64_t>(W);
        int64_t total = 0;
        for (int base = 0; base < W; base += kGiantThreads) {
            const int w = base + static_cast<int>(threadIdx.x);
            uint32_t word = w < W ? bm[w] : 0u;
            int all = 0;
            const int before = block_excl_scan(__popc(word), &all);
            if (indices) {
                int64_t pos = offs[cl] + total + before;
                while (word) {
                    const int bit = __ffs(word) - 1;
                    indices[pos++] = (w << 5) | bit;
                    word &= word - 1u;
                }
            }
            total += all;
        }
        if (!indices && threadIdx.x == 0) cnt[cl] = static_cast<int32_t>(total);
    }
}

// gc[giant index of c] = c for every giant
// Clears the giants' global bitmaps (rows 0 .. G-1 of W words, G read from
// the device).
__global__ void k_giant_zero(const int64_t* packed, int W, uint32_t* gbm) {
    const int64_t G = giant_index(*packed);
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x)
        for (int w = threadIdx.x; w < W; w += blockDim.x) gbm[g * W + w] = 0u;
}

__global__ void k_giant_list(const int64_t* segstart, const int64_t* pre, int64_t n_next, int32_t* gc) {
    GRID_STRIDE(c, n_next) {
        if (segstart[c + 1] - segstart[c] > kSegSmall) gc[giant_index(pre[c])] = static_cast<int32_t>(c);
    }
}

__global__ void k_iota_u32(uint32_t* a, int64_t n) {
    GRID_STRIDE(i, n) a[i] = static_cast<uint32_t>(i);
}

template <class Off>
__global__ void k_seg_offsets(const int64_t* offs, int64_t n_next, int64_t nnz_next, Off* offsets) {
    GRID_STRIDE(c, n_next + 1) offsets[c] = static_cast<Off>(c < n_next ? offs[c] : nnz_next);
}

// small segments: their distinct clusters (already in place, ascending) copied out; one wave per cluster
__global__ void k_small_out(const int64_t* segstart, int64_t n_next, const int32_t* cnt, const int64_t* offs,
                            const uint32_t* raw, int32_t* indices) {
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x >> 6;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6); c < n_next;
         c += static_cast<int64_t>(gridDim.x) * wpb) {
        const int64_t s0 = segstart[c];
        if (segstart[c + 1] - s0 > kSegSmall) continue;
        const int64_t o = offs[c], k = cnt[c];
        for (int64_t i = lane; i < k; i += 64) indices[o + i] = static_cast<int32_t>(raw[s0 + i]);
    }
}

// ---------------------------------------------------------------- validation
// Offsets must start at 0, end at nnz and never decrease before any kernel
// may read a row.
template <class Off>
__global__ void k_check_offsets(const Off* off, int64_t n, int64_t nnz, unsigned int* bad) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && (static_cast<int64_t>(off[0]) != 0 || static_cast<int64_t>(off[n]) != nnz))
        atomicOr(bad, 1u);
    GRID_STRIDE(v, n) {
        const int64_t b = off[v], e = off[v + 1];
        if (e < b || b < 0 || e > nnz) atomicOr(bad, 1u);
    }
}

// Entry checks once the rows are known to lie inside [0, nnz).
template <class Off>
__global__ void k_check_entries(const Off* off, const int32_t* src, const int32_t* idx, int64_t nnz, int64_t n,
                                unsigned int* bad) {
    unsigned int f = 0;
    GRID_STRIDE(p, nnz) {
        const int32_t v = src[p], u = idx[p];
        if (u < 0 || u >= n) f |= 2u;
        if (u == v) f |= 4u;
        if (p > static_cast<int64_t>(off[v]) && idx[p - 1] >= u) f |= 8u;
    }
    if (f) atomicOr(bad, f);
}

// (v,u) stored => (u,v) stored, by binary search in row u (rows sorted).
template <class Off>
__global__ void k_check_symmetry(const Off* off, const int32_t* src, const int32_t* idx, int64_t nnz,
                                 unsigned int* bad) {
    unsigned int f = 0;
    GRID_STRIDE(p, nnz) {
        const int32_t v = src[p], u = idx[p];
        int64_t lo = off[u], hi = off[u + 1];
        bool found = false;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const int32_t w = idx[mid];
            if (w == v) {
                found = true;
                break;
            }
            if (w < v) lo = mid + 1;
            else hi = mid;
        }
        if (!found) f |= 16u;
    }
    if (f) atomicOr(bad, f);
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

// One device value read back through a pinned slot of the context (one wait).
uint64_t read_u64(Ctx* c, const unsigned long long* p) {
    unsigned long long* h = reinterpret_cast<unsigned long long*>(c->pinned + 2);
    GOSH_HIP(hipMemcpyAsync(h, p, sizeof(*h), hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
    return *h;
}

template <class K>
int64_t build_coarse(Ctx* c, const int32_t* src, const int32_t* idx, int64_t nnz, const int32_t* map,
                     int64_t n_next, bool off64, void** off_out, int32_t** idx_out) {
    const int bb = std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(n_next - 1, 0))));
    // every entry gets a key; entries inside a cluster get the sentinel, which
    // the sort moves behind all others and the unique pass drops
    const K sent = 2 * bb >= static_cast<int>(8 * sizeof(K)) ? ~K(0) : (K(1) << (2 * bb)) - K(1);
    const int64_t m = nnz;
    DevBuf<K> keys(c, std::max<int64_t>(m, 1)), tmp(c, std::max<int64_t>(m, 1));
    DevBuf<int32_t> flag(c, std::max<int64_t>(m, 1));
    DevBuf<int64_t> pos(c, std::max<int64_t>(m, 1));
    int64_t nnz_next = 0;
    if (m > 0) {
        hipLaunchKernelGGL((k_write_pairs<K>), grid_for(nnz), dim3(kThreads), 0, c->stream, src, idx, nnz, map, bb,
                           sent, keys.p);
        GOSH_HIP(hipGetLastError());
        if constexpr (sizeof(K) == 4)
            radix_sort_u32(c, reinterpret_cast<uint32_t*>(keys.p), reinterpret_cast<uint32_t*>(tmp.p),
                           nullptr, nullptr, m, 2 * bb);
        else
            radix_sort_u64(c, reinterpret_cast<uint64_t*>(keys.p), reinterpret_cast<uint64_t*>(tmp.p), m,
                           2 * bb);
        hipLaunchKernelGGL((k_flag_unique<K>), grid_for(m), dim3(kThreads), 0, c->stream, keys.p, m, sent,
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

// Coarse CSR by cluster segments (see k_dedup_small, k_giant_chunks).  src:
// row of every entry.  Returns nnz' and sets *off_out / *idx_out, or returns
// -1 (nothing allocated) when the next level is too large for the LDS
// bitmaps; the caller then builds the level with build_coarse.
template <class Off>
int64_t build_coarse_seg(Ctx* c, const Off* off, const int32_t* src, const int32_t* idx, int64_t n, int64_t nnz,
                         const int32_t* map, int64_t n_next, bool off64, void** off_out, int32_t** idx_out) {
    const int bb = std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(n_next - 1, 0))));   // sort bits of a cluster id
    const int64_t W = ceil_div(std::max<int64_t>(n_next, 1), 32);   // bitmap words per wave and per giant
    if (W > kSegMaxWords) return -1;
    // members grouped by cluster, in id order within a cluster
    DevBuf<uint32_t> ckey(c, n), ckey_tmp(c, n), mem(c, n), mem_tmp(c, n);
    GOSH_HIP(hipMemcpyAsync(ckey.p, map, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_iota_u32, grid_for(n), dim3(kThreads), 0, c->stream, mem.p, n);
    GOSH_HIP(hipGetLastError());
    bool in_tmp = false;   // sorted into the _tmp buffers: swap instead of copying back
    radix_sort_u32(c, ckey.p, ckey_tmp.p, mem.p, mem_tmp.p, n, bb, &in_tmp);
    if (in_tmp) {
        std::swap(ckey, ckey_tmp);
        std::swap(mem, mem_tmp);
    }
    ckey_tmp.reset();
    mem_tmp.reset();
    DevBuf<int64_t> E(c, n);
    {
        DevBuf<int32_t> mdeg(c, n);
        hipLaunchKernelGGL((k_member_deg<Off>), grid_for(n), dim3(kThreads), 0, c->stream, off, mem.p, n, mdeg.p);
        GOSH_HIP(hipGetLastError());
        scan_i32_to_i64(c, mdeg.p, E.p, n, nullptr);
    }
    DevBuf<int64_t> segstart(c, n_next + 1);
    hipLaunchKernelGGL(k_seg_starts, grid_for(n_next + 1), dim3(kThreads), 0, c->stream, ckey.p, n, n_next, E.p, nnz,
                       segstart.p);
    GOSH_HIP(hipGetLastError());
    DevBuf<uint32_t> raw(c, std::max<int64_t>(nnz, 1));
    {
        DevBuf<int64_t> dbase(c, n);
        hipLaunchKernelGGL((k_dest_base<Off>), grid_for(n), dim3(kThreads), 0, c->stream, off, mem.p, E.p, n,
                           dbase.p);
        GOSH_HIP(hipGetLastError());
        if (nnz > 0) {
            hipLaunchKernelGGL(k_gather_raw, grid_for(nnz), dim3(kThreads), 0, c->stream, src, idx, nnz, dbase.p,
                               map, raw.p);
            GOSH_HIP(hipGetLastError());
        }
    }
    E.reset();
    mem.reset();
    ckey.reset();

    // giant segments: their count and chunks from one packed scan, whose
    // total stays on the device (pre[n_next]); the host sizes the giant
    // buffers and grids by upper bounds (a giant has more than kSegSmall
    // entries) instead of waiting for it, unless the bounds' bitmaps would
    // be too large, when it reads the total back
    DevBuf<int64_t> pre(c, n_next + 1);
    hipLaunchKernelGGL(k_giant_flags, grid_for(n_next + 1), dim3(kThreads), 0, c->stream, segstart.p, n_next, pre.p);
    GOSH_HIP(hipGetLastError());
    int64_t G = std::min<int64_t>(n_next, nnz / (kSegSmall + 1));
    int64_t chunks = nnz / kGiantChunk + G;
    if (G * W > kGiantBoundWords) {
        int64_t packed = 0;
        scan_i64(c, pre.p, pre.p, n_next + 1, false, ScanOp::Sum, &packed);
        G = packed & 0xFFFFFFFFll;
        chunks = packed >> 32;
    } else {
        scan_i64(c, pre.p, pre.p, n_next + 1, false, ScanOp::Sum, nullptr);
    }
    const int64_t* packed_dev = pre.p + n_next;

    DevBuf<int32_t> cnt(c, n_next);
    // as many workgroups as fit on the device at once: each wave clears its
    // bitmap once and then takes segment after segment
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>(W + ceil_div(W, 32)) * kSegWaves;
    // launch facts are queried once per context (each query is a host call
    // on the critical path right after the level's count was read back)
    if (!c->seg_lds_set) {
        const size_t lds_max = sizeof(uint32_t) * static_cast<size_t>(kSegMaxWords + kSegMaxWords / 32) * kSegWaves;
        GOSH_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dedup_small),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_max)));
        GOSH_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_giant_chunks),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(sizeof(uint32_t) * kSegMaxWords)));
        GOSH_HIP(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
        c->seg_lds_set = true;
    }
    int& per_cu = c->dedup_per_cu[lds];
    if (per_cu == 0)
        GOSH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_dedup_small),
                                                              64 * kSegWaves, lds));
    const int cus = c->cus;
    const int64_t dblocks = std::min<int64_t>(ceil_div(n_next, kSegWaves),
                                              static_cast<int64_t>(std::max(per_cu, 1)) * std::max(cus, 1));
    hipLaunchKernelGGL(k_dedup_small, dim3(static_cast<unsigned>(std::max<int64_t>(dblocks, 1))),
                       dim3(64 * kSegWaves), lds, c->stream, segstart.p, n_next, static_cast<int>(W), raw.p, cnt.p);
    GOSH_HIP(hipGetLastError());
    // G and chunks: the exact counts or upper bounds (the kernels read the
    // exact ones from packed_dev)
    DevBuf<int32_t> gc(c, std::max<int64_t>(G, 1));
    DevBuf<uint32_t> gbm(c, std::max<int64_t>(G * W, 1));
    const unsigned gblocks = static_cast<unsigned>(std::min<int64_t>(G, kGiantBlocks));
    if (G > 0) {
        hipLaunchKernelGGL(k_giant_zero, dim3(gblocks), dim3(kThreads), 0, c->stream, packed_dev,
                           static_cast<int>(W), gbm.p);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_giant_list, grid_for(n_next), dim3(kThreads), 0, c->stream, segstart.p, pre.p, n_next,
                           gc.p);
        GOSH_HIP(hipGetLastError());
        const size_t glds = sizeof(uint32_t) * static_cast<size_t>(W);
        hipLaunchKernelGGL(k_giant_chunks, dim3(static_cast<unsigned>(std::min<int64_t>(chunks, kGiantChunkBlocks))),
                           dim3(kGiantThreads), glds, c->stream, segstart.p, n_next, pre.p, static_cast<int>(W),
                           raw.p, gbm.p);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_giant_emit, dim3(gblocks), dim3(kGiantThreads), 0, c->stream, gc.p, packed_dev,
                           static_cast<int>(W), gbm.p, cnt.p, nullptr, nullptr);
        GOSH_HIP(hipGetLastError());
    }

    // offsets from the distinct counts, then the rows
    DevBuf<int64_t> offs(c, n_next);
    int64_t nnz_next = 0;
    scan_i32_to_i64(c, cnt.p, offs.p, n_next, &nnz_next);
    int32_t* indices = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * std::max<int64_t>(nnz_next, 1)));
    void* offsets = c->alloc((off64 ? 8 : 4) * (n_next + 1));
    if (off64)
        hipLaunchKernelGGL((k_seg_offsets<int64_t>), grid_for(n_next + 1), dim3(kThreads), 0, c->stream, offs.p,
                           n_next, nnz_next, static_cast<int64_t*>(offsets));
    else
        hipLaunchKernelGGL((k_seg_offsets<int32_t>), grid_for(n_next + 1), dim3(kThreads), 0, c->stream, offs.p,
                           n_next, nnz_next, static_cast<int32_t*>(offsets));
    GOSH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_small_out, grid_for(n_next, kThreads / 64), dim3(kThreads), 0, c->stream, segstart.p,
                       n_next, cnt.p, offs.p, raw.p, indices);
    GOSH_HIP(hipGetLastError());
    if (G > 0) {
        hipLaunchKernelGGL(k_giant_emit, dim3(gblocks), dim3(kGiantThreads), 0, c->stream, gc.p, packed_dev,
                           static_cast<int>(W), gbm.p, cnt.p, offs.p, indices);
        GOSH_HIP(hipGetLastError());
    }
    *off_out = offsets;
    *idx_out = indices;
    return nnz_next;
}

// Row of every entry (one wave per vertex streams its row).
template <class Off>
DevBuf<int32_t> expand_rows(Ctx* c, const Off* off, int64_t n, int64_t nnz) {
    DevBuf<int32_t> src(c, std::max<int64_t>(nnz, 1));
    if (nnz > 0 && n > 0) {
        hipLaunchKernelGGL((k_expand_rows<Off>), grid_for(n, kThreads / 64), dim3(kThreads), 0, c->stream, off, n,
                           src.p);
        GOSH_HIP(hipGetLastError());
    }
    return src;
}

unsigned int read_flags(Ctx* c, unsigned int* bad) {
    unsigned int* h = reinterpret_cast<unsigned int*>(c->pinned + 3);
    GOSH_HIP(hipMemcpyAsync(h, bad, 4, hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
    return *h;
}

// Structure checks of a caller's CSR; returns the row of every entry.
template <class Off>
DevBuf<int32_t> validate_structure(Ctx* c, const Off* off, const int32_t* idx, int64_t n, int64_t nnz,
                                   bool symmetry) {
    unsigned int* bad = reinterpret_cast<unsigned int*>(scratch_u64(c, 3));
    GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    hipLaunchKernelGGL((k_check_offsets<Off>), grid_for(n), dim3(kThreads), 0, c->stream, off, n, nnz, bad);
    GOSH_HIP(hipGetLastError());
    GOSH_REQUIRE(read_flags(c, bad) == 0, GOSH_E_BAD_GRAPH,
                 "offsets must start at 0, end at nnz and never decrease");
    DevBuf<int32_t> src = expand_rows(c, off, n, nnz);
    if (nnz > 0) {
        hipLaunchKernelGGL((k_check_entries<Off>), grid_for(nnz), dim3(kThreads), 0, c->stream, off, src.p, idx,
                           nnz, n, bad);
        GOSH_HIP(hipGetLastError());
        const unsigned int h = read_flags(c, bad);
        GOSH_REQUIRE(!(h & 2u), GOSH_E_BAD_GRAPH, "neighbour index out of range");
        GOSH_REQUIRE(!(h & 4u), GOSH_E_BAD_GRAPH, "self-loop");
        GOSH_REQUIRE(!(h & 8u), GOSH_E_BAD_GRAPH, "row not strictly ascending (unsorted or duplicate)");
        if (symmetry) {
            hipLaunchKernelGGL((k_check_symmetry<Off>), grid_for(nnz), dim3(kThreads), 0, c->stream, off, src.p,
                               idx, nnz, bad);
            GOSH_HIP(hipGetLastError());
            GOSH_REQUIRE(!(read_flags(c, bad) & 16u), GOSH_E_BAD_GRAPH, "graph is not symmetric");
        }
    }
    return src;
}

// Exact mapping: each vertex's eligible earlier neighbours, synchronous hub
// selection rounds, then the assignment.  Returns the cluster count.
template <class Off>
int64_t map_exact(Ctx* c, Level& L, const Off* off, const int32_t* idx, const int32_t* src, const uint32_t* perm,
                  const int32_t* rank_p, const uint8_t* light_p, bool dense, unsigned int* bad) {
    const int64_t n = L.n, nnz = L.nnz;
    DevBuf<int32_t> lower(c, std::max<int64_t>(nnz, 1));
    DevBuf<int64_t> lstart(c, n + 1);
    DevBuf<uint8_t> state(c, n);   // hub-round states, all undecided to start
    if (nnz > 0) {
        const int64_t tiles = ceil_div(nnz, kLowerTile);
        const int64_t words = ceil_div(nnz, int64_t(64));
        DevBuf<unsigned long long> bits(c, words);
        DevBuf<uint16_t> wpre(c, words);
        DevBuf<int64_t> tile(c, tiles + 1);
        DevBuf<uint32_t> rl(c, n);
        hipLaunchKernelGGL(k_pack_rank_light, grid_for(n), dim3(kThreads), 0, c->stream, rank_p, light_p, n, rl.p,
                           state.p);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lower_bits, dim3(static_cast<unsigned>(tiles)), dim3(kThreads), 0, c->stream, src, idx,
                           nnz, rl.p, bits.p, wpre.p, tile.p);
        GOSH_HIP(hipGetLastError());
        scan_i64(c, tile.p, tile.p, tiles + 1, false, ScanOp::Sum, nullptr);
        hipLaunchKernelGGL(k_lower_write, grid_for(nnz), dim3(kThreads), 0, c->stream, idx, nnz, bits.p, wpre.p,
                           tile.p, lower.p);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_lower_starts<Off>), grid_for(n + 1), dim3(kThreads), 0, c->stream, off, n, nnz, bits.p,
                           wpre.p, tile.p, tiles, lstart.p);
        GOSH_HIP(hipGetLastError());
    } else {
        fill(c, lstart.p, n + 1, 0);
        fill(c, state.p, n, 0);
    }

    // hub selection rounds; each round decides at least the earliest
    // undecided vertex, so the loop ends; dense levels (average degree >= 64)
    // scan each segment with a whole wave.  Three rounds per host check (a
    // round over decided vertices changes nothing, and the R-MAT levels take
    // 2-4); round g sets flag g mod 2 and clears the other for round g + 1,
    // so only the first flag needs a fill, and the flag read back is the
    // last round's.
    unsigned long long* flag[2] = {scratch_u64(c, 1), scratch_u64(c, 5)};
    GOSH_HIP(hipMemsetAsync(flag[0], 0, 8, c->stream));
    constexpr int kRoundsPerCheck = 3;
    for (int64_t round = 0;; round += kRoundsPerCheck) {
        GOSH_REQUIRE(round <= n + kRoundsPerCheck, GOSH_E_DEVICE, "coarsening rounds did not converge");
        for (int r = 0; r < kRoundsPerCheck; ++r) {
            const int g = static_cast<int>((round + r) & 1);
            if (dense)
                hipLaunchKernelGGL(k_round_group<64>, grid_for(n, kThreads / 64), dim3(kThreads), 0, c->stream, n,
                                   lstart.p, lower.p, state.p, flag[g], flag[g ^ 1]);
            else
                hipLaunchKernelGGL(k_round_group<kSparseGroup>, grid_for(n, kThreads / kSparseGroup), dim3(kThreads),
                                   0, c->stream, n, lstart.p, lower.p, state.p, flag[g], flag[g ^ 1]);
            GOSH_HIP(hipGetLastError());
        }
        if (read_u64(c, flag[(round + kRoundsPerCheck - 1) & 1]) == 0) break;
    }

    // cluster ids: hubs counted in pi order
    DevBuf<int32_t> hf(c, n);
    DevBuf<int64_t> cid(c, n);
    hipLaunchKernelGGL(k_hub_flags_by_rank, grid_for(n), dim3(kThreads), 0, c->stream, perm, n, state.p,
                       hf.p);
    GOSH_HIP(hipGetLastError());
    int64_t n_next = 0;
    scan_i32_to_i64(c, hf.p, cid.p, n, &n_next);
    hf.reset();
    L.map = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * n));
    if (dense)
        hipLaunchKernelGGL(k_assign_group<64>, grid_for(n, kThreads / 64), dim3(kThreads), 0, c->stream, n, lstart.p,
                           lower.p, state.p, rank_p, cid.p, L.map, bad);
    else
        hipLaunchKernelGGL(k_assign_group<kSparseGroup>, grid_for(n, kThreads / kSparseGroup), dim3(kThreads), 0,
                           c->stream, n, lstart.p, lower.p, state.p, rank_p, cid.p, L.map, bad);
    GOSH_HIP(hipGetLastError());
    return n_next;
}

// Lock-and-skip mapping (k_claim), in launches of c->claim_batch ranks (one
// wave over all ranks in deterministic mode).  Returns the cluster count.
template <class Off>
int64_t map_lock_skip(Ctx* c, Level& L, const Off* off, const int32_t* idx, const uint32_t* perm,
                      const int32_t* rank_p, const uint8_t* light_p, unsigned int* bad) {
    const int64_t n = L.n;
    DevBuf<int32_t> owner(c, n);
    fill(c, owner.p, n, 0xFF);
    if (c->deterministic) {
        hipLaunchKernelGGL((k_claim<Off>), dim3(1), dim3(64), 0, c->stream, off, idx, perm, int64_t{0}, n, light_p,
                           owner.p);
        GOSH_HIP(hipGetLastError());
    } else {
        const int64_t batch = c->claim_batch > 0 ? c->claim_batch : std::max<int64_t>(64, ceil_div(n, 64));
        for (int64_t r0 = 0; r0 < n; r0 += batch) {
            const int64_t r1 = std::min(n, r0 + batch);
            hipLaunchKernelGGL((k_claim<Off>), grid_for(r1 - r0, kThreads / 64), dim3(kThreads), 0, c->stream, off,
                               idx, perm, r0, r1, light_p, owner.p);
            GOSH_HIP(hipGetLastError());
        }
    }
    DevBuf<int32_t> hf(c, n);
    DevBuf<int64_t> cid(c, n);
    hipLaunchKernelGGL(k_owner_hub_flags, grid_for(n), dim3(kThreads), 0, c->stream, perm, n, owner.p, hf.p);
    GOSH_HIP(hipGetLastError());
    int64_t n_next = 0;
    scan_i32_to_i64(c, hf.p, cid.p, n, &n_next);
    hf.reset();
    L.map = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * n));
    hipLaunchKernelGGL(k_owner_assign, grid_for(n), dim3(kThreads), 0, c->stream, n, owner.p, rank_p, cid.p, L.map,
                       bad);
    GOSH_HIP(hipGetLastError());
    return n_next;
}

template <class Off>
void coarsen_one(Ctx* c, Level& L, Level& next, DevBuf<int32_t>* src_in) {
    const int64_t n = L.n, nnz = L.nnz;
    const Off* off = static_cast<const Off*>(L.offsets);
    const int32_t* idx = L.indices;

    // degrees, eligibility (hub^2 restriction) and the processing order pi:
    // a stable radix sort of the vertices on maxdeg - deg keeps ties in id order
    DevBuf<uint8_t> light(c, n);
    DevBuf<int64_t> deg(c, n);
    GOSH_HIP(hipMemsetAsync(scratch_u64(c, 0), 0, 8, c->stream));
    hipLaunchKernelGGL((k_degree<Off>), grid_reduce(n), dim3(kThreads), 0, c->stream, off, n, nnz,
                       light.p, deg.p, scratch_u64(c, 0), nullptr);
    GOSH_HIP(hipGetLastError());
    DevBuf<uint32_t> key(c, n), key_tmp(c, n), perm(c, n), perm_tmp(c, n);
    hipLaunchKernelGGL(k_sort_keys, grid_for(n), dim3(kThreads), 0, c->stream, deg.p, n,
                       reinterpret_cast<const unsigned long long*>(scratch_u64(c, 0)), key.p, perm.p);
    GOSH_HIP(hipGetLastError());
    // deg <= nnz/1 < 2^bits_for(max(n-1, nnz)) bounds maxdeg - deg
    bool in_tmp = false;   // sorted into the _tmp buffers: swap instead of copying back
    radix_sort_u32(c, key.p, key_tmp.p, perm.p, perm_tmp.p, n,
                   bits_for(static_cast<uint64_t>(std::min<int64_t>(std::max<int64_t>(n - 1, 0), nnz))), &in_tmp);
    if (in_tmp) std::swap(perm, perm_tmp);
    key_tmp.reset();
    perm_tmp.reset();
    key.reset();
    deg.reset();
    DevBuf<int32_t> rank(c, n);
    hipLaunchKernelGGL(k_rank_from_perm, grid_for(n), dim3(kThreads), 0, c->stream, perm.p, n, rank.p);
    GOSH_HIP(hipGetLastError());

    // row of every entry (for the coarse graph)
    DevBuf<int32_t> src_own;
    if (!src_in) src_own = expand_rows(c, off, n, nnz);
    const int32_t* src = src_in ? src_in->p : src_own.p;
    const bool dense = nnz >= 64 * n;
    unsigned int* bad = reinterpret_cast<unsigned int*>(scratch_u64(c, 4));
    GOSH_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
    int64_t n_next = 0;
    if (c->coarsen_mode == GOSH_COARSEN_LOCK_SKIP)
        n_next = map_lock_skip(c, L, off, idx, perm.p, rank.p, light.p, bad);
    else
        n_next = map_exact(c, L, off, idx, src, perm.p, rank.p, light.p, dense, bad);
    light.reset();
    rank.reset();
    perm.reset();

    // the assignment flag is copied now and read after the coarse build,
    // which waits for the stream when it reads its entry count back
    unsigned int* bad_h = reinterpret_cast<unsigned int*>(c->pinned + 4);
    *bad_h = 0xFFFFFFFFu;
    GOSH_HIP(hipMemcpyAsync(bad_h, bad, 4, hipMemcpyDeviceToHost, c->stream));

    // coarse graph: distinct pairs (map v, map u), map v != map u, rows
    // ascending; by cluster segments, or by one sort of all pair keys
    void* noff = nullptr;
    int32_t* nidx = nullptr;
    int64_t nnz_next = -1;
    if (c->coarse_build == 0 && n > 0 && nnz < (int64_t(1) << 31))
        nnz_next = build_coarse_seg<Off>(c, off, src, idx, n, nnz, L.map, n_next, L.off64, &noff, &nidx);
    if (nnz_next < 0) {
        if (2 * std::max(1, bits_for(static_cast<uint64_t>(std::max<int64_t>(n_next - 1, 0)))) <= 32)
            nnz_next = build_coarse<uint32_t>(c, src, idx, nnz, L.map, n_next, L.off64, &noff, &nidx);
        else
            nnz_next = build_coarse<uint64_t>(c, src, idx, nnz, L.map, n_next, L.off64, &noff, &nidx);
    }
    GOSH_REQUIRE(*bad_h != 0xFFFFFFFFu, GOSH_E_DEVICE, "coarse build returned before waiting for the stream");
    GOSH_REQUIRE(*bad_h == 0, GOSH_E_BAD_GRAPH, "coarsening left a vertex without a cluster (graph not symmetric?)");
    next.n = n_next;
    next.nnz = nnz_next;
    next.off64 = L.off64;
    next.offsets = next.own_offsets = noff;
    next.indices = next.own_indices = nidx;
    next.n_deg0 = -1;
}

}  // namespace

int64_t count_isolated(Ctx* c, const Level& L) {
    if (L.n_deg0 >= 0) return L.n_deg0;
    int64_t cnt = 0;
    if (L.n > 0) {
        GOSH_HIP(hipMemsetAsync(scratch_u64(c, 2), 0, 8, c->stream));
        if (L.off64)
            hipLaunchKernelGGL((k_degree<int64_t>), grid_reduce(L.n), dim3(kThreads), 0, c->stream,
                               static_cast<const int64_t*>(L.offsets), L.n, L.nnz, nullptr, nullptr, nullptr,
                               scratch_u64(c, 2));
        else
            hipLaunchKernelGGL((k_degree<int32_t>), grid_reduce(L.n), dim3(kThreads), 0, c->stream,
                               static_cast<const int32_t*>(L.offsets), L.n, L.nnz, nullptr, nullptr, nullptr,
                               scratch_u64(c, 2));
        GOSH_HIP(hipGetLastError());
        cnt = static_cast<int64_t>(read_u64(c, scratch_u64(c, 2)));
    }
    const_cast<Level&>(L).n_deg0 = cnt;
    return cnt;
}

const int32_t* cluster_sizes(Ctx* c, const Level& L, int64_t n_next) {
    if (!L.clsz && L.map) {
        Level& M = const_cast<Level&>(L);
        M.clsz = static_cast<int32_t*>(c->alloc(sizeof(int32_t) * std::max<int64_t>(n_next, 1)));
        fill(c, M.clsz, n_next, 0);
        if (L.n > 0) {
            hipLaunchKernelGGL(k_cluster_sizes, grid_for(L.n), dim3(kThreads), 0, c->stream, L.map, L.n, M.clsz);
            GOSH_HIP(hipGetLastError());
        }
    }
    return L.clsz;
}

void validate_csr(Ctx* c, const gosh_csr* g, bool symmetry) {
    GOSH_REQUIRE(g && g->n >= 0 && g->nnz >= 0, GOSH_E_INVALID_ARG, "bad csr shape");
    if (g->n == 0) {
        GOSH_REQUIRE(g->nnz == 0, GOSH_E_BAD_GRAPH, "an empty graph has no entries");
        return;
    }
    if (g->offsets_is_i64)
        validate_structure(c, static_cast<const int64_t*>(g->offsets), g->indices, g->n, g->nnz, symmetry);
    else
        validate_structure(c, static_cast<const int32_t*>(g->offsets), g->indices, g->n, g->nnz, symmetry);
}

void coarsen(Ctx* c, const gosh_csr* g0, int64_t threshold, double ratio, gosh_levels* out) {
    Level L0;
    L0.n = g0->n;
    L0.nnz = g0->nnz;
    L0.off64 = g0->offsets_is_i64 != 0;
    L0.offsets = g0->offsets;
    L0.indices = g0->indices;
    L0.n_deg0 = -1;
    out->lv.push_back(L0);
    if (L0.n == 0) {
        GOSH_REQUIRE(L0.nnz == 0, GOSH_E_BAD_GRAPH, "an empty graph has no entries");
        return;
    }
    // the caller's graph is checked before any kernel relies on it; the
    // row expansion made for the check is reused by the first level
    DevBuf<int32_t> src0 = L0.off64
        ? validate_structure(c, static_cast<const int64_t*>(L0.offsets), L0.indices, L0.n, L0.nnz, false)
        : validate_structure(c, static_cast<const int32_t*>(L0.offsets), L0.indices, L0.n, L0.nnz, false);
    constexpr int kMaxLevels = 128;
    while (static_cast<int>(out->lv.size()) < kMaxLevels) {
        Level next;
        Level& cur = out->lv.back();
        DevBuf<int32_t>* src = out->lv.size() == 1 ? &src0 : nullptr;
        if (cur.off64) coarsen_one<int64_t>(c, cur, next, src);
        else coarsen_one<int32_t>(c, cur, next, src);
        if (src) src0.reset();
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
    if (L.hub_bits) c->free(L.hub_bits);
    L.own_offsets = nullptr;
    L.own_indices = nullptr;
    L.map = nullptr;
    L.clsz = nullptr;
    L.hub_bits = nullptr;
}

}  // namespace gosh
