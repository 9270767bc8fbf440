// Embedding a level whose graph and matrix do not fit in device memory
// (Section 5): the vertex ids are split into K contiguous parts, the matrix
// and the graph stay in host memory, and rounds of kernels K_{i,j} run over
// the part pairs in inside-out order with at most P_GPU parts ("submatrix
// bins") and S_GPU sample pools resident at a time.
//
// * Host sampler threads build the pool S_{i,j} of a round: for every vertex
//   u of part i with c > 0 neighbours in part j, B positives drawn uniformly
//   among those neighbours (and, for i != j, the same for part j towards
//   part i).  The b-th positive of u in round r uses the Philox stream of
//   "epoch" r*B + b with the opposite part in the slot field, so that one
//   part and one sample per round is exactly Algorithm 3.
// * The device kernel K_{i,j} visits every pool entry like TrainInGPU: the
//   positive from the pool, k negatives drawn on the device uniformly from
//   the opposite part, UpdateEmbed on each (rows of two resident parts).
// * Rounds: ceil(e / B); lr' = lr * max(1 - r/rounds, 1e-4) in round r; the
//   positive visits stop after e * |V| (later pool entries are cut).
// * Execution is a dependency graph on HIP streams and events: one stream
//   per part bin (swap out, swap in), one per pool bin (host-to-device pool
//   copy) and two for the kernels, which may overlap; a kernel waits for
//   the events of its parts and its pool, a swap waits for the kernels that
//   used the bin, a pool copy waits for the kernel that used the pool bin.
//   A producer thread fills pinned host pool buffers ahead of the copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "device_util.hpp"
#include "gosh_internal.hpp"
#include "visit.hpp"

namespace gosh {
namespace part_detail {

using namespace train_detail;

constexpr uint32_t kPosBits = 27;                     // pool entry: pos_local | b << 27
constexpr uint32_t kPosMask = (1u << kPosBits) - 1u;
constexpr int64_t kMaxPartRows = int64_t(1) << kPosBits;
constexpr int kMaxB = 31;

// ------------------------------------------------------------ device
struct PairArgs {
    void* bin_a;               // rows of part a (source part of side 0)
    void* bin_b;               // rows of part b
    int64_t start_a, start_b, size_a, size_b;
    uint32_t part_a, part_b;
    const uint2* pool;         // entries: (source local id, positive local id | b << 27)
    int64_t n0, n1;            // entries on the device: side 0 (sources in a), side 1 (sources in b)
    int64_t f0, f1;            // entries of each side before the positive cap cut the pool
    int B;
    float lr;
    int k;
    uint32_t key0, key1, w2;
    uint32_t eps0;             // round * B
    unsigned long long* updates;
};

template <bool BF16, int D, int KMAX>
__device__ __forceinline__ void pair_visit(const PairArgs& P, int64_t e, int gl) {
    using Elem = typename RowIO<BF16>::Elem;
    const int k = P.k;
    const bool side1 = e >= P.n0;
    Elem* Ms = static_cast<Elem*>(side1 ? P.bin_b : P.bin_a);
    Elem* Mo = static_cast<Elem*>(side1 ? P.bin_a : P.bin_b);
    const int64_t start_s = side1 ? P.start_b : P.start_a;
    const int64_t start_o = side1 ? P.start_a : P.start_b;
    const int64_t size_o = side1 ? P.size_a : P.size_b;
    const uint32_t opp = side1 ? P.part_a : P.part_b;
    const uint2 ent = P.pool[e];
    const int64_t src = ent.x;                       // local in Ms
    const int64_t src_g = start_s + src;
    const uint32_t eps = P.eps0 + (ent.y >> kPosBits);

    int32_t u[KMAX + 1];
    u[0] = static_cast<int32_t>(ent.y & kPosMask);   // local in Mo
    {
        constexpr int NB = (KMAX + 1 + 3) / 4;
        uint32_t wd[4 * NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (4 * b <= k) {
                const uint4 r = philox10(make_uint4(static_cast<uint32_t>(src_g), eps, P.w2, stream_word3(0, opp, b)),
                                         P.key0, P.key1);
                wd[4 * b] = r.x; wd[4 * b + 1] = r.y; wd[4 * b + 2] = r.z; wd[4 * b + 3] = r.w;
            } else {
                wd[4 * b] = wd[4 * b + 1] = wd[4 * b + 2] = wd[4 * b + 3] = 0;
            }
        }
#pragma unroll
        for (int t = 1; t <= KMAX; ++t) u[t] = (t <= k) ? static_cast<int32_t>(scale_u32(wd[t], size_o)) : -1;
    }
    // a sample that is the source itself (only possible when both parts
    // coincide) is skipped
    const int64_t self = (src_g >= start_o && src_g < start_o + size_o) ? src_g - start_o : -1;
    update_chain<BF16, D, KMAX, false>(Ms, src, Mo, self, u, k, P.lr, static_cast<uint32_t>(src_g), eps, P.w2, 1u,
                                       opp, P.key0, P.key1, P.updates, gl);
}

// Launch shapes: one wave walks the entries in pool order (deterministic
// mode), one slot per lane group when one launch covers the pool, else a
// grid-stride loop (a pool may hold more entries than one launch has lanes).
// The loop is its own instantiation: inside a loop the visit holds more
// registers (100 against 84 VGPRs, 5 instead of 6 waves per SIMD).
enum PairShape { kPairSeq = 0, kPairOnce = 1, kPairStride = 2 };
constexpr int64_t kPairMaxBlocks = int64_t(1) << 20;

// A vertex owns B consecutive entries of its side; visiting b-major (slot
// i -> vertex i mod m, sample i div m) keeps the B visits of one source apart
// instead of in the same wave, where their atomic commits to the one source
// row would serialize.
template <bool BF16, int D, int KMAX>
__device__ __forceinline__ void pair_slot(const PairArgs& P, int64_t slot, int gl) {
    int64_t i = slot;
    const bool s1 = i >= P.f0;
    if (s1) i -= P.f0;
    const int64_t full = s1 ? P.f1 : P.f0;
    const int64_t m = full / P.B;
    const int64_t e = (i % m) * P.B + i / m;
    if (e < (s1 ? P.n1 : P.n0)) pair_visit<BF16, D, KMAX>(P, s1 ? P.n0 + e : e, gl);
}

template <bool BF16, int D, int KMAX, int SHAPE>
__global__ __launch_bounds__(kBlock) void k_pair(PairArgs P) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const int64_t total = P.n0 + P.n1;
    if (P.updates && blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(P.updates, static_cast<unsigned long long>(total) * static_cast<unsigned long long>(1 + P.k));
    if constexpr (SHAPE == kPairSeq) {
        for (int64_t e = 0; e < total; ++e) {
            if (grp == 0) pair_visit<BF16, D, KMAX>(P, e, gl);
            __threadfence();
        }
    } else {
        const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
        if constexpr (SHAPE == kPairOnce) {
            const int64_t slot = wave * G + grp;
            if (slot < P.f0 + P.f1) pair_slot<BF16, D, KMAX>(P, slot, gl);
        } else {
            const int64_t stride = static_cast<int64_t>(gridDim.x) * (kBlock / 64) * G;
            for (int64_t slot = wave * G + grp; slot < P.f0 + P.f1; slot += stride) pair_slot<BF16, D, KMAX>(P, slot, gl);
        }
    }
}

using PairLauncher = void (*)(const PairArgs&, hipStream_t, bool);

template <bool BF16, int D, int KMAX>
void launch_pair(const PairArgs& P, hipStream_t st, bool seq) {
    constexpr int G = Lanes<BF16, D>::kG;
    if (seq) {
        hipLaunchKernelGGL((k_pair<BF16, D, KMAX, kPairSeq>), dim3(1), dim3(64), 0, st, P);
        return;
    }
    const int64_t need = std::max<int64_t>(1, ceil_div(P.f0 + P.f1, (kBlock / 64) * G));
    if (need <= kPairMaxBlocks)
        hipLaunchKernelGGL((k_pair<BF16, D, KMAX, kPairOnce>), dim3(static_cast<unsigned>(need)), dim3(kBlock), 0, st, P);
    else
        hipLaunchKernelGGL((k_pair<BF16, D, KMAX, kPairStride>), dim3(static_cast<unsigned>(kPairMaxBlocks)), dim3(kBlock),
                           0, st, P);
}

template <bool BF16, int D>
PairLauncher pick_k(int k) {
    if (k <= 1) return &launch_pair<BF16, D, 1>;
    if (k <= 3) return &launch_pair<BF16, D, 3>;
    if (k <= 7) return &launch_pair<BF16, D, 7>;
    return &launch_pair<BF16, D, 15>;
}

template <bool BF16>
PairLauncher pick_d(int d, int k) {
    switch (d) {
        case 8: return pick_k<BF16, 8>(k);
        case 16: return pick_k<BF16, 16>(k);
        case 32: return pick_k<BF16, 32>(k);
        case 64: return pick_k<BF16, 64>(k);
        case 128: return pick_k<BF16, 128>(k);
        case 256: return pick_k<BF16, 256>(k);
        default: throw Error(GOSH_E_INVALID_ARG, "d must be one of 8, 16, 32, 64, 128, 256");
    }
}

// ------------------------------------------------------------ host: graph view and pools
struct HostGraph {
    int64_t n = 0, nnz = 0;
    const int64_t* off64 = nullptr;
    const int32_t* off32 = nullptr;
    const int32_t* idx = nullptr;
    int64_t beg(int64_t u) const { return off64 ? off64[u] : off32[u]; }
    int64_t end(int64_t u) const { return off64 ? off64[u + 1] : off32[u + 1]; }
    // first position of u's sorted row whose neighbour is >= x
    int64_t lower(int64_t u, int64_t x) const {
        int64_t lo = beg(u), hi = end(u);
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (idx[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    }
};

struct PoolSpec {
    int64_t start_a, end_a, start_b, end_b;   // parts a and b
    uint32_t part_a, part_b;
    int B;
    uint32_t eps0;                            // round * B
    uint32_t key0, key1, w2;
    // optional: bounds[u * (K + 1) + p] = position of u's first neighbour >= start of part p,
    // relative to the row start (the parts never change during a run)
    const int32_t* bounds = nullptr;
    int K = 0;
};

// Runs fn(t) on `threads` threads (the caller's thread is one of them).
template <class Fn>
void parallel(int threads, Fn&& fn) {
    if (threads <= 1) {
        fn(0);
        return;
    }
    std::vector<std::thread> th;
    std::exception_ptr err;
    std::mutex em;
    for (int t = 1; t < threads; ++t)
        th.emplace_back([&, t] {
            try {
                fn(t);
            } catch (...) {
                std::lock_guard<std::mutex> g(em);
                if (!err) err = std::current_exception();
            }
        });
    try {
        fn(0);
    } catch (...) {
        std::lock_guard<std::mutex> g(em);
        if (!err) err = std::current_exception();
    }
    for (auto& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Builds pool S_{a,b} into out (capacity entries); returns (n0, n1).  The
// work is split into chunks of consecutive source vertices: a counting pass
// sizes every chunk, then each chunk writes its entries at its offset.
std::pair<int64_t, int64_t> build_pool(const HostGraph& G, const PoolSpec& S, int threads, uint2* out,
                                       int64_t capacity) {
    struct Side {
        int64_t s0, s1, o0, o1;   // source part, opposite part
        uint32_t opp;
    };
    const Side sd[2] = {{S.start_a, S.end_a, S.start_b, S.end_b, S.part_b},
                        {S.start_b, S.end_b, S.start_a, S.end_a, S.part_a}};
    const int sides = S.part_a != S.part_b ? 2 : 1;
    const int cps = std::max(1, threads) * 4;   // chunks per side
    const int chunks = cps * sides;
    auto range = [&](int c, const Side*& sp, int64_t& lo, int64_t& hi) {
        sp = &sd[c / cps];
        const int64_t len = sp->s1 - sp->s0;
        const int cc = c % cps;
        lo = sp->s0 + len * cc / cps;
        hi = sp->s0 + len * (cc + 1) / cps;
    };
    std::vector<int64_t> cnt(chunks + 1, 0);
    std::atomic<int> next{0};
    parallel(threads, [&](int) {
        for (int c = next.fetch_add(1); c < chunks; c = next.fetch_add(1)) {
            const Side* sp;
            int64_t lo, hi, m = 0;
            range(c, sp, lo, hi);
            if (S.bounds) {
                const uint32_t o = sp->opp;
                for (int64_t u = lo; u < hi; ++u) {
                    const int32_t* bu = S.bounds + u * (S.K + 1);
                    if (bu[o + 1] > bu[o]) m += S.B;
                }
            } else {
                for (int64_t u = lo; u < hi; ++u)
                    if (G.lower(u, sp->o1) > G.lower(u, sp->o0)) m += S.B;
            }
            cnt[c + 1] = m;
        }
    });
    for (int c = 0; c < chunks; ++c) cnt[c + 1] += cnt[c];
    const int64_t n0 = cnt[cps], total = cnt[chunks];
    if (total > capacity) throw Error(GOSH_E_DEVICE, "sample pool larger than its buffer");
    next = 0;
    parallel(threads, [&](int) {
        for (int c = next.fetch_add(1); c < chunks; c = next.fetch_add(1)) {
            const Side* sp;
            int64_t lo, hi;
            range(c, sp, lo, hi);
            int64_t at = cnt[c];
            for (int64_t u = lo; u < hi; ++u) {
                int64_t first, cu;
                if (S.bounds) {
                    const int32_t* bu = S.bounds + u * (S.K + 1);
                    first = G.beg(u) + bu[sp->opp];
                    cu = bu[sp->opp + 1] - bu[sp->opp];
                } else {
                    first = G.lower(u, sp->o0);
                    cu = G.lower(u, sp->o1) - first;
                }
                if (cu == 0) continue;
                for (int b = 0; b < S.B; ++b) {
                    const uint4 r = philox10(make_uint4(static_cast<uint32_t>(u), S.eps0 + static_cast<uint32_t>(b),
                                                        S.w2, stream_word3(0, sp->opp, 0)),
                                             S.key0, S.key1);
                    const int64_t pos = G.idx[first + scale_u32(r.x, cu)];
                    out[at++] = make_uint2(static_cast<uint32_t>(u - sp->s0),
                                           static_cast<uint32_t>(pos - sp->o0) | (static_cast<uint32_t>(b) << kPosBits));
                }
            }
        }
    });
    return {n0, total - n0};
}

std::vector<std::pair<int, int>> inside_out(int K) {
    std::vector<std::pair<int, int>> v;
    int a = 0, b = 0;
    const int64_t len = int64_t(K) * (K + 1) / 2;
    for (int64_t j = 0; j < len; ++j) {
        if (j > 0) {
            if (a > b) ++b;
            else { ++a; b = 0; }
        }
        v.emplace_back(a, b);
    }
    return v;
}

int64_t part_start(int64_t n, int K, int p) {
    return static_cast<int64_t>((static_cast<__int128>(p) * n) / K);
}

// Device bytes of a plan with K parts.
// (blocks as the context's allocator sizes them, plus 1 MiB of slack).
uint64_t plan_bytes(int64_t n, int d, int esz, const gosh_part_params& p, int K) {
    const int64_t rows = ceil_div(std::max<int64_t>(n, 1), K);
    const uint64_t part = alloc_bucket(std::max<size_t>(static_cast<size_t>(rows) * d * esz, 16));
    const uint64_t pool = alloc_bucket(static_cast<size_t>(std::max<int64_t>(2 * rows * p.B, 1)) * sizeof(uint2));
    return static_cast<uint64_t>(p.sub_bins) * part + static_cast<uint64_t>(p.pool_bins) * pool + (1u << 20);
}

void check_params(const gosh_part_params& p) {
    GOSH_REQUIRE(p.sub_bins >= 2 && p.sub_bins <= 16, GOSH_E_INVALID_ARG, "sub_bins (P_GPU) must be in [2, 16]");
    GOSH_REQUIRE(p.pool_bins >= 1 && p.pool_bins <= 16, GOSH_E_INVALID_ARG, "pool_bins (S_GPU) must be in [1, 16]");
    GOSH_REQUIRE(p.B >= 1 && p.B <= kMaxB, GOSH_E_INVALID_ARG, "B must be in [1, 31]");
    GOSH_REQUIRE(p.parts >= 0 && p.parts <= 255, GOSH_E_INVALID_ARG, "parts must be in [0, 255]");
    GOSH_REQUIRE(p.threads >= 0 && p.threads <= 256, GOSH_E_INVALID_ARG, "threads must be in [0, 256]");
}

int choose_parts(int64_t n, int d, int esz, const gosh_part_params& p, uint64_t budget) {
    if (p.parts > 0) return p.parts;
    for (int K = p.sub_bins + 1; K <= 255; ++K) {
        if (ceil_div(n, K) > kMaxPartRows) continue;
        if (plan_bytes(n, d, esz, p, K) <= budget) return K;
    }
    throw Error(GOSH_E_CAP_EXCEEDED, "no part count up to 255 fits the device memory budget");
}

HostGraph host_graph(const gosh_csr* g) {
    GOSH_REQUIRE(g, GOSH_E_INVALID_ARG, "null graph");
    GOSH_REQUIRE(g->n >= 0 && g->nnz >= 0 && g->offsets && (g->nnz == 0 || g->indices), GOSH_E_INVALID_ARG,
                 "bad graph view");
    GOSH_REQUIRE(g->n < INT32_MAX, GOSH_E_UNSUPPORTED, "vertex ids are int32");
    HostGraph G;
    G.n = g->n;
    G.nnz = g->nnz;
    if (g->offsets_is_i64) G.off64 = static_cast<const int64_t*>(g->offsets);
    else G.off32 = static_cast<const int32_t*>(g->offsets);
    G.idx = g->indices;
    GOSH_REQUIRE(G.beg(0) == 0 && (G.n == 0 ? G.nnz == 0 : G.end(G.n - 1) == G.nnz), GOSH_E_BAD_GRAPH,
                 "offsets must run from 0 to nnz");
    return G;
}

int sampler_threads(int t) {
    if (t > 0) return t;
    const unsigned h = std::thread::hardware_concurrency();
    return static_cast<int>(std::min<unsigned>(h ? h : 4, 64));
}

}  // namespace part_detail

using namespace part_detail;

// ------------------------------------------------------------ the partitioned run
namespace {

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double s() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

struct EventSet {
    std::vector<hipEvent_t> ev;
    hipEvent_t make() {
        hipEvent_t e;
        GOSH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ev.push_back(e);
        return e;
    }
    ~EventSet() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

struct StreamSet {
    std::vector<hipStream_t> st;
    hipStream_t make() {
        hipStream_t s;
        GOSH_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        st.push_back(s);
        return s;
    }
    ~StreamSet() {
        for (auto s : st) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    explicit PinnedBuf(size_t b) : bytes(b) {
        if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(GOSH_E_OOM, "pinned host allocation of " + std::to_string(b) + " bytes failed");
        }
    }
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
};

}  // namespace

void train_partitioned(Ctx* c, const gosh_csr* g_host, void* emb_host, gosh_dtype dt, int d, int epochs, float lr,
                       int k, int32_t level, uint32_t tag, const gosh_part_params& prm, uint64_t* updates_dev,
                       gosh_part_stats* stats) {
    Timer wall;
    check_params(prm);
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
    GOSH_REQUIRE(k >= 0 && k <= 15, GOSH_E_INVALID_ARG, "k must be in [0, 15]");
    GOSH_REQUIRE(epochs >= 0, GOSH_E_INVALID_ARG, "epochs must be >= 0");
    GOSH_REQUIRE(std::isfinite(lr) && lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
    GOSH_REQUIRE(emb_host, GOSH_E_INVALID_ARG, "null embedding");
    const PairLauncher launch = dt == GOSH_BF16 ? pick_d<true>(d, k) : pick_d<false>(d, k);
    const HostGraph G = host_graph(g_host);
    const int64_t n = G.n;
    const int esz = dt == GOSH_BF16 ? 2 : 4;
    const size_t row_bytes = static_cast<size_t>(d) * esz;

    uint64_t budget;
    if (c->cap) {
        c->trim();
        budget = c->cap > c->in_use ? c->cap - c->in_use : 0;
    } else {
        size_t fr = 0, tot = 0;
        GOSH_HIP(hipMemGetInfo(&fr, &tot));
        budget = static_cast<uint64_t>(fr * 0.9);
    }
    const int K = choose_parts(n, d, esz, prm, budget);
    GOSH_REQUIRE(K >= 1 && ceil_div(std::max<int64_t>(n, 1), K) <= kMaxPartRows, GOSH_E_UNSUPPORTED,
                 "parts larger than 2^27 rows");
    const int P = std::min(prm.sub_bins, K);
    const int S = prm.pool_bins;
    const int threads = sampler_threads(prm.threads);
    const int B = prm.B;
    const int rounds = epochs > 0 ? (epochs + B - 1) / B : 0;
    const int64_t cap_pos = static_cast<int64_t>(epochs) * n;
    std::vector<int64_t> starts(K + 1);
    for (int p = 0; p <= K; ++p) starts[p] = part_start(n, K, p);
    int64_t max_rows = 0;
    for (int p = 0; p < K; ++p) max_rows = std::max(max_rows, starts[p + 1] - starts[p]);
    const auto pairs = inside_out(K);
    const int64_t npools = static_cast<int64_t>(rounds) * static_cast<int64_t>(pairs.size());
    const int64_t pool_cap = std::max<int64_t>(2 * max_rows * B, 1);
    const size_t pool_bytes = static_cast<size_t>(pool_cap) * sizeof(uint2);

    gosh_part_stats st{};
    st.parts = K;
    st.rounds = rounds;

    // device memory: part bins and pool bins
    std::vector<DevBuf<uint8_t>> bins, pools;
    for (int b = 0; b < P; ++b) bins.emplace_back(c, std::max<size_t>(max_rows * row_bytes, 16));
    for (int s = 0; s < S; ++s) pools.emplace_back(c, pool_bytes);
    st.device_bytes = c->in_use;

    GOSH_HIP(hipStreamSynchronize(c->stream));   // earlier work on the caller's stream (counters, rows)
    StreamSet streams;
    EventSet events;
    std::vector<hipStream_t> bin_st(P), pool_st(S), ker_st(2);
    for (auto& s : bin_st) s = streams.make();
    for (auto& s : pool_st) s = streams.make();
    for (auto& s : ker_st) s = streams.make();
    std::vector<hipEvent_t> bin_ready(P), pool_ready(S), ker_done(2), stored(K, nullptr);
    for (auto& e : bin_ready) e = events.make();
    for (auto& e : pool_ready) e = events.make();
    for (auto& e : ker_done) e = events.make();

    // host pool ring filled ahead by the producer thread
    const int H = S + 2;
    std::vector<std::unique_ptr<PinnedBuf>> ring;
    std::vector<hipEvent_t> ring_copied(H);
    for (int h = 0; h < H; ++h) {
        ring.emplace_back(new PinnedBuf(pool_bytes));
        ring_copied[h] = events.make();
    }
    struct Produced {
        int64_t n0 = 0, n1 = 0;
    };
    std::vector<Produced> made(H);
    std::mutex mu;
    std::condition_variable cv;
    int64_t produced = 0;      // pools ready on the host
    int64_t issued = 0;        // pools whose host-to-device copy is enqueued
    bool stop = false;
    std::exception_ptr prod_err;
    double sample_s = 0.0;
    const uint32_t key0 = static_cast<uint32_t>(c->seed), key1 = static_cast<uint32_t>(c->seed >> 32);
    const uint32_t w2 = stream_word2(level, tag);

    // part boundaries inside every row, found once (K+1 binary searches per
    // vertex) when the table is at most 8 GiB
    std::vector<int32_t> bounds;
    if (static_cast<double>(n) * (K + 1) * 4.0 <= 8.0 * (1u << 30)) {
        Timer tb;
        bounds.resize(static_cast<size_t>(n) * (K + 1));
        std::atomic<int64_t> nextv{0};
        constexpr int64_t kStep = 1 << 14;
        parallel(threads, [&](int) {
            for (int64_t v0 = nextv.fetch_add(kStep); v0 < n; v0 = nextv.fetch_add(kStep))
                for (int64_t u = v0; u < std::min(n, v0 + kStep); ++u) {
                    const int64_t b0 = G.beg(u);
                    for (int p = 0; p <= K; ++p)
                        bounds[static_cast<size_t>(u) * (K + 1) + p] = static_cast<int32_t>(G.lower(u, starts[p]) - b0);
                }
        });
        sample_s += tb.s();
    }

    std::thread producer([&] {
        try {
            for (int64_t q = 0; q < npools; ++q) {
                const int h = static_cast<int>(q % H);
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || issued > q - H; });
                    if (stop) return;
                }
                if (q >= H) GOSH_HIP(hipEventSynchronize(ring_copied[h]));   // its previous pool has left
                const int rho = static_cast<int>(q / static_cast<int64_t>(pairs.size()));
                const auto pr = pairs[q % pairs.size()];
                PoolSpec ps{starts[pr.first], starts[pr.first + 1], starts[pr.second], starts[pr.second + 1],
                            static_cast<uint32_t>(pr.first), static_cast<uint32_t>(pr.second), B,
                            static_cast<uint32_t>(rho * B), key0, key1, w2, bounds.empty() ? nullptr : bounds.data(), K};
                Timer t;
                auto nn = build_pool(G, ps, threads, static_cast<uint2*>(ring[h]->p), pool_cap);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    sample_s += t.s();
                    made[h] = Produced{nn.first, nn.second};
                    produced = q + 1;
                }
                cv.notify_all();
            }
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            prod_err = std::current_exception();
            stop = true;
            cv.notify_all();
        }
    });

    // residency bookkeeping
    std::vector<int> bin_part(P, -1);
    std::vector<int64_t> bin_last(P, -1);
    std::vector<std::array<bool, 2>> bin_users(P, {false, false});
    std::vector<int> pool_user(S, -1);   // kernel stream that last read the pool bin
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ktime;   // timing events around each kernel
    int64_t positives = 0;
    double h2d = 0, d2h = 0;

    auto wait_users = [&](int b) {
        for (int s = 0; s < 2; ++s)
            if (bin_users[b][s]) GOSH_HIP(hipStreamWaitEvent(bin_st[b], ker_done[s], 0));
        bin_users[b] = {false, false};
    };
    auto store = [&](int b) {   // bin b's part back to the host
        const int old = bin_part[b];
        if (old < 0) return;
        wait_users(b);
        const size_t bytes = static_cast<size_t>(starts[old + 1] - starts[old]) * row_bytes;
        GOSH_HIP(hipMemcpyAsync(static_cast<uint8_t*>(emb_host) + starts[old] * row_bytes, bins[b].p, bytes,
                                hipMemcpyDeviceToHost, bin_st[b]));
        if (!stored[old]) stored[old] = events.make();
        GOSH_HIP(hipEventRecord(stored[old], bin_st[b]));
        d2h += bytes;
        ++st.part_stores;
        bin_part[b] = -1;
    };
    auto ensure = [&](int part, int keep, int64_t q) -> int {
        for (int b = 0; b < P; ++b)
            if (bin_part[b] == part) {
                bin_last[b] = q;
                return b;
            }
        int victim = -1;
        for (int b = 0; b < P; ++b)
            if (bin_part[b] < 0) { victim = b; break; }
        if (victim < 0) {
            for (int b = 0; b < P; ++b) {
                if (bin_part[b] == keep) continue;
                if (victim < 0 || bin_last[b] < bin_last[victim]) victim = b;
            }
        }
        store(victim);
        wait_users(victim);
        if (stored[part]) GOSH_HIP(hipStreamWaitEvent(bin_st[victim], stored[part], 0));
        const size_t bytes = static_cast<size_t>(starts[part + 1] - starts[part]) * row_bytes;
        GOSH_HIP(hipMemcpyAsync(bins[victim].p, static_cast<const uint8_t*>(emb_host) + starts[part] * row_bytes, bytes,
                                hipMemcpyHostToDevice, bin_st[victim]));
        GOSH_HIP(hipEventRecord(bin_ready[victim], bin_st[victim]));
        h2d += bytes;
        ++st.part_loads;
        bin_part[victim] = part;
        bin_last[victim] = q;
        return victim;
    };

    std::exception_ptr run_err;
    try {
        for (int64_t q = 0; q < npools && positives < cap_pos; ++q) {
            const int h = static_cast<int>(q % H);
            Produced pr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || produced > q; });
                if (prod_err) std::rethrow_exception(prod_err);
                pr = made[h];
            }
            const int rho = static_cast<int>(q / static_cast<int64_t>(pairs.size()));
            const auto pa = pairs[q % pairs.size()];
            // the cap cuts the pool sequence in order
            const int64_t allowed = std::min(pr.n0 + pr.n1, cap_pos - positives);
            const int64_t n0 = std::min(pr.n0, allowed), n1 = allowed - n0;
            positives += allowed;
            const int ba = ensure(pa.first, pa.second, q);
            const int bb = pa.second == pa.first ? ba : ensure(pa.second, pa.first, q);
            const int s = static_cast<int>(q % S);
            if (pool_user[s] >= 0) GOSH_HIP(hipStreamWaitEvent(pool_st[s], ker_done[pool_user[s]], 0));
            const size_t bytes = static_cast<size_t>(n0 + n1) * sizeof(uint2);
            if (bytes) {
                // side 1 entries follow side 0 in the host buffer; cut entries are dropped
                GOSH_HIP(hipMemcpyAsync(pools[s].p, ring[h]->p, static_cast<size_t>(n0) * sizeof(uint2),
                                        hipMemcpyHostToDevice, pool_st[s]));
                if (n1)
                    GOSH_HIP(hipMemcpyAsync(static_cast<uint2*>(static_cast<void*>(pools[s].p)) + n0,
                                            static_cast<const uint2*>(ring[h]->p) + pr.n0,
                                            static_cast<size_t>(n1) * sizeof(uint2), hipMemcpyHostToDevice,
                                            pool_st[s]));
            }
            GOSH_HIP(hipEventRecord(pool_ready[s], pool_st[s]));
            GOSH_HIP(hipEventRecord(ring_copied[h], pool_st[s]));
            h2d += bytes;
            st.pool_entries += n0 + n1;
            {
                std::lock_guard<std::mutex> lk(mu);
                issued = q + 1;
            }
            cv.notify_all();

            const int ks = c->deterministic ? 0 : static_cast<int>(q % 2);
            hipStream_t kst = ker_st[ks];
            GOSH_HIP(hipStreamWaitEvent(kst, bin_ready[ba], 0));
            if (bb != ba) GOSH_HIP(hipStreamWaitEvent(kst, bin_ready[bb], 0));
            GOSH_HIP(hipStreamWaitEvent(kst, pool_ready[s], 0));
            if (n0 + n1 > 0) {
                const float f = 1.0f - static_cast<float>(static_cast<double>(rho) / rounds);
                PairArgs A{bins[ba].p, bins[bb].p, starts[pa.first], starts[pa.second],
                           starts[pa.first + 1] - starts[pa.first], starts[pa.second + 1] - starts[pa.second],
                           static_cast<uint32_t>(pa.first), static_cast<uint32_t>(pa.second),
                           static_cast<const uint2*>(static_cast<const void*>(pools[s].p)), n0, n1, pr.n0, pr.n1, B,
                           static_cast<float>(lr * std::max(static_cast<double>(f), 1e-4)), k, key0, key1, w2,
                           static_cast<uint32_t>(rho * B), reinterpret_cast<unsigned long long*>(updates_dev)};
                hipEvent_t t0, t1;
                GOSH_HIP(hipEventCreate(&t0));
                events.ev.push_back(t0);
                GOSH_HIP(hipEventCreate(&t1));
                events.ev.push_back(t1);
                GOSH_HIP(hipEventRecord(t0, kst));
                launch(A, kst, c->deterministic);
                GOSH_HIP(hipGetLastError());
                GOSH_HIP(hipEventRecord(t1, kst));
                ktime.emplace_back(t0, t1);
            }
            GOSH_HIP(hipEventRecord(ker_done[ks], kst));
            bin_users[ba][ks] = true;
            bin_users[bb][ks] = true;
            pool_user[s] = ks;
        }
        for (int b = 0; b < P; ++b) store(b);
        for (auto s : streams.st) GOSH_HIP(hipStreamSynchronize(s));
    } catch (...) {
        run_err = std::current_exception();
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    producer.join();
    if (run_err) {
        for (auto s : streams.st) (void)hipStreamSynchronize(s);
        std::rethrow_exception(run_err);
    }
    if (prod_err) std::rethrow_exception(prod_err);
    for (auto& kt : ktime) {
        float ms = 0.0f;
        GOSH_HIP(hipEventElapsedTime(&ms, kt.first, kt.second));
        st.kernel_seconds += ms * 1e-3;
    }
    st.kernels = static_cast<int64_t>(ktime.size());
    st.positives = positives;
    st.h2d_bytes = h2d;
    st.d2h_bytes = d2h;
    st.sample_seconds = sample_s;
    st.seconds = wall.s();
    if (stats) *stats = st;
}

int partition_parts(int64_t n, int d, gosh_dtype dt, uint64_t budget, const gosh_part_params& p, uint64_t* bytes) {
    check_params(p);
    const int esz = dt == GOSH_BF16 ? 2 : 4;
    const int K = choose_parts(n, d, esz, p, budget);
    if (bytes) *bytes = plan_bytes(n, d, esz, p, K);
    return K;
}

int64_t partition_pool(const gosh_csr* g, int K, int i, int j, int B, uint64_t seed, int32_t level, uint32_t tag,
                       int32_t round, int threads, int32_t* src, int32_t* pos, int32_t* bout, int64_t capacity) {
    GOSH_REQUIRE(K >= 1 && K <= 255 && i >= 0 && j >= 0 && i < K && j < K, GOSH_E_INVALID_ARG, "bad part pair");
    GOSH_REQUIRE(B >= 1 && B <= kMaxB, GOSH_E_INVALID_ARG, "B must be in [1, 31]");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
    const HostGraph G = host_graph(g);
    const int64_t sa = part_start(G.n, K, i), ea = part_start(G.n, K, i + 1);
    const int64_t sb = part_start(G.n, K, j), eb = part_start(G.n, K, j + 1);
    const int64_t cap = std::max<int64_t>((ea - sa + eb - sb) * B, 1);
    std::vector<uint2> buf(cap);
    PoolSpec ps{sa, ea, sb, eb, static_cast<uint32_t>(i), static_cast<uint32_t>(j), B,
                static_cast<uint32_t>(round * B), static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32),
                stream_word2(level, tag)};
    auto nn = build_pool(G, ps, sampler_threads(threads), buf.data(), cap);
    const int64_t total = nn.first + nn.second;
    if (src) {
        GOSH_REQUIRE(capacity >= total, GOSH_E_INVALID_ARG, "output arrays too small");
        for (int64_t e = 0; e < total; ++e) {
            const bool s1 = e >= nn.first;
            src[e] = static_cast<int32_t>((s1 ? sb : sa) + buf[e].x);
            pos[e] = static_cast<int32_t>((s1 ? sa : sb) + (buf[e].y & kPosMask));
            bout[e] = static_cast<int32_t>(buf[e].y >> kPosBits);
        }
    }
    return total;
}

void inside_out_pairs(int K, int32_t* out) {
    GOSH_REQUIRE(K >= 1 && K <= 255, GOSH_E_INVALID_ARG, "K must be in [1, 255]");
    const auto v = inside_out(K);
    for (size_t q = 0; q < v.size(); ++q) {
        out[2 * q] = v[q].first;
        out[2 * q + 1] = v[q].second;
    }
}

}  // namespace gosh
