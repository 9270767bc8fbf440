// Random-walk positive sampling (Section 3.2) on gfx950.
//
// The paper runs the walks on the host to spare device memory and to use the
// CPU's strength on irregular accesses; with 288 GB of HBM3E the walks of a
// whole epoch fit on the device with room to spare, and a host sampler would
// have to stream n * P pairs per epoch over PCIe.  So an epoch is four
// stream-ordered steps on the device:
//   1. k_walks: one lane per start vertex v walks `len` steps (Philox kind 4)
//      and stores the walk in row v of a [n][len+1] table (-1 past its end);
//   2. k_keys: every pair number q = v P + l (offset l of walk v) gets the
//      shuffle key word 0 of Philox kind 5 at counter q;
//   3. a stable LSD radix sort of (key, q) gives the visiting order (ties by q);
//   4. k_walk_train: rank r reads q, the two walk entries of its offset, draws
//      its k negatives (kind 6 at counter r) and runs the same update chain as
//      the per-epoch trainer, with rounding bits from kind 7 at counter r.
// Void pairs (offset past a walk that stopped at a vertex without
// neighbours) keep their rank and are skipped.  The walk table of a pair
// lives in one or two 64-byte lines, so the two walk reads of a rank cost
// little next to its 2 + k row reads and atomic row writes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.hpp"
#include "gosh_internal.hpp"
#include "primitives.hpp"
#include "visit.hpp"

namespace gosh {
namespace {

using namespace train_detail;

constexpr int kWalkThreads = 256;
constexpr int kMaxWalkLen = 1024;
constexpr int64_t kMaxGridBlocks = int64_t(1) << 20;   // 2^28 lanes per launch, far below the 2^32 limit
constexpr int kLdsSteps = 16;     // walks of up to 15 steps are counted from LDS (16 KiB per block)

struct WalkArgs {
    const void* offsets;
    const int32_t* indices;
    int64_t n, nnz;
    int32_t len;              // steps per walk
    int32_t P;                // pair offsets per walk
    const uint32_t* tab;      // offset l: a | b << 16
    int32_t* walks;           // [n][len + 1]
    uint32_t key0, key1, epoch, w2;
    int k;
    unsigned long long* updates;
};

// Pair offsets (a, b), 0 <= a < b <= len, b - a <= window, numbered by a
// then b.
__global__ void k_pair_table(int32_t len, int32_t window, uint32_t* tab) {
    int32_t l = 0;
    for (int32_t a = 0; a < len; ++a)
        for (int32_t b = a + 1; b <= len && b - a <= window; ++b)
            tab[l++] = static_cast<uint32_t>(a) | (static_cast<uint32_t>(b) << 16);
}

template <class Off>
__global__ __launch_bounds__(kWalkThreads) void k_walks(WalkArgs A) {
    __shared__ int32_t walk_lds[kLdsSteps * kWalkThreads];
    const int64_t v = static_cast<int64_t>(blockIdx.x) * kWalkThreads + threadIdx.x;
    unsigned long long cnt = 0;
    if (v < A.n) {
        const Off* off = static_cast<const Off*>(A.offsets);
        int32_t* w = A.walks + v * (A.len + 1);
        // LDS copy of the walk for the update count: column per lane, so the
        // lanes of a wave hit distinct banks
        const bool lds_ok = A.updates && A.len < kLdsSteps;
        int32_t* mine = walk_lds + threadIdx.x;
        int64_t cur = v;
        w[0] = static_cast<int32_t>(v);
        if (lds_ok) mine[0] = static_cast<int32_t>(v);
        int32_t wl = 1;
        uint4 r = make_uint4(0, 0, 0, 0);
        for (int32_t i = 0; i < A.len; ++i) {
            if ((i & 3) == 0)
                r = philox10(make_uint4(static_cast<uint32_t>(v), A.epoch, A.w2,
                                        stream_word3(4, 0, static_cast<uint32_t>(i >> 2))),
                             A.key0, A.key1);
            const uint32_t word = (i & 3) == 0 ? r.x : (i & 3) == 1 ? r.y : (i & 3) == 2 ? r.z : r.w;
            const int64_t beg = off[cur], end = off[cur + 1];
            // a malformed row is treated as empty instead of read out of bounds
            const int64_t deg = (beg >= 0 && beg <= end && end <= A.nnz) ? end - beg : 0;
            if (deg == 0) break;
            const int32_t nxt = A.indices[beg + scale_u32(word, deg)];
            if (nxt < 0 || nxt >= A.n) break;
            cur = nxt;
            if (lds_ok) mine[wl * kWalkThreads] = nxt;
            w[wl++] = nxt;
        }
        for (int32_t i = wl; i <= A.len; ++i) w[i] = -1;
        if (A.updates) {
            // executed updates of this walk's pairs: the positives that differ
            // from their source plus k negatives per pair (a negative equal to
            // the source is subtracted by the visit); the walk is read back
            // from the lane's own LDS copy when it fits
            for (int32_t l = 0; l < A.P; ++l) {
                const uint32_t ab = A.tab[l];
                const int32_t a = static_cast<int32_t>(ab & 0xFFFFu), b = static_cast<int32_t>(ab >> 16);
                if (b < wl) {
                    const int32_t wa = lds_ok ? mine[a * kWalkThreads] : w[a];
                    const int32_t wb = lds_ok ? mine[b * kWalkThreads] : w[b];
                    cnt += static_cast<unsigned long long>(A.k) + (wa != wb ? 1ull : 0ull);
                }
            }
        }
    }
    if (A.updates) {
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(A.updates, cnt);
    }
}

__global__ __launch_bounds__(kWalkThreads) void k_keys(uint32_t* keys, uint32_t* vals, int64_t m, uint32_t epoch,
                                                       uint32_t w2, uint32_t key0, uint32_t key1) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWalkThreads;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kWalkThreads + threadIdx.x; q < m; q += stride) {
        keys[q] = philox10(make_uint4(static_cast<uint32_t>(q), epoch, w2, stream_word3(5, 0, 0)), key0, key1).x;
        vals[q] = static_cast<uint32_t>(q);
    }
}

struct WalkTrain {
    void* emb;
    const int32_t* walks;     // [n][len + 1]
    const uint32_t* order;    // visiting order: pair numbers
    const uint32_t* tab;
    int64_t n, m;
    int32_t len, P;
    float lr;
    int k;
    uint32_t key0, key1, epoch, w2;
    unsigned long long* updates;
    int32_t plain_neg;        // negatives written with plain stores
    // with light_below > 0, rows of degree below it (source, positive and
    // negatives) are written with plain stores; hub_bits marks the others
    int64_t light_below;
    const uint32_t* hub_bits;
};

template <bool BF16, int D, int KMAX>
__device__ __forceinline__ void walk_visit(const WalkTrain& T, int64_t r, int gl) {
    using Elem = typename RowIO<BF16>::Elem;
    const uint32_t q = T.order[r];
    const uint32_t v = q / static_cast<uint32_t>(T.P);
    const uint32_t ab = T.tab[q - v * static_cast<uint32_t>(T.P)];
    const int32_t* w = T.walks + static_cast<int64_t>(v) * (T.len + 1);
    const int32_t pos = w[ab >> 16];
    if (pos < 0) return;      // void pair
    const int32_t src = w[ab & 0xFFFFu];
    int32_t u[KMAX + 1];
    u[0] = pos;
    {
        constexpr int NB = (KMAX + 1 + 3) / 4;
        uint32_t wd[4 * NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (4 * b <= T.k) {
                const uint4 x = philox10(make_uint4(static_cast<uint32_t>(r), T.epoch, T.w2, stream_word3(6, 0, b)),
                                         T.key0, T.key1);
                wd[4 * b] = x.x; wd[4 * b + 1] = x.y; wd[4 * b + 2] = x.z; wd[4 * b + 3] = x.w;
            } else {
                wd[4 * b] = wd[4 * b + 1] = wd[4 * b + 2] = wd[4 * b + 3] = 0;
            }
        }
#pragma unroll
        for (int t = 1; t <= KMAX; ++t) u[t] = (t <= T.k) ? static_cast<int32_t>(scale_u32(wd[t], T.n)) : -1;
    }
    uint32_t plain = T.plain_neg != 0 ? ((2u << KMAX) - 1u) & ~1u : 0u;
    if (T.light_below > 0) {
        const auto light = [&](int32_t x) {
            return ((T.hub_bits[static_cast<uint32_t>(x) >> 5] >> (static_cast<uint32_t>(x) & 31u)) & 1u) == 0u;
        };
        if (light(src)) plain |= 1u << 31;
#pragma unroll
        for (int t = 0; t <= KMAX; ++t)
            if (t <= T.k && u[t] >= 0 && light(u[t])) plain |= 1u << t;
    }
    Elem* M = static_cast<Elem*>(T.emb);
    update_chain<BF16, D, KMAX, false>(M, src, M, src, u, T.k, T.lr, static_cast<uint32_t>(r), T.epoch, T.w2, 7u, 0u,
                                       T.key0, T.key1, T.updates, gl, plain);
}

// Launch shapes: one wave in rank order (deterministic mode), one rank per
// lane group when one launch covers the epoch, else a grid-stride loop (an
// epoch can hold more ranks than one launch has lanes, n P up to 2^32).  The
// loop is its own instantiation: inside a loop the visit holds more registers
// (137 against 112 VGPRs, 3 instead of 4 waves per SIMD).
enum WalkShape { kWalkSeq = 0, kWalkOnce = 1, kWalkStride = 2 };

template <bool BF16, int D, int KMAX, int SHAPE>
__global__ __launch_bounds__(kBlock) void k_walk_train(WalkTrain T) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    if constexpr (SHAPE == kWalkSeq) {
        // one wave, ranks strictly in order
        for (int64_t r = 0; r < T.m; ++r) {
            if (grp == 0) walk_visit<BF16, D, KMAX>(T, r, gl);
            __threadfence();
        }
    } else {
        const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
        if constexpr (SHAPE == kWalkOnce) {
            const int64_t r = wave * G + grp;
            if (r < T.m) walk_visit<BF16, D, KMAX>(T, r, gl);
        } else {
            const int64_t stride = static_cast<int64_t>(gridDim.x) * (kBlock / 64) * G;
            for (int64_t r = wave * G + grp; r < T.m; r += stride) walk_visit<BF16, D, KMAX>(T, r, gl);
        }
    }
}

using WalkLauncher = void (*)(const WalkTrain&, hipStream_t, bool);

template <bool BF16, int D, int KMAX>
void launch_walk(const WalkTrain& T, hipStream_t st, bool seq) {
    constexpr int G = Lanes<BF16, D>::kG;
    if (seq) {
        hipLaunchKernelGGL((k_walk_train<BF16, D, KMAX, kWalkSeq>), dim3(1), dim3(64), 0, st, T);
        return;
    }
    const int64_t need = ceil_div(T.m, (kBlock / 64) * G);
    if (need <= kMaxGridBlocks)
        hipLaunchKernelGGL((k_walk_train<BF16, D, KMAX, kWalkOnce>), dim3(static_cast<unsigned>(std::max<int64_t>(need, 1))),
                           dim3(kBlock), 0, st, T);
    else
        hipLaunchKernelGGL((k_walk_train<BF16, D, KMAX, kWalkStride>), dim3(static_cast<unsigned>(kMaxGridBlocks)),
                           dim3(kBlock), 0, st, T);
}

template <bool BF16, int D>
WalkLauncher pick_k(int k) {
    if (k <= 1) return &launch_walk<BF16, D, 1>;
    if (k <= 3) return &launch_walk<BF16, D, 3>;
    if (k <= 7) return &launch_walk<BF16, D, 7>;
    return &launch_walk<BF16, D, 15>;
}

template <bool BF16>
WalkLauncher pick_d(int d, int k) {
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

// Pairs of an epoch in visiting order (-1, -1 for void ones).
__global__ __launch_bounds__(kWalkThreads) void k_emit(const int32_t* walks, const uint32_t* order,
                                                       const uint32_t* tab, int64_t m, int32_t len, int32_t P,
                                                       int32_t* src, int32_t* pos) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWalkThreads;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * kWalkThreads + threadIdx.x; r < m; r += stride) {
        const uint32_t q = order[r];
        const uint32_t v = q / static_cast<uint32_t>(P);
        const uint32_t ab = tab[q - v * static_cast<uint32_t>(P)];
        const int32_t* w = walks + static_cast<int64_t>(v) * (len + 1);
        const int32_t b = w[ab >> 16];
        src[r] = b < 0 ? -1 : w[ab & 0xFFFFu];
        pos[r] = b;
    }
}

// Device state of one call: pair table, walk table and the sort buffers,
// reused by every epoch.
struct WalkEpochs {
    Ctx* c;
    const Level& L;
    int64_t P, m;
    DevBuf<uint32_t> tab, keys, keys_tmp, order, order_tmp;
    DevBuf<int32_t> walks;
    WalkArgs A{};

    WalkEpochs(Ctx* ctx, const Level& lvl, int32_t level, uint32_t tag, int32_t len, int32_t window, int k,
               unsigned long long* updates)
        : c(ctx), L(lvl), P(walk_pair_count(len, window)), m(lvl.n * P) {
        GOSH_REQUIRE(m < (int64_t{1} << 32), GOSH_E_UNSUPPORTED,
                     "vertices times pairs per walk must stay below 2^32");
        if (m == 0) return;
        tab = DevBuf<uint32_t>(c, static_cast<size_t>(P));
        walks = DevBuf<int32_t>(c, static_cast<size_t>(L.n) * static_cast<size_t>(len + 1));
        keys = DevBuf<uint32_t>(c, static_cast<size_t>(m));
        keys_tmp = DevBuf<uint32_t>(c, static_cast<size_t>(m));
        order = DevBuf<uint32_t>(c, static_cast<size_t>(m));
        order_tmp = DevBuf<uint32_t>(c, static_cast<size_t>(m));
        hipLaunchKernelGGL(k_pair_table, dim3(1), dim3(1), 0, c->stream, len, window, tab.p);
        GOSH_HIP(hipGetLastError());
        A.offsets = L.offsets;
        A.indices = L.indices;
        A.n = L.n;
        A.nnz = L.nnz;
        A.len = len;
        A.P = static_cast<int32_t>(P);
        A.tab = tab.p;
        A.walks = walks.p;
        A.key0 = static_cast<uint32_t>(c->seed);
        A.key1 = static_cast<uint32_t>(c->seed >> 32);
        A.w2 = stream_word2(level, tag);
        A.k = k;
        A.updates = updates;
    }

    // walks, shuffle keys and visiting order of epoch j
    void prepare(int32_t j) {
        A.epoch = static_cast<uint32_t>(j);
        const unsigned walk_blocks = static_cast<unsigned>(ceil_div(L.n, kWalkThreads));
        if (L.off64) hipLaunchKernelGGL(k_walks<int64_t>, dim3(walk_blocks), dim3(kWalkThreads), 0, c->stream, A);
        else hipLaunchKernelGGL(k_walks<int32_t>, dim3(walk_blocks), dim3(kWalkThreads), 0, c->stream, A);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_keys, dim3(grid(m)), dim3(kWalkThreads), 0, c->stream, keys.p, order.p, m, A.epoch,
                           A.w2, A.key0, A.key1);
        GOSH_HIP(hipGetLastError());
        radix_sort_u32(c, keys.p, keys_tmp.p, order.p, order_tmp.p, m, 32);
    }

    static unsigned grid(int64_t items) {
        return static_cast<unsigned>(std::min<int64_t>(ceil_div(items, kWalkThreads), 65536));
    }
};

void check_walk_args(int32_t len, int32_t window, uint32_t tag) {
    GOSH_REQUIRE(len >= 0 && len <= kMaxWalkLen, GOSH_E_INVALID_ARG, "walk length must be in [0, 1024]");
    GOSH_REQUIRE(window >= 0, GOSH_E_INVALID_ARG, "window must be >= 0");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
}

}  // namespace

int64_t walk_pair_count(int32_t len, int32_t window) {
    const int64_t g = std::min(window, len);
    return g * len - g * (g - 1) / 2;
}

void train_walks(Ctx* c, const Level& L, int32_t level, void* emb, gosh_dtype dt, int d, int epochs, float lr,
                 int k, int32_t len, int32_t window, uint32_t tag, uint64_t* updates_dev,
                 gosh_walk_timing* timing) {
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
    GOSH_REQUIRE(k >= 0 && k <= 15, GOSH_E_INVALID_ARG, "k must be in [0, 15]");
    GOSH_REQUIRE(std::isfinite(lr) && lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
    GOSH_REQUIRE(epochs >= 0, GOSH_E_INVALID_ARG, "epochs must be >= 0");
    check_walk_args(len, window, tag);
    WalkLauncher fn = dt == GOSH_BF16 ? pick_d<true>(d, k) : pick_d<false>(d, k);
    GOSH_REQUIRE(L.n == 0 || emb, GOSH_E_INVALID_ARG, "null embedding");
    if (timing) *timing = gosh_walk_timing{0.0, 0.0, 0};
    if (L.n == 0 || epochs == 0 || walk_pair_count(len, window) == 0) return;
    WalkEpochs W(c, L, level, tag, len, window, k, reinterpret_cast<unsigned long long*>(updates_dev));

    WalkTrain T{};
    T.emb = emb;
    T.walks = W.walks.p;
    T.order = W.order.p;
    T.tab = W.tab.p;
    T.n = L.n;
    T.m = W.m;
    T.len = len;
    T.P = static_cast<int32_t>(W.P);
    T.k = k;
    T.key0 = W.A.key0;
    T.key1 = W.A.key1;
    T.w2 = W.A.w2;
    T.updates = W.A.updates;
    T.plain_neg = (!c->deterministic && c->plain_neg_min > 0 && L.n >= c->plain_neg_min) ? 1 : 0;
    // light rows stored plainly (also in deterministic mode, where it changes no bit)
    T.light_below = (c->plain_light_min > 0 && L.n >= c->plain_light_min) ? L.nnz / L.n + 1 : 0;
    if (T.light_below > 0) T.hub_bits = hub_bits(c, L, T.light_below);
    // optional timing: events before the sampling, between sampling and
    // training, and after the training of every epoch
    std::vector<hipEvent_t> ev;
    struct EventGuard {
        std::vector<hipEvent_t>& v;
        ~EventGuard() {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } guard{ev};
    if (timing) {
        ev.resize(3 * static_cast<size_t>(epochs), nullptr);
        for (auto& e : ev) GOSH_HIP(hipEventCreate(&e));
    }
    for (int j = 0; j < epochs; ++j) {
        if (timing) GOSH_HIP(hipEventRecord(ev[3 * j], c->stream));
        W.prepare(j);
        if (timing) GOSH_HIP(hipEventRecord(ev[3 * j + 1], c->stream));
        T.epoch = static_cast<uint32_t>(j);
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(epochs);
        T.lr = static_cast<float>(static_cast<double>(lr) * (f > 1e-4 ? f : 1e-4));
        fn(T, c->stream, c->deterministic);
        GOSH_HIP(hipGetLastError());
        if (timing) GOSH_HIP(hipEventRecord(ev[3 * j + 2], c->stream));
    }
    if (timing) {
        GOSH_HIP(hipEventSynchronize(ev.back()));
        for (int j = 0; j < epochs; ++j) {
            float a = 0.0f, b = 0.0f;
            GOSH_HIP(hipEventElapsedTime(&a, ev[3 * j], ev[3 * j + 1]));
            GOSH_HIP(hipEventElapsedTime(&b, ev[3 * j + 1], ev[3 * j + 2]));
            timing->sample_ms += a;
            timing->train_ms += b;
        }
        timing->epochs = epochs;
    }
}

int64_t walk_pairs(Ctx* c, const Level& L, int32_t level, int32_t epoch, int32_t len, int32_t window, uint32_t tag,
                   int32_t* src, int32_t* pos, int64_t capacity) {
    check_walk_args(len, window, tag);
    GOSH_REQUIRE(epoch >= 0, GOSH_E_INVALID_ARG, "epoch must be >= 0");
    const int64_t m = L.n * walk_pair_count(len, window);
    if (!src && !pos) return m;
    GOSH_REQUIRE(src && pos, GOSH_E_INVALID_ARG, "null output");
    GOSH_REQUIRE(capacity >= m, GOSH_E_INVALID_ARG, "output arrays hold fewer than n * P pairs");
    if (m == 0) return 0;
    WalkEpochs W(c, L, level, tag, len, window, 0, nullptr);
    W.prepare(epoch);
    hipLaunchKernelGGL(k_emit, dim3(WalkEpochs::grid(m)), dim3(kWalkThreads), 0, c->stream, W.walks.p, W.order.p,
                       W.tab.p, m, len, static_cast<int32_t>(W.P), src, pos);
    GOSH_HIP(hipGetLastError());
    return m;
}

}  // namespace gosh
