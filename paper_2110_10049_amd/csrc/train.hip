// TrainInGPU (Algorithm 3, Section 3.1) with UpdateEmbed (Algorithm 1) for
// gfx950.
//
// Layout: every lane owns 8 elements of a row, so a source with dimension d
// is served by a group of L = d/8 lanes and one wave64 carries 64/L sources
// (d=128: 4 sources per wave, d=32: 16); the elements are interleaved across
// the group (see RowIO) so that each memory instruction covers contiguous
// bytes.  The dot product is reduced inside
// the group with DPP (no LDS round trip).  Each group draws its samples from
// Philox, issues the loads of the source row and of all 1+k sample rows at
// once, then runs the dependent chain of updates from registers; the source
// row plays the role of the paper's shared-memory staged row (Section 3.1),
// here kept in registers.  A sample that repeats within one source is
// forwarded from the earlier update's registers, so the chain has the
// sequential semantics of Algorithm 3.  Sources of one epoch run
// concurrently without locks; an epoch is one launch, so epochs never
// overlap (Section 3.1).  Each sample row's change and, at the end, the
// source row's change are applied atomically to memory (see RowIO).
//
// BF16 storage: rows are widened to FP32, all arithmetic is FP32, and each
// written row is stochastically rounded with Philox bits (kind 1, slot =
// update index or 255 for the source write-back): element e lies in 32-bit
// word w = e/2, which draws block w mod L and takes half 2*(w div L) + e mod 2,
// so lane gl draws exactly one block (block gl) per row update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "gosh_internal.hpp"

namespace gosh {
namespace {

constexpr int kEPL = 8;       // row elements per lane
constexpr int kBlock = 256;   // 4 waves

struct TrainParams {
    const void* offsets;
    const int32_t* indices;
    int64_t n;                // vertices of the level (negatives are drawn from [0, n))
    void* emb;
    int64_t n_rows;           // rows addressable in emb
    float lr;
    int k;
    uint32_t key0, key1;
    uint32_t epoch;
    uint32_t w2;              // level | tag << 8
    unsigned long long* updates;   // optional executed-update counter
    const int32_t* src_list;       // explicit-sample mode
    const int32_t* samples;
    int64_t nsrc;
};

enum Mode { kEpoch = 0, kExplicit = 1, kSequential = 2 };

// Row access.  A lane of the group of L = d/8 lanes owns row elements
// gl + L*i (FP32) or 32-bit words gl + L*i (BF16, two elements each), so
// every load and every atomic instruction of a group covers one contiguous
// run of the row.
//
// Writes are atomic: sources of an epoch run concurrently and share rows, and
// a plain read-modify-write store would drop every concurrent update but the
// last one -- on small levels, where a whole epoch is in flight at once,
// nearly all of them.  FP32 rows receive their changes with atomic adds.
// BF16 rows receive, per 32-bit word, the exact difference between the
// stochastically rounded new value and the value this visit started from,
// through the packed BF16 atomic add: uncontended, the stored row becomes
// exactly the rounded value (the difference of two nearby BF16 values is
// itself a BF16 value); contended, the concurrent changes add up in value
// space.  (Adding bit-pattern differences with integer atomics would be
// faster but wraps through the sign when many concurrent updates move one
// element across zero.)  The L2 atomic units sustain about half the
// bandwidth of plain stores, so they bound the training kernel.
template <bool BF16>
struct RowIO;

template <>
struct RowIO<false> {
    using Elem = float;
    template <int L>
    __device__ static void load(const float* M, int64_t row, int gl, float (&x)[kEPL]) {
        const float* p = M + row * (L * kEPL) + gl;
#pragma unroll
        for (int i = 0; i < kEPL; ++i) x[i] = p[L * i];
    }
    template <int L>
    __device__ static void add(float* M, int64_t row, int gl, const float (&dx)[kEPL]) {
        float* p = M + row * (L * kEPL) + gl;
#pragma unroll
        for (int i = 0; i < kEPL; ++i)
            __hip_atomic_fetch_add(p + L * i, dx[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

typedef __bf16 __attribute__((ext_vector_type(2))) bf16x2_t;

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

template <>
struct RowIO<true> {
    using Elem = uint16_t;
    template <int L>
    __device__ static void load(const uint16_t* M, int64_t row, int gl, float (&x)[kEPL]) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(M + row * (L * kEPL)) + gl;
#pragma unroll
        for (int i = 0; i < kEPL / 2; ++i) {
            const uint32_t w = p[L * i];
            x[2 * i] = bf16_lo(w);
            x[2 * i + 1] = bf16_hi(w);
        }
    }
    // cur: the values this visit last saw (exact BF16), v: the FP32 results.
    // Element h of the lane uses random half h of r.  out: the rounded values.
    template <int L>
    __device__ static void commit(uint16_t* M, int64_t row, int gl, const float (&cur)[kEPL],
                                  const float (&v)[kEPL], uint4 r, float (&out)[kEPL]) {
        uint32_t* p = reinterpret_cast<uint32_t*>(M + row * (L * kEPL)) + gl;
        const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < kEPL / 2; ++i) {
            const uint32_t t0 = bf16_sr(v[2 * i], rw[i] & 0xFFFFu);
            const uint32_t t1 = bf16_sr(v[2 * i + 1], rw[i] >> 16);
            out[2 * i] = __uint_as_float(t0 << 16);
            out[2 * i + 1] = __uint_as_float(t1 << 16);
            const uint32_t d = bf16_rne_bits(out[2 * i] - cur[2 * i]) |
                               (bf16_rne_bits(out[2 * i + 1] - cur[2 * i + 1]) << 16);
            if (d != 0u)
                __builtin_amdgcn_global_atomic_fadd_v2bf16(
                    (__attribute__((address_space(1))) bf16x2_t*)(p + L * i),
                    __builtin_bit_cast(bf16x2_t, d));
        }
    }
};

__device__ __forceinline__ float sigmoidf_(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}

// One source visit: draws (or reads) the samples and applies the updates.
template <bool BF16, int D, int KMAX, class Off, int MODE>
__device__ __forceinline__ void visit(const TrainParams& P, int64_t slot, bool active, int gl) {
    constexpr int L = D / kEPL;
    using IO = RowIO<BF16>;
    using Elem = typename IO::Elem;
    Elem* M = static_cast<Elem*>(P.emb);
    const int k = P.k;

    int64_t src = slot;
    int32_t u[KMAX + 1];
#pragma unroll
    for (int t = 0; t <= KMAX; ++t) u[t] = -1;

    if constexpr (MODE == kExplicit) {
        if (active) {
            src = P.src_list[slot];
            active = src >= 0 && src < P.n_rows;
        }
        if (active) {
#pragma unroll
            for (int t = 0; t <= KMAX; ++t) {
                if (t <= k) {
                    const int32_t v = P.samples[slot * (1 + k) + t];
                    u[t] = (v >= 0 && v < P.n_rows) ? v : -1;
                }
            }
        }
    } else {
        if (active) {
            constexpr int NB = (KMAX + 1 + 3) / 4;
            uint32_t wd[4 * NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (4 * b <= k) {
                    const uint4 r = philox10(
                        make_uint4(static_cast<uint32_t>(src), P.epoch, P.w2, stream_word3(0, 0, b)),
                        P.key0, P.key1);
                    wd[4 * b] = r.x; wd[4 * b + 1] = r.y; wd[4 * b + 2] = r.z; wd[4 * b + 3] = r.w;
                } else {
                    wd[4 * b] = wd[4 * b + 1] = wd[4 * b + 2] = wd[4 * b + 3] = 0;
                }
            }
            const Off* off = static_cast<const Off*>(P.offsets);
            const int64_t beg = off[src], end = off[src + 1];
            const int64_t deg = end - beg;
#pragma unroll
            for (int t = 1; t <= KMAX; ++t)
                if (t <= k) u[t] = static_cast<int32_t>(scale_u32(wd[t], P.n));
            if (deg > 0) {
                const int32_t pos = P.indices[beg + scale_u32(wd[0], deg)];
                u[0] = (pos >= 0 && pos < P.n) ? pos : -1;
            }
        }
    }
    if (!active) return;

    float s[kEPL];
    float m[KMAX + 1][kEPL];
    IO::template load<L>(M, src, gl, s);
#pragma unroll
    for (int t = 0; t <= KMAX; ++t) {
        if (u[t] >= 0 && u[t] != src) {
            IO::template load<L>(M, u[t], gl, m[t]);
        } else {
#pragma unroll
            for (int e = 0; e < kEPL; ++e) m[t][e] = 0.0f;
        }
    }

    int done = 0;
    const float lr = P.lr;
    float s0[kEPL];
#pragma unroll
    for (int e = 0; e < kEPL; ++e) s0[e] = s[e];
#pragma unroll
    for (int t = 0; t <= KMAX; ++t) {
        if (t > k) break;
        const int32_t ut = u[t];
        if (ut < 0 || ut == src) {
            if (t > 0 && ut == src && P.updates && gl == 0) atomicAdd(P.updates, ~0ull);  // -1
            continue;
        }
        // a row sampled earlier in this visit continues from its updated value
#pragma unroll
        for (int tp = 0; tp < t; ++tp) {
            if (u[tp] == ut) {
#pragma unroll
                for (int e = 0; e < kEPL; ++e) m[t][e] = m[tp][e];
            }
        }
        float x = 0.0f;
#pragma unroll
        for (int e = 0; e < kEPL; ++e) x = fmaf(s[e], m[t][e], x);
        x = group_sum<L>(x);
        const float b = (t == 0) ? 1.0f : 0.0f;
        const float g = (b - sigmoidf_(x)) * lr;
#pragma unroll
        for (int e = 0; e < kEPL; ++e) s[e] = fmaf(g, m[t][e], s[e]);
        if constexpr (BF16) {
            const uint4 bits = philox10(make_uint4(static_cast<uint32_t>(src), P.epoch, P.w2,
                                                   stream_word3(1, static_cast<uint32_t>(t),
                                                                static_cast<uint32_t>(gl))),
                                        P.key0, P.key1);
            float v[kEPL], out[kEPL];
#pragma unroll
            for (int e = 0; e < kEPL; ++e) v[e] = fmaf(g, s[e], m[t][e]);
            IO::template commit<L>(M, ut, gl, m[t], v, bits, out);
#pragma unroll
            for (int e = 0; e < kEPL; ++e) m[t][e] = out[e];
        } else {
            float dx[kEPL];
#pragma unroll
            for (int e = 0; e < kEPL; ++e) {
                dx[e] = g * s[e];
                m[t][e] += dx[e];
            }
            IO::template add<L>(M, ut, gl, dx);
        }
        ++done;
    }
    if (done) {
        if constexpr (BF16) {
            const uint4 bits = philox10(make_uint4(static_cast<uint32_t>(src), P.epoch, P.w2,
                                                   stream_word3(1, 0xFFu, static_cast<uint32_t>(gl))),
                                        P.key0, P.key1);
            float out[kEPL];
            IO::template commit<L>(M, src, gl, s0, s, bits, out);
        } else {
            float dx[kEPL];
#pragma unroll
            for (int e = 0; e < kEPL; ++e) dx[e] = s[e] - s0[e];
            IO::template add<L>(M, src, gl, dx);
        }
    }
}

template <bool BF16, int D, int KMAX, class Off, int MODE>
__global__ __launch_bounds__(kBlock) void k_train(TrainParams P) {
    constexpr int L = D / kEPL;
    constexpr int G = 64 / L;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    if constexpr (MODE == kSequential) {
        // one wave, sources strictly in ascending id order
        for (int64_t s = 0; s < P.n; ++s) {
            visit<BF16, D, KMAX, Off, MODE>(P, s, grp == 0, gl);
            __threadfence();
        }
    } else {
        const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
        const int64_t slot = wave * G + grp;
        const int64_t limit = (MODE == kExplicit) ? P.nsrc : P.n;
        visit<BF16, D, KMAX, Off, MODE>(P, slot, slot < limit, gl);
    }
}

template <class Off>
__global__ void k_draw(TrainParams P, int32_t* out) {
    const int64_t src = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (src >= P.n) return;
    const int k = P.k;
    const Off* off = static_cast<const Off*>(P.offsets);
    const int64_t beg = off[src], deg = static_cast<int64_t>(off[src + 1]) - beg;
    for (int b = 0; 4 * b <= k; ++b) {
        const uint4 r = philox10(make_uint4(static_cast<uint32_t>(src), P.epoch, P.w2, stream_word3(0, 0, b)),
                                 P.key0, P.key1);
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
        for (int j = 0; j < 4; ++j) {
            const int t = 4 * b + j;
            if (t > k) break;
            int32_t v;
            if (t == 0) v = deg > 0 ? P.indices[beg + scale_u32(w[0], deg)] : -1;
            else v = static_cast<int32_t>(scale_u32(w[j], P.n));
            out[src * (1 + k) + t] = v;
        }
    }
}

// Adds the UpdateEmbed calls of `epochs` epochs without self-negatives:
// one positive per vertex with neighbours plus k negatives per vertex
// (negatives equal to the source are subtracted by the training kernel).
template <class Off>
__global__ void k_add_updates(const Off* off, int64_t n, int k, int epochs, unsigned long long* p) {
    unsigned long long cnt = 0;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<int64_t>(gridDim.x) * blockDim.x)
        cnt += (off[v + 1] != off[v]) ? 1ull : 0ull;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    unsigned long long add = ((threadIdx.x & 63) == 0) ? cnt * static_cast<unsigned long long>(epochs) : 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        add += static_cast<unsigned long long>(k) * static_cast<unsigned long long>(n) * epochs;
    if (add) atomicAdd(p, add);
}

// ---------------------------------------------------------------- dispatch
using Launcher = void (*)(const TrainParams&, int64_t, hipStream_t);

template <bool BF16, int D, int KMAX, class Off, int MODE>
void launch(const TrainParams& P, int64_t items, hipStream_t st) {
    constexpr int G = 64 / (D / kEPL);
    if constexpr (MODE == kSequential) {
        hipLaunchKernelGGL((k_train<BF16, D, KMAX, Off, MODE>), dim3(1), dim3(64), 0, st, P);
    } else {
        const int64_t per_block = (kBlock / 64) * G;
        const int64_t blocks = ceil_div(items, per_block);
        hipLaunchKernelGGL((k_train<BF16, D, KMAX, Off, MODE>), dim3(static_cast<unsigned>(blocks)),
                           dim3(kBlock), 0, st, P);
    }
}

template <bool BF16, int D, int KMAX, int MODE>
Launcher pick_off(bool off64) {
    if constexpr (MODE == kExplicit) return &launch<BF16, D, KMAX, int32_t, MODE>;
    else return off64 ? &launch<BF16, D, KMAX, int64_t, MODE> : &launch<BF16, D, KMAX, int32_t, MODE>;
}

template <bool BF16, int D, int MODE>
Launcher pick_k(int k, bool off64) {
    if (k <= 1) return pick_off<BF16, D, 1, MODE>(off64);
    if (k <= 3) return pick_off<BF16, D, 3, MODE>(off64);
    if (k <= 7) return pick_off<BF16, D, 7, MODE>(off64);
    return pick_off<BF16, D, 15, MODE>(off64);
}

template <bool BF16, int MODE>
Launcher pick_d(int d, int k, bool off64) {
    switch (d) {
        case 8: return pick_k<BF16, 8, MODE>(k, off64);
        case 16: return pick_k<BF16, 16, MODE>(k, off64);
        case 32: return pick_k<BF16, 32, MODE>(k, off64);
        case 64: return pick_k<BF16, 64, MODE>(k, off64);
        case 128: return pick_k<BF16, 128, MODE>(k, off64);
        case 256: return pick_k<BF16, 256, MODE>(k, off64);
    }
    return nullptr;
}

template <int MODE>
Launcher pick(gosh_dtype dt, int d, int k, bool off64) {
    return dt == GOSH_BF16 ? pick_d<true, MODE>(d, k, off64) : pick_d<false, MODE>(d, k, off64);
}

void check_train_args(gosh_dtype dt, int d, int k, float lr) {
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
    GOSH_REQUIRE(d == 8 || d == 16 || d == 32 || d == 64 || d == 128 || d == 256, GOSH_E_INVALID_ARG,
                 "d must be one of 8, 16, 32, 64, 128, 256");
    GOSH_REQUIRE(k >= 0 && k <= 15, GOSH_E_INVALID_ARG, "k must be in [0, 15]");
    GOSH_REQUIRE(std::isfinite(lr) && lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
}

TrainParams base_params(Ctx* c, int32_t level, uint32_t tag) {
    TrainParams P{};
    P.key0 = static_cast<uint32_t>(c->seed);
    P.key1 = static_cast<uint32_t>(c->seed >> 32);
    P.w2 = stream_word2(level, tag);
    return P;
}

}  // namespace

void train_level(Ctx* c, const Level& L, int32_t level, void* emb, gosh_dtype dt, int d, int epochs,
                 float lr, int k, uint32_t tag, uint64_t* updates_dev) {
    check_train_args(dt, d, k, lr);
    GOSH_REQUIRE(epochs >= 0, GOSH_E_INVALID_ARG, "epochs must be >= 0");
    GOSH_REQUIRE(L.n == 0 || emb, GOSH_E_INVALID_ARG, "null embedding");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
    if (L.n == 0 || epochs == 0) return;
    TrainParams P = base_params(c, level, tag);
    P.offsets = L.offsets;
    P.indices = L.indices;
    P.n = L.n;
    P.emb = emb;
    P.n_rows = L.n;
    P.k = k;
    P.updates = reinterpret_cast<unsigned long long*>(updates_dev);
    Launcher fn = c->deterministic ? pick<kSequential>(dt, d, k, L.off64) : pick<kEpoch>(dt, d, k, L.off64);
    GOSH_REQUIRE(fn, GOSH_E_INVALID_ARG, "unsupported training shape");
    for (int j = 0; j < epochs; ++j) {
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(epochs);
        P.lr = static_cast<float>(static_cast<double>(lr) * (f > 1e-4 ? f : 1e-4));
        P.epoch = static_cast<uint32_t>(j);
        fn(P, L.n, c->stream);
        GOSH_HIP(hipGetLastError());
    }
    if (updates_dev) {
        const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(L.n, 256), 1024));
        auto* cnt = reinterpret_cast<unsigned long long*>(updates_dev);
        if (L.off64)
            hipLaunchKernelGGL(k_add_updates<int64_t>, dim3(blocks), dim3(256), 0, c->stream,
                               static_cast<const int64_t*>(L.offsets), L.n, k, epochs, cnt);
        else
            hipLaunchKernelGGL(k_add_updates<int32_t>, dim3(blocks), dim3(256), 0, c->stream,
                               static_cast<const int32_t*>(L.offsets), L.n, k, epochs, cnt);
        GOSH_HIP(hipGetLastError());
    }
}

void update_batch(Ctx* c, void* emb, gosh_dtype dt, int d, int64_t n_rows, int nsrc, const int32_t* src,
                  const int32_t* samples, int k, float lr, int32_t level, uint32_t tag, int32_t epoch) {
    check_train_args(dt, d, k, lr);
    GOSH_REQUIRE(n_rows >= 0 && nsrc >= 0 && epoch >= 0, GOSH_E_INVALID_ARG, "negative size");
    GOSH_REQUIRE(nsrc == 0 || (emb && src && samples), GOSH_E_INVALID_ARG, "null pointer");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
    if (nsrc == 0) return;
    TrainParams P = base_params(c, level, tag);
    P.emb = emb;
    P.n_rows = n_rows;
    P.n = n_rows;
    P.lr = lr;
    P.k = k;
    P.epoch = static_cast<uint32_t>(epoch);
    P.src_list = src;
    P.samples = samples;
    P.nsrc = nsrc;
    Launcher fn = pick<kExplicit>(dt, d, k, false);
    fn(P, nsrc, c->stream);
    GOSH_HIP(hipGetLastError());
}

void draw_samples(Ctx* c, const Level& L, int32_t level, int32_t epoch, int k, uint32_t tag, int32_t* out) {
    GOSH_REQUIRE(k >= 0 && k <= 15, GOSH_E_INVALID_ARG, "k must be in [0, 15]");
    GOSH_REQUIRE(epoch >= 0, GOSH_E_INVALID_ARG, "epoch must be >= 0");
    GOSH_REQUIRE(L.n == 0 || out, GOSH_E_INVALID_ARG, "null output");
    if (L.n == 0) return;
    TrainParams P = base_params(c, level, tag);
    P.offsets = L.offsets;
    P.indices = L.indices;
    P.n = L.n;
    P.k = k;
    P.epoch = static_cast<uint32_t>(epoch);
    const unsigned blocks = static_cast<unsigned>(ceil_div(L.n, 256));
    if (L.off64) hipLaunchKernelGGL(k_draw<int64_t>, dim3(blocks), dim3(256), 0, c->stream, P, out);
    else hipLaunchKernelGGL(k_draw<int32_t>, dim3(blocks), dim3(256), 0, c->stream, P, out);
    GOSH_HIP(hipGetLastError());
}

}  // namespace gosh
