// Per-source visit of TrainInGPU (Algorithm 3) with UpdateEmbed (Algorithm 1)
// for gfx950: the row layout, the row access with its write discipline and
// the update chain shared by the per-epoch, batched, partitioned and
// random-walk trainers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_util.hpp"

namespace gosh {
namespace train_detail {


constexpr int kBlock = 256;   // 4 waves

struct TrainParams {
    const void* offsets;
    const int32_t* indices;
    int64_t n;                // vertices of the level (negatives are drawn from [0, n))
    int64_t nnz;              // entries of the level's CSR
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
    // epochs in one launch (kEpoch mode): slot s runs epoch epoch + s / n with
    // lr0 * max(1 - epoch / e_total, 1e-4); span 1 uses epoch and lr as given
    int32_t span;
    int32_t e_total;
    float lr0;
    int32_t plain_neg;        // negatives written with plain stores instead of atomic adds
    // rows of degree below light_below written with plain stores (sources,
    // positives and negatives alike), 0 for none; the host sets it to
    // floor(nnz / n) + 1, so light rows are the complement of Section 4.1's
    // hubs (deg * n <= nnz), and hub rows keep their atomic commits
    int64_t light_below;
    const uint32_t* hub_bits; // with light_below > 0: bit v set iff deg(v) >= light_below
    int32_t* record;          // optional: samples drawn by each visit, [n][1+k]
    double* loss;             // optional: running loss per epoch of the launch (index = epoch - first)
};

enum Mode { kEpoch = 0, kExplicit = 1, kSequential = 2, kPersistent = 3, kLds = 4, kTable = 5 };

// Lane layout of a d-wide row.  A group of L lanes serves one row; lane gl
// owns the 32-bit words gl + L*i, i < WPL (FP32: one element per word, BF16:
// two), so every load and atomic instruction of a group covers one contiguous
// run of L words.  The L2 atomic units take at most 64 bytes of a wave
// instruction per request and sustain about 20 G requests/s next to about
// 330 G atomic words/s, so a row is split over up to 16 lanes: rows of at
// most 16 words take a single request per update (d = 8, 16, 32 in BF16),
// wider rows stay at the word limit.  L is also a multiple of d/8, the number
// of 4-word Philox blocks of a row's rounding bits, so every lane draws one
// block per row update.
template <bool BF16, int D>
struct Lanes {
    static constexpr int kWords = BF16 ? D / 2 : D;          // 32-bit words per row
    static constexpr int kWide = D / 8 > 16 ? D / 8 : 16;
    static constexpr int kL = kWords < kWide ? kWords : kWide;  // lanes per row
    static constexpr int kWPL = kWords / kL;                  // words per lane
    static constexpr int kEPL = BF16 ? 2 * kWPL : kWPL;       // elements per lane
    static constexpr int kG = 64 / kL;                        // rows (sources) per wave
    static constexpr int kBlocks = D / 8;                     // Philox blocks of rounding bits
    static_assert(kL * kWPL == kWords && kL % kBlocks == 0 && 64 % kL == 0, "row layout");
};

// Row access.
//
// Writes are atomic: sources of an epoch run concurrently and share rows, and
// a plain read-modify-write store would drop every concurrent update but the
// last one -- on small levels, where a whole epoch is in flight at once,
// nearly all of them.  FP32 rows receive their changes with atomic adds.
// BF16 rows: per 32-bit word (two elements), the change from the pair this
// visit started from (cur) to the stochastically rounded new pair (out).
// When both differences out - cur are BF16 values (so cur + diff is exactly
// out), the word takes the packed BF16 atomic add of the differences:
// uncontended it becomes exactly out, contended the concurrent changes add
// up in value space.  Otherwise (a difference needs more than 8 significant
// bits: a sign crossing, or a change much larger or much smaller than the
// element) one packed add would round the difference and then the sum, so
// that half takes two adds through zero instead, -cur then +out, each exact
// (x - x = 0 and 0 + out = out); a concurrent add landing between them still
// adds up, and a concurrent reader may meanwhile see 0, which lies within
// |out - cur| of both ends for these halves.  Uncontended, every word of a
// committed row therefore holds exactly the stochastically rounded result,
// and no commit waits for a returned value.  (Adding
// bit-pattern differences with integer atomics would be faster but wraps
// through the sign when many concurrent updates move one element across
// zero.)  The L2 atomic units bound the training kernel.
template <bool BF16>
struct RowIO;

template <>
struct RowIO<false> {
    using Elem = float;
    template <int D, bool COH>
    __device__ static void load(const float* M, int64_t row, int gl, float (&x)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        const float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i) {
            if constexpr (COH)
                x[i] = __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t*>(p + L * i),
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            else
                x[i] = p[L * i];
        }
    }
    template <int D>
    __device__ static void store(float* M, int64_t row, int gl, const float (&x)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i) p[L * i] = x[i];
    }
    template <int D>
    __device__ static void add(float* M, int64_t row, int gl, const float (&dx)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i)
            __hip_atomic_fetch_add(p + L * i, dx[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

typedef __bf16 __attribute__((ext_vector_type(2))) bf16x2_t;

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void atomic_add_bf16x2(uint32_t* p, uint32_t d) {
    __builtin_amdgcn_global_atomic_fadd_v2bf16((__attribute__((address_space(1))) bf16x2_t*)p,
                                               __builtin_bit_cast(bf16x2_t, d));
}

// BF16 rows are held in registers as their 32-bit words (two elements each,
// low half the even element) and widened to FP32 where the arithmetic reads
// them, which halves the registers a visit's 1+k sample rows take.
template <>
struct RowIO<true> {
    using Elem = uint16_t;
    template <int D, bool COH>
    __device__ static void load(const uint16_t* M, int64_t row, int gl, uint32_t (&w)[Lanes<true, D>::kWPL]) {
        constexpr int L = Lanes<true, D>::kL;
        const uint32_t* p = reinterpret_cast<const uint32_t*>(M + row * D) + gl;
#pragma unroll
        for (int i = 0; i < Lanes<true, D>::kWPL; ++i) {
            if constexpr (COH)
                w[i] = __hip_atomic_load(p + L * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                w[i] = p[L * i];
        }
    }
    // cur: the words this visit last saw, v: the FP32 results, r: the lane's
    // Philox block (block gl mod d/8 of the row).  Word w of the row takes
    // 32-bit output word w div (d/8) of its block (low half for the even
    // element).  out: the rounded words.
    // PLAIN: store the rounded words instead of committing the change.
    template <int D, bool PLAIN = false>
    __device__ static void commit(uint16_t* M, int64_t row, int gl, const uint32_t (&cur)[Lanes<true, D>::kWPL],
                                  const float (&v)[Lanes<true, D>::kEPL], uint4 r,
                                  uint32_t (&out)[Lanes<true, D>::kWPL]) {
        using Ly = Lanes<true, D>;
        constexpr int L = Ly::kL;
        uint32_t* p = reinterpret_cast<uint32_t*>(M + row * D) + gl;
        const int q0 = gl / Ly::kBlocks;
#pragma unroll
        for (int i = 0; i < Ly::kWPL; ++i) {
            // output word q of the block, selected without indexing a
            // register array by a lane-dependent value (that would go to scratch)
            const int q = q0 + i * (L / Ly::kBlocks);
            const uint32_t bits = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
            const uint32_t t0 = bf16_sr(v[2 * i], bits & 0xFFFFu);
            const uint32_t t1 = bf16_sr(v[2 * i + 1], bits >> 16);
            const uint32_t want = (t0 & 0xFFFFu) | (t1 << 16);
            out[i] = want;
            if constexpr (PLAIN) {
                p[L * i] = want;
            } else {
                // per half: the exact rounded difference in one add, or,
                // when out - cur is not a BF16 value, two exact adds through
                // zero (-cur, then +out)
                // the FP32 difference of two BF16 values is exact unless
                // their exponents lie far apart; it is a BF16 value when its
                // low half is zero, and then adding it back gives out again
                const float c0 = bf16_lo(cur[i]), c1 = bf16_hi(cur[i]);
                const float o0 = bf16_lo(want), o1 = bf16_hi(want);
                const float d0 = o0 - c0, d1 = o1 - c1;
                const uint32_t h0 = __float_as_uint(d0) >> 16, h1 = __float_as_uint(d1) >> 16;
                const bool x0 = (__float_as_uint(d0) & 0xFFFFu) == 0u && c0 + d0 == o0;
                const bool x1 = (__float_as_uint(d1) & 0xFFFFu) == 0u && c1 + d1 == o1;
                const uint32_t a = (x0 ? h0 : (cur[i] & 0xFFFFu) ^ 0x8000u) |
                                   ((x1 ? h1 : (cur[i] >> 16) ^ 0x8000u) << 16);
                const uint32_t b2 = (x0 ? 0u : want & 0xFFFFu) | (x1 ? 0u : want & 0xFFFF0000u);
                if ((a & 0x7FFF7FFFu) != 0u) atomic_add_bf16x2(p + L * i, a);
                if ((b2 & 0x7FFF7FFFu) != 0u) atomic_add_bf16x2(p + L * i, b2);
            }
        }
    }
};

// Rows held in one workgroup's LDS (a level or job trained inside a single
// workgroup): the same interface as RowIO, with the workgroup as the only
// writer.  FP32 changes are LDS atomic adds; a BF16 word is committed by
// compare-and-swap: uncontended it becomes exactly the stochastically
// rounded pair, and a half that another wave changed in the meantime gets
// this visit's change v - cur added to its current value and rounded again
// with the same bits (LDS swaps take a few cycles, so the loop is cheap).
template <bool BF16>
struct LdsRowIO;

template <>
struct LdsRowIO<false> {
    using Elem = float;
    template <int D, bool COH>
    __device__ static void load(const float* M, int64_t row, int gl, float (&x)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        const float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i) x[i] = p[L * i];
    }
    template <int D>
    __device__ static void store(float* M, int64_t row, int gl, const float (&x)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i) p[L * i] = x[i];
    }
    template <int D>
    __device__ static void add(float* M, int64_t row, int gl, const float (&dx)[Lanes<false, D>::kEPL]) {
        constexpr int L = Lanes<false, D>::kL;
        float* p = M + row * D + gl;
#pragma unroll
        for (int i = 0; i < Lanes<false, D>::kWPL; ++i)
            __hip_atomic_fetch_add(p + L * i, dx[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

template <>
struct LdsRowIO<true> {
    using Elem = uint16_t;
    template <int D, bool COH>
    __device__ static void load(const uint16_t* M, int64_t row, int gl, uint32_t (&w)[Lanes<true, D>::kWPL]) {
        constexpr int L = Lanes<true, D>::kL;
        const uint32_t* p = reinterpret_cast<const uint32_t*>(M + row * D) + gl;
#pragma unroll
        for (int i = 0; i < Lanes<true, D>::kWPL; ++i) w[i] = p[L * i];
    }
    template <int D, bool PLAIN = false>
    __device__ static void commit(uint16_t* M, int64_t row, int gl, const uint32_t (&cur)[Lanes<true, D>::kWPL],
                                  const float (&v)[Lanes<true, D>::kEPL], uint4 r,
                                  uint32_t (&out)[Lanes<true, D>::kWPL]) {
        using Ly = Lanes<true, D>;
        constexpr int L = Ly::kL;
        uint32_t* p = reinterpret_cast<uint32_t*>(M + row * D) + gl;
        const int q0 = gl / Ly::kBlocks;
#pragma unroll
        for (int i = 0; i < Ly::kWPL; ++i) {
            const int q = q0 + i * (L / Ly::kBlocks);
            const uint32_t bits = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
            const uint32_t t0 = bf16_sr(v[2 * i], bits & 0xFFFFu) & 0xFFFFu;
            const uint32_t t1 = bf16_sr(v[2 * i + 1], bits >> 16) & 0xFFFFu;
            const uint32_t want = t0 | (t1 << 16);
            out[i] = want;
            uint32_t expected = cur[i];
            uint32_t desired = want;
            // bounded: a word changes at most once per other visit in flight
            for (int it = 0; it < 1024; ++it) {
                if (__hip_atomic_compare_exchange_strong(p + L * i, &expected, desired, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                const uint32_t h0 = expected & 0xFFFFu, h1 = expected >> 16;
                const uint32_t s0 = cur[i] & 0xFFFFu, s1 = cur[i] >> 16;
                const uint32_t n0 = h0 == s0 ? t0
                                             : bf16_sr(bf16_lo(h0) + (v[2 * i] - bf16_lo(s0)), bits & 0xFFFFu) & 0xFFFFu;
                const uint32_t n1 = h1 == s1 ? t1
                                             : bf16_sr(bf16_lo(h1) + (v[2 * i + 1] - bf16_lo(s1)), bits >> 16) & 0xFFFFu;
                desired = n0 | (n1 << 16);
            }
        }
    }
};

__device__ __forceinline__ float sigmoidf_(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}

// softplus(z) = log(1 + e^z) in FP32: the logistic loss of Section 2 is
// softplus(-x) for a positive (-log sigma(x)) and softplus(x) for a negative
// (-log(1 - sigma(x))).
__device__ __forceinline__ float softplusf_(float z) {
    return fmaxf(z, 0.0f) + __logf(1.0f + __expf(-fabsf(z)));
}

// UpdateEmbed (Algorithm 1) on samples u[0..k] of one source, u[0] the
// positive: the source row (row `src` of Ms) is updated in registers along
// the chain and written back once at the end; the samples are rows of Mo.
// Samples that are -1 or equal to `self` (the source's index in Mo, -1 if it
// has none) are skipped; a skipped negative is subtracted from `updates`,
// which the callers precount.  BF16 rounding bits come from the stream (sid,
// epoch, w2, kind sr_kind | slot t or 255 | block blk_hi << 8 | gl mod d/8).
// COH: loads bypass the non-coherent caches (rows written by other waves of
// the same launch).  plain: rows written with plain stores of the new values
// instead of atomic commits of the change (bit t sample slot t, bit 31 the
// source).  Returns, when want_loss, the visit's running loss: the
// Section 2 objective of each executed update at the dot it reads (the same
// value on every lane of the group); 0 otherwise.
// HUB: the positive (u[0]) is a hub row held by the workgroup: its words
// are read from hub_words (LDS, the row's layout) and its change is added to
// hub_delta (LDS, FP32 per element) instead of being committed; the caller
// commits the summed change once.
template <bool BF16, int D, int KMAX, bool COH, class IO = RowIO<BF16>, bool HUB = false>
__device__ __forceinline__ float update_chain(typename RowIO<BF16>::Elem* Ms, int64_t src,
                                              typename RowIO<BF16>::Elem* Mo, int64_t self,
                                              const int32_t (&u)[KMAX + 1], int k, float lr, uint32_t sid,
                                              uint32_t epoch, uint32_t w2, uint32_t sr_kind, uint32_t blk_hi,
                                              uint32_t key0, uint32_t key1, unsigned long long* updates, int gl,
                                              uint32_t plain = 0u, bool want_loss = false,
                                              const uint32_t* hub_words = nullptr, float* hub_delta = nullptr) {
    using Ly = Lanes<BF16, D>;
    constexpr int L = Ly::kL;
    constexpr int E = Ly::kEPL;
    constexpr int W = Ly::kWPL;
    const uint32_t blk = (blk_hi << 8) | static_cast<uint32_t>(gl % Ly::kBlocks);
    int done = 0;
    float lsum = 0.0f;
    if constexpr (BF16) {
        // rows as packed BF16 words; element 2i is the low half of word i
        uint32_t sw[W];
        uint32_t mw[KMAX + 1][W];
        IO::template load<D, COH>(Ms, src, gl, sw);
#pragma unroll
        for (int t = 0; t <= KMAX; ++t) {
            if (HUB && t == 0) {
#pragma unroll
                for (int i = 0; i < W; ++i) mw[0][i] = hub_words[gl + L * i];
            } else if (t <= k && u[t] >= 0 && u[t] != self) {
                IO::template load<D, COH>(Mo, u[t], gl, mw[t]);
            } else {
#pragma unroll
                for (int i = 0; i < W; ++i) mw[t][i] = 0u;
            }
        }
        float s[E];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            s[2 * i] = bf16_lo(sw[i]);
            s[2 * i + 1] = bf16_hi(sw[i]);
        }
#pragma unroll
        for (int t = 0; t <= KMAX; ++t) {
            if (t > k) break;
            const int32_t ut = u[t];
            if (ut < 0 || ut == self) {
                if (t > 0 && ut >= 0 && ut == self && updates && gl == 0) atomicAdd(updates, ~0ull);  // -1
                continue;
            }
            // a row sampled earlier in this visit continues from its updated value
#pragma unroll
            for (int tp = 0; tp < t; ++tp) {
                if (u[tp] == ut) {
#pragma unroll
                    for (int i = 0; i < W; ++i) mw[t][i] = mw[tp][i];
                }
            }
            float x = 0.0f;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                x = fmaf(s[2 * i], bf16_lo(mw[t][i]), x);
                x = fmaf(s[2 * i + 1], bf16_hi(mw[t][i]), x);
            }
            x = group_sum<L>(x);
            const float b = (t == 0) ? 1.0f : 0.0f;
            const float g = (b - sigmoidf_(x)) * lr;
            if (want_loss) lsum += softplusf_(t == 0 ? -x : x);
#pragma unroll
            for (int i = 0; i < W; ++i) {
                s[2 * i] = fmaf(g, bf16_lo(mw[t][i]), s[2 * i]);
                s[2 * i + 1] = fmaf(g, bf16_hi(mw[t][i]), s[2 * i + 1]);
            }
            const uint4 bits = philox10(
                make_uint4(sid, epoch, w2, stream_word3(sr_kind, static_cast<uint32_t>(t), blk)), key0, key1);
            float v[E];
#pragma unroll
            for (int i = 0; i < W; ++i) {
                v[2 * i] = fmaf(g, s[2 * i], bf16_lo(mw[t][i]));
                v[2 * i + 1] = fmaf(g, s[2 * i + 1], bf16_hi(mw[t][i]));
            }
            if (HUB && t == 0) {
                // the hub's change, summed over the workgroup's visits
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    atomicAdd(&hub_delta[2 * (gl + L * i)], v[2 * i] - bf16_lo(mw[0][i]));
                    atomicAdd(&hub_delta[2 * (gl + L * i) + 1], v[2 * i + 1] - bf16_hi(mw[0][i]));
                }
                ++done;
                continue;
            }
            uint32_t out[W];
            if ((plain >> t) & 1u) IO::template commit<D, true>(Mo, ut, gl, mw[t], v, bits, out);
            else IO::template commit<D>(Mo, ut, gl, mw[t], v, bits, out);
#pragma unroll
            for (int i = 0; i < W; ++i) mw[t][i] = out[i];
            ++done;
        }
        if (done) {
            const uint4 bits = philox10(make_uint4(sid, epoch, w2, stream_word3(sr_kind, 0xFFu, blk)), key0, key1);
            uint32_t out[W];
            if (plain >> 31) IO::template commit<D, true>(Ms, src, gl, sw, s, bits, out);
            else IO::template commit<D>(Ms, src, gl, sw, s, bits, out);
        }
    } else {
        float s[E];
        float m[KMAX + 1][E];
        IO::template load<D, COH>(Ms, src, gl, s);
#pragma unroll
        for (int t = 0; t <= KMAX; ++t) {
            if (HUB && t == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) m[0][e] = __uint_as_float(hub_words[gl + L * e]);
            } else if (t <= k && u[t] >= 0 && u[t] != self) {
                IO::template load<D, COH>(Mo, u[t], gl, m[t]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) m[t][e] = 0.0f;
            }
        }
        float s0[E];
#pragma unroll
        for (int e = 0; e < E; ++e) s0[e] = s[e];
#pragma unroll
        for (int t = 0; t <= KMAX; ++t) {
            if (t > k) break;
            const int32_t ut = u[t];
            if (ut < 0 || ut == self) {
                if (t > 0 && ut >= 0 && ut == self && updates && gl == 0) atomicAdd(updates, ~0ull);  // -1
                continue;
            }
            // a row sampled earlier in this visit continues from its updated value
#pragma unroll
            for (int tp = 0; tp < t; ++tp) {
                if (u[tp] == ut) {
#pragma unroll
                    for (int e = 0; e < E; ++e) m[t][e] = m[tp][e];
                }
            }
            float x = 0.0f;
#pragma unroll
            for (int e = 0; e < E; ++e) x = fmaf(s[e], m[t][e], x);
            x = group_sum<L>(x);
            const float b = (t == 0) ? 1.0f : 0.0f;
            const float g = (b - sigmoidf_(x)) * lr;
            if (want_loss) lsum += softplusf_(t == 0 ? -x : x);
#pragma unroll
            for (int e = 0; e < E; ++e) s[e] = fmaf(g, m[t][e], s[e]);
            float dx[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                // not contracted: the row in registers is the rounded change
                // added to the row, the value an uncontended atomic add leaves
#pragma clang fp contract(off)
                dx[e] = g * s[e];
                m[t][e] += dx[e];
            }
            if (HUB && t == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) atomicAdd(&hub_delta[gl + L * e], dx[e]);
            } else if ((plain >> t) & 1u) {
                IO::template store<D>(Mo, ut, gl, m[t]);
            } else {
                IO::template add<D>(Mo, ut, gl, dx);
            }
            ++done;
        }
        if (done) {
            float dx[E];
#pragma unroll
            for (int e = 0; e < E; ++e) dx[e] = s[e] - s0[e];
            if (plain >> 31) {
                // the value an uncontended atomic add of dx leaves
#pragma unroll
                for (int e = 0; e < E; ++e) s[e] = s0[e] + dx[e];
                IO::template store<D>(Ms, src, gl, s);
            } else {
                IO::template add<D>(Ms, src, gl, dx);
            }
        }
    }
    return lsum;
}

// One source visit: draws (or reads) the samples and applies the updates.
// Returns the visit's running loss when P.loss is set (see update_chain), 0
// for an inactive slot.  With P.record set, the drawn samples are written to
// record[src * (1 + k) + t].
template <bool BF16, int D, int KMAX, class Off, int MODE, class IO = RowIO<BF16>>
__device__ __forceinline__ float visit(const TrainParams& P, int64_t slot, bool active, int gl) {
    using Elem = typename RowIO<BF16>::Elem;
    Elem* M = static_cast<Elem*>(P.emb);
    const int k = P.k;

    int64_t src = slot;
    uint32_t plain = 0u;   // rows stored plainly: bit t sample slot t, bit 31 the source
    int32_t u[KMAX + 1];
#pragma unroll
    for (int t = 0; t <= KMAX; ++t) u[t] = -1;

    if constexpr (MODE == kLds || MODE == kTable) {
        // the epoch's samples were drawn into the table P.samples beforehand;
        // in kTable a first entry below -1 marks a visit another pass takes
        if (active) {
#pragma unroll
            for (int t = 0; t <= KMAX; ++t)
                if (t <= k) u[t] = P.samples[slot * (1 + k) + t];
            if (MODE == kTable && u[0] < -1) active = false;
        }
    } else if constexpr (MODE == kExplicit) {
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
            // a malformed row is treated as empty instead of read out of bounds
            const int64_t deg = (beg >= 0 && beg <= end && end <= P.nnz) ? end - beg : 0;
#pragma unroll
            for (int t = 1; t <= KMAX; ++t)
                if (t <= k) u[t] = static_cast<int32_t>(scale_u32(wd[t], P.n));
            if (deg > 0) {
                const int32_t pos = P.indices[beg + scale_u32(wd[0], deg)];
                u[0] = (pos >= 0 && pos < P.n) ? pos : -1;
            }
            if (P.record && gl == 0) {
#pragma unroll
                for (int t = 0; t <= KMAX; ++t)
                    if (t <= k) P.record[src * (1 + k) + t] = u[t];
            }
            if constexpr (MODE == kEpoch || MODE == kSequential) {
                if (P.light_below > 0) {
                    // light rows are stored plainly; a sample's class comes
                    // from the level's hub bitmap (n / 8 bytes, cache-resident),
                    // read beside the row loads of the chain
                    if (deg < P.light_below) plain |= 1u << 31;
#pragma unroll
                    for (int t = 0; t <= KMAX; ++t) {
                        if (t <= k && u[t] >= 0) {
                            const uint32_t w = P.hub_bits[static_cast<uint32_t>(u[t]) >> 5];
                            if (((w >> (static_cast<uint32_t>(u[t]) & 31u)) & 1u) == 0u) plain |= 1u << t;
                        }
                    }
                }
            }
        }
    }
    if (!active) return 0.0f;
    if ((MODE == kEpoch || MODE == kExplicit || MODE == kSequential || MODE == kTable) && P.plain_neg != 0)
        plain |= ((2u << KMAX) - 1u) & ~1u;   // every negative slot
    return update_chain<BF16, D, KMAX, MODE == kPersistent, IO>(
        M, src, M, src, u, k, P.lr, static_cast<uint32_t>(src), P.epoch, P.w2, 1u, 0u, P.key0, P.key1, P.updates,
        gl, plain, P.loss != nullptr);
}

// Samples of source `src` in epoch P.epoch (kind 0 of the Philox stream), as
// the per-epoch kernel draws them: out[0] the positive (-1 without
// neighbours), out[t] negative t.
template <class Off>
__device__ __forceinline__ void draw_source(const TrainParams& P, int64_t src, int32_t* out) {
    const Off* off = static_cast<const Off*>(P.offsets);
    const int64_t beg = off[src], end = off[src + 1];
    const int64_t deg = (beg >= 0 && beg <= end && end <= P.nnz) ? end - beg : 0;
    for (int b = 0; 4 * b <= P.k; ++b) {
        const uint4 r = philox10(make_uint4(static_cast<uint32_t>(src), P.epoch, P.w2, stream_word3(0, 0, b)),
                                 P.key0, P.key1);
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
        for (int j = 0; j < 4; ++j) {
            const int t = 4 * b + j;
            if (t > P.k) break;
            int32_t v;
            if (t == 0) {
                v = -1;
                if (deg > 0) {
                    const int32_t pos = P.indices[beg + scale_u32(w[0], deg)];
                    v = (pos >= 0 && pos < P.n) ? pos : -1;
                }
            } else {
                v = static_cast<int32_t>(scale_u32(w[j], P.n));
            }
            out[t] = v;
        }
    }
}

// Adds the running losses of the wave's groups (`l` on every lane of a
// group, L lanes per group) to *dst: an FP32 sum over the wave, one FP64
// atomic add per wave.
template <int L>
__device__ __forceinline__ void wave_add_loss(double* dst, float l, int gl) {
    float v = (gl == 0) ? l : 0.0f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v != 0.0f)
        __hip_atomic_fetch_add(dst, static_cast<double>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kLdsBlock = 1024;   // one workgroup of 16 waves trains a level held in LDS

// LDS bytes a level trained in one workgroup needs: its rows plus the
// sample table of one epoch.
__host__ __device__ constexpr int64_t lds_level_bytes(int64_t n, int d, int elem_bytes, int k) {
    return n * d * elem_bytes + n * (1 + k) * 4;
}

// Trains all P.e_total epochs of one level (or batched job) inside the
// calling workgroup of kLdsBlock threads, its rows held in `lds` (the LDS
// hot copy: read from HBM once, written back once).  Every epoch first draws
// the samples of all sources into an LDS table (all threads at once, the
// same Philox draws as the per-epoch kernel), then the waves visit the
// sources with the update chain on the LDS rows, a workgroup barrier after
// each phase: Algorithm 3's epochs in order, the sources of an epoch
// concurrent over the workgroup's 16 waves.  lr' = P.lr0 max(1 - j/e, 1e-4).
template <bool BF16, int D, int KMAX, class Off>
__device__ __forceinline__ void train_rows_in_lds(TrainParams P, unsigned char* lds) {
    using Elem = typename RowIO<BF16>::Elem;
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const int wave = threadIdx.x >> 6;
    Elem* rows = reinterpret_cast<Elem*>(lds);
    int32_t* table = reinterpret_cast<int32_t*>(lds + P.n * D * sizeof(Elem));
    const int64_t words = P.n * D * static_cast<int64_t>(sizeof(Elem)) / 4;
    uint32_t* glob = static_cast<uint32_t*>(P.emb);
    for (int64_t i = threadIdx.x; i < words; i += kLdsBlock) reinterpret_cast<uint32_t*>(rows)[i] = glob[i];
    __syncthreads();
    TrainParams Q = P;
    Q.emb = rows;
    Q.samples = table;
    for (int j = 0; j < P.e_total; ++j) {
        Q.epoch = static_cast<uint32_t>(j);
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(P.e_total);
        Q.lr = static_cast<float>(static_cast<double>(P.lr0) * (f > 1e-4 ? f : 1e-4));
        Q.loss = P.loss ? P.loss + j : nullptr;
        for (int64_t v = threadIdx.x; v < P.n; v += kLdsBlock) {
            draw_source<Off>(Q, v, table + v * (1 + P.k));
            if (Q.record) {
                for (int t = 0; t <= P.k; ++t) Q.record[v * (1 + P.k) + t] = table[v * (1 + P.k) + t];
            }
        }
        __syncthreads();
        for (int64_t base = static_cast<int64_t>(wave) * G; base < P.n; base += (kLdsBlock / 64) * G) {
            const int64_t slot = base + grp;
            const float l = visit<BF16, D, KMAX, Off, kLds, LdsRowIO<BF16>>(Q, slot, slot < P.n, gl);
            if (Q.loss) wave_add_loss<L>(Q.loss, l, gl);
        }
        __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < words; i += kLdsBlock) glob[i] = reinterpret_cast<uint32_t*>(rows)[i];
}

}  // namespace train_detail
}  // namespace gosh
