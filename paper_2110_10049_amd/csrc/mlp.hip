// Learned prolongation: a two-layer network that predicts a fine row from
// the coarse row ExpandEmbedding (Algorithm 2) would copy,
//
//   x = [c, log1p(deg(v)), log(clsz(map v))],  c = coarse[map v]   (d + 2)
//   y = c + W2 GELU(W1 x + b1) + b2,
//
// so W2 = 0, b2 = 0 is copy prolongation.  BF16 MFMA (16x16x32) with FP32
// accumulation; FP32 master weights, biases added in FP32; Adam on the
// master weights.
//
// Layout of the products.  Both layers are computed transposed, weights as
// the A operand and batch rows as the B operand: Z1^T = W1 X^T and
// Y^T = W2 A1^T.  A wave owns NT*16 batch rows; lane l of a 16x16 tile
// holds batch row l%16.  The X operand is then eight consecutive features
// of one row, a single 16-byte load from the coarse row; the layer-1
// result already sits in registers in the layout the layer-2 B operand
// needs, once the K order of W2 is permuted to match (a contraction is
// invariant under a common permutation of K in both operands).  Weights
// are stored pre-packed in operand order ("fragments": 64 lanes x 16 B per
// 16x32 tile), so staging them into LDS is a linear copy and every operand
// read is one conflict-free 16-byte LDS load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.hpp"
#include "gosh_internal.hpp"


namespace gosh {
namespace mlp_detail {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr float kRsqrt2 = 0.70710678118654752f;
constexpr float kRsqrt2Pi = 0.39894228040143268f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr int kLdsLimitFrags = 160;        // 16x32 BF16 fragments (1 KiB each) that fit in LDS
constexpr int kFwdThreads = 512;      // forward blocks for d = 256 (two row tiles per wave)
constexpr int kFwdThreadsWide = 1024; // forward blocks for d <= 128 (one row tile per wave)
constexpr int kTrainThreads = 256;

// ------------------------------------------------------------ shapes
struct Shape {
    int D, H;
    int F() const { return D + 2; }
    int K1() const { return D + 32; }                       // D + 2 padded to 32
    int64_t nparams() const { return int64_t(H) * F() + H + int64_t(D) * H + D; }
    int64_t off_b1() const { return int64_t(H) * F(); }
    int64_t off_w2() const { return off_b1() + H; }
    int64_t off_b2() const { return off_w2() + int64_t(D) * H; }
    int64_t w1f_elems() const { return int64_t(H) * K1(); }
    int64_t w2f_elems() const { return int64_t(D) * H; }
};

// ------------------------------------------------------------ scalar helpers
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (one v_cvt_pk_bf16_f32 per pair)
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    bf16x2 v;
    v[0] = static_cast<__bf16>(lo);
    v[1] = static_cast<__bf16>(hi);
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint32_t f2bf(float x) { return pack2(x, 0.0f) & 0xFFFFu; }

// Lower tail Phi(-|z|) = erfc(|z| / sqrt 2) / 2 from the complementary error
// function of Abramowitz and Stegun, Handbook of Mathematical Functions,
// 7.1.26 (absolute error of erf at most 1.5e-7): for x >= 0,
// erfc(x) ~= t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), t = 1 / (1 + p x),
// here with x = |z| / sqrt 2 and the factor 1/2 folded into the a_i.  Also
// returns exp(-z^2 / 2), which the derivative of GELU reuses.
__device__ __forceinline__ float phi_lower(float z, float& ez) {
    constexpr float kP = 0.3275911f * kRsqrt2;
    constexpr float c1 = 0.5f * 0.254829592f, c2 = 0.5f * -0.284496736f, c3 = 0.5f * 1.421413741f,
                    c4 = 0.5f * -1.453152027f, c5 = 0.5f * 1.061405429f;
    constexpr float kNegHalfLog2e = -0.72134752044448170f;   // -log2(e) / 2
    const float t = __builtin_amdgcn_rcpf(fmaf(fabsf(z), kP, 1.0f));
    const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, c5, c4), c3), c2), c1);
    ez = __builtin_amdgcn_exp2f((z * z) * kNegHalfLog2e);
    return poly * ez;
}
// GELU(z) = z Phi(z) (Hendrycks and Gimpel); GELU'(z) = Phi(z) + z exp(-z^2/2) / sqrt(2 pi).

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// K position (q, j) of a lane group q (= lane/16) and element j -> index in
// a 32-wide K block, for operands whose K block is made of two 16-row
// accumulator tiles (rows 4q..4q+3 of each).
__host__ __device__ __forceinline__ int perm_k(int q, int j) { return j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4); }
// inverse: column c of a 32-wide block -> (q, j)
__host__ __device__ __forceinline__ void perm_inv(int c, int& q, int& j) {
    if (c < 16) { q = c >> 2; j = c & 3; }
    else { q = (c - 16) >> 2; j = 4 + ((c - 16) & 3); }
}

// ------------------------------------------------------------ row sources
// Where batch row r takes its coarse row, degree and cluster size from.
// Level form: coarse index map[r], degree from the fine level's offsets,
// cluster size clsz[map[r]].  Batch form (map == nullptr): coarse index r,
// deg[r], clsz[r].
struct RowSrc {
    const void* coarse;
    const int32_t* map;
    const void* offsets;
    int off64;
    const int32_t* deg;
    const int32_t* clsz;
    int64_t rows;
};

template <bool BF16>
__device__ __forceinline__ u32x4 load_row8(const void* rows, int64_t r, int D, int f0) {
    if constexpr (BF16) {
        return *reinterpret_cast<const u32x4*>(static_cast<const uint16_t*>(rows) + r * D + f0);
    } else {
        const float* p = static_cast<const float*>(rows) + r * D + f0;
        const f32x4 a = *reinterpret_cast<const f32x4*>(p);
        const f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
        return u32x4{pack2(a[0], a[1]), pack2(a[2], a[3]), pack2(b[0], b[1]), pack2(b[2], b[3])};
    }
}

template <bool BF16>
__device__ __forceinline__ f32x4 load_row4(const void* rows, int64_t r, int D, int f0) {
    if constexpr (BF16) {
        const u32x2 w = *reinterpret_cast<const u32x2*>(static_cast<const uint16_t*>(rows) + r * D + f0);
        return f32x4{bf16_lo(w[0]), bf16_hi(w[0]), bf16_lo(w[1]), bf16_hi(w[1])};
    } else {
        return *reinterpret_cast<const f32x4*>(static_cast<const float*>(rows) + r * D + f0);
    }
}

template <bool BF16>
__device__ __forceinline__ void store_row4(void* rows, int64_t r, int D, int f0, f32x4 y) {
    if constexpr (BF16) {
        *reinterpret_cast<u32x2*>(static_cast<uint16_t*>(rows) + r * D + f0) =
            u32x2{pack2(y[0], y[1]), pack2(y[2], y[3])};
    } else {
        *reinterpret_cast<f32x4*>(static_cast<float*>(rows) + r * D + f0) = y;
    }
}

// B-operand fragments of X for NT row tiles starting at `base`: xf[nt][kb]
// holds features kb*32 + 8q .. +7 of row base + 16 nt + l%16.
template <int D, int NT, bool BF16>
__device__ __forceinline__ void load_x(const RowSrc& S, int64_t base, int lane, u32x4 (&xf)[NT][D / 32 + 1],
                                       int64_t (&cid)[NT], bool (&ok)[NT]) {
    constexpr int KB1 = D / 32 + 1;
    const int r16 = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t r = base + nt * 16 + r16;
        ok[nt] = r < S.rows;
        cid[nt] = ok[nt] ? (S.map ? static_cast<int64_t>(S.map[r]) : r) : 0;
        float fdeg = 0.0f, fcs = 0.0f;
        if (ok[nt] && q == 0) {
            int64_t deg;
            if (S.offsets) {
                deg = S.off64 ? static_cast<const int64_t*>(S.offsets)[r + 1] - static_cast<const int64_t*>(S.offsets)[r]
                              : static_cast<int64_t>(static_cast<const int32_t*>(S.offsets)[r + 1] -
                                                     static_cast<const int32_t*>(S.offsets)[r]);
            } else {
                deg = S.deg[r];
            }
            // ln(deg + 1) and ln(clsz) of integers >= 1 through the hardware
            // base-2 logarithm (a few FP32 ulps; the features are rounded
            // to BF16 next); a degree fits in 32 bits (indices are int32)
            fdeg = __builtin_amdgcn_logf(static_cast<float>(static_cast<int32_t>(deg) + 1)) * kLn2;
            fcs = __builtin_amdgcn_logf(static_cast<float>(S.clsz[cid[nt]])) * kLn2;
        }
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int f0 = kb * 32 + 8 * q;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (kb < KB1 - 1) {
                if (ok[nt]) v = load_row8<BF16>(S.coarse, cid[nt], D, f0);
            } else if (q == 0) {
                v[0] = pack2(fdeg, fcs);
            }
            xf[nt][kb] = v;
        }
    }
}

// One 32-wide hidden block: layer 1 for hidden rows 32 kb2 .. +31 and the
// GELU, returned as layer-2 B fragments hb[nt] (permuted K order).  w1b
// points at the block's 2 * (D/32 + 1) W1 fragments and b1b at its 32
// biases.  z, Phi(-|z|) and exp(-z^2/2) are handed to `keep` for the
// backward pass.
template <int D, int H, int NT, class WPtr, class BPtr, class Keep>
__device__ __forceinline__ void hidden_block(WPtr w1b, BPtr b1b, int kb2, int lane,
                                             const u32x4 (&xf)[NT][D / 32 + 1], u32x4 (&hb)[NT], Keep&& keep) {
    constexpr int KB1 = D / 32 + 1;
    const int q = lane >> 4;
    // the accumulators start at the bias, so z needs no add after the product
    f32x4 a1[2][NT];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const f32x4 bb = *reinterpret_cast<const f32x4*>(b1b + m * 16 + 4 * q);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) a1[m][nt] = bb;
    }
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const u32x4 w = w1b[(m * KB1 + kb) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) a1[m][nt] = mfma(w, xf[nt][kb], a1[m][nt]);
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int h0 = (2 * kb2 + m) * 16 + 4 * q;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float g[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = a1[m][nt][i];
                float ez;
                const float lo = phi_lower(z, ez);        // Phi(-|z|)
                // z Phi(z) = max(z, 0) - |z| Phi(-|z|) for either sign of z;
                // max(z, 0) as a median with a finite bound, one instruction
                // on the MFMA result with no canonicalising copy first
                g[i] = fmaf(-fabsf(z), lo, __builtin_amdgcn_fmed3f(z, 0.0f, 3.0e38f));
                keep(nt, h0 + i, z, lo, ez);
            }
            hb[nt][2 * m] = pack2(g[0], g[1]);
            hb[nt][2 * m + 1] = pack2(g[2], g[3]);
        }
    }
}

// ------------------------------------------------------------ inference
// Every wave loops over 16*NT-row tiles; W1, W2 and b1 are staged in LDS
// once per workgroup when they fit (WLDS), else read through L2.  The LDS
// copy is grouped by hidden block: W1 fragments, W2 fragments and biases of
// one block lie together, so each operand read is a constant offset from
// one block address.
template <int D, int H, int NT, bool BF16, bool WLDS, int THREADS>
__global__ __launch_bounds__(THREADS) void k_forward(RowSrc S, const u32x4* __restrict__ W1f,
                                                         const u32x4* __restrict__ W2f,
                                                         const float* __restrict__ b1,
                                                         const float* __restrict__ b2, void* __restrict__ out,
                                                         int64_t ntiles) {
    constexpr int KB1 = D / 32 + 1, KB2 = H / 32, MT2 = D / 16;
    constexpr int W1B = 2 * KB1 * 64;               // W1 fragments of one hidden block (u32x4)
    constexpr int BLK = W1B + MT2 * 64 + 8;         // + its W2 fragments + 32 biases
    __shared__ u32x4 lds[WLDS ? KB2 * BLK + D / 4 : 1];
    const float* bias2 = b2;
    if constexpr (WLDS) {
        for (int i = threadIdx.x; i < KB2 * BLK; i += blockDim.x) {
            const int b = i / BLK, o = i - b * BLK;
            u32x4 v;
            if (o < W1B) {
                v = W1f[b * W1B + o];
            } else if (o < W1B + MT2 * 64) {
                const int f = o - W1B;
                v = W2f[((f >> 6) * KB2 + b) * 64 + (f & 63)];
            } else {
                v = *reinterpret_cast<const u32x4*>(b1 + b * 32 + (o - W1B - MT2 * 64) * 4);
            }
            lds[i] = v;
        }
        float* lb2 = reinterpret_cast<float*>(lds + KB2 * BLK);
        for (int i = threadIdx.x; i < D; i += blockDim.x) lb2[i] = b2[i];
        bias2 = lb2;
    }
    // BF16 rows: the residual c is added by one MFMA per output tile, with a
    // 0/1 selection matrix as the A operand and the X fragment that already
    // holds c as the B operand: tile mt with sel[mt & 1] and X block mt / 2
    // gives c[mt * 16 + m] (exact products, FP32 accumulation)
    __shared__ u32x4 lsel[BF16 ? 128 : 1];
    if constexpr (BF16) {
        for (int i = threadIdx.x; i < 128; i += blockDim.x) {
            const int sel = (i >> 6) * 16 + (i & 15), k0 = 8 * ((i & 63) >> 4);
            u32x4 v;
#pragma unroll
            for (int w = 0; w < 4; ++w)
                v[w] = (k0 + 2 * w == sel ? 0x3F80u : 0u) | (k0 + 2 * w + 1 == sel ? 0x3F800000u : 0u);
            lsel[i] = v;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
    const int nw = blockDim.x >> 6;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * nw;
    int64_t t = static_cast<int64_t>(blockIdx.x) * nw + (threadIdx.x >> 6);
    // no prefetch of the next tile's X: its registers would spill, and the
    // other waves of the SIMD cover the gather
    u32x4 xf[NT][KB1];
    int64_t cid[NT];
    bool ok[NT];
    for (; t < ntiles; t += stride) {
        const int64_t base = t * (16 * NT);
        load_x<D, NT, BF16>(S, t * (16 * NT), lane, xf, cid, ok);
        // the output accumulators start at b2
        f32x4 acc[MT2][NT];
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt) {
            const f32x4 bb = *reinterpret_cast<const f32x4*>(bias2 + mt * 16 + 4 * q);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = bb;
        }
#pragma unroll 1
        for (int kb2 = 0; kb2 < KB2; ++kb2) {
            const u32x4* w1b;
            const u32x4* w2b;
            const float* b1b;
            int w2s;
            if constexpr (WLDS) {
                w1b = lds + kb2 * BLK;
                w2b = w1b + W1B;
                w2s = 64;
                b1b = reinterpret_cast<const float*>(w2b + MT2 * 64);
            } else {
                w1b = W1f + kb2 * W1B;
                w2b = W2f + kb2 * 64;
                w2s = KB2 * 64;
                b1b = b1 + kb2 * 32;
            }
            u32x4 hb[NT];
            hidden_block<D, H, NT>(w1b, b1b, kb2, lane, xf, hb, [](int, int, float, float, float) {});
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt) {
                const u32x4 w = w2b[mt * w2s + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma(w, hb[nt], acc[mt][nt]);
            }
        }
        if constexpr (BF16) {
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt) {
                const u32x4 sw = lsel[(mt & 1) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma(sw, xf[nt][mt >> 1], acc[mt][nt]);
            }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (!ok[nt]) continue;
            const int64_t r = base + nt * 16 + r16;
#pragma unroll
            for (int mt = 0; mt < MT2; ++mt) {
                const int f0 = mt * 16 + 4 * q;
                f32x4 y = acc[mt][nt];
                if constexpr (!BF16) {   // FP32 rows: the residual in full precision
                    const f32x4 c = load_row4<BF16>(S.coarse, cid[nt], D, f0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) y[i] += c[i];
                }
                store_row4<BF16>(out, r, D, f0, y);
            }
        }
    }
}

// ------------------------------------------------------------ training
// Forward, loss and backward-data for one 32-row tile per wave (rows padded
// to Bp, a multiple of 32; rows >= S.rows contribute nothing).  Writes
// feature-major (transposed) BF16 copies of X, A1, dY and dZ1 for the
// weight-gradient products, and each tile's squared error.
struct TrainBufs {
    uint16_t* xt;    // [K1][Bp]
    uint16_t* a1t;   // [H][Bp]
    float* gp;       // [H][Bp]  gelu'(z1)
    uint16_t* dyt;   // [D][Bp]
    uint16_t* dzt;   // [H][Bp]
    float* lossp;    // [Bp/32]
    int64_t bp;
};

template <int D, int H, bool BF16>
__global__ __launch_bounds__(kTrainThreads) void k_train_fwd(RowSrc S, const void* __restrict__ target,
                                                             const u32x4* __restrict__ W1f,
                                                             const u32x4* __restrict__ W2f,
                                                             const u32x4* __restrict__ W2tf,
                                                             const float* __restrict__ b1,
                                                             const float* __restrict__ b2, TrainBufs T,
                                                             float dscale) {
    constexpr int NT = 2, KB1 = D / 32 + 1, KB2 = H / 32, MT1 = H / 16, MT2 = D / 16, KBD = D / 32;
    const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t * 32 >= T.bp) return;   // wave-uniform
    const int64_t base = t * 32;
    const int64_t bp = T.bp;

    u32x4 xf[NT][KB1];
    int64_t cid[NT];
    bool ok[NT];
    load_x<D, NT, BF16>(S, base, lane, xf, cid, ok);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t r = base + nt * 16 + r16;
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t w = xf[nt][kb][j >> 1];
                T.xt[static_cast<int64_t>(kb * 32 + 8 * q + j) * bp + r] =
                    static_cast<uint16_t>((j & 1) ? (w >> 16) : (w & 0xFFFFu));
            }
    }

    f32x4 acc[MT2][NT];
#pragma unroll
    for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int kb2 = 0; kb2 < KB2; ++kb2) {
        u32x4 hb[NT];
        hidden_block<D, H, NT>(W1f + kb2 * 2 * KB1 * 64, b1 + kb2 * 32, kb2, lane, xf, hb,
                               [&](int nt, int h, float z, float lo, float ez) {
            const float P = z >= 0.0f ? 1.0f - lo : lo;
            T.gp[static_cast<int64_t>(h) * bp + base + nt * 16 + r16] = fmaf(z * ez, kRsqrt2Pi, P);   // GELU'(z)
        });
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t r = base + nt * 16 + r16;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int h = (2 * kb2 + m) * 16 + 4 * q + i;
                    const uint32_t w = hb[nt][2 * m + (i >> 1)];
                    T.a1t[static_cast<int64_t>(h) * bp + r] = static_cast<uint16_t>((i & 1) ? (w >> 16) : (w & 0xFFFFu));
                }
        }
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt) {
            const u32x4 w = W2f[(mt * KB2 + kb2) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma(w, hb[nt], acc[mt][nt]);
        }
    }

    // output, loss and dY = dscale * (y - target), BF16 for the products
    float loss = 0.0f;
    uint32_t dyb[NT][MT2][2];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t r = base + nt * 16 + r16;
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt) {
            const int f0 = mt * 16 + 4 * q;
            float dy[4] = {0.f, 0.f, 0.f, 0.f};
            if (ok[nt]) {
                const f32x4 c = load_row4<BF16>(S.coarse, cid[nt], D, f0);
                const f32x4 tg = load_row4<BF16>(target, r, D, f0);
                const f32x4 bb = *reinterpret_cast<const f32x4*>(b2 + f0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float y = c[i] + (acc[mt][nt][i] + bb[i]);
                    const float diff = y - tg[i];
                    loss += diff * diff;
                    dy[i] = dscale * diff;
                }
            }
            dyb[nt][mt][0] = pack2(dy[0], dy[1]);
            dyb[nt][mt][1] = pack2(dy[2], dy[3]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                T.dyt[static_cast<int64_t>(f0 + i) * bp + r] =
                    static_cast<uint16_t>((i & 1) ? (dyb[nt][mt][i >> 1] >> 16) : (dyb[nt][mt][i >> 1] & 0xFFFFu));
        }
    }
    loss = group_sum<32>(loss);
    loss += __shfl_xor(loss, 32);
    if (lane == 0) T.lossp[t] = loss;

    // backward data: dA1^T = W2^T dY^T, dZ1 = dA1 * gelu'(z1)
#pragma unroll 1
    for (int mt = 0; mt < MT1; ++mt) {
        f32x4 g[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) g[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KBD; ++kb) {
            const u32x4 w = W2tf[(mt * KBD + kb) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const u32x4 b = {dyb[nt][2 * kb][0], dyb[nt][2 * kb][1], dyb[nt][2 * kb + 1][0],
                                 dyb[nt][2 * kb + 1][1]};
                g[nt] = mfma(w, b, g[nt]);
            }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t r = base + nt * 16 + r16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t h = mt * 16 + 4 * q + i;
                const float dz = g[nt][i] * T.gp[h * bp + r];
                T.dzt[h * bp + r] = static_cast<uint16_t>(f2bf(dz));
            }
        }
    }
}

// Weight gradients out[m][n] = sum_r Pt[m][r] Qt[n][r] over one chunk of
// kChunk rows; one wave per 32x32 output block.  Job 0: dW2 = dY^T A1
// (Pt = dY^T, Qt = A1^T); job 1: dW1 = dZ1^T X (Pt = dZ1^T, Qt = X^T).
// Results go to partial slice `chunk` of the parameter-ordered buffer.
constexpr int kChunk = 256;

template <int D, int H>
__global__ __launch_bounds__(256) void k_wgrad(TrainBufs T, float* __restrict__ gpart, int64_t nparams) {
    constexpr int F = D + 2, K1 = D + 32;
    constexpr int NB0 = (D / 32) * (H / 32);     // blocks of job 0
    constexpr int NB1 = (H / 32) * (K1 / 32);    // blocks of job 1
    const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= NB0 + NB1) return;               // wave-uniform
    const int chunk = blockIdx.y;
    const int64_t bp = T.bp;
    const int64_t r0 = static_cast<int64_t>(chunk) * kChunk;
    const int64_t r1 = std::min<int64_t>(r0 + kChunk, bp);
    const bool job1 = item >= NB0;
    const int b = job1 ? item - NB0 : item;
    const int ncols = job1 ? K1 / 32 : H / 32;
    const int m0 = (b / ncols) * 32, n0 = (b % ncols) * 32;
    const uint16_t* P = job1 ? T.dzt : T.dyt;
    const uint16_t* Q = job1 ? T.xt : T.a1t;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t r = r0; r < r1; r += 32) {
        u32x4 a[2], bq[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const u32x4*>(P + static_cast<int64_t>(m0 + 16 * i + r16) * bp + r + 8 * q);
            bq[i] = *reinterpret_cast<const u32x4*>(Q + static_cast<int64_t>(n0 + 16 * i + r16) * bp + r + 8 * q);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], bq[j], acc[i][j]);
    }
    float* out = gpart + static_cast<int64_t>(chunk) * nparams;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 16 * i + 4 * q + e;
                const int n = n0 + 16 * j + r16;
                if (!job1) {
                    out[static_cast<int64_t>(H) * F + H + static_cast<int64_t>(m) * H + n] = acc[i][j][e];
                } else if (n < F) {
                    out[static_cast<int64_t>(m) * F + n] = acc[i][j][e];
                }
            }
}

// Bias gradients over one chunk: db1[h] = sum_r dZ1[r][h], db2[f] = sum_r dY[r][f].
template <int D, int H>
__global__ __launch_bounds__(256) void k_colsum(TrainBufs T, float* __restrict__ gpart, int64_t nparams) {
    constexpr int F = D + 2;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= H + D) return;
    const int chunk = blockIdx.y;
    const int64_t r0 = static_cast<int64_t>(chunk) * kChunk;
    const int64_t r1 = std::min<int64_t>(r0 + kChunk, T.bp);
    const uint16_t* row = col < H ? T.dzt + static_cast<int64_t>(col) * T.bp : T.dyt + static_cast<int64_t>(col - H) * T.bp;
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += __uint_as_float(static_cast<uint32_t>(row[r]) << 16);
    float* out = gpart + static_cast<int64_t>(chunk) * nparams;
    if (col < H) out[static_cast<int64_t>(H) * F + col] = s;
    else out[static_cast<int64_t>(H) * F + H + static_cast<int64_t>(D) * H + (col - H)] = s;
}

// Positions of parameter p in the packed BF16 fragments (-1: not packed).
template <int D, int H>
__device__ __forceinline__ void frag_slots(int64_t p, int64_t& s1, int64_t& s2, int64_t& s3) {
    constexpr int F = D + 2, KB1 = D / 32 + 1, KB2 = H / 32, KBD = D / 32;
    s1 = s2 = s3 = -1;
    if (p < static_cast<int64_t>(H) * F) {
        const int h = static_cast<int>(p / F), f = static_cast<int>(p % F);
        const int c = f & 31, q = c >> 3, j = c & 7;
        s1 = ((static_cast<int64_t>(h >> 4) * KB1 + (f >> 5)) * 64 + q * 16 + (h & 15)) * 8 + j;
        return;
    }
    p -= static_cast<int64_t>(H) * F + H;
    if (p < 0 || p >= static_cast<int64_t>(D) * H) return;
    const int m = static_cast<int>(p / H), h = static_cast<int>(p % H);
    int q, j;
    perm_inv(h & 31, q, j);
    s2 = ((static_cast<int64_t>(m >> 4) * KB2 + (h >> 5)) * 64 + q * 16 + (m & 15)) * 8 + j;
    perm_inv(m & 31, q, j);
    s3 = ((static_cast<int64_t>(h >> 4) * KBD + (m >> 5)) * 64 + q * 16 + (h & 15)) * 8 + j;
}

struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
    int mode;                              // 0: gradient only, 1: Adam step, 2: pack only
};

// Sums the chunk partials in order (gradient), optionally applies Adam to
// the master weights, and refreshes the BF16 fragments.
template <int D, int H>
__global__ __launch_bounds__(256) void k_update(const float* __restrict__ gpart, int nchunks, float* __restrict__ grad_out,
                                               float* __restrict__ master, float* __restrict__ mom1,
                                               float* __restrict__ mom2, uint16_t* __restrict__ w1f,
                                               uint16_t* __restrict__ w2f, uint16_t* __restrict__ w2tf,
                                               int64_t nparams, AdamArgs A) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nparams) return;
    float w = master[p];
    if (A.mode != 2) {
        float g = 0.0f;
        for (int c = 0; c < nchunks; ++c) g += gpart[static_cast<int64_t>(c) * nparams + p];
        if (grad_out) grad_out[p] = g;
        if (A.mode == 0) return;
        const float m = A.beta1 * mom1[p] + (1.0f - A.beta1) * g;
        const float v = A.beta2 * mom2[p] + (1.0f - A.beta2) * g * g;
        mom1[p] = m;
        mom2[p] = v;
        w -= A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
        master[p] = w;
    }
    int64_t s1, s2, s3;
    frag_slots<D, H>(p, s1, s2, s3);
    const uint16_t b = static_cast<uint16_t>(f2bf(w));
    if (s1 >= 0) w1f[s1] = b;
    if (s2 >= 0) w2f[s2] = b;
    if (s3 >= 0) w2tf[s3] = b;
}

__global__ void k_loss(const float* __restrict__ lossp, int64_t ntiles, float scale, float* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.0f;
    for (int64_t i = 0; i < ntiles; ++i) s += lossp[i];
    *out = s * scale;
}

// W1 ~ U(-1/sqrt(d+2), 1/sqrt(d+2)) from Philox (kind 3), everything else 0.
__global__ void k_init(float* __restrict__ master, int64_t n_w1, int64_t nparams, float lim, uint32_t k0, uint32_t k1) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nparams) return;
    float w = 0.0f;
    if (p < n_w1) {
        const uint4 r = philox10(make_uint4(static_cast<uint32_t>(p), static_cast<uint32_t>(p >> 32), 0u,
                                            stream_word3(3u, 0u, 0u)),
                                 k0, k1);
        w = lim * (2.0f * (static_cast<float>(r.x >> 8) * (1.0f / 16777216.0f)) - 1.0f);
    }
    master[p] = w;
}

// Minibatch of training pairs: row b draws a pair uniformly over all
// sources' fine vertices (Philox kind 2, counter (b, step)), then copies the
// coarse row, the target row, the degree and the cluster size.
struct PairSrc {
    const void* offsets;
    int off64;
    const int32_t* map;
    const int32_t* clsz;
    const void* coarse;
    const void* fine;
    int64_t start;   // first pair index of this source
    int64_t n;
};

template <int D, bool BF16>
__global__ void k_sample(const PairSrc* __restrict__ srcs, int nsrc, int64_t total, int64_t B, int32_t step,
                         uint32_t tag, uint32_t k0, uint32_t k1, void* __restrict__ cb, void* __restrict__ tb,
                         int32_t* __restrict__ degb, int32_t* __restrict__ clszb) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint4 r = philox10(make_uint4(static_cast<uint32_t>(b), static_cast<uint32_t>(step), stream_word2(0, tag),
                                        stream_word3(2u, 0u, 0u)),
                             k0, k1);
    const int64_t u = static_cast<int64_t>(((static_cast<uint64_t>(r.x) << 32 | r.y) >> 16) % static_cast<uint64_t>(total));
    int s = 0;
    while (s + 1 < nsrc && srcs[s + 1].start <= u) ++s;
    const PairSrc P = srcs[s];
    const int64_t v = u - P.start;
    const int64_t c = P.map[v];
    int64_t deg = P.off64 ? static_cast<const int64_t*>(P.offsets)[v + 1] - static_cast<const int64_t*>(P.offsets)[v]
                          : static_cast<int64_t>(static_cast<const int32_t*>(P.offsets)[v + 1] -
                                                 static_cast<const int32_t*>(P.offsets)[v]);
    degb[b] = static_cast<int32_t>(std::min<int64_t>(deg, INT32_MAX));
    clszb[b] = P.clsz[c];
    constexpr int W = D * (BF16 ? 2 : 4) / 16;
    const u32x4* cs = static_cast<const u32x4*>(P.coarse) + c * W;
    const u32x4* fs = static_cast<const u32x4*>(P.fine) + v * W;
    u32x4* cd = static_cast<u32x4*>(cb) + b * W;
    u32x4* td = static_cast<u32x4*>(tb) + b * W;
    for (int i = 0; i < W; ++i) {
        cd[i] = cs[i];
        td[i] = fs[i];
    }
}

// ------------------------------------------------------------ host side
bool supported(int d, int h) {
    return (d == 32 || d == 64 || d == 128 || d == 256) && (h == 64 || h == 128 || h == 256);
}

template <int D, int H>
constexpr bool fits_lds() {   // weight fragments plus the biases (under one fragment)
    return (H / 16) * (D / 32 + 1) + (D / 16) * (H / 32) + 1 + 2 <= kLdsLimitFrags;   // + 2 selection fragments
}

int num_cus(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    return n;
}

template <class Fn>
void dispatch(int d, int h, Fn&& fn) {
#define GOSH_MLP_CASE(DD, HH) \
    if (d == DD && h == HH) return fn(std::integral_constant<int, DD>{}, std::integral_constant<int, HH>{});
    GOSH_MLP_CASE(32, 64) GOSH_MLP_CASE(32, 128) GOSH_MLP_CASE(32, 256)
    GOSH_MLP_CASE(64, 64) GOSH_MLP_CASE(64, 128) GOSH_MLP_CASE(64, 256)
    GOSH_MLP_CASE(128, 64) GOSH_MLP_CASE(128, 128) GOSH_MLP_CASE(128, 256)
    GOSH_MLP_CASE(256, 64) GOSH_MLP_CASE(256, 128) GOSH_MLP_CASE(256, 256)
#undef GOSH_MLP_CASE
    throw Error(GOSH_E_INVALID_ARG, "unsupported (d, hidden)");
}

void run_update(Ctx* c, gosh_mlp* M, const float* gpart, int nchunks, float* grad_out, AdamArgs A) {
    const Shape s{M->d, M->hidden};
    const unsigned blocks = static_cast<unsigned>(ceil_div(s.nparams(), 256));
    dispatch(M->d, M->hidden, [&](auto dd, auto hh) {
        constexpr int D = decltype(dd)::value, H = decltype(hh)::value;
        hipLaunchKernelGGL((k_update<D, H>), dim3(blocks), dim3(256), 0, c->stream, gpart, nchunks, grad_out,
                           M->master, M->m1, M->m2, M->w1f, M->w2f, M->w2tf, s.nparams(), A);
    });
    GOSH_HIP(hipGetLastError());
}

// Scratch of one training step for Bp padded rows.
struct StepBufs {
    DevBuf<uint16_t> xt, a1t, dyt, dzt;
    DevBuf<float> gp, gpart, lossp;
    TrainBufs tb{};
    int nchunks = 0;
    StepBufs(Ctx* c, const Shape& s, int64_t bp)
        : xt(c, s.K1() * bp), a1t(c, s.H * bp), dyt(c, s.D * bp), dzt(c, s.H * bp), gp(c, s.H * bp),
          gpart(c, ceil_div(bp, kChunk) * s.nparams()), lossp(c, bp / 32) {
        tb = TrainBufs{xt.p, a1t.p, gp.p, dyt.p, dzt.p, lossp.p, bp};
        nchunks = static_cast<int>(ceil_div(bp, kChunk));
    }
};

// Forward + backward over the batch described by S (S.rows rows) and the
// target rows; leaves the gradient partials in B.gpart.
void grad_pass(Ctx* c, gosh_mlp* M, gosh_dtype dt, const RowSrc& S, const void* target, StepBufs& B) {
    const int64_t bp = B.tb.bp;
    const float dscale = static_cast<float>(2.0 / (static_cast<double>(S.rows) * M->d));
    dispatch(M->d, M->hidden, [&](auto dd, auto hh) {
        constexpr int D = decltype(dd)::value, H = decltype(hh)::value;
        const unsigned wblocks = static_cast<unsigned>(ceil_div(bp / 32, kTrainThreads / 64));
        const u32x4* w1 = reinterpret_cast<const u32x4*>(M->w1f);
        const u32x4* w2 = reinterpret_cast<const u32x4*>(M->w2f);
        const u32x4* w2t = reinterpret_cast<const u32x4*>(M->w2tf);
        const float* b1 = M->master + Shape{D, H}.off_b1();
        const float* b2 = M->master + Shape{D, H}.off_b2();
        if (dt == GOSH_BF16)
            hipLaunchKernelGGL((k_train_fwd<D, H, true>), dim3(wblocks), dim3(kTrainThreads), 0, c->stream, S, target,
                               w1, w2, w2t, b1, b2, B.tb, dscale);
        else
            hipLaunchKernelGGL((k_train_fwd<D, H, false>), dim3(wblocks), dim3(kTrainThreads), 0, c->stream, S, target,
                               w1, w2, w2t, b1, b2, B.tb, dscale);
        GOSH_HIP(hipGetLastError());
        constexpr int items = (D / 32) * (H / 32) + (H / 32) * ((D + 32) / 32);
        hipLaunchKernelGGL((k_wgrad<D, H>), dim3(static_cast<unsigned>(ceil_div(items, 4)), B.nchunks), dim3(256), 0,
                           c->stream, B.tb, B.gpart.p, M->nparams);
        GOSH_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_colsum<D, H>), dim3(static_cast<unsigned>(ceil_div(D + H, 256)), B.nchunks), dim3(256), 0,
                           c->stream, B.tb, B.gpart.p, M->nparams);
        GOSH_HIP(hipGetLastError());
    });
}

void check_dt(gosh_dtype dt) {
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
}

}  // namespace mlp_detail

using namespace mlp_detail;

// ------------------------------------------------------------ entry points (called from api.hip)
gosh_mlp* mlp_create(gosh_ctx* owner, int d, int hidden) {
    Ctx* c = &owner->c;
    GOSH_REQUIRE(supported(d, hidden), GOSH_E_INVALID_ARG,
                 "learned prolongation needs d in {32, 64, 128, 256} and hidden in {64, 128, 256}");
    const Shape s{d, hidden};
    gosh_mlp* M = new gosh_mlp();
    M->owner = owner;
    M->ctx = c;
    M->d = d;
    M->hidden = hidden;
    M->nparams = s.nparams();
    try {
        M->master = static_cast<float*>(c->alloc(sizeof(float) * s.nparams()));
        M->m1 = static_cast<float*>(c->alloc(sizeof(float) * s.nparams()));
        M->m2 = static_cast<float*>(c->alloc(sizeof(float) * s.nparams()));
        M->w1f = static_cast<uint16_t*>(c->alloc(2 * s.w1f_elems()));
        M->w2f = static_cast<uint16_t*>(c->alloc(2 * s.w2f_elems()));
        M->w2tf = static_cast<uint16_t*>(c->alloc(2 * s.w2f_elems()));
        GOSH_HIP(hipMemsetAsync(M->m1, 0, sizeof(float) * s.nparams(), c->stream));
        GOSH_HIP(hipMemsetAsync(M->m2, 0, sizeof(float) * s.nparams(), c->stream));
        GOSH_HIP(hipMemsetAsync(M->w1f, 0, 2 * s.w1f_elems(), c->stream));   // padding columns stay 0
        const float lim = static_cast<float>(1.0 / std::sqrt(static_cast<double>(s.F())));
        hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>(ceil_div(s.nparams(), 256))), dim3(256), 0, c->stream,
                           M->master, static_cast<int64_t>(hidden) * s.F(), s.nparams(), lim,
                           static_cast<uint32_t>(c->seed), static_cast<uint32_t>(c->seed >> 32));
        GOSH_HIP(hipGetLastError());
        run_update(c, M, nullptr, 0, nullptr, AdamArgs{0, 0, 0, 0, 0, 0, 2});
    } catch (...) {
        mlp_free(M);
        delete M;
        throw;
    }
    return M;
}

void mlp_free(gosh_mlp* M) {
    if (!M || !M->ctx) return;
    Ctx* c = M->ctx;
    for (void* p : {static_cast<void*>(M->master), static_cast<void*>(M->m1), static_cast<void*>(M->m2),
                    static_cast<void*>(M->w1f), static_cast<void*>(M->w2f), static_cast<void*>(M->w2tf)})
        c->free(p);
    M->master = M->m1 = M->m2 = nullptr;
    M->w1f = M->w2f = M->w2tf = nullptr;
}

void mlp_set_weights(Ctx* c, gosh_mlp* M, const float* host) {
    GOSH_REQUIRE(host, GOSH_E_INVALID_ARG, "null weights");
    GOSH_HIP(hipMemcpyAsync(M->master, host, sizeof(float) * M->nparams, hipMemcpyHostToDevice, c->stream));
    GOSH_HIP(hipMemsetAsync(M->m1, 0, sizeof(float) * M->nparams, c->stream));
    GOSH_HIP(hipMemsetAsync(M->m2, 0, sizeof(float) * M->nparams, c->stream));
    M->t = 0;
    run_update(c, M, nullptr, 0, nullptr, AdamArgs{0, 0, 0, 0, 0, 0, 2});
    GOSH_HIP(hipStreamSynchronize(c->stream));   // the host buffer may go away after return
}

void mlp_get_weights(Ctx* c, const gosh_mlp* M, float* host) {
    GOSH_REQUIRE(host, GOSH_E_INVALID_ARG, "null output");
    GOSH_HIP(hipMemcpyAsync(host, M->master, sizeof(float) * M->nparams, hipMemcpyDeviceToHost, c->stream));
    GOSH_HIP(hipStreamSynchronize(c->stream));
}

void mlp_prolong(Ctx* c, const gosh_mlp* M, const Level& fine, int64_t n_coarse, const void* coarse, void* fine_emb,
                 gosh_dtype dt, int d) {
    check_dt(dt);
    GOSH_REQUIRE(d == M->d, GOSH_E_INVALID_ARG, "d differs from the network's");
    GOSH_REQUIRE(fine.map, GOSH_E_INVALID_ARG, "level has no map to a coarser level");
    if (fine.n == 0) return;
    GOSH_REQUIRE(coarse && fine_emb, GOSH_E_INVALID_ARG, "null embedding");
    const int32_t* clsz = cluster_sizes(c, fine, n_coarse);
    RowSrc S{coarse, fine.map, fine.offsets, fine.off64 ? 1 : 0, nullptr, clsz, fine.n};
    const int ncu = num_cus(c->device);
    dispatch(M->d, M->hidden, [&](auto dd, auto hh) {
        constexpr int D = decltype(dd)::value, H = decltype(hh)::value;
        // d <= 128: one 16-row tile per wave and 16 waves per workgroup, so
        // that each SIMD holds 4 waves against the one copy of the weights in
        // LDS (the GELU between the two products needs waves to hide its
        // latency); d = 256 keeps 8 waves of one tile each
        constexpr int NT = 1;
        constexpr int T = D >= 256 ? kFwdThreads : kFwdThreadsWide;
        constexpr bool WL = fits_lds<D, H>();
        const int64_t ntiles = ceil_div(fine.n, 16 * NT);
        const int64_t per_block = T / 64;
        const unsigned blocks =
            static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(ntiles, per_block), int64_t(ncu) * (WL ? 1 : 2))));
        const u32x4* w1 = reinterpret_cast<const u32x4*>(M->w1f);
        const u32x4* w2 = reinterpret_cast<const u32x4*>(M->w2f);
        const float* b1 = M->master + Shape{D, H}.off_b1();
        const float* b2 = M->master + Shape{D, H}.off_b2();
        if (dt == GOSH_BF16)
            hipLaunchKernelGGL((k_forward<D, H, NT, true, WL, T>), dim3(blocks), dim3(T), 0, c->stream, S, w1, w2,
                               b1, b2, fine_emb, ntiles);
        else
            hipLaunchKernelGGL((k_forward<D, H, NT, false, WL, T>), dim3(blocks), dim3(T), 0, c->stream, S, w1,
                               w2, b1, b2, fine_emb, ntiles);
    });
    GOSH_HIP(hipGetLastError());
}

void mlp_grad(Ctx* c, gosh_mlp* M, gosh_dtype dt, const gosh_mlp_batch* b, float* grads, float* loss) {
    check_dt(dt);
    GOSH_REQUIRE(b && b->rows > 0, GOSH_E_INVALID_ARG, "empty batch");
    GOSH_REQUIRE(b->rows <= (int64_t(1) << 24), GOSH_E_INVALID_ARG, "batch too large");
    GOSH_REQUIRE(b->coarse && b->deg && b->clsz && b->target, GOSH_E_INVALID_ARG, "null batch array");
    GOSH_REQUIRE(grads, GOSH_E_INVALID_ARG, "null gradient output");
    const Shape s{M->d, M->hidden};
    const int64_t bp = ceil_div(b->rows, 32) * 32;
    StepBufs B(c, s, bp);
    RowSrc S{b->coarse, nullptr, nullptr, 0, b->deg, b->clsz, b->rows};
    grad_pass(c, M, dt, S, b->target, B);
    run_update(c, M, B.gpart.p, B.nchunks, grads, AdamArgs{0, 0, 0, 0, 0, 0, 0});
    if (loss) {
        hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, c->stream, B.lossp.p, bp / 32,
                           static_cast<float>(1.0 / (static_cast<double>(b->rows) * M->d)), loss);
        GOSH_HIP(hipGetLastError());
    }
    GOSH_HIP(hipStreamSynchronize(c->stream));   // scratch is released on return
}

namespace {
AdamArgs adam_args(gosh_mlp* M, float lr) {
    ++M->t;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, static_cast<double>(M->t)));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, static_cast<double>(M->t)));
    return AdamArgs{lr, 0.9f, 0.999f, 1e-8f, static_cast<float>(c1), static_cast<float>(c2), 1};
}
}  // namespace

void mlp_adam_step(Ctx* c, gosh_mlp* M, const float* grads, float lr) {
    GOSH_REQUIRE(grads, GOSH_E_INVALID_ARG, "null gradients");
    GOSH_REQUIRE(std::isfinite(lr) && lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
    run_update(c, M, grads, 1, nullptr, adam_args(M, lr));
}

void mlp_train(Ctx* c, gosh_mlp* M, gosh_dtype dt, const std::vector<PairSrcHost>& srcs, int steps, int batch,
               float lr, uint32_t tag, float* loss_dev) {
    check_dt(dt);
    GOSH_REQUIRE(steps >= 0, GOSH_E_INVALID_ARG, "steps must be >= 0");
    GOSH_REQUIRE(batch >= 1 && batch <= (1 << 20), GOSH_E_INVALID_ARG, "batch must be in [1, 2^20]");
    GOSH_REQUIRE(std::isfinite(lr) && lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
    GOSH_REQUIRE(tag < (1u << 24), GOSH_E_INVALID_ARG, "tag must fit in 24 bits");
    std::vector<PairSrc> hs;
    int64_t total = 0;
    for (const PairSrcHost& p : srcs) {
        GOSH_REQUIRE(p.L && p.L->map, GOSH_E_INVALID_ARG, "source level has no map to a coarser level");
        GOSH_REQUIRE(p.coarse && p.fine, GOSH_E_INVALID_ARG, "null source embedding");
        if (p.L->n == 0) continue;
        const int32_t* clsz = cluster_sizes(c, *p.L, p.n_coarse);
        hs.push_back(PairSrc{p.L->offsets, p.L->off64 ? 1 : 0, p.L->map, clsz, p.coarse, p.fine, total, p.L->n});
        total += p.L->n;
    }
    GOSH_REQUIRE(total > 0, GOSH_E_INVALID_ARG, "no training pairs");
    if (steps == 0) return;
    const Shape s{M->d, M->hidden};
    const int64_t bp = ceil_div(batch, 32) * 32;
    const size_t esz = dt == GOSH_BF16 ? 2 : 4;
    DevBuf<PairSrc> dsrc(c, hs.size());
    GOSH_HIP(hipMemcpyAsync(dsrc.p, hs.data(), sizeof(PairSrc) * hs.size(), hipMemcpyHostToDevice, c->stream));
    DevBuf<uint8_t> cb(c, bp * s.D * esz), tb(c, bp * s.D * esz);
    DevBuf<int32_t> degb(c, bp), clszb(c, bp);
    StepBufs B(c, s, bp);
    RowSrc S{cb.p, nullptr, nullptr, 0, degb.p, clszb.p, batch};
    const uint32_t k0 = static_cast<uint32_t>(c->seed), k1 = static_cast<uint32_t>(c->seed >> 32);
    for (int step = 0; step < steps; ++step) {
        dispatch(M->d, M->hidden, [&](auto dd, auto) {
            constexpr int D = decltype(dd)::value;
            if (dt == GOSH_BF16)
                hipLaunchKernelGGL((k_sample<D, true>), dim3(static_cast<unsigned>(ceil_div(batch, 256))), dim3(256), 0,
                                   c->stream, dsrc.p, static_cast<int>(hs.size()), total, static_cast<int64_t>(batch),
                                   step, tag, k0, k1, cb.p, tb.p, degb.p, clszb.p);
            else
                hipLaunchKernelGGL((k_sample<D, false>), dim3(static_cast<unsigned>(ceil_div(batch, 256))), dim3(256), 0,
                                   c->stream, dsrc.p, static_cast<int>(hs.size()), total, static_cast<int64_t>(batch),
                                   step, tag, k0, k1, cb.p, tb.p, degb.p, clszb.p);
        });
        GOSH_HIP(hipGetLastError());
        grad_pass(c, M, dt, S, tb.p, B);
        run_update(c, M, B.gpart.p, B.nchunks, nullptr, adam_args(M, lr));
        if (loss_dev) {
            hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, c->stream, B.lossp.p, bp / 32,
                               static_cast<float>(1.0 / (static_cast<double>(batch) * M->d)), loss_dev + step);
            GOSH_HIP(hipGetLastError());
        }
    }
    GOSH_HIP(hipStreamSynchronize(c->stream));   // scratch is released on return
}

}  // namespace gosh
