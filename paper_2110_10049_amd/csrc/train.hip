// TrainInGPU (Algorithm 3, Section 3.1) with UpdateEmbed (Algorithm 1) for
// gfx950.
//
// Layout: a source is served by a group of L lanes (Lanes in visit.hpp: up
// to 16 lanes, d/8 for d = 256), one wave64 carries 64/L sources (BF16:
// d=128 4 sources per wave, d=8 16), and the row's 32-bit words are
// interleaved across the group so that each memory instruction covers
// contiguous bytes.  The dot product is reduced inside the group with DPP
// (no LDS round trip).  Each group draws its samples from
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
// so lane gl draws exactly one block (block gl mod d/8) per row update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "gosh_internal.hpp"

#include "visit.hpp"

namespace gosh {
namespace {

using namespace train_detail;

// LOOP (per-epoch mode, one epoch per launch): each wave takes its slots in
// a grid-stride loop over a capped grid instead of one slot group per wave.
// Measured faster on levels below kLoopMaxVertices and slower on level 0 of
// the scale-20 graph, even at one iteration per wave, so it is a separate
// kernel.
template <bool BF16, int D, int KMAX, class Off, int MODE, bool LOOP = false>
__global__ __launch_bounds__(kBlock) void k_train(TrainParams P) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    if constexpr (MODE == kSequential) {
        // one wave, sources strictly in ascending id order; the running loss
        // is summed per visit in FP64
        double acc = 0.0;
        for (int64_t s = 0; s < P.n; ++s) {
            acc += visit<BF16, D, KMAX, Off, MODE>(P, s, grp == 0, gl);
            __threadfence();
        }
        if (P.loss && lane == 0 && acc != 0.0)
            __hip_atomic_fetch_add(P.loss, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
        const int64_t slot = wave * G + grp;
        if constexpr (MODE == kEpoch) {
            if (P.span > 1) {
                // several epochs in flight: this slot's epoch and its decayed lr
                const int64_t ep = slot / P.n;
                TrainParams Q = P;
                Q.epoch = P.epoch + static_cast<uint32_t>(ep);
                const double f = 1.0 - static_cast<double>(Q.epoch) / static_cast<double>(P.e_total);
                Q.lr = static_cast<float>(static_cast<double>(P.lr0) * (f > 1e-4 ? f : 1e-4));
                const float l = visit<BF16, D, KMAX, Off, MODE>(Q, slot - ep * P.n, slot < P.n * P.span, gl);
                if (P.loss && gl == 0 && l != 0.0f)
                    __hip_atomic_fetch_add(P.loss + ep, static_cast<double>(l), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }
        const int64_t limit = (MODE == kExplicit) ? P.nsrc : P.n;
        if constexpr (LOOP) {
            const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBlock / 64);
            for (int64_t w = wave; w * G < limit; w += waves) {   // wave-uniform bound
                const int64_t s = w * G + grp;
                const float l = visit<BF16, D, KMAX, Off, MODE>(P, s, s < limit, gl);
                if (P.loss) wave_add_loss<L>(P.loss, l, gl);
            }
        } else {
            const float l = visit<BF16, D, KMAX, Off, MODE>(P, slot, slot < limit, gl);
            if (P.loss) wave_add_loss<L>(P.loss, l, gl);
        }
    }
}

// Device-wide barrier of a cooperative launch: every block adds one to
// *count once all its waves arrived, then waits until the count reaches
// `target` (= blocks x barriers passed).  The wait is bounded: after
// spin_limit polls the block sets *error and goes on (the results are then
// invalid, but every wave still exits).
// The arrival is a release and the poll an acquire at device scope, which
// make the block's row updates visible to, and the other blocks' updates
// visible in, the next epoch (the L1 of the block's CU is invalidated by
// the acquire; __syncthreads orders the block's other waves around it).  The
// cost grows with the number of arriving blocks (about 1.6 us for 32 blocks
// against 3-6 us for a kernel launch), so resident launches use few blocks
// of 16 waves.
__device__ __forceinline__ void grid_barrier(unsigned int* count, unsigned int target, unsigned int* error,
                                             unsigned long long spin_limit) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        for (unsigned long long spins = 0;; ++spins) {
            if (__hip_atomic_load(count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (spins >= spin_limit) {
                atomicOr(error, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

constexpr int kResBlock = 1024;   // 16 waves per block of a resident launch

// All epochs of a small level in one cooperative launch (Algorithm 3's
// barrier between epochs kept as a device-wide barrier instead of a launch
// boundary).  Waves take the level's sources in a grid-stride loop, so every
// epoch runs exactly the per-epoch launch's visits (same samples, lr and
// rounding bits); rows written in earlier epochs of the launch are read with
// coherent loads (kPersistent).  P.e_total epochs; P.loss, when set, has one
// entry per epoch.
template <bool BF16, int D, int KMAX, class Off>
__global__ __launch_bounds__(kResBlock) void k_train_resident(TrainParams P, unsigned int* barrier,
                                                              unsigned int* error, unsigned long long spin_limit) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kResBlock / 64) + (threadIdx.x >> 6);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (kResBlock / 64) * G;
    for (int j = 0; j < P.e_total; ++j) {
        TrainParams Q = P;
        Q.epoch = static_cast<uint32_t>(j);
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(P.e_total);
        Q.lr = static_cast<float>(static_cast<double>(P.lr0) * (f > 1e-4 ? f : 1e-4));
        Q.loss = P.loss ? P.loss + j : nullptr;
        for (int64_t base = wave * G; base < P.n; base += stride) {
            const int64_t slot = base + grp;
            const float l = visit<BF16, D, KMAX, Off, kPersistent>(Q, slot, slot < P.n, gl);
            if (Q.loss) wave_add_loss<L>(Q.loss, l, gl);
        }
        if (j + 1 < P.e_total) grid_barrier(barrier, static_cast<unsigned int>(j + 1) * gridDim.x, error, spin_limit);
    }
}

// A level whose rows fit in one workgroup's LDS: all epochs inside one
// workgroup (train_rows_in_lds); dynamic LDS = lds_level_bytes.
template <bool BF16, int D, int KMAX, class Off>
__global__ __launch_bounds__(kLdsBlock) void k_train_lds(TrainParams P) {
    extern __shared__ __align__(16) unsigned char lds_rows[];
    train_rows_in_lds<BF16, D, KMAX, Off>(P, lds_rows);
}

constexpr int64_t kLdsMaxBytes = 160 * 1024;   // LDS of one CU

__global__ void k_zero_word(unsigned int* p) { *p = 0u; }

constexpr int64_t kResidentBlocks = 128;  // blocks of a resident launch at most (fastest in a sweep of 8-256)

template <class Off>
__global__ void k_draw(TrainParams P, int32_t* out) {
    const int64_t src = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (src >= P.n) return;
    const int k = P.k;
    const Off* off = static_cast<const Off*>(P.offsets);
    const int64_t beg = off[src], end = off[src + 1];
    const int64_t deg = (beg >= 0 && beg <= end && end <= P.nnz) ? end - beg : 0;
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
// One add per workgroup (a per-wave add put thousands of atomics on one
// counter); blocks of 256 threads.
template <class Off>
__global__ __launch_bounds__(256) void k_add_updates(const Off* off, int64_t n, int k, int epochs,
                                                     unsigned long long* p) {
    __shared__ unsigned long long part[4];
    unsigned long long cnt = 0;
    for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<int64_t>(gridDim.x) * blockDim.x)
        cnt += (off[v + 1] != off[v]) ? 1ull : 0ull;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long add = (part[0] + part[1] + part[2] + part[3]) * static_cast<unsigned long long>(epochs);
        if (blockIdx.x == 0) add += static_cast<unsigned long long>(k) * static_cast<unsigned long long>(n) * epochs;
        if (add) atomicAdd(p, add);
    }
}

// ---------------------------------------------------------------- dispatch
using Launcher = void (*)(const TrainParams&, int64_t, hipStream_t);

constexpr int64_t kLoopMaxVertices = 262144;   // levels below it run the LOOP kernel
constexpr int64_t kLoopBlocks = 2560;           // its grid cap: two rounds of resident workgroups on 256 CUs

template <bool BF16, int D, int KMAX, class Off, int MODE>
void launch(const TrainParams& P, int64_t items, hipStream_t st) {
    constexpr int G = Lanes<BF16, D>::kG;
    if constexpr (MODE == kSequential) {
        hipLaunchKernelGGL((k_train<BF16, D, KMAX, Off, MODE>), dim3(1), dim3(64), 0, st, P);
    } else {
        const int64_t per_block = (kBlock / 64) * G;
        const int64_t blocks = ceil_div(items, per_block);
        if constexpr (MODE == kEpoch) {
            if (items == P.n && P.n < kLoopMaxVertices) {   // one epoch per launch
                hipLaunchKernelGGL((k_train<BF16, D, KMAX, Off, MODE, true>),
                                   dim3(static_cast<unsigned>(std::min(blocks, kLoopBlocks))), dim3(kBlock), 0, st, P);
                return;
            }
        }
        hipLaunchKernelGGL((k_train<BF16, D, KMAX, Off, MODE>), dim3(static_cast<unsigned>(blocks)),
                           dim3(kBlock), 0, st, P);
    }
}

// Resident (all epochs in one cooperative launch) kernels.
struct ResidentKernel {
    const void* fn;
    int per_wave;
};

template <bool BF16, int D, int KMAX>
ResidentKernel resident_off(bool off64, bool lds) {
    if (lds)
        return ResidentKernel{off64 ? reinterpret_cast<const void*>(&k_train_lds<BF16, D, KMAX, int64_t>)
                                    : reinterpret_cast<const void*>(&k_train_lds<BF16, D, KMAX, int32_t>),
                              Lanes<BF16, D>::kG};
    return ResidentKernel{off64 ? reinterpret_cast<const void*>(&k_train_resident<BF16, D, KMAX, int64_t>)
                                : reinterpret_cast<const void*>(&k_train_resident<BF16, D, KMAX, int32_t>),
                          Lanes<BF16, D>::kG};
}

template <bool BF16, int D>
ResidentKernel resident_k(int k, bool off64, bool lds) {
    if (k <= 1) return resident_off<BF16, D, 1>(off64, lds);
    if (k <= 3) return resident_off<BF16, D, 3>(off64, lds);
    if (k <= 7) return resident_off<BF16, D, 7>(off64, lds);
    return resident_off<BF16, D, 15>(off64, lds);
}

template <bool BF16>
ResidentKernel resident_d(int d, int k, bool off64, bool lds = false) {
    switch (d) {
        case 8: return resident_k<BF16, 8>(k, off64, lds);
        case 16: return resident_k<BF16, 16>(k, off64, lds);
        case 32: return resident_k<BF16, 32>(k, off64, lds);
        case 64: return resident_k<BF16, 64>(k, off64, lds);
        case 128: return resident_k<BF16, 128>(k, off64, lds);
        case 256: return resident_k<BF16, 256>(k, off64, lds);
    }
    return ResidentKernel{nullptr, 0};
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

// Lanes serving one row (Lanes::kL) for a runtime dtype and d.
template <bool BF16>
int lanes_for(int d) {
    switch (d) {
        case 8: return Lanes<BF16, 8>::kL;
        case 16: return Lanes<BF16, 16>::kL;
        case 32: return Lanes<BF16, 32>::kL;
        case 64: return Lanes<BF16, 64>::kL;
        case 128: return Lanes<BF16, 128>::kL;
        default: return Lanes<BF16, 256>::kL;
    }
}
int lanes_per_row(gosh_dtype dt, int d) { return dt == GOSH_BF16 ? lanes_for<true>(d) : lanes_for<false>(d); }

// Hub bitmap of a level: bit v of word v / 32 set iff deg(v) >= light_below.
// One thread per vertex; a wave's 64 flags are one ballot, written by lane 0
// as two words (waves start at multiples of 64 vertices).
template <class Off>
__global__ void k_hub_bits(const Off* off, int64_t n, int64_t light_below, uint32_t* bits) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t v0 = static_cast<int64_t>(blockIdx.x) * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        const bool hub = v < n && static_cast<int64_t>(off[v + 1]) - static_cast<int64_t>(off[v]) >= light_below;
        const unsigned long long m = __ballot(hub);
        if ((threadIdx.x & 63) == 0) {
            const int64_t w = (v0 + threadIdx.x) >> 5;   // v is a multiple of 64 here
            if (w * 32 < n) bits[w] = static_cast<uint32_t>(m);
            if ((w + 1) * 32 < n) bits[w + 1] = static_cast<uint32_t>(m >> 32);
        }
    }
}

TrainParams base_params(Ctx* c, int32_t level, uint32_t tag) {
    TrainParams P{};
    P.key0 = static_cast<uint32_t>(c->seed);
    P.key1 = static_cast<uint32_t>(c->seed >> 32);
    P.w2 = stream_word2(level, tag);
    return P;
}

}  // namespace

const uint32_t* hub_bits(Ctx* c, const Level& L, int64_t light_below) {
    if (!L.hub_bits) {
        Level& M = const_cast<Level&>(L);
        const int64_t words = ceil_div(L.n, 32);
        M.hub_bits = static_cast<uint32_t*>(c->alloc(sizeof(uint32_t) * static_cast<size_t>(std::max<int64_t>(words, 1))));
        const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(L.n, 256), 65536));
        if (L.off64)
            hipLaunchKernelGGL(k_hub_bits<int64_t>, dim3(blocks), dim3(256), 0, c->stream,
                               static_cast<const int64_t*>(L.offsets), L.n, light_below, M.hub_bits);
        else
            hipLaunchKernelGGL(k_hub_bits<int32_t>, dim3(blocks), dim3(256), 0, c->stream,
                               static_cast<const int32_t*>(L.offsets), L.n, light_below, M.hub_bits);
        GOSH_HIP(hipGetLastError());
    }
    return L.hub_bits;
}

bool train_level_grouped(Ctx* c, const Level& L, train_detail::TrainParams P, gosh_dtype dt, int d, int epochs,
                         float lr);

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
    P.nnz = L.nnz;
    P.emb = emb;
    P.n_rows = L.n;
    P.k = k;
    P.updates = reinterpret_cast<unsigned long long*>(updates_dev);
    Launcher fn = c->deterministic ? pick<kSequential>(dt, d, k, L.off64) : pick<kEpoch>(dt, d, k, L.off64);
    GOSH_REQUIRE(fn, GOSH_E_INVALID_ARG, "unsupported training shape");
    // epochs run one launch each (Section 3.1), unless the context lets
    // `overlap` epochs share a launch on levels of at least overlap_min vertices
    int span = (!c->deterministic && c->overlap > 1 && L.n >= c->overlap_min) ? c->overlap : 1;
    // one launch covers n * span sources with L lanes each; a 1-D launch
    // holds fewer than 2^32 lanes
    const int64_t lanes_per_source = lanes_per_row(dt, d);
    constexpr int64_t kMaxLanes = (int64_t(1) << 32) - 4096;
    GOSH_REQUIRE(c->deterministic || L.n * lanes_per_source <= kMaxLanes, GOSH_E_UNSUPPORTED,
                 "level too large for one epoch launch at this d");
    while (span > 1 && L.n * span * lanes_per_source > kMaxLanes) span /= 2;
    P.span = 1;
    P.e_total = epochs;
    P.lr0 = lr;
    P.plain_neg = (!c->deterministic && c->plain_neg_min > 0 && L.n >= c->plain_neg_min) ? 1 : 0;
    // light rows stored plainly; also in deterministic mode, where one visit
    // at a time makes a plain store equal to the atomic commit
    P.light_below = (c->plain_light_min > 0 && L.n >= c->plain_light_min) ? L.nnz / L.n + 1 : 0;
    if (P.light_below > 0) P.hub_bits = hub_bits(c, L, P.light_below);
    if (c->record) {
        GOSH_REQUIRE(c->record_cap >= L.n * (1 + k), GOSH_E_INVALID_ARG,
                     "draw record buffer holds fewer than n * (1 + k) entries");
        P.record = c->record;
    }
    GOSH_REQUIRE(!c->loss || c->loss_cap >= epochs, GOSH_E_INVALID_ARG,
                 "loss record buffer holds fewer entries than the call's epochs");
    const int64_t lds_bytes = lds_level_bytes(L.n, d, dt == GOSH_BF16 ? 2 : 4, k);
    const bool plain = P.plain_neg != 0 || P.light_below != 0;
    const bool grouped = !c->deterministic && span == 1 && P.light_below == 0 && c->group_max > 0 &&
                         L.n >= c->group_min && L.n <= c->group_max && L.n < (int64_t(1) << 31) &&
                         train_level_grouped(c, L, P, dt, d, epochs, lr);
    if (grouped) {
        // epochs ran with the visits of hot positives grouped (grouped.hip)
    } else if (!c->deterministic && span == 1 && !plain && L.n <= c->lds_max && lds_bytes <= kLdsMaxBytes) {
        // the level's rows and one epoch's samples in one workgroup's LDS
        const ResidentKernel R = dt == GOSH_BF16 ? resident_d<true>(d, k, L.off64, true)
                                                 : resident_d<false>(d, k, L.off64, true);
        GOSH_REQUIRE(R.fn, GOSH_E_INVALID_ARG, "unsupported training shape");
        GOSH_HIP(hipFuncSetAttribute(R.fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
        P.lr = lr;
        P.epoch = 0;
        P.loss = c->loss;
        void* args[] = {&P};
        GOSH_HIP(hipLaunchKernel(R.fn, dim3(1), dim3(kLdsBlock), args, static_cast<size_t>(lds_bytes), c->stream));
    } else if (!c->deterministic && span == 1 && epochs > 1 && L.n <= c->resident_max && !plain) {
        // all epochs in one cooperative launch with device-wide barriers
        const ResidentKernel R = dt == GOSH_BF16 ? resident_d<true>(d, k, L.off64) : resident_d<false>(d, k, L.off64);
        GOSH_REQUIRE(R.fn, GOSH_E_INVALID_ARG, "unsupported training shape");
        int per_cu = 0, cus = 0;
        GOSH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, R.fn, kResBlock, 0));
        GOSH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        const int64_t need = ceil_div(L.n, static_cast<int64_t>(kResBlock / 64) * R.per_wave);
        const int64_t cap = std::min<int64_t>(static_cast<int64_t>(std::max(per_cu, 1)) * cus, kResidentBlocks);
        const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(1, std::min(need, cap)));
        unsigned int* bar = reinterpret_cast<unsigned int*>(static_cast<char*>(c->scratch) + 512);
        unsigned int* err = reinterpret_cast<unsigned int*>(static_cast<char*>(c->scratch) + 516);
        hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, c->stream, bar);
        GOSH_HIP(hipGetLastError());
        P.lr = lr;
        P.epoch = 0;
        P.loss = c->loss;
        unsigned long long spin_limit = 1ull << 22;   // a few seconds of polling
        void* args[] = {&P, &bar, &err, &spin_limit};
        GOSH_HIP(hipLaunchCooperativeKernel(R.fn, dim3(blocks), dim3(kResBlock), args, 0, c->stream));
    } else {
    for (int j = 0; j < epochs; j += span) {
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(epochs);
        P.lr = static_cast<float>(static_cast<double>(lr) * (f > 1e-4 ? f : 1e-4));
        P.epoch = static_cast<uint32_t>(j);
        P.span = std::min(span, epochs - j);
        P.loss = c->loss ? c->loss + j : nullptr;
        fn(P, L.n * P.span, c->stream);
        GOSH_HIP(hipGetLastError());
    }
    }
    if (updates_dev) {
        const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(L.n, 256), 512)));
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
    P.plain_neg = (!c->deterministic && c->plain_neg_min > 0 && n_rows >= c->plain_neg_min) ? 1 : 0;
    P.loss = c->loss;   // the batch's running loss goes to entry 0
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
    P.nnz = L.nnz;
    P.k = k;
    P.epoch = static_cast<uint32_t>(epoch);
    const unsigned blocks = static_cast<unsigned>(ceil_div(L.n, 256));
    if (L.off64) hipLaunchKernelGGL(k_draw<int64_t>, dim3(blocks), dim3(256), 0, c->stream, P, out);
    else hipLaunchKernelGGL(k_draw<int32_t>, dim3(blocks), dim3(256), 0, c->stream, P, out);
    GOSH_HIP(hipGetLastError());
}

}  // namespace gosh
