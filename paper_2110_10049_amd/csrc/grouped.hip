// TrainInGPU epochs with the visits of hot positives grouped (an opt-in
// schedule of Algorithm 3's concurrent sources, Section 3.1).
//
// On a coarse level most positive samples land on a few hub rows, and every
// visit commits its change to the positive's row: thousands of commits per
// epoch meet on the same rows and serialise at the L2.  Here every source's
// samples are first drawn (the same Philox draws as the per-epoch kernel)
// into a table, and the visits whose positive is a hot hub (degree at least
// hot_factor times the level's average) are filed into one bucket per hub.
// The draws do not depend on the rows, so one launch draws a batch of
// epochs.  One launch per epoch then runs, concurrently, the other visits
// from the table and, per chunk of kChunk bucketed visits, a workgroup that
// reads its hub row once into LDS, runs the chunk's visits against that
// copy (each visit's hub change is summed in LDS, FP32) and commits the sum
// to the hub row once.  The visits of a chunk read the hub row as it was
// when the chunk started -- one of the interleavings concurrent sources
// allow -- and no change is lost: the chunk commits with the same exact
// atomic commit as a visit.  Source rows and negatives are committed as in
// the per-epoch kernel; a visit whose negative repeats its positive stays
// ungrouped, so repeated samples keep their sequential semantics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "gosh_internal.hpp"
#include "primitives.hpp"

#include "visit.hpp"

namespace gosh {
namespace {

using namespace train_detail;

constexpr int kThreads = 256;
inline dim3 grid_for(int64_t items) {
    return dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div(std::max<int64_t>(items, 1), kThreads), 1 << 20)));
}
#define GRID_STRIDE(i, N) \
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (N); \
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)

constexpr int kMaxHot = 4096;        // hub buckets at most (a level's hottest ids)
constexpr int kDrawThreads = 1024;   // sources per workgroup of the draw kernel
constexpr int kHotBlocks = 4096;     // workgroups taking the bucket chunks
constexpr int kMaxBatch = 16;        // epochs drawn per draw launch, at most
constexpr int64_t kBatchBytes = int64_t(256) << 20;   // a batch's tables and bucket lists, at most

// flag[v] = 1 for a hub of degree >= hot_deg
template <class Off>
__global__ void k_hot_flags(const Off* off, int64_t n, int64_t hot_deg, int32_t* flag) {
    GRID_STRIDE(v, n) {
        flag[v] = static_cast<int64_t>(off[v + 1]) - static_cast<int64_t>(off[v]) >= hot_deg ? 1 : 0;
    }
}

// slot[v] = bucket of hub v (-1: not bucketed), hub_of[slot] = v, cap[slot]
// = deg(v): a hub is the positive of its neighbours only, at most deg(v) a
// epoch (the bucket write also checks it, for graphs that are not symmetric)
template <class Off>
__global__ void k_hot_slots(const Off* off, const int32_t* flag, const int64_t* pre, int64_t n, int32_t* slot,
                            int32_t* hub_of, int64_t* cap) {
    GRID_STRIDE(v, n) {
        const bool hot = flag[v] && pre[v] < kMaxHot;
        slot[v] = hot ? static_cast<int32_t>(pre[v]) : -1;
        if (hot) {
            hub_of[pre[v]] = static_cast<int32_t>(v);
            cap[pre[v]] = static_cast<int64_t>(off[v + 1]) - static_cast<int64_t>(off[v]);
        }
    }
}

// One thread per source: its samples into the table; a visit whose positive
// is a bucketed hub (and no negative repeats it) is filed into the hub's
// bucket and marked -2 - slot in the table.  Bucket positions: ranks within
// the workgroup from LDS counters, one global add per workgroup and hub.
// Epoch P.epoch + blockIdx.y of a batch is drawn into its own table, counts
// and bucket lists (strides table_stride, cnt_stride, list_stride); the
// draw record, when set, keeps the draws of epoch record_epoch.
template <class Off>
__global__ __launch_bounds__(kDrawThreads) void k_group_draw(TrainParams P, uint32_t record_epoch,
                                                             const int32_t* slot_of, int32_t n_hot,
                                                             const int64_t* bstart, const int64_t* cap, int32_t* cnt,
                                                             int64_t cnt_stride, int32_t* list, int64_t list_stride,
                                                             int32_t* table, int64_t table_stride) {
    __shared__ int32_t lcnt[kMaxHot];
    __shared__ int32_t lbase[kMaxHot];
    for (int i = threadIdx.x; i < n_hot; i += kDrawThreads) lcnt[i] = 0;
    __syncthreads();
    P.epoch += blockIdx.y;
    cnt += blockIdx.y * cnt_stride;
    list += blockIdx.y * list_stride;
    table += blockIdx.y * table_stride;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * kDrawThreads + threadIdx.x;
    const int k = P.k;
    int32_t u[16];
    int hs = -1, rank = 0;
    if (s < P.n) {
        draw_source<Off>(P, s, u);
        for (int t = 0; t <= k; ++t) table[s * (1 + k) + t] = u[t];
        if (P.record && P.epoch == record_epoch)
            for (int t = 0; t <= k; ++t) P.record[s * (1 + k) + t] = u[t];
        if (u[0] >= 0) {
            hs = slot_of[u[0]];
            for (int t = 1; t <= k; ++t)
                if (u[t] == u[0]) hs = -1;
        }
        if (hs >= 0) rank = atomicAdd(&lcnt[hs], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_hot; i += kDrawThreads) {
        const int c = lcnt[i];
        lbase[i] = c > 0 ? atomicAdd(&cnt[i], c) : 0;
    }
    __syncthreads();
    if (hs >= 0) {
        const int64_t at = static_cast<int64_t>(lbase[hs]) + rank;
        if (at < cap[hs]) {
            list[bstart[hs] + at] = static_cast<int32_t>(s);
            table[s * (1 + k)] = -2 - hs;
        }
    }
}

// cstart[i] = chunks of the buckets before i (chunks of kChunk visits), for
// i in [0, n_hot]; one workgroup of 1024 threads per epoch of the batch
// (counts at cnt + blockIdx.x * cnt_stride, result at cstart + blockIdx.x *
// cstart_stride), n_hot <= 4096.
__global__ __launch_bounds__(1024) void k_group_chunks(const int32_t* cnt, int64_t cnt_stride, const int64_t* cap,
                                                       int32_t n_hot, int chunk, int64_t* cstart,
                                                       int64_t cstart_stride) {
    __shared__ int64_t part[1024];
    cnt += blockIdx.x * cnt_stride;
    cstart += blockIdx.x * cstart_stride;
    const int per = (n_hot + 1023) / 1024;
    const int i0 = threadIdx.x * per;
    int64_t local = 0;
    for (int i = i0; i < i0 + per && i < n_hot; ++i)
        local += (min(static_cast<int64_t>(cnt[i]), cap[i]) + chunk - 1) / chunk;
    part[threadIdx.x] = local;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan of the per-thread sums
        const int64_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int i = i0; i < i0 + per && i < n_hot; ++i) {
        cstart[i] = run;
        run += (min(static_cast<int64_t>(cnt[i]), cap[i]) + chunk - 1) / chunk;
    }
    if (threadIdx.x == 1023) cstart[n_hot] = part[1023];
}

struct GroupArgs {
    const int32_t* hub_of;
    const int64_t* bstart;
    const int64_t* cap;
    const int32_t* cnt;
    const int32_t* list;
    const int64_t* cstart;
    int32_t n_hot;
    int64_t hot_blocks;
};

// hot_blocks of the launch's workgroups take the bucket chunks, the others
// visit one source per lane group from the table (grouped visits skipped).
// The hot workgroups sit evenly among the others (workgroup floor(j T / H)
// is hot workgroup j, T workgroups in all, H hot).  The chunks are numbered
// in bit-reversed order over [0, 2^lg) ⊇ [0, total), and position q goes to
// hot workgroup floor(q H / 2^lg) when 2^lg <= H -- one chunk per workgroup
// at most, spread evenly over the launch -- else to workgroups q mod H in
// turn.  The chunks then run while the other visits do, and the chunks of
// one hub -- consecutive items -- spread over the whole launch, so a hub's
// visits meet its row at many different times, as in one launch per epoch.
// Taking the chunks from a counter instead bunched them at the launch's
// start (the first hot workgroups took them all, in chains), and running
// them all at the start made the hub rows of a 93k-vertex level overshoot.
template <bool BF16, int D, int KMAX, class Off>
__global__ __launch_bounds__(kBlock) void k_train_grouped(TrainParams P, GroupArgs A) {
    using Ly = Lanes<BF16, D>;
    using Elem = typename RowIO<BF16>::Elem;
    constexpr int L = Ly::kL;
    constexpr int G = Ly::kG;
    constexpr int W = Ly::kWPL;
    constexpr int kChunk = (kBlock / 64) * G;   // visits per chunk: every lane group of the workgroup
    constexpr int kWords = BF16 ? D / 2 : D;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const int64_t b = blockIdx.x, T = gridDim.x, H = A.hot_blocks;
    const int64_t hj = (b * H + T - 1) / T;   // hot workgroups before b: ceil(b H / T)
    if (!(hj < H && hj * T / H == b)) {
        const int64_t wave = (b - hj) * (kBlock / 64) + (threadIdx.x >> 6);
        const int64_t slot = wave * G + grp;
        const float l = visit<BF16, D, KMAX, Off, kTable>(P, slot, slot < P.n, gl);
        if (P.loss) wave_add_loss<L>(P.loss, l, gl);
        return;
    }
    __shared__ uint32_t hub_words[kWords];
    __shared__ float hub_delta[D];
    Elem* M = static_cast<Elem*>(P.emb);
    const int64_t total = A.cstart[A.n_hot];
    int lg = 0;
    while ((int64_t(1) << lg) < total) ++lg;
    const int64_t N2 = int64_t(1) << lg;
    int64_t q0 = hj, qend = N2, qstep = H;
    if (N2 <= H) {   // the one position q with floor(q H / N2) = hj, if any
        q0 = (hj * N2 + H - 1) / H;
        qend = (q0 < N2 && q0 * H / N2 == hj) ? q0 + 1 : 0;
        qstep = 1;
    }
    for (int64_t q = q0; q < qend; q += qstep) {
        const int64_t t = lg > 0 ? static_cast<int64_t>(__brev(static_cast<uint32_t>(q)) >> (32 - lg)) : 0;
        if (t >= total) continue;
        int lo = 0, hi = A.n_hot;   // last bucket whose first chunk is <= t
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.cstart[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int64_t i0 = (t - A.cstart[lo]) * kChunk;
        const int64_t count = min(static_cast<int64_t>(kChunk), min(static_cast<int64_t>(A.cnt[lo]), A.cap[lo]) - i0);
        const int64_t hub = A.hub_of[lo];
        const uint32_t* hrow = reinterpret_cast<const uint32_t*>(M + hub * D);
        // the hub row as committed so far (loads that bypass the workgroup's
        // non-coherent cache, which may hold the row from earlier in the launch)
        for (int i = threadIdx.x; i < kWords; i += kBlock)
            hub_words[i] = __hip_atomic_load(hrow + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int i = threadIdx.x; i < D; i += kBlock) hub_delta[i] = 0.0f;
        __syncthreads();
        const int j = (threadIdx.x >> 6) * G + grp;   // this lane group's visit of the chunk
        float l = 0.0f;
        if (j < count) {
            const int64_t src = A.list[A.bstart[lo] + i0 + j];
            int32_t u[KMAX + 1];
#pragma unroll
            for (int q = 0; q <= KMAX; ++q) u[q] = (q <= P.k) ? P.samples[src * (1 + P.k) + q] : -1;
            u[0] = static_cast<int32_t>(hub);
            const uint32_t plain = P.plain_neg != 0 ? ((2u << KMAX) - 1u) & ~1u : 0u;
            l = update_chain<BF16, D, KMAX, false, RowIO<BF16>, true>(
                M, src, M, src, u, P.k, P.lr, static_cast<uint32_t>(src), P.epoch, P.w2, 1u, 0u, P.key0, P.key1,
                P.updates, gl, plain, P.loss != nullptr, hub_words, hub_delta);
        }
        if (P.loss) wave_add_loss<L>(P.loss, l, gl);
        __syncthreads();
        if (threadIdx.x < L) {
            // the chunk's summed change, committed once: stochastically rounded
            // from the chunk's starting row (stream kind 9, counter chunk id)
            if constexpr (BF16) {
                uint32_t cur[W];
                float v[2 * W];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    cur[i] = hub_words[gl + L * i];
                    v[2 * i] = bf16_lo(cur[i]) + hub_delta[2 * (gl + L * i)];
                    v[2 * i + 1] = bf16_hi(cur[i]) + hub_delta[2 * (gl + L * i) + 1];
                }
                const uint4 bits = philox10(
                    make_uint4(static_cast<uint32_t>(t), P.epoch, P.w2,
                               stream_word3(9u, 0u, static_cast<uint32_t>(gl % Ly::kBlocks))),
                    P.key0, P.key1);
                uint32_t out[W];
                RowIO<true>::commit<D>(reinterpret_cast<uint16_t*>(M), hub, gl, cur, v, bits, out);
            } else {
                float dx[W];
#pragma unroll
                for (int e = 0; e < W; ++e) dx[e] = hub_delta[gl + L * e];
                RowIO<false>::add<D>(reinterpret_cast<float*>(M), hub, gl, dx);
            }
        }
        __syncthreads();
    }
}

using GroupLauncher = void (*)(const TrainParams&, const GroupArgs&, int64_t, hipStream_t);

template <bool BF16, int D, int KMAX, class Off>
void launch_grouped(const TrainParams& P, const GroupArgs& A, int64_t n, hipStream_t st) {
    constexpr int G = Lanes<BF16, D>::kG;
    const int64_t cold = ceil_div(n, static_cast<int64_t>(kBlock / 64) * G);
    hipLaunchKernelGGL((k_train_grouped<BF16, D, KMAX, Off>), dim3(static_cast<unsigned>(A.hot_blocks + cold)),
                       dim3(kBlock), 0, st, P, A);
}

template <bool BF16, int D, int KMAX>
GroupLauncher pick_goff(bool off64) {
    return off64 ? &launch_grouped<BF16, D, KMAX, int64_t> : &launch_grouped<BF16, D, KMAX, int32_t>;
}
template <bool BF16, int D>
GroupLauncher pick_gk(int k, bool off64) {
    if (k <= 1) return pick_goff<BF16, D, 1>(off64);
    if (k <= 3) return pick_goff<BF16, D, 3>(off64);
    if (k <= 7) return pick_goff<BF16, D, 7>(off64);
    return pick_goff<BF16, D, 15>(off64);
}
template <bool BF16>
GroupLauncher pick_gd(int d, int k, bool off64) {
    switch (d) {
        case 8: return pick_gk<BF16, 8>(k, off64);
        case 16: return pick_gk<BF16, 16>(k, off64);
        case 32: return pick_gk<BF16, 32>(k, off64);
        case 64: return pick_gk<BF16, 64>(k, off64);
        case 128: return pick_gk<BF16, 128>(k, off64);
        case 256: return pick_gk<BF16, 256>(k, off64);
    }
    return nullptr;
}

int chunk_visits(gosh_dtype dt, int d) {
    auto g = [&](auto bf) -> int {
        constexpr bool B = decltype(bf)::value;
        switch (d) {
            case 8: return (kBlock / 64) * Lanes<B, 8>::kG;
            case 16: return (kBlock / 64) * Lanes<B, 16>::kG;
            case 32: return (kBlock / 64) * Lanes<B, 32>::kG;
            case 64: return (kBlock / 64) * Lanes<B, 64>::kG;
            case 128: return (kBlock / 64) * Lanes<B, 128>::kG;
            default: return (kBlock / 64) * Lanes<B, 256>::kG;
        }
    };
    return dt == GOSH_BF16 ? g(std::true_type{}) : g(std::false_type{});
}

}  // namespace

bool train_level_grouped(Ctx* c, const Level& L, TrainParams P, gosh_dtype dt, int d, int epochs, float lr) {
    const int64_t n = L.n;
    const int64_t hot_deg = std::max<int64_t>(1, static_cast<int64_t>(c->group_factor * static_cast<double>(L.nnz) /
                                                                      static_cast<double>(n)));
    // bucketed hubs of the level: the first kMaxHot ids of degree >= hot_deg
    DevBuf<int32_t> flag(c, n);
    DevBuf<int64_t> pre(c, n);
    if (L.off64)
        hipLaunchKernelGGL(k_hot_flags<int64_t>, grid_for(n), dim3(kThreads), 0, c->stream,
                           static_cast<const int64_t*>(L.offsets), n, hot_deg, flag.p);
    else
        hipLaunchKernelGGL(k_hot_flags<int32_t>, grid_for(n), dim3(kThreads), 0, c->stream,
                           static_cast<const int32_t*>(L.offsets), n, hot_deg, flag.p);
    GOSH_HIP(hipGetLastError());
    int64_t hot = 0;
    scan_i32_to_i64(c, flag.p, pre.p, n, &hot);
    const int32_t n_hot = static_cast<int32_t>(std::min<int64_t>(hot, kMaxHot));
    if (n_hot == 0) return false;
    DevBuf<int32_t> slot(c, n), hub_of(c, n_hot);
    DevBuf<int64_t> cap(c, n_hot), bstart(c, n_hot);
    if (L.off64)
        hipLaunchKernelGGL(k_hot_slots<int64_t>, grid_for(n), dim3(kThreads), 0, c->stream,
                           static_cast<const int64_t*>(L.offsets), flag.p, pre.p, n, slot.p, hub_of.p, cap.p);
    else
        hipLaunchKernelGGL(k_hot_slots<int32_t>, grid_for(n), dim3(kThreads), 0, c->stream,
                           static_cast<const int32_t*>(L.offsets), flag.p, pre.p, n, slot.p, hub_of.p, cap.p);
    GOSH_HIP(hipGetLastError());
    flag.reset();
    pre.reset();
    int64_t capacity = 0;
    scan_i64(c, cap.p, bstart.p, n_hot, false, ScanOp::Sum, &capacity);
    // Draws do not depend on the rows, so a batch of epochs is drawn in one
    // launch (and its chunks laid out in another); the batch is sized so
    // that its tables and lists stay within kBatchBytes.
    const int64_t tstride = n * (1 + P.k);
    const int64_t lstride = std::max<int64_t>(capacity, 1);
    const int64_t cstride = (n_hot + 63) / 64 * 64;   // an epoch's counts, whole 256-byte lines
    const int64_t per_epoch = 4 * (tstride + lstride);
    const int batch = static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>({static_cast<int64_t>(kMaxBatch), static_cast<int64_t>(epochs),
                                                kBatchBytes / per_epoch})));
    DevBuf<int32_t> list(c, lstride * batch), table(c, tstride * batch), cnt(c, cstride * batch);
    DevBuf<int64_t> cstart(c, (n_hot + 1) * static_cast<int64_t>(batch));
    GroupLauncher fn = dt == GOSH_BF16 ? pick_gd<true>(d, P.k, L.off64) : pick_gd<false>(d, P.k, L.off64);
    GOSH_REQUIRE(fn, GOSH_E_INVALID_ARG, "unsupported training shape");
    const int chunk = chunk_visits(dt, d);
    const unsigned dblocks = static_cast<unsigned>(ceil_div(n, kDrawThreads));
    const uint32_t last = static_cast<uint32_t>(epochs - 1);
    for (int j = 0; j < epochs; ++j) {
        const int jb = j % batch;
        if (jb == 0) {
            const int nb = std::min(batch, epochs - j);
            TrainParams Q = P;
            Q.epoch = static_cast<uint32_t>(j);
            GOSH_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * cstride * nb, c->stream));
            const dim3 grid(dblocks, static_cast<unsigned>(nb));
            if (L.off64)
                hipLaunchKernelGGL(k_group_draw<int64_t>, grid, dim3(kDrawThreads), 0, c->stream, Q, last, slot.p,
                                   n_hot, bstart.p, cap.p, cnt.p, cstride, list.p, lstride, table.p, tstride);
            else
                hipLaunchKernelGGL(k_group_draw<int32_t>, grid, dim3(kDrawThreads), 0, c->stream, Q, last, slot.p,
                                   n_hot, bstart.p, cap.p, cnt.p, cstride, list.p, lstride, table.p, tstride);
            GOSH_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_group_chunks, dim3(static_cast<unsigned>(nb)), dim3(1024), 0, c->stream, cnt.p,
                               cstride, cap.p, n_hot, chunk, cstart.p, static_cast<int64_t>(n_hot + 1));
            GOSH_HIP(hipGetLastError());
        }
        const double f = 1.0 - static_cast<double>(j) / static_cast<double>(epochs);
        P.lr = static_cast<float>(static_cast<double>(lr) * (f > 1e-4 ? f : 1e-4));
        P.epoch = static_cast<uint32_t>(j);
        P.span = 1;
        P.loss = c->loss ? c->loss + j : nullptr;
        P.samples = table.p + jb * tstride;
        const GroupArgs A{hub_of.p, bstart.p, cap.p, cnt.p + jb * cstride, list.p + jb * lstride,
                          cstart.p + jb * (n_hot + 1), n_hot, kHotBlocks};
        fn(P, A, n, c->stream);
        GOSH_HIP(hipGetLastError());
    }
    return true;
}

}  // namespace gosh
