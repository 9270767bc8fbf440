// Batched TrainInGPU: many independent graphs (or coarse levels) trained by
// one call.  Each job is trained exactly as by gosh_train on its own graph
// (same Philox streams given its level and tag): its epochs never overlap,
// its sources run concurrently.  Jobs are independent of one another.
//
// Two executions, chosen by a small autotuner:
//  * persistent: one launch.  Work is cut into tasks (a chunk of one job's
//    sources in one epoch) numbered epoch-major: all tasks of epoch round 0
//    (every job, job by job), then round 1, ...  Waves take task numbers
//    from one global counter.  Before starting a task of epoch e a wave
//    waits until the job's completion counter shows all its tasks of epoch
//    e-1 done; those tasks carry smaller numbers, so they were taken by
//    waves that are already running and the wait ends.  Rows are read with
//    agent-scope loads (coherent across the XCDs) because epochs of one job
//    follow each other inside the launch.
//  * epoch graph: one launch per epoch round over the sources of all jobs
//    that still train in that round, the rounds recorded as a chain of
//    kernel nodes of one hipGraph and launched together.
// The autotuner times both (persistent with several grid sizes and chunk
// lengths) on a dry run of up to 8 epochs over scratch copies of the embeddings and
// caches the winner per (dtype, d, k, size class).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "device_util.hpp"
#include "gosh_internal.hpp"
#include "visit.hpp"

namespace gosh {
namespace {

using namespace train_detail;

struct BJob {
    const void* offsets;
    const int32_t* indices;
    void* emb;
    int64_t n;
    int64_t nnz;
    int64_t nchunks;     // tasks per epoch (persistent execution)
    float lr;
    int32_t epochs;
    uint32_t w2;         // level | tag << 8
    int32_t off64;
};

struct PersistArgs {
    const BJob* jobs;
    int32_t njobs;
    int32_t k;
    uint32_t key0, key1;
    int64_t chunk;                   // sources per task
    const int64_t* round_start;      // [max_e + 1]: first task number of each epoch round
    const int32_t* round_jobs;       // [max_e]: jobs still training in that round (a prefix)
    const int64_t* job_task0;        // [njobs + 1]: prefix of nchunks over the job list
    int32_t max_e;
    unsigned long long* next_task;
    unsigned long long* done;        // [njobs]: finished tasks of each job, all epochs
    unsigned long long* updates;     // self-negative decrements (may be null)
    unsigned int* error;
    unsigned long long spin_limit;
    int32_t seq;                     // deterministic: a task is a whole job epoch, visited in source order
};

struct MultiArgs {
    const BJob* jobs;
    const int64_t* job_src0;         // [njobs + 1]: prefix of n over the job list
    int32_t active;                  // jobs[0 .. active) train in this round
    int32_t epoch;
    int32_t k;
    uint32_t key0, key1;
    unsigned long long* updates;
};

__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ TrainParams job_params(const BJob& J, int epoch, int k, uint32_t key0, uint32_t key1,
                                                  unsigned long long* updates) {
    TrainParams P{};
    P.offsets = J.offsets;
    P.indices = J.indices;
    P.n = J.n;
    P.nnz = J.nnz;
    P.emb = J.emb;
    P.n_rows = J.n;
    const double f = 1.0 - static_cast<double>(epoch) / static_cast<double>(J.epochs);
    P.lr = static_cast<float>(static_cast<double>(J.lr) * (f > 1e-4 ? f : 1e-4));
    P.k = k;
    P.key0 = key0;
    P.key1 = key1;
    P.epoch = static_cast<uint32_t>(epoch);
    P.w2 = J.w2;
    P.updates = updates;
    return P;
}

template <bool BF16, int D, int KMAX, int MODE>
__device__ __forceinline__ void visit_job(const BJob& J, const TrainParams& P, int64_t src, bool active, int gl) {
    if (J.off64) visit<BF16, D, KMAX, int64_t, MODE>(P, src, active, gl);
    else visit<BF16, D, KMAX, int32_t, MODE>(P, src, active, gl);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Every wave schedules itself: it takes a task number, waits for the job's
// previous epoch, trains the task's sources and counts the task done.  The
// scheduling loop has no lane-dependent branch: all lanes take part in each
// scheduling atomic (lane 0 adds 1, the others 0, so the value read back
// through the first lane is the counter before the wave's addition) and in
// each load of a completion counter, and every decision is taken on values
// made wave-uniform, so the whole wave always runs the same iteration.
template <bool BF16, int D, int KMAX>
__global__ __launch_bounds__(kBlock) void k_persist(PersistArgs A) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const uint64_t one = lane == 0 ? 1ull : 0ull;
    const int64_t total = A.round_start[A.max_e];
    for (;;) {
        const int64_t t = static_cast<int64_t>(uniform64(
            __hip_atomic_fetch_add(A.next_task, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
        if (t >= total) break;
        // decode (epoch, job, chunk)
        const int e = static_cast<int>(upper_bound_i64(A.round_start, 0, A.max_e + 1, t) - 1);
        const int64_t r = t - A.round_start[e];
        const int j = static_cast<int>(upper_bound_i64(A.job_task0, 0, A.round_jobs[e] + 1, r) - 1);
        const int64_t c = r - A.job_task0[j];
        const BJob J = A.jobs[j];
        // the job's previous epoch must be complete
        const uint64_t need = static_cast<uint64_t>(e) * static_cast<uint64_t>(J.nchunks);
        bool skip = false;
        for (uint64_t spins = 0;; ++spins) {
            const uint64_t seen =
                uniform64(__hip_atomic_load(A.done + j, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
            if (seen >= need) break;
            if (spins >= A.spin_limit) {
                atomicOr(A.error, 1u);
                skip = true;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!skip) {
            const TrainParams P = job_params(J, e, A.k, A.key0, A.key1, A.updates);
            const int64_t beg = c * A.chunk;
            const int64_t end = min(J.n, beg + A.chunk);
            if (A.seq) {
                // one source at a time in ascending id order (Algorithm 3's
                // loop run sequentially, as gosh_train's deterministic mode)
                for (int64_t src = beg; src < end; ++src) {
                    visit_job<BF16, D, KMAX, kPersistent>(J, P, src, grp == 0, gl);
                    __threadfence();
                }
            } else {
                for (int64_t base = beg; base < end; base += G) {
                    const int64_t src = base + grp;
                    visit_job<BF16, D, KMAX, kPersistent>(J, P, src, src < end, gl);
                }
            }
        }
        // the wave's updates are performed before the task counts as done
        __threadfence();
        __hip_atomic_fetch_add(A.done + j, one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <bool BF16, int D, int KMAX>
__global__ __launch_bounds__(kBlock) void k_multi(MultiArgs A) {
    constexpr int L = Lanes<BF16, D>::kL;
    constexpr int G = Lanes<BF16, D>::kG;
    const int lane = threadIdx.x & 63;
    const int grp = lane / L, gl = lane % L;
    const int64_t slot = (static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6)) * G + grp;
    const int64_t total = A.job_src0[A.active];
    if (slot >= total) return;
    const int j = static_cast<int>(upper_bound_i64(A.job_src0, 0, A.active + 1, slot) - 1);
    const BJob J = A.jobs[j];
    const TrainParams P = job_params(J, A.epoch, A.k, A.key0, A.key1, A.updates);
    visit_job<BF16, D, KMAX, kEpoch>(J, P, slot - A.job_src0[j], true, gl);
}

// Jobs whose rows fit in LDS, one workgroup each: every epoch of job
// blockIdx.x inside the workgroup (train_rows_in_lds), rows read from HBM
// once and written back once.
template <bool BF16, int D, int KMAX>
__global__ __launch_bounds__(kLdsBlock) void k_batched_lds(const BJob* jobs, int k, uint32_t key0, uint32_t key1,
                                                           unsigned long long* updates) {
    extern __shared__ __align__(16) unsigned char lds_rows[];
    const BJob J = jobs[blockIdx.x];
    TrainParams P = job_params(J, 0, k, key0, key1, updates);
    P.e_total = J.epochs;
    P.lr0 = J.lr;
    if (J.off64) train_rows_in_lds<BF16, D, KMAX, int64_t>(P, lds_rows);
    else train_rows_in_lds<BF16, D, KMAX, int32_t>(P, lds_rows);
}

// Clears `n` 64-bit words (a kernel rather than a memset node, so that the
// call stays valid inside a captured stream).
__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0ull;
}

// Base count of UpdateEmbed calls of each job (self-negatives are
// subtracted by the training kernels): one block per job.
__global__ void k_add_job_updates(const BJob* jobs, int k, unsigned long long* updates) {
    const BJob J = jobs[blockIdx.x];
    unsigned long long cnt = 0;
    for (int64_t v = threadIdx.x; v < J.n; v += blockDim.x) {
        int64_t b, e;
        if (J.off64) {
            b = static_cast<const int64_t*>(J.offsets)[v];
            e = static_cast<const int64_t*>(J.offsets)[v + 1];
        } else {
            b = static_cast<const int32_t*>(J.offsets)[v];
            e = static_cast<const int32_t*>(J.offsets)[v + 1];
        }
        cnt += (e != b) ? 1ull : 0ull;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    unsigned long long add = ((threadIdx.x & 63) == 0) ? cnt * static_cast<unsigned long long>(J.epochs) : 0ull;
    if (threadIdx.x == 0)
        add += static_cast<unsigned long long>(k) * static_cast<unsigned long long>(J.n) * J.epochs;
    if (add) atomicAdd(updates, add);
}

// ---------------------------------------------------------------- dispatch
struct Kernels {
    const void* persist;
    const void* multi;
    int per_wave;      // sources per wave
    const void* lds;
};

template <bool BF16, int D, int KMAX>
Kernels kernels_for() {
    return Kernels{reinterpret_cast<const void*>(&k_persist<BF16, D, KMAX>),
                   reinterpret_cast<const void*>(&k_multi<BF16, D, KMAX>), Lanes<BF16, D>::kG,
                   reinterpret_cast<const void*>(&k_batched_lds<BF16, D, KMAX>)};
}

template <bool BF16, int D>
Kernels pick_k(int k) {
    if (k <= 1) return kernels_for<BF16, D, 1>();
    if (k <= 3) return kernels_for<BF16, D, 3>();
    if (k <= 7) return kernels_for<BF16, D, 7>();
    return kernels_for<BF16, D, 15>();
}

template <bool BF16>
Kernels pick_d(int d, int k) {
    switch (d) {
        case 8: return pick_k<BF16, 8>(k);
        case 16: return pick_k<BF16, 16>(k);
        case 32: return pick_k<BF16, 32>(k);
        case 64: return pick_k<BF16, 64>(k);
        case 128: return pick_k<BF16, 128>(k);
        case 256: return pick_k<BF16, 256>(k);
    }
    return Kernels{nullptr, nullptr, 0, nullptr};
}


// Device-side description of one batched call.
struct Plan {
    std::vector<BJob> jobs;          // sorted by epochs, descending
    int max_e = 0;
    DevBuf<BJob> djobs;
    DevBuf<int64_t> job_src0;        // prefix of n
    std::vector<int64_t> h_src0;
    std::vector<int32_t> h_active;   // jobs still training in each round
};

void build_plan(Ctx* c, const gosh_job* in, int njobs, Plan& P) {
    P.jobs.resize(njobs);
    for (int i = 0; i < njobs; ++i) {
        const gosh_job& q = in[i];
        BJob& J = P.jobs[i];
        J.offsets = q.g.offsets;
        J.indices = q.g.indices;
        J.emb = q.emb;
        J.n = q.g.n;
        J.nnz = q.g.nnz;
        J.lr = q.lr;
        J.epochs = q.epochs;
        J.w2 = stream_word2(q.level, q.tag);
        J.off64 = q.g.offsets_is_i64 ? 1 : 0;
        J.nchunks = 0;
    }
    std::stable_sort(P.jobs.begin(), P.jobs.end(), [](const BJob& a, const BJob& b) { return a.epochs > b.epochs; });
    P.max_e = njobs ? P.jobs[0].epochs : 0;
    P.h_src0.assign(njobs + 1, 0);
    for (int i = 0; i < njobs; ++i) P.h_src0[i + 1] = P.h_src0[i] + P.jobs[i].n;
    P.h_active.assign(P.max_e, 0);
    for (int e = 0; e < P.max_e; ++e) {
        int a = 0;
        while (a < njobs && P.jobs[a].epochs > e) ++a;
        P.h_active[e] = a;
    }
    P.job_src0 = DevBuf<int64_t>(c, njobs + 1);
    GOSH_HIP(hipMemcpyAsync(P.job_src0.p, P.h_src0.data(), sizeof(int64_t) * (njobs + 1), hipMemcpyHostToDevice,
                            c->stream));
}

struct RunShape {
    int mode;            // GOSH_BATCH_PERSISTENT or GOSH_BATCH_EPOCH_GRAPH
    int blocks_per_cu;
    int chunk_iters;     // sources per task = chunk_iters * sources per wave (0: a whole job, visited in order)
};

// Device tables of one persistent launch (see PersistArgs).
struct PersistTables {
    BJob* jobs;                      // [njobs]
    int64_t* round_start;            // [max_e + 1]
    int64_t* task0;                  // [njobs + 1]
    int32_t* active;                 // [max_e]
    unsigned long long* ctr;         // [njobs + 1]: done counters, then the task counter
    unsigned int* error;             // one word (cleared by the caller)
};

// Host side of the persistent execution: tasks per job and epoch round, the
// tables copied into `T`, counters cleared, one launch.  `jobs` holds the
// jobs sorted by epochs (descending) with epochs already capped.
void launch_persistent(Ctx* c, std::vector<BJob>& jobs, const std::vector<int32_t>& active, const RunShape& R,
                       const Kernels& K, int k, unsigned long long* updates, const PersistTables& T) {
    const int njobs = static_cast<int>(jobs.size());
    const int max_e = static_cast<int>(active.size());
    const bool seq = R.chunk_iters == 0;
    int64_t chunk = static_cast<int64_t>(K.per_wave) * R.chunk_iters;
    if (seq) {
        chunk = 1;
        for (const auto& J : jobs) chunk = std::max<int64_t>(chunk, J.n);
    }
    std::vector<int64_t> task0(njobs + 1, 0);
    for (int i = 0; i < njobs; ++i) {
        jobs[i].nchunks = ceil_div(jobs[i].n, chunk);
        task0[i + 1] = task0[i] + jobs[i].nchunks;
    }
    std::vector<int64_t> round_start(max_e + 1, 0);
    for (int e = 0; e < max_e; ++e) round_start[e + 1] = round_start[e] + task0[active[e]];
    GOSH_HIP(hipMemcpyAsync(T.jobs, jobs.data(), sizeof(BJob) * njobs, hipMemcpyHostToDevice, c->stream));
    GOSH_HIP(hipMemcpyAsync(T.round_start, round_start.data(), sizeof(int64_t) * (max_e + 1), hipMemcpyHostToDevice,
                            c->stream));
    GOSH_HIP(hipMemcpyAsync(T.task0, task0.data(), sizeof(int64_t) * (njobs + 1), hipMemcpyHostToDevice, c->stream));
    GOSH_HIP(hipMemcpyAsync(T.active, active.data(), sizeof(int32_t) * max_e, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_zero_u64, dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div(njobs + 1, 256), 64))),
                       dim3(256), 0, c->stream, T.ctr, static_cast<int64_t>(njobs + 1));
    GOSH_HIP(hipGetLastError());
    PersistArgs A{};
    A.jobs = T.jobs;
    A.njobs = njobs;
    A.k = k;
    A.key0 = static_cast<uint32_t>(c->seed);
    A.key1 = static_cast<uint32_t>(c->seed >> 32);
    A.chunk = chunk;
    A.round_start = T.round_start;
    A.round_jobs = T.active;
    A.job_task0 = T.task0;
    A.max_e = max_e;
    A.next_task = T.ctr + njobs;
    A.done = T.ctr;
    A.updates = updates;
    A.error = T.error;
    A.spin_limit = 1ull << 22;   // a few seconds of polling
    A.seq = seq ? 1 : 0;
    int cus = 0;
    GOSH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    // no more waves than tasks in the first (largest) epoch round: extra
    // waves could only poll the done counters of epochs not yet reached
    const int64_t round0 = round_start[1] - round_start[0];
    const int64_t waves =
        std::min<int64_t>(static_cast<int64_t>(cus) * std::max(R.blocks_per_cu, 1) * (kBlock / 64), round0);
    const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(1, ceil_div(waves, kBlock / 64)));
    void* args[] = {&A};
    GOSH_HIP(hipLaunchKernel(K.persist, dim3(blocks), dim3(kBlock), args, 0, c->stream));
}

// Runs the plan's jobs (with their epochs capped at `epochs_cap` if > 0).
void run(Ctx* c, Plan& P, const RunShape& R, const Kernels& K, int d, int k, int epochs_cap,
         unsigned long long* updates) {
    const int njobs = static_cast<int>(P.jobs.size());
    std::vector<BJob> jobs = P.jobs;
    if (epochs_cap > 0)
        for (auto& J : jobs) J.epochs = std::min(J.epochs, epochs_cap);
    const int max_e = njobs ? jobs[0].epochs : 0;
    if (max_e == 0) return;
    std::vector<int32_t> active(max_e);
    for (int e = 0; e < max_e; ++e) {
        int a = 0;
        while (a < njobs && jobs[a].epochs > e) ++a;
        active[e] = a;
    }
    const uint32_t key0 = static_cast<uint32_t>(c->seed), key1 = static_cast<uint32_t>(c->seed >> 32);
    if (R.mode == GOSH_BATCH_PERSISTENT) {
        DevBuf<BJob> dj(c, njobs);
        DevBuf<int64_t> drs(c, max_e + 1), dt0(c, njobs + 1);
        DevBuf<int32_t> dact(c, max_e);
        DevBuf<unsigned long long> ctr(c, njobs + 1);
        PersistTables T{dj.p, drs.p, dt0.p, dact.p, ctr.p,
                        reinterpret_cast<unsigned int*>(static_cast<char*>(c->scratch) + 256)};
        launch_persistent(c, jobs, active, R, K, k, updates, T);
        // the small buffers above are released to the context cache only; the
        // stream orders their reuse after this launch
    } else {
        DevBuf<BJob> dj(c, njobs);
        GOSH_HIP(hipMemcpyAsync(dj.p, jobs.data(), sizeof(BJob) * njobs, hipMemcpyHostToDevice, c->stream));
        const int per_block = (kBlock / 64) * K.per_wave;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        GOSH_HIP(hipGraphCreate(&graph, 0));
        try {
            std::vector<MultiArgs> margs(max_e);
            hipGraphNode_t prev = nullptr;
            for (int e = 0; e < max_e; ++e) {
                MultiArgs& M = margs[e];
                M.jobs = dj.p;
                M.job_src0 = P.job_src0.p;
                M.active = active[e];
                M.epoch = e;
                M.k = k;
                M.key0 = key0;
                M.key1 = key1;
                M.updates = updates;
                void* args[] = {&margs[e]};
                hipKernelNodeParams kp{};
                kp.func = const_cast<void*>(K.multi);
                kp.gridDim = dim3(static_cast<unsigned>(std::max<int64_t>(1, ceil_div(P.h_src0[active[e]], per_block))));
                kp.blockDim = dim3(kBlock);
                kp.sharedMemBytes = 0;
                kp.kernelParams = args;
                kp.extra = nullptr;
                hipGraphNode_t node;
                GOSH_HIP(hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
                prev = node;
            }
            GOSH_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            GOSH_HIP(hipGraphLaunch(exec, c->stream));
            GOSH_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            if (exec) (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            throw;
        }
        GOSH_HIP(hipGraphExecDestroy(exec));
        GOSH_HIP(hipGraphDestroy(graph));
    }
    GOSH_HIP(hipGetLastError());
}

int log2_bucket(int64_t x) {
    int b = 0;
    while ((int64_t(1) << b) < std::max<int64_t>(x, 1)) ++b;
    return b;
}

std::string tune_key(gosh_dtype dt, int d, int k, const Plan& P) {
    int64_t work = 0;
    for (const auto& J : P.jobs) work += J.n;
    return std::string(dt == GOSH_BF16 ? "bf16" : "f32") + "/d" + std::to_string(d) + "/k" + std::to_string(k) +
           "/S" + std::to_string(log2_bucket(work)) + "/J" + std::to_string(log2_bucket(static_cast<int64_t>(P.jobs.size()))) +
           "/E" + std::to_string(log2_bucket(P.max_e));
}

RunShape autotune(Ctx* c, Plan& P, const Kernels& K, gosh_dtype dt, int d, int k) {
    // candidates timed on a dry run of up to 8 epochs over scratch copies of
    // the rows (two epochs hide the cost of waiting on earlier epochs, which
    // dominates a job with many short epochs)
    const int dry = std::max(1, std::min(P.max_e, 8));
    const size_t elem = dt == GOSH_BF16 ? 2 : 4;
    size_t bytes = 0;
    for (const auto& J : P.jobs) bytes += static_cast<size_t>(J.n) * d * elem;
    DevBuf<char> scratch(c, std::max<size_t>(bytes, 256));
    Plan T;
    T.jobs = P.jobs;
    T.max_e = P.max_e;
    T.h_src0 = P.h_src0;
    T.h_active = P.h_active;
    T.job_src0 = DevBuf<int64_t>(c, P.jobs.size() + 1);
    GOSH_HIP(hipMemcpyAsync(T.job_src0.p, P.job_src0.p, sizeof(int64_t) * (P.jobs.size() + 1),
                            hipMemcpyDeviceToDevice, c->stream));
    size_t at = 0;
    for (auto& J : T.jobs) {
        const size_t nb = static_cast<size_t>(J.n) * d * elem;
        GOSH_HIP(hipMemcpyAsync(scratch.p + at, J.emb, nb, hipMemcpyDeviceToDevice, c->stream));
        J.emb = scratch.p + at;
        at += nb;
    }
    std::vector<RunShape> cand = {{GOSH_BATCH_EPOCH_GRAPH, 0, 0}};
    for (int bpc : {1, 2, 4})
        for (int it : {1, 4, 16}) cand.push_back({GOSH_BATCH_PERSISTENT, bpc, it});
    hipEvent_t a, b;
    GOSH_HIP(hipEventCreate(&a));
    GOSH_HIP(hipEventCreate(&b));
    RunShape best = cand[1];
    float best_ms = 1e30f;
    try {
        run(c, T, cand[1], K, d, k, 1, nullptr);   // warm-up
        for (const auto& R : cand) {
            GOSH_HIP(hipEventRecord(a, c->stream));
            run(c, T, R, K, d, k, dry, nullptr);
            GOSH_HIP(hipEventRecord(b, c->stream));
            GOSH_HIP(hipEventSynchronize(b));
            float ms = 0;
            GOSH_HIP(hipEventElapsedTime(&ms, a, b));
            if (ms < best_ms) {
                best_ms = ms;
                best = R;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    GOSH_HIP(hipStreamSynchronize(c->stream));
    return best;
}

void load_tune_file(Ctx* c) {
    if (c->tune_loaded) return;
    c->tune_loaded = true;
    const char* path = std::getenv("GOSH_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    int mode, bpc, it;
    while (std::fscanf(f, "%255s %d %d %d", key, &mode, &bpc, &it) == 4)
        c->tune[key] = {mode, bpc, it};
    std::fclose(f);
}

void save_tune_entry(const std::string& key, const RunShape& R) {
    const char* path = std::getenv("GOSH_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d\n", key.c_str(), R.mode, R.blocks_per_cu, R.chunk_iters);
    std::fclose(f);
}

// Checks the job list of a batched call and keeps the jobs with work.
std::vector<gosh_job> checked_jobs(const gosh_job* jobs, int njobs, gosh_dtype dt, int d, int k) {
    GOSH_REQUIRE(njobs >= 0 && (njobs == 0 || jobs), GOSH_E_INVALID_ARG, "bad job list");
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
    GOSH_REQUIRE(d == 8 || d == 16 || d == 32 || d == 64 || d == 128 || d == 256, GOSH_E_INVALID_ARG,
                 "d must be one of 8, 16, 32, 64, 128, 256");
    GOSH_REQUIRE(k >= 0 && k <= 15, GOSH_E_INVALID_ARG, "k must be in [0, 15]");
    std::vector<gosh_job> kept;
    for (int i = 0; i < njobs; ++i) {
        const gosh_job& q = jobs[i];
        GOSH_REQUIRE(q.g.n >= 0 && q.g.nnz >= 0 && q.g.n < INT32_MAX, GOSH_E_INVALID_ARG, "bad job graph shape");
        GOSH_REQUIRE(q.g.offsets && (q.g.nnz == 0 || q.g.indices), GOSH_E_INVALID_ARG, "null job graph");
        GOSH_REQUIRE(q.g.offsets_is_i64 || q.g.nnz <= INT32_MAX, GOSH_E_INVALID_ARG, "nnz needs int64 offsets");
        GOSH_REQUIRE(q.epochs >= 0, GOSH_E_INVALID_ARG, "epochs must be >= 0");
        GOSH_REQUIRE(std::isfinite(q.lr) && q.lr >= 0.0f, GOSH_E_INVALID_ARG, "lr must be finite and >= 0");
        GOSH_REQUIRE(q.tag < (1u << 24) && q.level >= 0, GOSH_E_INVALID_ARG, "bad level or tag");
        GOSH_REQUIRE(q.g.n == 0 || q.emb, GOSH_E_INVALID_ARG, "null job embedding");
        if (q.g.n > 0 && q.epochs > 0) kept.push_back(q);
    }
    return kept;
}

// ---------------------------------------------------------------- no-allocation entry
// The device tables of gosh_train_batched_noalloc live in this file-scope
// array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only names a stand-in
// symbol): its device address is looked up once per device and kept in
// g_scratch_dev.
constexpr int kNoAllocMaxJobs = 4096;
constexpr int kNoAllocMaxEpochs = 16384;
constexpr size_t kTabJobs = 0;
constexpr size_t kTabRounds = kTabJobs + sizeof(BJob) * kNoAllocMaxJobs;
constexpr size_t kTabTask0 = kTabRounds + sizeof(int64_t) * (kNoAllocMaxEpochs + 1);
constexpr size_t kTabActive = kTabTask0 + sizeof(int64_t) * (kNoAllocMaxJobs + 1);
constexpr size_t kTabCtr = (kTabActive + sizeof(int32_t) * kNoAllocMaxEpochs + 255) / 256 * 256;
constexpr size_t kTabEnd = kTabCtr + sizeof(unsigned long long) * (kNoAllocMaxJobs + 2);   // + error word
constexpr size_t kScratchBytes = (kTabEnd + 255) / 256 * 256;
static_assert(kTabRounds % 8 == 0 && kTabTask0 % 8 == 0 && kTabActive % 8 == 0, "table alignment");
static_assert(sizeof(BJob) == 64 && kScratchBytes == 524800, "size stated in gosh.h");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

void batched_noalloc_init(int device) {
    GOSH_REQUIRE(device >= 0 && device < kMaxDevices, GOSH_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return;
    void* ptr = nullptr;
    // called with `device` current: its own copy of the array
    GOSH_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    GOSH_REQUIRE(ptr != nullptr, GOSH_E_DEVICE, "no device address for the batched scratch array");
    g_scratch_dev[device] = ptr;
}

void train_batched_noalloc(Ctx* c, const gosh_job* jobs, int njobs, gosh_dtype dt, int d, int k,
                           uint64_t* updates_dev) {
    std::vector<gosh_job> kept = checked_jobs(jobs, njobs, dt, d, k);
    GOSH_REQUIRE(kept.size() <= static_cast<size_t>(kNoAllocMaxJobs), GOSH_E_INVALID_ARG,
                 "gosh_train_batched_noalloc takes at most 4096 jobs with work");
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = static_cast<char*>(c->device >= 0 && c->device < kMaxDevices ? g_scratch_dev[c->device] : nullptr);
    }
    GOSH_REQUIRE(base, GOSH_E_DEVICE, "batched scratch array not set up on this device");
    std::vector<BJob> bj(kept.size());
    for (size_t i = 0; i < kept.size(); ++i) {
        const gosh_job& q = kept[i];
        BJob& J = bj[i];
        J.offsets = q.g.offsets;
        J.indices = q.g.indices;
        J.emb = q.emb;
        J.n = q.g.n;
        J.nnz = q.g.nnz;
        J.lr = q.lr;
        J.epochs = q.epochs;
        J.w2 = stream_word2(q.level, q.tag);
        J.off64 = q.g.offsets_is_i64 ? 1 : 0;
        J.nchunks = 0;
    }
    std::stable_sort(bj.begin(), bj.end(), [](const BJob& a, const BJob& b) { return a.epochs > b.epochs; });
    const int max_e = bj.empty() ? 0 : bj[0].epochs;
    GOSH_REQUIRE(max_e <= kNoAllocMaxEpochs, GOSH_E_INVALID_ARG,
                 "gosh_train_batched_noalloc takes at most 16384 epochs per job");
    // error word first (one 64-bit slot), then the done counters and the task counter
    PersistTables T{reinterpret_cast<BJob*>(base + kTabJobs), reinterpret_cast<int64_t*>(base + kTabRounds),
                    reinterpret_cast<int64_t*>(base + kTabTask0), reinterpret_cast<int32_t*>(base + kTabActive),
                    reinterpret_cast<unsigned long long*>(base + kTabCtr + sizeof(unsigned long long)),
                    reinterpret_cast<unsigned int*>(base + kTabCtr)};
    // a call keeps the array's last contents: clear the error word (and the counters)
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c->stream,
                       reinterpret_cast<unsigned long long*>(base + kTabCtr), static_cast<int64_t>(bj.size() + 2));
    GOSH_HIP(hipGetLastError());
    if (bj.empty()) return;
    std::vector<int32_t> active(max_e);
    for (int e = 0; e < max_e; ++e) {
        int a = 0;
        while (a < static_cast<int>(bj.size()) && bj[a].epochs > e) ++a;
        active[e] = a;
    }
    const Kernels K = dt == GOSH_BF16 ? pick_d<true>(d, k) : pick_d<false>(d, k);
    const RunShape R = c->deterministic ? RunShape{GOSH_BATCH_PERSISTENT, 2, 0} : RunShape{GOSH_BATCH_PERSISTENT, 2, 4};
    auto* upd = reinterpret_cast<unsigned long long*>(updates_dev);
    // launch_persistent clears the counters again (the same words) before its launch
    launch_persistent(c, bj, active, R, K, k, upd, T);
    if (upd) {
        hipLaunchKernelGGL(k_add_job_updates, dim3(static_cast<unsigned>(bj.size())), dim3(256), 0, c->stream, T.jobs,
                           k, upd);
        GOSH_HIP(hipGetLastError());
    }
}

unsigned int batched_noalloc_error(Ctx* c) {
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = static_cast<char*>(c->device >= 0 && c->device < kMaxDevices ? g_scratch_dev[c->device] : nullptr);
    }
    GOSH_REQUIRE(base, GOSH_E_DEVICE, "batched scratch array not set up on this device");
    GOSH_HIP(hipStreamSynchronize(c->stream));
    unsigned int err = 0;
    GOSH_HIP(hipMemcpy(&err, base + kTabCtr, sizeof(err), hipMemcpyDeviceToHost));
    return err;
}

void train_batched(Ctx* c, const gosh_job* jobs, int njobs, gosh_dtype dt, int d, int k, int mode,
                   uint64_t* updates_dev, int32_t* chosen) {
    GOSH_REQUIRE(mode >= GOSH_BATCH_AUTO && mode <= GOSH_BATCH_EPOCH_GRAPH, GOSH_E_INVALID_ARG, "bad batch mode");
    std::vector<gosh_job> kept = checked_jobs(jobs, njobs, dt, d, k);
    if (chosen) chosen[0] = chosen[1] = chosen[2] = 0;
    if (kept.empty()) return;
    const Kernels K = dt == GOSH_BF16 ? pick_d<true>(d, k) : pick_d<false>(d, k);
    if (!c->deterministic && c->lds_max > 0) {
        // jobs whose rows fit in one workgroup's LDS: one workgroup each
        std::vector<BJob> lj;
        std::vector<gosh_job> rest;
        int64_t bytes = 0;
        for (const auto& q : kept) {
            const int64_t b = lds_level_bytes(q.g.n, d, dt == GOSH_BF16 ? 2 : 4, k);
            if (q.g.n <= c->lds_max && b <= 160 * 1024) {
                BJob J{};
                J.offsets = q.g.offsets;
                J.indices = q.g.indices;
                J.emb = q.emb;
                J.n = q.g.n;
                J.nnz = q.g.nnz;
                J.lr = q.lr;
                J.epochs = q.epochs;
                J.w2 = stream_word2(q.level, q.tag);
                J.off64 = q.g.offsets_is_i64 ? 1 : 0;
                lj.push_back(J);
                bytes = std::max(bytes, b);
            } else {
                rest.push_back(q);
            }
        }
        if (!lj.empty()) {
            DevBuf<BJob> dj(c, lj.size());
            GOSH_HIP(hipMemcpyAsync(dj.p, lj.data(), sizeof(BJob) * lj.size(), hipMemcpyHostToDevice, c->stream));
            GOSH_HIP(hipFuncSetAttribute(K.lds, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)));
            auto* upd = reinterpret_cast<unsigned long long*>(updates_dev);
            const uint32_t key0 = static_cast<uint32_t>(c->seed), key1 = static_cast<uint32_t>(c->seed >> 32);
            const BJob* jp = dj.p;
            void* args[] = {&jp, &k, const_cast<uint32_t*>(&key0), const_cast<uint32_t*>(&key1), &upd};
            GOSH_HIP(hipLaunchKernel(K.lds, dim3(static_cast<unsigned>(lj.size())), dim3(kLdsBlock), args,
                                     static_cast<size_t>(bytes), c->stream));
            if (upd) {
                hipLaunchKernelGGL(k_add_job_updates, dim3(static_cast<unsigned>(lj.size())), dim3(256), 0,
                                   c->stream, dj.p, k, upd);
                GOSH_HIP(hipGetLastError());
            }
        }
        kept.swap(rest);
        if (kept.empty()) return;
    }
    Plan P;
    build_plan(c, kept.data(), static_cast<int>(kept.size()), P);
    RunShape R{GOSH_BATCH_PERSISTENT, 2, 4};
    if (c->deterministic) {
        // each job epoch one task visited in source order: per job exactly
        // gosh_train's deterministic mode; jobs still run side by side
        R = {GOSH_BATCH_PERSISTENT, 2, 0};
    } else if (mode == GOSH_BATCH_EPOCH_GRAPH) {
        R = {GOSH_BATCH_EPOCH_GRAPH, 0, 0};
    } else if (mode == GOSH_BATCH_AUTO) {
        load_tune_file(c);
        const std::string key = tune_key(dt, d, k, P);
        auto it = c->tune.find(key);
        if (it != c->tune.end()) {
            R = {it->second[0], it->second[1], it->second[2]};
        } else {
            R = autotune(c, P, K, dt, d, k);
            c->tune[key] = {R.mode, R.blocks_per_cu, R.chunk_iters};
            save_tune_entry(key, R);
        }
    }
    unsigned int* err = reinterpret_cast<unsigned int*>(static_cast<char*>(c->scratch) + 256);
    GOSH_HIP(hipMemsetAsync(err, 0, 4, c->stream));
    auto* upd = reinterpret_cast<unsigned long long*>(updates_dev);
    run(c, P, R, K, d, k, 0, upd);
    if (upd) {
        DevBuf<BJob> dj(c, P.jobs.size());
        GOSH_HIP(hipMemcpyAsync(dj.p, P.jobs.data(), sizeof(BJob) * P.jobs.size(), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_add_job_updates, dim3(static_cast<unsigned>(P.jobs.size())), dim3(256), 0, c->stream,
                           dj.p, k, upd);
        GOSH_HIP(hipGetLastError());
    }
    if (chosen) {
        chosen[0] = R.mode;
        chosen[1] = R.blocks_per_cu;
        chosen[2] = R.chunk_iters;
    }
}

}  // namespace gosh
