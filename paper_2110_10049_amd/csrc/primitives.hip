// Device-wide scans and a stable LSD radix sort for gfx950 (wave64).
#include "primitives.hpp"

#include "device_util.hpp"

namespace gosh {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <ScanOp OP>
__host__ __device__ __forceinline__ int64_t apply(int64_t a, int64_t b) {
    if constexpr (OP == ScanOp::Sum) return a + b;
    else return a > b ? a : b;
}

// Inclusive scan across a wave64.
template <ScanOp OP>
__device__ __forceinline__ int64_t wave_inclusive(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v = apply<OP>(v, t);
    }
    return v;
}

// Exclusive scan of one value per thread across the block; *total receives
// the block total.
template <ScanOp OP>
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* total) {
    __shared__ int64_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t inc = wave_inclusive<OP>(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0;
    int64_t all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w) before = apply<OP>(before, wsum[i]);
        all = apply<OP>(all, wsum[i]);
    }
    __syncthreads();
    *total = all;
    const int64_t ex_in_wave = __shfl_up(inc, 1, 64);
    return apply<OP>(before, lane ? ex_in_wave : 0);
}

template <class T, ScanOp OP>
__global__ __launch_bounds__(kScanThreads) void k_tile_reduce(const T* in, int64_t n, int64_t* part) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i * kScanThreads + threadIdx.x;
        if (idx < n) acc = apply<OP>(acc, static_cast<int64_t>(in[idx]));
    }
    int64_t total;
    block_exclusive<OP>(acc, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// A thread's kScanItems consecutive items: 16-byte accesses when the run is
// whole and aligned (the scans are bandwidth-bound), element-wise otherwise.
template <class T>
__device__ __forceinline__ void load_run(const T* in, int64_t start, int64_t n, int64_t (&v)[kScanItems]) {
    static_assert(kScanItems * sizeof(T) % 16 == 0, "whole 16-byte chunks");
    if (start + kScanItems <= n && (reinterpret_cast<uintptr_t>(in + start) & 15u) == 0) {
        constexpr int per = 16 / sizeof(T);
#pragma unroll
        for (int c = 0; c < kScanItems / per; ++c) {
            const int4 w = reinterpret_cast<const int4*>(in + start)[c];
            T t[per];
            __builtin_memcpy(t, &w, 16);
#pragma unroll
            for (int j = 0; j < per; ++j) v[c * per + j] = static_cast<int64_t>(t[j]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) v[i] = start + i < n ? static_cast<int64_t>(in[start + i]) : 0;
    }
}

__device__ __forceinline__ void store_run(int64_t* out, int64_t start, int64_t n, const int64_t (&r)[kScanItems]) {
    if (start + kScanItems <= n && (reinterpret_cast<uintptr_t>(out + start) & 15u) == 0) {
#pragma unroll
        for (int c = 0; c < kScanItems / 2; ++c) {
            int4 w;
            __builtin_memcpy(&w, &r[2 * c], 16);
            reinterpret_cast<int4*>(out + start)[c] = w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            if (start + i < n) out[start + i] = r[i];
    }
}

// Scans one tile per block (blocked arrangement: thread t owns items
// [t*kScanItems, (t+1)*kScanItems) of the tile), adding prefix[block].  With
// all_out set, the thread holding item n-1 writes the reduction of all n
// inputs there (a pinned host slot: no copy back).
template <class T, ScanOp OP>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T* in, int64_t* out, int64_t n,
                                                             const int64_t* prefix, int inclusive, int64_t* all_out) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    const int64_t start = base + static_cast<int64_t>(threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    load_run(in, start, n, v);
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) acc = apply<OP>(acc, v[i]);
    int64_t total;
    int64_t run = block_exclusive<OP>(acc, &total);
    if (prefix) run = apply<OP>(prefix[blockIdx.x], run);
    int64_t r[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t nxt = apply<OP>(run, v[i]);
        r[i] = inclusive ? nxt : run;
        if (all_out && start + i == n - 1) *all_out = nxt;
        run = nxt;
    }
    store_run(out, start, n, r);
}

template <class T, ScanOp OP>
void scan_launch(Ctx* c, const T* in, int64_t* out, int64_t n, bool inclusive, int64_t* total) {
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL((k_tile_scan<T, OP>), dim3(1), dim3(kScanThreads), 0, c->stream, in, out,
                           n, nullptr, inclusive ? 1 : 0, total);
        GOSH_HIP(hipGetLastError());
        return;
    }
    DevBuf<int64_t> part(c, nb);
    hipLaunchKernelGGL((k_tile_reduce<T, OP>), dim3(nb), dim3(kScanThreads), 0, c->stream, in, n,
                       part.p);
    GOSH_HIP(hipGetLastError());
    scan_launch<int64_t, OP>(c, part.p, part.p, nb, false, nullptr);
    hipLaunchKernelGGL((k_tile_scan<T, OP>), dim3(nb), dim3(kScanThreads), 0, c->stream, in, out, n,
                       part.p, inclusive ? 1 : 0, total);
    GOSH_HIP(hipGetLastError());
}

template <class T, ScanOp OP>
void scan_impl(Ctx* c, const T* in, int64_t* out, int64_t n, bool inclusive, int64_t* total_host) {
    if (n <= 0) {
        if (total_host) *total_host = 0;
        return;
    }
    // The scan kernel writes the total into a pinned slot of the context
    // (no copy kernel), and the host waits once.
    scan_launch<T, OP>(c, in, out, n, inclusive, total_host ? c->pinned_dev + 1 : nullptr);
    if (total_host) {
        GOSH_HIP(hipStreamSynchronize(c->stream));
        *total_host = c->pinned[1];
    }
}

// ---------------------------------------------------------------- radix sort
constexpr int kSortThreads = 256;
constexpr int kRadix = 256;
constexpr int kWaves = kSortThreads / 64;

// ITEMS keys per thread: a tile of ITEMS * 256 keys per workgroup (16 for
// large inputs; 4 when 16 would leave most compute units without a tile)
template <class K, int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* keys, int64_t n, int shift,
                                                             int64_t* hist, int64_t nb) {
    constexpr int kSortItems = ITEMS;
    constexpr int kSortTile = kSortThreads * ITEMS;
    __shared__ int cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t idx = base + i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[static_cast<int>((keys[idx] >> shift) & (kRadix - 1))], 1);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Scatters one tile, stable (keys of equal digit keep their input order).
// All keys of the tile are loaded first; the tile is then ranked in rounds of
// 256 consecutive keys (a key's rank among equal digits: earlier rounds,
// earlier waves of its round, earlier lanes of its wave found with 8 ballots)
// and placed at its tile-local position in LDS, so that the final copy to
// the output writes each digit's run of the tile with consecutive lanes.
template <class K, bool VALS, int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K* keys, K* keys_out,
                                                                const uint32_t* vals,
                                                                uint32_t* vals_out, int64_t n,
                                                                int shift, const int64_t* offs,
                                                                int64_t nb) {
    constexpr int kSortItems = ITEMS;
    constexpr int kSortTile = kSortThreads * ITEMS;
    __shared__ int64_t base_off[kRadix];     // output position of the tile's first key of each digit
    __shared__ int local_start[kRadix];      // tile position of the first key of each digit
    __shared__ int placed[kRadix];           // keys of each digit placed by earlier rounds
    __shared__ int wave_cnt[kWaves][kRadix];
    __shared__ int wave_tot[kWaves];
    __shared__ K sk[kSortTile];
    __shared__ uint32_t sv[VALS ? kSortTile : 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * kSortTile;
    const int len = static_cast<int>(n - tile < kSortTile ? n - tile : kSortTile);

    K key[kSortItems];
    uint32_t val[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = r * kSortThreads + tid;
        key[r] = i < len ? keys[tile + i] : K(0);
        val[r] = (VALS && i < len) ? vals[tile + i] : 0u;
    }
    base_off[tid] = offs[static_cast<int64_t>(tid) * nb + blockIdx.x];
    local_start[tid] = 0;
    placed[tid] = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) wave_cnt[i][tid] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (r * kSortThreads + tid < len) atomicAdd(&local_start[static_cast<int>((key[r] >> shift) & (kRadix - 1))], 1);
    __syncthreads();
    {
        // exclusive scan of the 256 digit counts, one per thread
        const int cnt = local_start[tid];
        int inc = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) wave_tot[w] = inc;
        __syncthreads();
        int before = 0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i)
            if (i < w) before += wave_tot[i];
        local_start[tid] = before + inc - cnt;
    }
    __syncthreads();

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (r * kSortThreads >= len) break;   // the same for the whole block
        const bool valid = r * kSortThreads + tid < len;
        const int digit = static_cast<int>((key[r] >> shift) & (kRadix - 1));
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1;
            const uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wave_cnt[w][digit] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = local_start[digit] + placed[digit] + rank;
            for (int i = 0; i < w; ++i) pos += wave_cnt[i][digit];
            sk[pos] = key[r];
            if constexpr (VALS) sv[pos] = val[r];
        }
        __syncthreads();
        {
            int add = 0;
#pragma unroll
            for (int i = 0; i < kWaves; ++i) {
                add += wave_cnt[i][tid];
                wave_cnt[i][tid] = 0;
            }
            placed[tid] += add;
        }
        __syncthreads();
    }
    for (int i = tid; i < len; i += kSortThreads) {
        const K k = sk[i];
        const int digit = static_cast<int>((k >> shift) & (kRadix - 1));
        const int64_t pos = base_off[digit] + (i - local_start[digit]);
        keys_out[pos] = k;
        if constexpr (VALS) vals_out[pos] = sv[i];
    }
}


template <class K, bool VALS, int ITEMS>
void radix_sort_impl(Ctx* c, K* keys, K* keys_tmp, uint32_t* vals, uint32_t* vals_tmp, int64_t n,
                     int bits, bool* in_tmp) {
    if (in_tmp) *in_tmp = false;
    if (n <= 1 || bits <= 0) return;
    const int64_t nb = ceil_div(n, static_cast<int64_t>(kSortThreads) * ITEMS);
    DevBuf<int64_t> hist(c, static_cast<size_t>(nb) * kRadix);
    K* src = keys;
    K* dst = keys_tmp;
    uint32_t* vsrc = vals;
    uint32_t* vdst = vals_tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL((k_radix_hist<K, ITEMS>), dim3(nb), dim3(kSortThreads), 0, c->stream, src, n,
                           shift, hist.p, nb);
        GOSH_HIP(hipGetLastError());
        scan_impl<int64_t, ScanOp::Sum>(c, hist.p, hist.p, nb * kRadix, false, nullptr);
        hipLaunchKernelGGL((k_radix_scatter<K, VALS, ITEMS>), dim3(nb), dim3(kSortThreads), 0, c->stream,
                           src, dst, vsrc, vdst, n, shift, hist.p, nb);
        GOSH_HIP(hipGetLastError());
        std::swap(src, dst);
        std::swap(vsrc, vdst);
    }
    if (src != keys && in_tmp) {
        *in_tmp = true;   // the caller takes the result from the _tmp buffers
    } else if (src != keys) {
        GOSH_HIP(hipMemcpyAsync(keys, src, sizeof(K) * n, hipMemcpyDeviceToDevice, c->stream));
        if (VALS)
            GOSH_HIP(hipMemcpyAsync(vals, vsrc, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice,
                                    c->stream));
    }
}

}  // namespace

void scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n, bool inclusive, ScanOp op,
              int64_t* total_host) {
    if (op == ScanOp::Sum) scan_impl<int64_t, ScanOp::Sum>(c, in, out, n, inclusive, total_host);
    else scan_impl<int64_t, ScanOp::Max>(c, in, out, n, inclusive, total_host);
}

void scan_i32_to_i64(Ctx* c, const int32_t* in, int64_t* out, int64_t n, int64_t* total_host) {
    scan_impl<int32_t, ScanOp::Sum>(c, in, out, n, false, total_host);
}

// Inputs below kLargeSort keys sort in tiles of 1,024 keys (a tile of 4,096
// would leave most of the 256 compute units idle on a coarse level).
constexpr int64_t kLargeSort = int64_t(4) << 20;

void radix_sort_u32(Ctx* c, uint32_t* keys, uint32_t* keys_tmp, uint32_t* vals,
                    uint32_t* vals_tmp, int64_t n, int bits, bool* in_tmp) {
    if (n >= kLargeSort) {
        if (vals) radix_sort_impl<uint32_t, true, 16>(c, keys, keys_tmp, vals, vals_tmp, n, bits, in_tmp);
        else radix_sort_impl<uint32_t, false, 16>(c, keys, keys_tmp, nullptr, nullptr, n, bits, in_tmp);
    } else {
        if (vals) radix_sort_impl<uint32_t, true, 4>(c, keys, keys_tmp, vals, vals_tmp, n, bits, in_tmp);
        else radix_sort_impl<uint32_t, false, 4>(c, keys, keys_tmp, nullptr, nullptr, n, bits, in_tmp);
    }
}

void radix_sort_u64(Ctx* c, uint64_t* keys, uint64_t* keys_tmp, int64_t n, int bits, bool* in_tmp) {
    if (n >= kLargeSort) radix_sort_impl<uint64_t, false, 16>(c, keys, keys_tmp, nullptr, nullptr, n, bits, in_tmp);
    else radix_sort_impl<uint64_t, false, 4>(c, keys, keys_tmp, nullptr, nullptr, n, bits, in_tmp);
}

}  // namespace gosh
