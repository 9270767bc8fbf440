// ExpandEmbedding of Algorithm 2 (Section 3): every fine vertex starts from
// the trained row of its super vertex, fine[v] = coarse[map[v]].  A plain
// row gather: each thread moves 16 B, consecutive threads cover consecutive
// 16 B chunks of the fine matrix (coalesced stores, row-contiguous loads).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "gosh_internal.hpp"

namespace gosh {
namespace {

template <int CHUNKS>
__global__ __launch_bounds__(256) void k_prolong(const uint4* __restrict__ coarse, uint4* __restrict__ fine,
                                                 const int32_t* __restrict__ map, int64_t n_fine) {
    const int64_t total = n_fine * CHUNKS;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t v = i / CHUNKS;
        const int c = static_cast<int>(i - v * CHUNKS);
        fine[i] = coarse[static_cast<int64_t>(map[v]) * CHUNKS + c];
    }
}

template <int CHUNKS>
void launch(const void* coarse, void* fine, const int32_t* map, int64_t n, hipStream_t st) {
    const int64_t total = n * CHUNKS;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(total, 256), int64_t(1) << 20));
    hipLaunchKernelGGL((k_prolong<CHUNKS>), dim3(blocks), dim3(256), 0, st, static_cast<const uint4*>(coarse),
                       static_cast<uint4*>(fine), map, n);
}

}  // namespace

void prolong_copy(Ctx* c, const Level& fine, const void* coarse, void* fine_emb, gosh_dtype dt, int d) {
    GOSH_REQUIRE(dt == GOSH_F32 || dt == GOSH_BF16, GOSH_E_INVALID_ARG, "dtype must be F32 or BF16");
    GOSH_REQUIRE(d == 8 || d == 16 || d == 32 || d == 64 || d == 128 || d == 256, GOSH_E_INVALID_ARG,
                 "d must be one of 8, 16, 32, 64, 128, 256");
    GOSH_REQUIRE(fine.map, GOSH_E_INVALID_ARG, "level has no map to a coarser level");
    if (fine.n == 0) return;
    GOSH_REQUIRE(coarse && fine_emb, GOSH_E_INVALID_ARG, "null embedding");
    const int row_bytes = d * (dt == GOSH_BF16 ? 2 : 4);
    switch (row_bytes / 16) {
        case 1: launch<1>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 2: launch<2>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 4: launch<4>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 8: launch<8>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 16: launch<16>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 32: launch<32>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        case 64: launch<64>(coarse, fine_emb, fine.map, fine.n, c->stream); break;
        default: throw Error(GOSH_E_INVALID_ARG, "unsupported row size");
    }
    GOSH_HIP(hipGetLastError());
}

}  // namespace gosh
