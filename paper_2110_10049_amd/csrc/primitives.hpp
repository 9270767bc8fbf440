// Device-wide primitives written for gfx950: exclusive/inclusive scans and a
// stable LSD radix sort.  All run on the context stream and allocate their
// temporaries from the context.
#pragma once

#include "gosh_internal.hpp"

namespace gosh {

enum class ScanOp { Sum, Max };

// out[i] = op(in[0..i-1]) (exclusive, identity 0) or op(in[0..i]) (inclusive).
// `in` and `out` may alias.  If total_host != nullptr the reduction of all n
// inputs is copied back (synchronising the stream).
void scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n, bool inclusive, ScanOp op,
              int64_t* total_host);
void scan_i32_to_i64(Ctx* c, const int32_t* in, int64_t* out, int64_t n, int64_t* total_host);

// Stable LSD radix sort on bits [0, bits) of the keys, 8 bits per pass.
// Sorted keys (and values, if vals != nullptr) end up in `keys`/`vals`;
// `keys_tmp`/`vals_tmp` are scratch of the same length.  With in_tmp set,
// an odd pass count leaves them in `keys_tmp`/`vals_tmp` instead (no copy
// back) and *in_tmp says so.
void radix_sort_u32(Ctx* c, uint32_t* keys, uint32_t* keys_tmp, uint32_t* vals,
                    uint32_t* vals_tmp, int64_t n, int bits, bool* in_tmp = nullptr);
void radix_sort_u64(Ctx* c, uint64_t* keys, uint64_t* keys_tmp, int64_t n, int bits, bool* in_tmp = nullptr);

}  // namespace gosh
