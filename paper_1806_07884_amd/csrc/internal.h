// Host-side launch wrappers shared between the translation units of librbf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace rbf {

// ---- sort_scan.hip -------------------------------------------------------
// Exclusive prefix sums; `out` may alias `in`.  `temp` must hold
// scan_temp_bytes(n) bytes.
size_t scan_temp_bytes(int64_t n);
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s);
hipError_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `key_bits` bits.  The
// sorted pairs end in (keys, vals) when the pass count is even, else in the
// `_alt` buffers; *in_alt tells which.
size_t radix_temp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                            int64_t n, int key_bits, void* temp, hipStream_t s, bool* in_alt);

// cell_start[c] = first sorted index whose key >> shift >= c, for c in
// [0, ncell + 1]; cell_start[ncell + 1] = n.  Keys must be sorted and
// key >> shift <= ncell.
hipError_t cell_starts(const uint32_t* sorted_keys, int64_t n, int32_t ncell, int shift,
                       int32_t* cell_start, hipStream_t s);

}  // namespace rbf
