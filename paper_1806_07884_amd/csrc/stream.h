// Launch wrappers of the chunked assembly (stream_kernels.hip).
#pragma once

#include "plan_kernels.h"

namespace rbf {

// Candidate lists of the m centres of P (centre hash, radii): cnt[j] = their
// number (err[0] set when one exceeds kMaxCand), then, with ptr the exclusive
// scan of cnt, col[ptr[j] ..] the candidates in ascending order and up[j] the
// start of the upper part (l >= j).
hipError_t launch_cand_count(const PlanView& P, int64_t* cnt, int32_t* err, hipStream_t s);
hipError_t launch_cand_fill(const PlanView& P, const int64_t* ptr, int64_t* up, int32_t* col,
                            hipStream_t s);
// bad[0] |= 1 when a coordinate (SoA [dim][n]) or a value of the chunk is not finite.
hipError_t launch_chunk_check(const double* x, const double* h, int64_t n, int dim, int32_t* bad,
                              hipStream_t s);
// inbox[0] += *sentinel_start (the chunk's points inside the hash grid).
hipError_t launch_stream_inbox(const int32_t* sentinel_start, int64_t* inbox, hipStream_t s);
// One chunk's terms: P's point hash is the chunk's (n points, values hs in
// sorted order); acc/mark over the candidates, count and g over the centres.
// grouped: the grouped path (candidate lists longer than one wave on average).
hipError_t launch_stream_accum(const PlanView& P, int phi, bool fp32, bool grouped,
                               const double* hs, const int64_t* cptr, const int64_t* cup,
                               const int32_t* ccol, double* acc, uint8_t* mark, int64_t* count,
                               double* g, hipStream_t s);
// support[j] = min(count[j], INT32_MAX), active[j] = count[j] >= min_support.
hipError_t launch_stream_active(const int64_t* count, int64_t m, int32_t min_support,
                                int32_t* support, uint8_t* active, hipStream_t s);
// Full-row and lower-part sizes of the kept entries (marked, both ends
// active) and the largest |l - j| (maxdelta, max-combined).
hipError_t launch_stream_rows(const int64_t* cptr, const int64_t* cup, const int32_t* ccol,
                              const uint8_t* mark, const uint8_t* active, int64_t m,
                              int64_t* full_cnt, int32_t* lower_cnt, int32_t* maxdelta,
                              hipStream_t s);
// Columns of the full CSR at row_ptr, and src[e] = the accumulator of entry e.
hipError_t launch_stream_fill(const int64_t* cptr, const int64_t* cup, const int32_t* ccol,
                              const uint8_t* mark, const uint8_t* active, int64_t m,
                              const int64_t* row_ptr, int32_t* col, int64_t* src, hipStream_t s);
// Values (float32 or float64) into the solver's sliced-ELL layout, the
// diagonals, and diag = g = 0 for inactive centres.
hipError_t launch_stream_values(const int64_t* row_ptr, const int32_t* col, const int64_t* src,
                                const int32_t* amap, const uint8_t* active, const double* acc,
                                const int64_t* sptr, int lanes, int64_t m, bool fp32, void* val,
                                double* diag, double* g, hipStream_t s);

}  // namespace rbf
