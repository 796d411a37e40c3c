// Host-side decisions of the mixed-precision solve (plain C++, no HIP): when
// the float32 iteration counts as stalled, and what a stalled or broken-down
// float32 solve does next.
#pragma once

#include <stdint.h>

namespace rbf {

// Default number of consecutive reliable updates without progress after which
// a float32 solve gives up.
constexpr int kDefaultStallLimit = 8;

// Progress of the float32 iteration, seen at its reliable updates: an update
// whose float64 residual ||r||^2 is above a quarter of the previous update's
// (||r|| fell by less than 2x) counts as a stall; `limit` stalls in a row end
// the float32 solve.  The first update has nothing to compare with.
struct StallWatch {
  int limit;
  int count = 0;
  double last = -1.0;
  explicit StallWatch(int stall_limit) : limit(stall_limit) {}
  // true when the float32 solve should stop at this update
  bool update(double rr_true) {
    if (last >= 0.0 && rr_true > 0.25 * last)
      ++count;
    else
      count = 0;
    last = rr_true;
    return count >= limit;
  }
};

enum class Fallback {
  kNone,             // return the float32 result and its status as they are
  kReassemble,       // assemble B and g in float64 from the points, solve in float64
  kFromAccumulators  // no points (chunked plan): the float64 accumulators become
                     // the float64 matrix, solve in float64
};

// What follows a float32 solve that ended with `status` after using part of
// the iteration budget (`iters_left` iterations remain).  Only a stall
// (status `warn_fallback`) or a breakdown (`err_breakdown`) with iterations
// left goes on in float64; the iteration cap (or any other status) returns as
// is, and so does a stall or breakdown with nothing left.  A plan that holds
// its points re-assembles in float64; a plan made from point chunks has no
// points left and takes its float64 accumulators instead.
inline Fallback fallback_action(int status, int warn_fallback, int err_breakdown, bool mixed,
                                bool has_points, int64_t iters_left) {
  if (!mixed || iters_left <= 0) return Fallback::kNone;
  if (status != warn_fallback && status != err_breakdown) return Fallback::kNone;
  return has_points ? Fallback::kReassemble : Fallback::kFromAccumulators;
}

}  // namespace rbf
