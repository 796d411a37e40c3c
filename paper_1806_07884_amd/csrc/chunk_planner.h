// Host-side sizing of the chunks of CG launches (plain C++, no HIP).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>

namespace rbf {

// Right-hand sides one planner tracks (the batched solve's maximum).
constexpr int kPlanMaxRhs = 4;

// Sizes of the chunks of CG launches queued between host checks.  A launch
// queued past a raised flag (reliable update, convergence) returns at entry
// but still costs a few us, and the chunk after the one that raises the flag
// is always queued too.  So chunks shrink as the flag nears: the decay of
// ||r||^2 between the last two snapshots gives the iterations left to the
// trigger (the soonest over the right-hand sides still iterating), and a
// chunk takes half of what remains past the chunk still in flight, between
// 4 launches and check_every.  Without a decay to go by (after a refresh,
// which may have converged, or when ||r|| grew) chunks start small and double.
struct ChunkPlanner {
  int64_t cmin, cmax, ramp;
  int nr = 0;
  double rr0[kPlanMaxRhs], rr1[kPlanMaxRhs], trig[kPlanMaxRhs];
  bool on[kPlanMaxRhs];
  int64_t it0 = -1, it1 = -1;

  explicit ChunkPlanner(int64_t check_every)
      : cmin(std::min<int64_t>(4, check_every)), cmax(check_every), ramp(cmin) {}
  void restart() {
    it0 = it1 = -1;
    ramp = cmin;
  }
  // a snapshot after `iter` iterations: ||r||^2, trigger and activity per
  // right-hand side
  void seen(int64_t iter, int n, const double* rr, const double* trigger2, const int32_t* active) {
    nr = n;
    it0 = it1;
    it1 = iter;
    for (int k = 0; k < n; ++k) {
      rr0[k] = rr1[k];
      rr1[k] = rr[k];
      trig[k] = trigger2[k];
      on[k] = active == nullptr || active[k] != 0;
    }
  }
  int64_t next(int64_t inflight) {
    double left = -1.0;
    if (it0 >= 0 && it1 > it0) {
      for (int k = 0; k < nr; ++k) {
        if (!on[k]) continue;
        if (!(rr0[k] > 0.0 && rr1[k] > 0.0 && rr1[k] < rr0[k] && trig[k] > 0.0)) {
          left = -1.0;  // a right-hand side without a decay: no estimate
          break;
        }
        const double rate = std::log(rr1[k] / rr0[k]) / (double)(it1 - it0);
        const double lk = rr1[k] > trig[k] ? std::log(trig[k] / rr1[k]) / rate : 0.0;
        if (left < 0.0 || lk < left) left = lk;
      }
    }
    if (left < 0.0) {
      const int64_t n = ramp;
      ramp = std::min(cmax, 2 * ramp);
      return n;
    }
    const double want = 0.5 * left - (double)inflight;
    const int64_t n = want <= (double)cmin ? cmin : (want >= (double)cmax ? cmax : (int64_t)want);
    ramp = n;
    return n;
  }
};

}  // namespace rbf
