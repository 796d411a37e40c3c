// Device scalars and argument bundles of the conjugate-gradient kernels.
#pragma once

#include "internal.h"

namespace rbf {

// Most blocks of any CG kernel; bounds the partial-sum arrays.
constexpr int kCgMaxBlocks = 2048;

// Scalars of one CG solve, kept in device memory.  Each is written by block 0
// of one kernel and read by later kernels (or the host) only.
struct CgScalars {
  double rzh[2];     // r . z of iterate k at [k & 1]
  double beta_fixed; // beta of the next spmv after a float64 residual
  double alpha, beta, pq;
  double rr;         // ||r||^2 of the iterated residual (last seen)
  double rr_true;    // ||g - (B + lambda I) x||^2 at the last float64 recomputation
  double gg;         // ||g||^2
  double tol2;       // rtol^2 * gg
  double delta2;     // reliable-update factor squared
  double trigger2;   // iterated ||r||^2 at which the spmv raises the flag
  int64_t iter;      // executed iterations
  int32_t done;      // 0 running, 1 trigger reached, 2 breakdown, 3 converged
  int32_t pad_;
};

template <typename XT>
struct CgArgs {
  int64_t m;
  XT* p[2];
  XT* q;
  XT* r;
  XT* z;
  XT* xlo;            // iterated correction
  const XT* dinv;
  double* xhi;        // float64 solution
  double* r64;        // float64 true residual
  CgScalars* sc;
  double* part_spmv;  // [spmv_blocks] partials of p . q
  double* part_upd;   // [2 * update_blocks] partials of r . z and r . r
  int spmv_blocks;
  int update_blocks;
};

// The stored matrix in the solver's sliced-ELL layout.  Rows are taken in
// slices of S = 64 / L consecutive rows; each row of a slice gets L lanes of a
// wave.  Slice s starts at sptr[s] and holds slen[s] entries per row (the
// longest row of the slice, rounded up to a multiple of L); entry k of row
// i = j - s S sits at sptr[s] + (k / L) * 64 + i * L + (k % L), so every
// wave-wide load is one contiguous 64-entry run.  Columns are stored as
// l - j (int16 when every |l - j| fits, else int32); padding entries have
// delta 0 and value 0.
struct CgMatrix {
  const int64_t* sptr;
  const int32_t* slen;
  int64_t nslices;
  const void* col;
  bool col16;
  const void* val;  // VT
  int lanes;        // L: lanes per row (2, 4 or 8)
};

__host__ __device__ inline int64_t sell_pos(const int64_t* sptr, int lanes, int64_t j, int64_t k) {
  const int64_t rows = 64 / lanes;
  const int64_t s = j / rows, i = j - s * rows;
  return sptr[s] + (k / lanes) * 64 + i * lanes + (k % lanes);
}

int sell_lanes(double mean_row);
int cg_grid_blocks(int64_t nslices);
int cg_update_blocks(int64_t m);

// Iteration k = cg_spmv(parity = k & 1) then cg_update(parity).  fixed_beta:
// the spmv takes beta from the last float64 residual (first iteration after
// set-up or a reliable update).  With e0/e1 (may be null) the launch stamps
// the two events at the kernel's start and end.
template <typename VT, typename XT>
hipError_t cg_spmv(const CgArgs<XT>& a, const CgMatrix& A, int parity, int fixed_beta,
                   hipEvent_t e0, hipEvent_t e1, hipStream_t s);
template <typename XT>
hipError_t cg_update(const CgArgs<XT>& a, int parity, hipStream_t s);
// x_hi += x_lo; float64 residual; r, z from it; scalars for the next spmv.
template <typename VT, typename XT>
hipError_t cg_true_residual(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int restart,
                            int parity, hipStream_t s);
template <typename XT>
hipError_t cg_setup(const CgArgs<XT>& a, const uint8_t* active, const double* g, double rtol,
                    double delta, hipStream_t s);

}  // namespace rbf
