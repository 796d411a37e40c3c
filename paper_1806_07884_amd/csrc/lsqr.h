// Vector steps of the LSQR solve (lsqr_kernels.hip).
#pragma once

#include "internal.h"
#include "solver.h"

namespace rbf {

// Most partial sums a reduction of these kernels writes (its `part` holds
// kLsqrParts * kMaxPoly doubles).
constexpr int kLsqrParts = 512;

// out[0] = sum of x_i^2 (fixed order: block partials over contiguous ranges).
hipError_t lsqr_sumsq(const double* x, int64_t n, double* part, double* out, hipStream_t s);
// y = a x + b y.
hipError_t lsqr_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
// x *= a.
hipError_t lsqr_scale(int64_t n, double a, double* x, hipStream_t s);
// x_j = 0 where centre j is inactive.
hipError_t lsqr_mask(const uint8_t* active, int64_t m, double* x, hipStream_t s);
// x += c1 w, then w = v + c2 w.
hipError_t lsqr_step(int64_t n, double c1, double c2, const double* v, double* w, double* x,
                     hipStream_t s);
// out[0..dim] = P^T u over the n sorted points ps (SoA), P in the scaled basis
// ((x - o) / s, 1).
hipError_t lsqr_poly_adjoint(const double* ps, int64_t n, int dim, const PolyBasis& B,
                             const double* u, double* part, double* out, hipStream_t s);

}  // namespace rbf
