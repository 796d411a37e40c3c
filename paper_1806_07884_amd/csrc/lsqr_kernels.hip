// Vector kernels of the LSQR solve (Paige and Saunders, ACM TOMS 8 (1982)) of
// the least-squares problem of Section 2, eq. 4-5 (with the polynomial columns
// of Section 3, eq. 9), min || [A P] (c, k) - h ||^2 + lambda ||c||^2, on the
// design matrix itself: A v is an evaluation at the data points (eq. 3) and
// A^T u the assembly's right-hand-side pass, so the conditioning is that of
// A, not of A^T A.  The scalar recurrences run on the host; these kernels
// are the vector steps.  Every reduction is a fixed-order sum of per-block
// partials over contiguous ranges, so a solve is deterministic.
#include "lsqr.h"
#include "plan_kernels.h"

namespace rbf {
namespace {

constexpr int kLB = 256;

__device__ __forceinline__ void block_range(int64_t n, int64_t* lo, int64_t* hi) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  *lo = (int64_t)blockIdx.x * per;
  *hi = *lo + per < n ? *lo + per : n;
}

// Sum of the block's values v[0..W) of every wave, in wave order, into out.
template <int N>
__device__ __forceinline__ void block_total(double (&v)[N], double* out) {
  __shared__ double ws[N][kLB / kWave];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) ws[k][threadIdx.x / kWave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double t = 0.0;
      for (int w = 0; w < kLB / kWave; ++w) t += ws[k][w];
      out[k] = t;
    }
  }
}

// part[b] = sum of x_i^2 over block b's range.
__global__ __launch_bounds__(kLB) void k_sumsq_part(const double* __restrict__ x, int64_t n,
                                                    double* __restrict__ part) {
  int64_t lo, hi;
  block_range(n, &lo, &hi);
  double v[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) v[0] += x[i] * x[i];
  block_total<1>(v, part + blockIdx.x);
}

// out[0] = sum over k of part[k] (k < nb), in order.
__global__ __launch_bounds__(kLB) void k_sum_parts(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
  double v[1] = {0.0};
  for (int k = threadIdx.x; k < nb; k += kLB) v[0] += part[k];
  block_total<1>(v, out);
}

// y = a x + b y.
__global__ __launch_bounds__(kLB) void k_axpby(int64_t n, double a, const double* __restrict__ x,
                                               double b, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

// x *= a.
__global__ __launch_bounds__(kLB) void k_scale(int64_t n, double a, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i < n) x[i] *= a;
}

// x_j = 0 where centre j is inactive.
__global__ __launch_bounds__(kLB) void k_mask(const uint8_t* __restrict__ active, int64_t m,
                                              double* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (j < m && !active[j]) x[j] = 0.0;
}

// x += c1 w; then w = v + c2 w.
__global__ __launch_bounds__(kLB) void k_lsqr_step(int64_t n, double c1, double c2,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ w,
                                                   double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x;
  if (i < n) {
    const double wi = w[i];
    x[i] += c1 * wi;
    w[i] = v[i] + c2 * wi;
  }
}

// Per block, the sums of u_i t_i over its range of the sorted points, t_i the
// point's row of P in the scaled basis ((x - o) / s, 1): part[b * kMaxPoly + k].
__global__ __launch_bounds__(kLB) void k_poly_adjoint_part(const double* __restrict__ ps,
                                                           int64_t n, int dim, PolyBasis B,
                                                           const double* __restrict__ u,
                                                           double* __restrict__ part) {
  int64_t lo, hi;
  block_range(n, &lo, &hi);
  double v[kMaxPoly] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kLB) {
    const double ui = u[i];
    for (int d = 0; d < dim; ++d) v[d] += ui * ((ps[d * n + i] - B.o[d]) / B.s[d]);
    v[dim] += ui;
  }
  block_total<kMaxPoly>(v, part + (int64_t)blockIdx.x * kMaxPoly);
}

// out[k] = sum over blocks of part[b * kMaxPoly + k], k < np, in block order.
__global__ __launch_bounds__(kLB) void k_poly_adjoint_final(const double* __restrict__ part,
                                                            int nb, int np,
                                                            double* __restrict__ out) {
  double v[kMaxPoly] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kLB) {
#pragma unroll
    for (int k = 0; k < kMaxPoly; ++k) v[k] += part[(int64_t)b * kMaxPoly + k];
  }
  double t[kMaxPoly];
  block_total<kMaxPoly>(v, t);
  if (threadIdx.x == 0)
    for (int k = 0; k < np; ++k) out[k] = t[k];
}

inline int blocks_for(int64_t n) {
  const int64_t b = (n + 4 * kLB - 1) / (4 * kLB);
  return (int)(b < 1 ? 1 : (b > kLsqrParts ? kLsqrParts : b));
}

}  // namespace

hipError_t lsqr_sumsq(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
  if (n <= 0) {
    return hipMemsetAsync(out, 0, sizeof(double), s);
  }
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_sumsq_part, dim3(nb), dim3(kLB), 0, s, x, n, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kLB), 0, s, (const double*)part, nb, out);
  return hipGetLastError();
}

hipError_t lsqr_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + kLB - 1) / kLB)), dim3(kLB), 0, s, n, a, x, b,
                     y);
  return hipGetLastError();
}

hipError_t lsqr_scale(int64_t n, double a, double* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + kLB - 1) / kLB)), dim3(kLB), 0, s, n, a, x);
  return hipGetLastError();
}

hipError_t lsqr_mask(const uint8_t* active, int64_t m, double* x, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((m + kLB - 1) / kLB)), dim3(kLB), 0, s, active, m, x);
  return hipGetLastError();
}

hipError_t lsqr_step(int64_t n, double c1, double c2, const double* v, double* w, double* x,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lsqr_step, dim3((unsigned)((n + kLB - 1) / kLB)), dim3(kLB), 0, s, n, c1,
                     c2, v, w, x);
  return hipGetLastError();
}

hipError_t lsqr_poly_adjoint(const double* ps, int64_t n, int dim, const PolyBasis& B,
                             const double* u, double* part, double* out, hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_poly_adjoint_part, dim3(nb), dim3(kLB), 0, s, ps, n, dim, B, u, part);
  hipLaunchKernelGGL(k_poly_adjoint_final, dim3(1), dim3(kLB), 0, s, (const double*)part, nb,
                     dim + 1, out);
  return hipGetLastError();
}

}  // namespace rbf
