// Evaluation of the approximant (Section 2, eq. 3):
//     f(y) = sum_j c_j phi(||y - xi_j|| / rho_j)   over centres with y in supp(j),
// plus, with polynomial reproduction, a^T y + a_0 (Section 3, eq. 6-7); one
// thread per query point, centres found through the centre hash, and the
// root-mean-square error against given values.
#define RBF_CHECK_FILE 4  // place ids of the checked build's device checks
#include "plan_kernels.h"

namespace rbf {
namespace {

// One wave per query: the centres of the 3^(d-1) rows of cells around the
// query's cell, taken as one list, are split over the lanes (consecutive
// sorted centres on consecutive lanes, so the loads coalesce and every lane
// has the same number of steps); the lanes' partial sums are added by a
// butterfly of fixed order, so the value is deterministic.
template <int DIM, int PHI>
__global__ __launch_bounds__(256) void k_eval(PlanView P, int64_t nq, const double* __restrict__ y,
                                              const double* __restrict__ cs,
                                              const double* __restrict__ rho2_s,
                                              const double* __restrict__ irho_s,
                                              const double* __restrict__ kpoly,
                                              double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (q >= nq) return;
  double p[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) p[d] = y[d * nq + q];
  int c[3] = {0, 0, 0};
  double acc = 0.0;
  if (cell_of<DIM>(P.grid, p, c)) {
    NbrWalk<DIM> walk(P.grid, c, 1);
    constexpr int R = DIM == 2 ? 3 : 9;
    // row k's first sorted centre and the prefix of the row lengths, one row per lane
    int lo = 0, len = 0;
    if (lane < R) {
      int lo_id, hi_id;
      if (walk.range(lane, lo_id, hi_id)) {
        lo = P.ccs[lo_id];
        len = P.ccs[hi_id + 1] - lo;
      }
    }
    int pre = len;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int t = __shfl_up(pre, off, kWave);
      if (lane >= off) pre += t;
    }
    // every lane takes the whole table (all lanes active here)
    int rpre[R], rlo[R], rlen[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rpre[r] = __shfl(pre, r, kWave);
      rlo[r] = __shfl(lo, r, kWave);
      rlen[r] = __shfl(len, r, kWave);
    }
    const int total = rpre[R - 1];
    for (int t = lane; t < total; t += kWave) {
      // the row holding list position t (rows of no centres hold none)
      int start = 0, lok = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (t >= rpre[r] - rlen[r] && t < rpre[r]) {
          start = rpre[r] - rlen[r];
          lok = rlo[r];
        }
      }
      const int i = lok + (t - start);
      if (!RBF_CHECK(P, (unsigned)i < (unsigned)P.m)) continue;
      double xl[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) xl[d] = P.ctr_s[d * P.m + i];
      const double s = sqdist<DIM>(p, xl);
      if (s < rho2_s[i]) acc += cs[i] * wendland<PHI, double>(__builtin_sqrt(s) * irho_s[i]);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    if (kpoly) {
      double pv = kpoly[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) pv += kpoly[d] * p[d];
      acc += pv;
    }
    out[q] = acc;
  }
}

__global__ void k_gather(const double* __restrict__ src, const int32_t* __restrict__ perm,
                         int64_t n, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_scatter_rows(const double* __restrict__ src, const int32_t* __restrict__ amap,
                               int64_t m, double* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) dst[j] = amap[j] >= 0 ? src[amap[j]] : 0.0;
}

constexpr int kRed = 256;

__global__ __launch_bounds__(kRed) void k_sq_err(const double* __restrict__ f,
                                                 const double* __restrict__ h, int64_t n,
                                                 double* __restrict__ part) {
  __shared__ double ws[kRed / kWave];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRed) {
    const double d = f[i] - h[i];
    s += d * d;
  }
  s = wave_sum(s);
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRed / kWave; ++w) t += ws[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kRed) void k_sum_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
  __shared__ double ws[kRed / kWave];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += kRed) s += part[k];
  s = wave_sum(s);
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRed / kWave; ++w) t += ws[w];
    out[0] = t;
  }
}

template <int DIM>
void eval_dim(const PlanView& P, int phi, int64_t nq, const double* y, const double* cs,
              const double* rho2_s, const double* irho_s, const double* kp, double* out,
              hipStream_t s) {
  const int bs = 256;
  const dim3 grid((unsigned)((nq + bs / kWave - 1) / (bs / kWave)));
  switch (phi) {
    case 0: hipLaunchKernelGGL((k_eval<DIM, 0>), grid, dim3(bs), 0, s, P, nq, y, cs, rho2_s, irho_s, kp, out); break;
    case 1: hipLaunchKernelGGL((k_eval<DIM, 1>), grid, dim3(bs), 0, s, P, nq, y, cs, rho2_s, irho_s, kp, out); break;
    case 2: hipLaunchKernelGGL((k_eval<DIM, 2>), grid, dim3(bs), 0, s, P, nq, y, cs, rho2_s, irho_s, kp, out); break;
    default: hipLaunchKernelGGL((k_eval<DIM, 3>), grid, dim3(bs), 0, s, P, nq, y, cs, rho2_s, irho_s, kp, out); break;
  }
}

}  // namespace

hipError_t launch_gather(const double* src, const int32_t* perm, int64_t n, double* dst,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, src, perm, n,
                     dst);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const double* src, const int32_t* amap, int64_t m, double* dst,
                               hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, src,
                     amap, m, dst);
  return hipGetLastError();
}

hipError_t launch_eval(const PlanView& P, int phi, int64_t nq, const double* y, const double* cs,
                       const double* rho2_s, const double* irho_s, const double* kpoly,
                       double* out, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  if (P.dim == 2)
    eval_dim<2>(P, phi, nq, y, cs, rho2_s, irho_s, kpoly, out, s);
  else
    eval_dim<3>(P, phi, nq, y, cs, rho2_s, irho_s, kpoly, out, s);
  return hipGetLastError();
}

int sq_err_blocks(int64_t n) {
  int64_t b = (n + kRed - 1) / kRed;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_sq_err(const double* f, const double* h, int64_t n, double* part, int nb,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sq_err, dim3(nb), dim3(kRed), 0, s, f, h, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kRed), 0, s, (const double*)part, nb, out);
  return hipGetLastError();
}

}  // namespace rbf
