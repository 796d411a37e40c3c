// Linear polynomial reproduction (Section 3, eq. 6-10): the blocks that the
// polynomial adds to the normal equations,
//
//     Q = A^T P   (M x (d+1)),    C = P^T P   ((d+1) x (d+1)),    e = P^T h,
//
// with P_i the linear basis at point i.  The kernels use the scaled basis
// P_i = ((x_i - o) / s, 1), o and s the centre and half-extent of the points'
// bounding box, which spans the same functions as the paper's (x_i^T, 1) but
// keeps C well conditioned whatever the coordinates' offset; coefficients are
// converted to the paper's basis at the boundary (k_poly_coeffs).
//
// Q is summed per centre over its support, like g = A^T h (one block of four
// waves per centre, the waves' sums added in wave order), with phi evaluated
// in the assembly's precision (float32 for the mixed path, as for B and g, so
// the stored system is the normal equations of one matrix A), products and
// sums in float64; C and e over all points (block partials, then one block in
// a fixed order).  Every sum is deterministic.
#include "plan_kernels.h"
#include "solver.h"

namespace rbf {
namespace {

constexpr int kPolyWaves = 4;
constexpr int kPolyChunk = 256;
constexpr int kGramVals = 14;  // upper triangle of a 4 x 4 C and 4 of e
constexpr int kRed = 256;

template <typename T>
__device__ __forceinline__ double phi_arg(double s, double irho);
template <>
__device__ __forceinline__ double phi_arg<double>(double s, double irho) {
  return __builtin_sqrt(s) * irho;
}
template <>
__device__ __forceinline__ double phi_arg<float>(double s, double irho) {
  return (double)(__builtin_sqrtf((float)s) * (float)irho);
}

template <int DIM, int PHI, typename T>
__global__ __launch_bounds__(kWave* kPolyWaves) void k_poly_moments(PlanView P, PolyBasis B,
                                                                    int64_t ms,
                                                                    double* __restrict__ q64) {
  __shared__ double sp[kPolyWaves][DIM][kPolyChunk];
  __shared__ double red[DIM + 1][kPolyWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = blockIdx.x;
  const int32_t row = P.amap[j];
  if (row < 0) return;
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double r2j = P.rho2[j], irj = P.irho[j];
  double acc[DIM + 1];
#pragma unroll
  for (int t = 0; t <= DIM; ++t) acc[t] = 0.0;
  double(*wsp)[kPolyChunk] = sp[w];
  stream_support_part<DIM, kPolyChunk>(P, xj, r2j, w, kPolyWaves, wsp, nullptr, [&](int np) {
    for (int q = lane; q < np; q += kWave) {
      double p[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
      const double phi =
          (double)wendland<PHI, T>((T)phi_arg<T>(sqdist<DIM>(p, xj), irj));
#pragma unroll
      for (int d = 0; d < DIM; ++d) acc[d] += phi * ((p[d] - B.o[d]) / B.s[d]);
      acc[DIM] += phi;
    }
  });
#pragma unroll
  for (int t = 0; t <= DIM; ++t) {
    const double v = wave_sum(acc[t]);
    if (lane == 0) red[t][w] = v;
  }
  __syncthreads();
  if (threadIdx.x <= DIM) {
    double v = 0.0;
    for (int u = 0; u < kPolyWaves; ++u) v += red[threadIdx.x][u];
    q64[(int64_t)threadIdx.x * ms + row] = v;
  }
}

// Block partials of C (upper triangle, row by row) and e over the points
// (sorted order; every block covers a fixed range, so the sums are
// deterministic).
template <int DIM>
__global__ __launch_bounds__(kRed) void k_poly_gram(const double* __restrict__ ps,
                                                    const double* __restrict__ hs, int64_t n,
                                                    PolyBasis B, double* __restrict__ part) {
  constexpr int NP = DIM + 1;
  __shared__ double ws[kGramVals][kRed / kWave];
  double v[kGramVals];
#pragma unroll
  for (int k = 0; k < kGramVals; ++k) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRed) {
    double b[NP];
#pragma unroll
    for (int d = 0; d < DIM; ++d) b[d] = (ps[d * n + i] - B.o[d]) / B.s[d];
    b[DIM] = 1.0;
    const double h = hs[i];
    int k = 0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
#pragma unroll
      for (int c = a; c < NP; ++c) v[k++] += b[a] * b[c];
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) v[10 + a] += b[a] * h;
  }
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int k = 0; k < kGramVals; ++k) {
    const double t = wave_sum(v[k]);
    if (lane == 0) ws[k][threadIdx.x / kWave] = t;
  }
  __syncthreads();
  if (threadIdx.x < kGramVals) {
    double t = 0.0;
    for (int u = 0; u < kRed / kWave; ++u) t += ws[threadIdx.x][u];
    part[(int64_t)blockIdx.x * kGramVals + threadIdx.x] = t;
  }
}

// C, e and C^-1 (Cholesky, then the inverse column by column) from the
// partials; S->bad when C is not numerically positive definite (points on a
// line or plane).
__global__ __launch_bounds__(kRed) void k_poly_finish(const double* __restrict__ part, int nb,
                                                      int np, PolySys* __restrict__ S) {
  __shared__ double tot[kGramVals];
  if (threadIdx.x < kGramVals) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(int64_t)b * kGramVals + threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double C[kMaxPoly][kMaxPoly] = {};
  int k = 0;
  for (int a = 0; a < np; ++a)
    for (int c = a; c < np; ++c) {
      C[a][c] = tot[k];
      C[c][a] = tot[k];
      ++k;
    }
  // lower Cholesky factor
  double Lf[kMaxPoly][kMaxPoly] = {};
  int bad = 0;
  for (int c = 0; c < np && !bad; ++c) {
    double d = C[c][c];
    for (int u = 0; u < c; ++u) d -= Lf[c][u] * Lf[c][u];
    if (!(d > 1e-12 * C[c][c]) || !__builtin_isfinite(d)) {
      bad = 1;
      break;
    }
    Lf[c][c] = __builtin_sqrt(d);
    for (int r = c + 1; r < np; ++r) {
      double v = C[r][c];
      for (int u = 0; u < c; ++u) v -= Lf[r][u] * Lf[c][u];
      Lf[r][c] = v / Lf[c][c];
    }
  }
  double Ci[kMaxPoly][kMaxPoly] = {};
  if (!bad) {
    for (int col = 0; col < np; ++col) {
      double y[kMaxPoly] = {};
      for (int r = 0; r < np; ++r) {
        double v = r == col ? 1.0 : 0.0;
        for (int u = 0; u < r; ++u) v -= Lf[r][u] * y[u];
        y[r] = v / Lf[r][r];
      }
      for (int r = np - 1; r >= 0; --r) {
        double v = y[r];
        for (int u = r + 1; u < np; ++u) v -= Lf[u][r] * Ci[u][col];
        Ci[r][col] = v / Lf[r][r];
      }
    }
  }
  for (int a = 0; a < kMaxPoly; ++a) {
    for (int c = 0; c < kMaxPoly; ++c) {
      S->C[a][c] = C[a][c];
      S->Ci[a][c] = Ci[a][c];
    }
    S->e[a] = a < np ? tot[10 + a] : 0.0;
  }
  S->np = np;
  S->bad = bad;
}

__global__ void k_poly_cast(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Coefficients between the scaled basis (x_s) and the paper's (x^T, 1) basis
// (k): k_d = x_s,d / s_d, k_0 = x_s,0 - sum_d x_s,d o_d / s_d, and back.
__global__ void k_poly_coeffs(const double* __restrict__ in, PolyBasis B, int dim, int to_paper,
                              double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (to_paper) {
    double a0 = in[dim];
    for (int d = 0; d < dim; ++d) {
      out[d] = in[d] / B.s[d];
      a0 -= in[d] * B.o[d] / B.s[d];
    }
    out[dim] = a0;
  } else {
    double a0 = in[dim];
    for (int d = 0; d < dim; ++d) {
      out[d] = in[d] * B.s[d];
      a0 += in[d] * B.o[d];
    }
    out[dim] = a0;
  }
}

// No row of B: the polynomial alone, x = C^-1 e.
__global__ void k_poly_only(const PolySys* __restrict__ S, double* __restrict__ x) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int t = 0; t < kMaxPoly; ++t) {
    double v = 0.0;
    for (int k = 0; k < S->np; ++k) v += S->Ci[t][k] * S->e[k];
    x[t] = t < S->np ? v : 0.0;
  }
}

template <int DIM, typename T>
void moments_dim(const PlanView& P, int phi, const PolyBasis& B, int64_t ms, double* q64,
                 hipStream_t s) {
  const dim3 grid((unsigned)P.m), block(kWave * kPolyWaves);
  switch (phi) {
    case 0: hipLaunchKernelGGL((k_poly_moments<DIM, 0, T>), grid, block, 0, s, P, B, ms, q64); break;
    case 1: hipLaunchKernelGGL((k_poly_moments<DIM, 1, T>), grid, block, 0, s, P, B, ms, q64); break;
    case 2: hipLaunchKernelGGL((k_poly_moments<DIM, 2, T>), grid, block, 0, s, P, B, ms, q64); break;
    default: hipLaunchKernelGGL((k_poly_moments<DIM, 3, T>), grid, block, 0, s, P, B, ms, q64); break;
  }
}

}  // namespace

int poly_gram_blocks(int64_t n) {
  const int64_t b = (n + kRed - 1) / kRed;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_poly_system(const PlanView& P, int phi, const PolyBasis& B, int64_t ms,
                              const double* hs, double* q64, float* q32, double* part, int nb,
                              PolySys* S, hipStream_t s) {
  if (P.m > 0 && ms > 0) {
    if (P.dim == 2) {
      if (q32) moments_dim<2, float>(P, phi, B, ms, q64, s);
      else moments_dim<2, double>(P, phi, B, ms, q64, s);
    } else {
      if (q32) moments_dim<3, float>(P, phi, B, ms, q64, s);
      else moments_dim<3, double>(P, phi, B, ms, q64, s);
    }
    if (q32) {
      const int64_t cnt = (int64_t)(P.dim + 1) * ms;
      hipLaunchKernelGGL(k_poly_cast, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                         (const double*)q64, q32, cnt);
    }
  }
  return launch_poly_gram(P, B, hs, part, nb, S, s);
}

hipError_t launch_poly_gram(const PlanView& P, const PolyBasis& B, const double* hs, double* part,
                            int nb, PolySys* S, hipStream_t s) {
  if (P.dim == 2)
    hipLaunchKernelGGL(k_poly_gram<2>, dim3(nb), dim3(kRed), 0, s, P.ps, hs, P.n, B, part);
  else
    hipLaunchKernelGGL(k_poly_gram<3>, dim3(nb), dim3(kRed), 0, s, P.ps, hs, P.n, B, part);
  hipLaunchKernelGGL(k_poly_finish, dim3(1), dim3(kRed), 0, s, (const double*)part, nb,
                     P.dim + 1, S);
  return hipGetLastError();
}

hipError_t launch_poly_coeffs(const double* in, const PolyBasis& B, int dim, bool to_paper,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_coeffs, dim3(1), dim3(64), 0, s, in, B, dim, to_paper ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_poly_only(const PolySys* S, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_only, dim3(1), dim3(64), 0, s, S, x);
  return hipGetLastError();
}

}  // namespace rbf
