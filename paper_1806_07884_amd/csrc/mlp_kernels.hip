// Learned support radius: density features per block of centres, the
// 16-64-64-1 tanh MLP (training with Adam, gradients, BF16 inference) and the
// broadcast of the predicted radius to the centres of each block.
//
// The paper observes that CS-RBF accuracy depends on data density and on the
// shape parameter, picks alpha = 1/rho experimentally (Section 6, Table 3)
// and leaves optimal shape parameters to future work (Section 7); the network
// regresses log(rho / spacing) from the counts of Algorithm 1's range query at
// a sweep of radii.
//
// Parameter layout (5313 floats): W1[16][64] (input-major), b1[64],
// W2[64][64], b2[64], W3[64], b3.
#include <hip/hip_bf16.h>

#include "mlp_kernels.h"
#include "plan_kernels.h"

namespace rbf {
namespace {

constexpr int kIn = kMlpInputs, kH = kMlpHidden;
constexpr int oW1 = 0, ob1 = kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH;
static_assert(ob3 + 1 == kMlpParams, "parameter layout");
constexpr int kT = 256;                                // threads of the MLP kernels
constexpr int kOwn = (kMlpParams + kT - 1) / kT;       // parameters owned per thread (21)
constexpr int kB = 32;                                 // samples per forward/backward chunk

// ---------------------------------------------------------------- features
// counts[j * R + s] = #{points : s(x, xi_j) < radii[s]^2}, one wave per centre;
// the candidate cells reach `reach` cells around the centre's cell.
template <int DIM>
__global__ __launch_bounds__(256) void k_density_counts(PlanView P, const double* __restrict__ radii,
                                                        int R, int reach,
                                                        int32_t* __restrict__ counts) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (j >= P.m) return;
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  double r2[kMaxRadii];
  int n[kMaxRadii];
  for (int s = 0; s < kMaxRadii; ++s) {
    r2[s] = s < R ? radii[s] * radii[s] : 0.0;
    n[s] = 0;
  }
  int c[3];
  if (cell_of<DIM>(P.grid, xj, c)) {
    NbrWalk<DIM> walk(P.grid, c, reach);
    for (int k = 0; k < walk.rows(); ++k) {
      int lo_id, hi_id;
      if (!walk.range(k, lo_id, hi_id)) continue;
      const int lo = P.pcs[lo_id], hi = P.pcs[hi_id + 1];
      for (int i = lo + lane; i < hi; i += kWave) {
        double p[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = P.ps[d * P.n + i];
        const double sq = sqdist<DIM>(p, xj);
#pragma unroll
        for (int s = 0; s < kMaxRadii; ++s) n[s] += (s < R && sq < r2[s]) ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kMaxRadii; ++s) {
    const int t = wave_sum_int(n[s]);
    if (lane == 0 && s < R) counts[j * R + s] = t;
  }
}

// Block of every centre: t = (xi - min) / (max - min), b = min(nb - 1,
// floor(t nb)) per dimension, first coordinate fastest (float64, as the
// oracle).  box = {min_0, max_0, min_1, max_1, ...}.
__device__ __forceinline__ int block_index(const double* x, const double* box, int dim, int nb,
                                           bool clamp_low) {
  int idx = 0, mul = 1;
  for (int d = 0; d < dim; ++d) {
    const double lo = box[2 * d], ext = box[2 * d + 1] - lo;
    const double t = ext > 0.0 ? (x[d] - lo) / ext : 0.0;
    double f = floor(t * (double)nb);
    if (clamp_low && f < 0.0) f = 0.0;
    int b = f > (double)(nb - 1) ? nb - 1 : (int)f;
    idx += b * mul;
    mul *= nb;
  }
  return idx;
}

__global__ void k_centre_blocks(const double* __restrict__ ctr, int64_t m, int dim,
                                const double* __restrict__ box, int nb,
                                int32_t* __restrict__ blk) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double x[3];
  for (int d = 0; d < dim; ++d) x[d] = ctr[d * m + j];
  blk[j] = block_index(x, box, dim, nb, false);
}

// One workgroup per block of centres: mean and population standard deviation
// of log(1 + count) for every radius, summed over the block's centres in
// index order (thread-strided, then a fixed tree), stored as float32.
__global__ __launch_bounds__(256) void k_block_features(const int32_t* __restrict__ counts,
                                                        const int32_t* __restrict__ blk,
                                                        int64_t m, int R,
                                                        float* __restrict__ feats) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  for (int s = 0; s < R; ++s) {
    double sum = 0.0, cnt = 0.0;
    for (int64_t j = threadIdx.x; j < m; j += 256) {
      if (blk[j] == b) {
        sum += log1p((double)counts[j * R + s]);
        cnt += 1.0;
      }
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double n = red[0];
    __syncthreads();
    const double mean = n > 0.0 ? total / n : 0.0;
    double dev = 0.0;
    for (int64_t j = threadIdx.x; j < m; j += 256) {
      if (blk[j] == b) {
        const double d = log1p((double)counts[j * R + s]) - mean;
        dev += d * d;
      }
    }
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      feats[b * 2 * R + 2 * s] = (float)mean;
      feats[b * 2 * R + 2 * s + 1] = (float)(n > 0.0 ? sqrt(red[0] / n) : 0.0);
    }
    __syncthreads();
  }
}

// Per block of the centres' box: sum of (f - h)^2 over the queries that fall
// in it, and their count (one workgroup per block, fixed summation order).
__global__ __launch_bounds__(256) void k_block_sq_err(const double* __restrict__ y, int64_t nq,
                                                      int dim, const double* __restrict__ f,
                                                      const double* __restrict__ h,
                                                      const double* __restrict__ box, int nb,
                                                      double* __restrict__ sums,
                                                      int64_t* __restrict__ counts) {
  __shared__ double red[256];
  __shared__ int64_t redc[256];
  const int b = blockIdx.x;
  double s = 0.0;
  int64_t c = 0;
  for (int64_t q = threadIdx.x; q < nq; q += 256) {
    double x[3];
    for (int d = 0; d < dim; ++d) x[d] = y[d * nq + q];
    if (block_index(x, box, dim, nb, true) == b) {
      const double e = f[q] - h[q];
      s += e * e;
      c += 1;
    }
  }
  red[threadIdx.x] = s;
  redc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      redc[threadIdx.x] += redc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[b] = red[0];
    counts[b] = redc[0];
  }
}

// rho_j = clamp(spacing exp(pred[block(j)]), rho_min, rho_max); a non-finite
// prediction gives rho_fallback.
__global__ void k_radius_broadcast(const float* __restrict__ pred, const int32_t* __restrict__ blk,
                                   int64_t m, double spacing, double rho_min, double rho_max,
                                   double rho_fallback, double* __restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const double p = (double)pred[blk[j]];
  double r = spacing * exp(p);
  r = r < rho_min ? rho_min : (r > rho_max ? rho_max : r);
  rho[j] = __builtin_isfinite(p) ? r : rho_fallback;
}

// ---------------------------------------------------------------- MLP
struct MlpLds {
  float W[kMlpParams];
  float X[kB][kIn];
  float y[kB];
  float H1[kB][kH];
  float H2[kB][kH];
  float dZ2[kB][kH];
  float dZ1[kB][kH];
  float dout[kB];
  float lossv[kB];
};

// Forward and backward of one chunk of nb <= kB samples whose inputs sit in
// L.X / L.y, with weights in L.W; d_out = 2 r / scale.  Adds the gradient of
// every parameter this thread owns (k = tid + kT * i) to g[i] and returns the
// chunk's sum of squared residuals in L.lossv[0] (thread 0 after a barrier).
__device__ void mlp_chunk(MlpLds& L, int nb, float scale, float* g) {
  const int tid = threadIdx.x;
  const int u = tid & (kH - 1);
  // layer 1 and 2 (four samples per pass of the 256 threads)
  for (int s = tid >> 6; s < nb; s += kT / kH) {
    float a = L.W[ob1 + u];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a += L.X[s][i] * L.W[oW1 + i * kH + u];
    L.H1[s][u] = tanhf(a);
  }
  __syncthreads();
  for (int s = tid >> 6; s < nb; s += kT / kH) {
    float a = L.W[ob2 + u];
    for (int i = 0; i < kH; ++i) a += L.H1[s][i] * L.W[oW2 + i * kH + u];
    L.H2[s][u] = tanhf(a);
  }
  __syncthreads();
  if (tid < nb) {
    float o = L.W[ob3];
    for (int i = 0; i < kH; ++i) o += L.H2[tid][i] * L.W[oW3 + i];
    const float r = o - L.y[tid];
    L.dout[tid] = 2.0f * r / scale;
    L.lossv[tid] = r * r;
  }
  __syncthreads();
  for (int s = tid >> 6; s < nb; s += kT / kH) {
    const float h2 = L.H2[s][u];
    L.dZ2[s][u] = L.dout[s] * L.W[oW3 + u] * (1.0f - h2 * h2);
  }
  __syncthreads();
  for (int s = tid >> 6; s < nb; s += kT / kH) {
    float a = 0.0f;
    for (int v = 0; v < kH; ++v) a += L.dZ2[s][v] * L.W[oW2 + u * kH + v];
    const float h1 = L.H1[s][u];
    L.dZ1[s][u] = a * (1.0f - h1 * h1);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = tid + kT * i;
    if (k >= kMlpParams) break;
    float acc = 0.0f;
    if (k < ob1) {
      const int a = k / kH, v = k % kH;
      for (int s = 0; s < nb; ++s) acc += L.X[s][a] * L.dZ1[s][v];
    } else if (k < oW2) {
      const int v = k - ob1;
      for (int s = 0; s < nb; ++s) acc += L.dZ1[s][v];
    } else if (k < ob2) {
      const int a = (k - oW2) / kH, v = (k - oW2) % kH;
      for (int s = 0; s < nb; ++s) acc += L.H1[s][a] * L.dZ2[s][v];
    } else if (k < oW3) {
      const int v = k - ob2;
      for (int s = 0; s < nb; ++s) acc += L.dZ2[s][v];
    } else if (k < ob3) {
      const int v = k - oW3;
      for (int s = 0; s < nb; ++s) acc += L.H2[s][v] * L.dout[s];
    } else {
      for (int s = 0; s < nb; ++s) acc += L.dout[s];
    }
    g[i] += acc;
  }
  if (tid == 0) {
    float t = 0.0f;
    for (int s = 0; s < nb; ++s) t += L.lossv[s];
    L.lossv[0] = t;
  }
  __syncthreads();
}

// Rows of the chunk into LDS, each input standardised: (x_i - mean_i) / std_i
// in float32 (scale = {mean[16], std[16]}).
__device__ void load_chunk(MlpLds& L, const float* __restrict__ x, const float* __restrict__ y,
                           const float* __restrict__ scale, const int32_t* __restrict__ idx,
                           int64_t first, int nb) {
  for (int t = threadIdx.x; t < nb * kIn; t += kT) {
    const int s = t / kIn, i = t % kIn;
    const int64_t row = idx ? (int64_t)idx[first + s] : first + s;
    L.X[s][i] = (x[row * kIn + i] - scale[i]) / scale[kIn + i];
  }
  for (int s = threadIdx.x; s < nb; s += kT) {
    const int64_t row = idx ? (int64_t)idx[first + s] : first + s;
    L.y[s] = y[row];
  }
  __syncthreads();
}

// Full-batch gradient of the mean squared error over n samples (chunks of kB
// in order), and the loss.
__global__ __launch_bounds__(kT) void k_mlp_grad(const float* __restrict__ params,
                                                 const float* __restrict__ scale,
                                                 const float* __restrict__ x,
                                                 const float* __restrict__ y, int64_t n,
                                                 float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  __shared__ MlpLds L;
  for (int k = threadIdx.x; k < kMlpParams; k += kT) L.W[k] = params[k];
  __syncthreads();
  float g[kOwn];
#pragma unroll
  for (int i = 0; i < kOwn; ++i) g[i] = 0.0f;
  float lsum = 0.0f;
  for (int64_t first = 0; first < n; first += kB) {
    const int nb = (int)(n - first < kB ? n - first : kB);
    load_chunk(L, x, y, scale, nullptr, first, nb);
    mlp_chunk(L, nb, (float)n, g);
    lsum += L.lossv[0];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = threadIdx.x + kT * i;
    if (k < kMlpParams) grad[k] = g[i];
  }
  if (threadIdx.x == 0) loss[0] = lsum / (float)n;
}

// `steps` Adam steps on mini-batches of `batch` rows listed in order[]; the
// parameters live in LDS for the whole run and every thread keeps the Adam
// moments of the parameters it owns in registers.  losses[k] = batch loss.
__global__ __launch_bounds__(kT) void k_mlp_train(float* __restrict__ params,
                                                  float* __restrict__ mom1,
                                                  float* __restrict__ mom2,
                                                  const float* __restrict__ scale,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ y,
                                                  const int32_t* __restrict__ order, int steps,
                                                  int batch, float lr, int t0,
                                                  float* __restrict__ losses) {
  __shared__ MlpLds L;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int k = threadIdx.x; k < kMlpParams; k += kT) L.W[k] = params[k];
  float m1[kOwn], m2[kOwn];
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = threadIdx.x + kT * i;
    m1[i] = k < kMlpParams ? mom1[k] : 0.0f;
    m2[i] = k < kMlpParams ? mom2[k] : 0.0f;
  }
  __syncthreads();
  for (int st = 0; st < steps; ++st) {
    float g[kOwn];
#pragma unroll
    for (int i = 0; i < kOwn; ++i) g[i] = 0.0f;
    float lsum = 0.0f;
    for (int first = 0; first < batch; first += kB) {
      const int nb = batch - first < kB ? batch - first : kB;
      load_chunk(L, x, y, scale, order, (int64_t)st * batch + first, nb);
      mlp_chunk(L, nb, (float)batch, g);
      lsum += L.lossv[0];
      __syncthreads();
    }
    if (threadIdx.x == 0) losses[st] = lsum / (float)batch;
    const int t = t0 + st + 1;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
#pragma unroll
    for (int i = 0; i < kOwn; ++i) {
      const int k = threadIdx.x + kT * i;
      if (k >= kMlpParams) break;
      m1[i] = b1 * m1[i] + (1.0f - b1) * g[i];
      m2[i] = b2 * m2[i] + (1.0f - b2) * g[i] * g[i];
      const float mh = m1[i] / c1, vh = m2[i] / c2;
      L.W[k] -= lr * mh / (sqrtf(vh) + eps);
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < kMlpParams; k += kT) params[k] = L.W[k];
#pragma unroll
  for (int i = 0; i < kOwn; ++i) {
    const int k = threadIdx.x + kT * i;
    if (k < kMlpParams) {
      mom1[k] = m1[i];
      mom2[k] = m2[i];
    }
  }
}

// BF16 inference: weights, inputs and hidden activations rounded to bfloat16
// (nearest even), products accumulated in float32; one thread per sample.
__global__ __launch_bounds__(256) void k_mlp_infer_bf16(const float* __restrict__ params,
                                                        const float* __restrict__ scale,
                                                        const float* __restrict__ x, int64_t n,
                                                        float* __restrict__ out) {
  __shared__ __hip_bfloat16 W[kMlpParams];
  for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) W[k] = __float2bfloat16(params[k]);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float xin[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i)
    xin[i] = __bfloat162float(__float2bfloat16((x[s * kIn + i] - scale[i]) / scale[kIn + i]));
  float h1[kH];
  for (int u = 0; u < kH; ++u) {
    float a = __bfloat162float(W[ob1 + u]);
#pragma unroll
    for (int i = 0; i < kIn; ++i) a += xin[i] * __bfloat162float(W[oW1 + i * kH + u]);
    h1[u] = __bfloat162float(__float2bfloat16(tanhf(a)));
  }
  float o = __bfloat162float(W[ob3]);
  for (int u = 0; u < kH; ++u) {
    float a = __bfloat162float(W[ob2 + u]);
    for (int i = 0; i < kH; ++i) a += h1[i] * __bfloat162float(W[oW2 + i * kH + u]);
    const float h2 = __bfloat162float(__float2bfloat16(tanhf(a)));
    o += h2 * __bfloat162float(W[oW3 + u]);
  }
  out[s] = o;
}

}  // namespace

template <int DIM>
static void counts_dim(const PlanView& P, const double* radii, int R, int reach, int32_t* counts,
                       hipStream_t s) {
  const dim3 grid((unsigned)((P.m + 3) / 4));
  hipLaunchKernelGGL(k_density_counts<DIM>, grid, dim3(256), 0, s, P, radii, R, reach, counts);
}

hipError_t launch_density_counts(const PlanView& P, const double* radii, int R, int reach,
                                 int32_t* counts, hipStream_t s) {
  if (P.dim == 2)
    counts_dim<2>(P, radii, R, reach, counts, s);
  else
    counts_dim<3>(P, radii, R, reach, counts, s);
  return hipGetLastError();
}

hipError_t launch_centre_blocks(const double* ctr, int64_t m, int dim, const double* box, int nb,
                                int32_t* blk, hipStream_t s) {
  hipLaunchKernelGGL(k_centre_blocks, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ctr, m,
                     dim, box, nb, blk);
  return hipGetLastError();
}

hipError_t launch_block_features(const int32_t* counts, const int32_t* blk, int64_t m, int R,
                                 int nblocks, float* feats, hipStream_t s) {
  hipLaunchKernelGGL(k_block_features, dim3(nblocks), dim3(256), 0, s, counts, blk, m, R, feats);
  return hipGetLastError();
}

hipError_t launch_block_sq_err(const double* y, int64_t nq, int dim, const double* f,
                               const double* h, const double* box, int nb, int nblocks,
                               double* sums, int64_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_block_sq_err, dim3(nblocks), dim3(256), 0, s, y, nq, dim, f, h, box, nb,
                     sums, counts);
  return hipGetLastError();
}

hipError_t launch_radius_broadcast(const float* pred, const int32_t* blk, int64_t m,
                                   double spacing, double rho_min, double rho_max,
                                   double rho_fallback, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_radius_broadcast, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, pred,
                     blk, m, spacing, rho_min, rho_max, rho_fallback, rho);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* scale, const float* x,
                           const float* y, int64_t n, float* grad, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(kT), 0, s, params, scale, x, y, n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_train(float* params, float* m1, float* m2, const float* scale,
                            const float* x, const float* y, const int32_t* order, int steps,
                            int batch, float lr, int t0, float* losses, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(kT), 0, s, params, m1, m2, scale, x, y, order,
                     steps, batch, lr, t0, losses);
  return hipGetLastError();
}

hipError_t launch_mlp_infer_bf16(const float* params, const float* scale, const float* x,
                                 int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_infer_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params,
                     scale, x, n, out);
  return hipGetLastError();
}

}  // namespace rbf
