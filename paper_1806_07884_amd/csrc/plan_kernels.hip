// Plan kernels: grid hash of points and centres, support counts and the
// structural sparsity pattern of B = A^T A (Section 5, eq. 11-13).
//
// Support of centre j (Algorithm 1, strict range query; eq. 18):
//     supp(j) = { points x : s(x, xi_j) < rho_j^2 }.
// Pattern of row j of B (both triangles are produced; the stored upper CSR is
// the suffix l >= j of each sorted row):
//     { l active : supp(j) and supp(l) share a point }.
#include "plan_kernels.h"

namespace rbf {
namespace {

constexpr int kRedThreads = 256;

// Per-block min / max / non-finite flag of one float64 array.
__global__ __launch_bounds__(kRedThreads) void k_minmax_partial(const double* __restrict__ a,
                                                                int64_t n,
                                                                double* __restrict__ pmin,
                                                                double* __restrict__ pmax,
                                                                int* __restrict__ pbad) {
  __shared__ double smin[kRedThreads / kWave], smax[kRedThreads / kWave];
  __shared__ int sbad[kRedThreads / kWave];
  double lo = __builtin_inf(), hi = -__builtin_inf();
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = a[i];
    if (!__builtin_isfinite(v)) {
      bad = 1;
    } else {
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o1 = __shfl_xor(lo, off, kWave), o2 = __shfl_xor(hi, off, kWave);
    int o3 = __shfl_xor(bad, off, kWave);
    lo = o1 < lo ? o1 : lo;
    hi = o2 > hi ? o2 : hi;
    bad |= o3;
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    smin[w] = lo;
    smax[w] = hi;
    sbad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kRedThreads / kWave; ++k) {
      lo = smin[k] < lo ? smin[k] : lo;
      hi = smax[k] > hi ? smax[k] : hi;
      bad |= sbad[k];
    }
    pmin[blockIdx.x] = lo;
    pmax[blockIdx.x] = hi;
    pbad[blockIdx.x] = bad;
  }
}

__global__ void k_minmax_final(const double* __restrict__ pmin, const double* __restrict__ pmax,
                               const int* __restrict__ pbad, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo = __builtin_inf(), hi = -__builtin_inf();
  int bad = 0;
  for (int k = 0; k < nb; ++k) {
    lo = pmin[k] < lo ? pmin[k] : lo;
    hi = pmax[k] > hi ? pmax[k] : hi;
    bad |= pbad[k];
  }
  out[0] = lo;
  out[1] = hi;
  out[2] = (double)bad;
}

template <int DIM>
__global__ void k_cell_keys(Grid G, const double* __restrict__ x, int64_t n,
                            uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) p[d] = x[d * n + i];
  int c[3];
  const bool in = cell_of<DIM>(G, p, c);
  keys[i] = in ? (uint32_t)cell_id<DIM>(G, c) : (uint32_t)G.ncell;
  idx[i] = (int32_t)i;
}

__global__ void k_gather_soa(const double* __restrict__ src, const int32_t* __restrict__ perm,
                             int64_t n, int dim, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = perm[i];
  for (int d = 0; d < dim; ++d) dst[d * n + i] = src[d * n + k];
}

__global__ void k_radius_tables(const double* __restrict__ rho_in, double rho, int64_t m,
                                double* __restrict__ rho_c, double* __restrict__ rho2_c,
                                double* __restrict__ irho_c) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const double r = rho_in ? rho_in[j] : rho;
  rho_c[j] = r;
  rho2_c[j] = r * r;
  irho_c[j] = 1.0 / r;
}

// One wave per centre: count the points of its support.
template <int DIM>
__global__ __launch_bounds__(256) void k_support_count(PlanView P, int32_t min_support,
                                                       int32_t* __restrict__ count,
                                                       uint8_t* __restrict__ active) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (j >= P.m) return;
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double r2 = P.rho2[j];
  int c[3];
  int n = 0;
  if (cell_of<DIM>(P.grid, xj, c)) {
    NbrWalk<DIM> walk(P.grid, c, 1);
    for (int k = 0; k < walk.rows(); ++k) {
      int lo_id, hi_id;
      if (!walk.range(k, lo_id, hi_id)) continue;
      const int lo = P.pcs[lo_id], hi = P.pcs[hi_id + 1];
      for (int i = lo + lane; i < hi; i += kWave) {
        double p[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = P.ps[d * P.n + i];
        n += sqdist<DIM>(p, xj) < r2 ? 1 : 0;
      }
    }
  }
  n = wave_sum_int(n);
  if (lane == 0) {
    count[j] = n;
    active[j] = n >= min_support ? 1 : 0;
  }
}

constexpr int kSymChunk = 256;

// Pattern of row j.  Count mode writes the full-row and lower-part sizes; fill
// mode writes the sorted columns of the full row.
template <int DIM, bool FILL>
__global__ __launch_bounds__(kWave) void k_symbolic(PlanView P, int64_t* __restrict__ full_cnt,
                                                    int32_t* __restrict__ lower_cnt,
                                                    const int64_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ col,
                                                    int32_t* __restrict__ err) {
  __shared__ int32_t cand[kMaxCand];
  __shared__ int32_t surv[kMaxCand];
  __shared__ uint8_t flag[kMaxCand];
  __shared__ double sp[DIM][kSymChunk];
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  const uint64_t lt = lanemask_lt();
  if (!P.active[j]) {
    if (!FILL && lane == 0) {
      full_cnt[j] = 0;
      lower_cnt[j] = 0;
    }
    return;
  }
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double rj = P.rho[j];
  int c[3];
  cell_of<DIM>(P.grid, xj, c);  // centres always lie inside the box

  // candidate columns: active centres whose ball can meet centre j's ball
  int nc = 0;
  {
    NbrWalk<DIM> walk(P.grid, c, 2);
    for (int k = 0; k < walk.rows(); ++k) {
      int lo_id, hi_id;
      if (!walk.range(k, lo_id, hi_id)) continue;
      const int lo = P.ccs[lo_id], hi = P.ccs[hi_id + 1];
      for (int i0 = lo; i0 < hi; i0 += kWave) {
        const int i = i0 + lane;
        bool ok = false;
        int l = 0;
        if (i < hi) {
          l = P.cperm[i];
          if (P.active[l]) {
            double xl[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xl[d] = P.ctr_s[d * P.m + i];
            const double reach = (rj + P.rho[l]) * (1.0 + 1e-9);
            ok = sqdist<DIM>(xl, xj) <= reach * reach;
          }
        }
        const uint64_t m = __ballot(ok);
        const int pos = nc + __popcll(m & lt);
        if (ok && pos < kMaxCand) cand[pos] = l;
        nc += __popcll(m);
      }
    }
  }
  if (nc > kMaxCand) {
    if (lane == 0) atomicExch(err, 1);
    if (!FILL && lane == 0) {
      full_cnt[j] = 0;
      lower_cnt[j] = 0;
    }
    return;
  }
  for (int t = lane; t < nc; t += kWave) flag[t] = 0;
  __syncthreads();

  // a candidate survives when one supported point of j lies in its support
  stream_support<DIM, kSymChunk>(P, xj, P.rho2[j], sp, nullptr, [&](int np) {
    for (int t = lane; t < nc; t += kWave) {
      if (flag[t]) continue;
      const int l = cand[t];
      double xl[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) xl[d] = P.ctr[d * P.m + l];
      const double r2l = P.rho2[l];
      for (int q = 0; q < np; ++q) {
        double p[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = sp[d][q];
        if (sqdist<DIM>(p, xl) < r2l) {
          flag[t] = 1;
          break;
        }
      }
    }
  });
  __syncthreads();

  // compact the survivors, keeping candidate order
  int ns = 0, nlow = 0;
  for (int t0 = 0; t0 < nc; t0 += kWave) {
    const int t = t0 + lane;
    const bool s = t < nc && flag[t];
    const uint64_t m = __ballot(s);
    const uint64_t ml = __ballot(s && cand[t] < j);
    if (s) surv[ns + __popcll(m & lt)] = cand[t];
    ns += __popcll(m);
    nlow += __popcll(ml);
  }
  __syncthreads();
  if (!FILL) {
    if (lane == 0) {
      full_cnt[j] = ns;
      lower_cnt[j] = nlow;
    }
    return;
  }
  // ascending columns: rank of each survivor among the survivors
  const int64_t base = row_ptr[j];
  for (int t = lane; t < ns; t += kWave) {
    const int l = surv[t];
    int rank = 0;
    for (int u = 0; u < ns; ++u) rank += surv[u] < l ? 1 : 0;
    col[base + rank] = l;
  }
}

}  // namespace

hipError_t launch_minmax(const double* a, int64_t n, double* partial_min, double* partial_max,
                         int* partial_bad, int nblocks, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_partial, dim3(nblocks), dim3(kRedThreads), 0, s, a, n, partial_min,
                     partial_max, partial_bad);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, s, (const double*)partial_min,
                     (const double*)partial_max, (const int*)partial_bad, nblocks, out3);
  return hipGetLastError();
}

hipError_t launch_cell_keys(int dim, const Grid& G, const double* x, int64_t n, uint32_t* keys,
                            int32_t* idx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  const dim3 grid((unsigned)((n + bs - 1) / bs));
  if (dim == 2)
    hipLaunchKernelGGL(k_cell_keys<2>, grid, dim3(bs), 0, s, G, x, n, keys, idx);
  else
    hipLaunchKernelGGL(k_cell_keys<3>, grid, dim3(bs), 0, s, G, x, n, keys, idx);
  return hipGetLastError();
}

hipError_t launch_gather_soa(const double* src, const int32_t* perm, int64_t n, int dim,
                             double* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_gather_soa, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, src, perm,
                     n, dim, dst);
  return hipGetLastError();
}

hipError_t launch_radius_tables(const double* rho_in, double rho, int64_t m, double* rho_c,
                                double* rho2_c, double* irho_c, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(k_radius_tables, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, rho_in,
                     rho, m, rho_c, rho2_c, irho_c);
  return hipGetLastError();
}

hipError_t launch_support_count(const PlanView& P, int32_t min_support, int32_t* count,
                                uint8_t* active, hipStream_t s) {
  const int waves = 4;
  const dim3 grid((unsigned)((P.m + waves - 1) / waves));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_support_count<2>, grid, dim3(waves * kWave), 0, s, P, min_support, count,
                       active);
  else
    hipLaunchKernelGGL(k_support_count<3>, grid, dim3(waves * kWave), 0, s, P, min_support, count,
                       active);
  return hipGetLastError();
}

hipError_t launch_symbolic(const PlanView& P, bool fill, int64_t* full_cnt, int32_t* lower_cnt,
                           const int64_t* row_ptr, int32_t* col, int32_t* err, hipStream_t s) {
  const dim3 grid((unsigned)P.m);
  if (P.dim == 2) {
    if (fill)
      hipLaunchKernelGGL((k_symbolic<2, true>), grid, dim3(kWave), 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err);
    else
      hipLaunchKernelGGL((k_symbolic<2, false>), grid, dim3(kWave), 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err);
  } else {
    if (fill)
      hipLaunchKernelGGL((k_symbolic<3, true>), grid, dim3(kWave), 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err);
    else
      hipLaunchKernelGGL((k_symbolic<3, false>), grid, dim3(kWave), 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err);
  }
  return hipGetLastError();
}

}  // namespace rbf
