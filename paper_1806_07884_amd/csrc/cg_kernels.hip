// Jacobi-preconditioned conjugate gradients on the assembled normal equations.
//
// One CG iteration k is two kernels, with every cross-block scalar carried
// from one kernel to the next through plain per-block partial sums:
//
//   spmv(k):   every block reduces the previous update's partials of r.z and
//              r.r (same fixed order in every block, so all blocks agree),
//              checks the trigger, forms beta = rz_k / rz_{k-1}, then
//              p_new = z + beta p_old (on the fly for every column it reads),
//              q = (B + lambda I) p_new and a partial of p_new . q.
//   update(k): every block reduces the partials of p . q, forms
//              alpha = rz_k / (p . q); x += alpha p; r -= alpha q;
//              z = D^-1 r; partials of r . z and r . r.
//
// Kernel boundaries make the partials of one kernel visible to every block of
// the next on all XCDs, so no device-scope fence (an L2 write-back per block
// on this chip) is ever executed.  Scalars the host reads are written by block
// 0 of each kernel.  Once a flag is raised the remaining launched kernels
// return at entry.
//
// Precision: the matrix and the iterated vectors are VT / XT (float64, or
// float32 for the mixed path); every dot product is accumulated in float64.
// The solution is kept in float64; at a reliable update the float64 residual
// g - (B + lambda I) x is recomputed and replaces the iterated one.
#include <hip/hip_ext.h>

#include "plan_kernels.h"
#include "solver.h"

namespace rbf {
namespace {

constexpr int kBlock = 256;

template <typename T, int G>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of one double per thread in a fixed order; every thread gets it.
__device__ __forceinline__ double block_sum(double v, double* ws) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) t += ws[w];
  return t;
}

// Sum of n partials part[stride * k + off], identical in every block.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int n,
                                                  int stride, int off, double* ws) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) s += part[stride * k + off];
  return block_sum(s, ws);
}

constexpr int kWavesPerBlock = kBlock / kWave;

// For the slice of S = 64 / L rows owned by this wave, the row sums
// az = sum_e b_e z[col_e] and ap = sum_e b_e p[col_e], complete in the lane
// with (lane % L) == 0 of every row.  Four independent loads per lane are in
// flight per step; rows past m gather from row m - 1 with value 0.
template <typename VT, typename XT, typename CT, int L>
__device__ __forceinline__ void slice_products(int64_t m, int64_t slice, const CgMatrix& A,
                                               const XT* __restrict__ z,
                                               const XT* __restrict__ p, XT* az, XT* ap,
                                               int64_t* row_out) {
  constexpr int S = kWave / L;
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t row = slice * S + lane / L;
  const int32_t rowc = (int32_t)(row < m ? row : m - 1);
  const int64_t base = A.sptr[slice] + lane;
  const int steps = A.slen[slice] / L;
  XT a0 = (XT)0, a1 = (XT)0, a2 = (XT)0, a3 = (XT)0;
  XT b0 = (XT)0, b1 = (XT)0, b2 = (XT)0, b3 = (XT)0;
  int st = 0;
  for (; st + 3 < steps; st += 4) {
    const int64_t o = base + (int64_t)st * kWave;
    const int32_t l0 = rowc + (int32_t)col[o];
    const int32_t l1 = rowc + (int32_t)col[o + kWave];
    const int32_t l2 = rowc + (int32_t)col[o + 2 * kWave];
    const int32_t l3 = rowc + (int32_t)col[o + 3 * kWave];
    const XT v0 = (XT)val[o], v1 = (XT)val[o + kWave];
    const XT v2 = (XT)val[o + 2 * kWave], v3 = (XT)val[o + 3 * kWave];
    a0 += v0 * z[l0];
    b0 += v0 * p[l0];
    a1 += v1 * z[l1];
    b1 += v1 * p[l1];
    a2 += v2 * z[l2];
    b2 += v2 * p[l2];
    a3 += v3 * z[l3];
    b3 += v3 * p[l3];
  }
  for (; st < steps; ++st) {
    const int64_t o = base + (int64_t)st * kWave;
    const int32_t l0 = rowc + (int32_t)col[o];
    const XT v0 = (XT)val[o];
    a0 += v0 * z[l0];
    b0 += v0 * p[l0];
  }
  XT a = (a0 + a1) + (a2 + a3), b = (b0 + b1) + (b2 + b3);
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  *az = a;
  *ap = b;
  *row_out = row;
}

// q = (B + lambda I) p_new with p_new = z + beta p_old, factored as
// q = B z + beta B p_old so that the matrix is streamed before beta is known.
// One wave per slice (grid-stride over slices).
template <typename VT, typename XT, typename CT, int L>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(
    int64_t m, CgMatrix A, const XT* __restrict__ z, const XT* __restrict__ pold,
    XT* __restrict__ pnew, XT* __restrict__ q, CgScalars* __restrict__ sc,
    const double* __restrict__ part_in, int n_in, double* __restrict__ part_out, int parity,
    int fixed_beta) {
  __shared__ double ws[kBlock / kWave];
  if (sc->done) return;
  // partials of the previous update: loaded first, reduced after the first
  // slice's matrix loads are in flight
  double prz = 0.0, prr = 0.0;
  for (int k = threadIdx.x; k < n_in; k += kBlock) {
    prz += part_in[2 * k];
    prr += part_in[2 * k + 1];
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  int64_t slice = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  XT az = (XT)0, ap = (XT)0;
  int64_t row = m;
  if (slice < A.nslices) slice_products<VT, XT, CT, L>(m, slice, A, z, pold, &az, &ap, &row);
  const double rz = block_sum(prz, ws);
  const double rr = block_sum(prr, ws);
  if (!__builtin_isfinite(rz) || !__builtin_isfinite(rr)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = 2;
    return;
  }
  if (rr <= sc->trigger2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->rr = rr;
      sc->done = 1;
    }
    return;
  }
  const double beta_d = fixed_beta ? sc->beta_fixed : rz / sc->rzh[parity ^ 1];
  const XT beta = (XT)beta_d;
  double contrib = 0.0;
  while (slice < A.nslices) {
    if ((lane & (L - 1)) == 0 && row < m) {
      const XT pj = z[row] + beta * pold[row];
      const XT qj = az + beta * ap;
      pnew[row] = pj;
      q[row] = qj;
      contrib += (double)pj * (double)qj;
    }
    slice += wstride;
    if (slice < A.nslices) slice_products<VT, XT, CT, L>(m, slice, A, z, pold, &az, &ap, &row);
  }
  const double bs = block_sum(contrib, ws);
  if (threadIdx.x == 0) {
    part_out[blockIdx.x] = bs;
    if (blockIdx.x == 0) {
      sc->rzh[parity] = rz;
      sc->rr = rr;
      sc->beta = beta_d;
    }
  }
}

template <typename XT>
__global__ __launch_bounds__(kBlock) void k_cg_update(
    int64_t m, const XT* __restrict__ p, const XT* __restrict__ q, XT* __restrict__ x,
    XT* __restrict__ r, XT* __restrict__ z, const XT* __restrict__ dinv,
    CgScalars* __restrict__ sc, const double* __restrict__ part_in, int n_in,
    double* __restrict__ part_out, int parity) {
  __shared__ double ws[kBlock / kWave];
  if (sc->done) return;
  double ppq = 0.0;
  for (int k = threadIdx.x; k < n_in; k += kBlock) ppq += part_in[k];
  // the first element's operands are loaded before alpha is known
  int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  XT pj = (XT)0, qj = (XT)0, xj = (XT)0, rj = (XT)0, dj = (XT)0;
  if (j < m) {
    pj = p[j];
    qj = q[j];
    xj = x[j];
    rj = r[j];
    dj = dinv[j];
  }
  const double pq = block_sum(ppq, ws);
  if (!(pq > 0.0) || !__builtin_isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = 2;
    return;
  }
  const double alpha_d = sc->rzh[parity] / pq;
  const XT alpha = (XT)alpha_d;
  double rz = 0.0, rr = 0.0;
  while (j < m) {
    xj += alpha * pj;
    rj -= alpha * qj;
    const XT zj = dj * rj;
    x[j] = xj;
    r[j] = rj;
    z[j] = zj;
    rz += (double)rj * (double)zj;
    rr += (double)rj * (double)rj;
    j += stride;
    if (j < m) {
      pj = p[j];
      qj = q[j];
      xj = x[j];
      rj = r[j];
      dj = dinv[j];
    }
  }
  const double brz = block_sum(rz, ws);
  const double brr = block_sum(rr, ws);
  if (threadIdx.x == 0) {
    part_out[2 * blockIdx.x] = brz;
    part_out[2 * blockIdx.x + 1] = brr;
    if (blockIdx.x == 0) {
      sc->alpha = alpha_d;
      sc->pq = pq;
      sc->iter += 1;
    }
  }
}

// x_hi += x_lo; x_lo = 0 (x_lo is the iterated correction).
template <typename XT>
__global__ void k_fold_solution(int64_t m, double* __restrict__ xhi, XT* __restrict__ xlo) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  xhi[j] += (double)xlo[j];
  xlo[j] = (XT)0;
}

// Float64 residual of the stored system: r64 = g - (B + lambda I) x_hi, then
// r = (XT) r64 and z = D^-1 r (one wave per slice).
template <typename VT, typename XT, typename CT, int L>
__global__ __launch_bounds__(kBlock) void k_true_residual(int64_t m, CgMatrix A,
                                                          const double* __restrict__ xhi,
                                                          const double* __restrict__ g,
                                                          const XT* __restrict__ dinv,
                                                          double* __restrict__ r64,
                                                          XT* __restrict__ r, XT* __restrict__ z) {
  constexpr int S = kWave / L;
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t slice = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
       slice < A.nslices; slice += (int64_t)gridDim.x * kWavesPerBlock) {
    const int64_t row = slice * S + lane / L;
    const int32_t rowc = (int32_t)(row < m ? row : m - 1);
    const int64_t base = A.sptr[slice] + lane;
    const int steps = A.slen[slice] / L;
    double acc = 0.0;
    for (int st = 0; st < steps; ++st) {
      const int64_t o = base + (int64_t)st * kWave;
      acc += (double)val[o] * xhi[rowc + (int32_t)col[o]];
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((lane & (L - 1)) == 0 && row < m) {
      const double rv = g[row] - acc;
      const XT ri = (XT)rv;
      r64[row] = rv;
      r[row] = ri;
      z[row] = dinv[row] * ri;
    }
  }
}

// Partials of r.z and r64.r64 in the update kernel's layout.
template <typename XT>
__global__ __launch_bounds__(kBlock) void k_residual_dots(int64_t m, const double* __restrict__ r64,
                                                          const XT* __restrict__ r,
                                                          const XT* __restrict__ z,
                                                          double* __restrict__ part_out) {
  __shared__ double ws[kBlock / kWave];
  double rz = 0.0, rr = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * kBlock) {
    rz += (double)r[j] * (double)z[j];
    rr += r64[j] * r64[j];
  }
  const double brz = block_sum(rz, ws);
  const double brr = block_sum(rr, ws);
  if (threadIdx.x == 0) {
    part_out[2 * blockIdx.x] = brz;
    part_out[2 * blockIdx.x + 1] = brr;
  }
}

// After a float64 residual: sets the true residual norm, the convergence flag,
// the next trigger, and the beta the next spmv takes (0 on a restart,
// rz_true / rz_{k-1} on a reliable update).
__global__ __launch_bounds__(kBlock) void k_residual_scalars(CgScalars* __restrict__ sc,
                                                             const double* __restrict__ part,
                                                             int n, int restart, int parity) {
  __shared__ double ws[kBlock / kWave];
  const double rz = reduce_partials(part, n, 2, 0, ws);
  const double rr = reduce_partials(part, n, 2, 1, ws);
  if (threadIdx.x == 0) {
    sc->rr_true = rr;
    sc->rr = rr;
    sc->beta_fixed = restart ? 0.0 : rz / sc->rzh[parity ^ 1];
    const double trig = sc->delta2 * rr;
    sc->trigger2 = trig > sc->tol2 ? trig : sc->tol2;
    if (!__builtin_isfinite(rr) || !__builtin_isfinite(rz)) {
      sc->done = 2;
    } else if (rr <= sc->tol2) {
      sc->done = 3;
    } else {
      sc->done = 0;
    }
  }
}

template <typename XT>
__global__ void k_zero_inactive(int64_t m, const uint8_t* __restrict__ active,
                                double* __restrict__ xhi, XT* __restrict__ xlo,
                                XT* __restrict__ p0, XT* __restrict__ p1) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  if (!active[j]) xhi[j] = 0.0;
  xlo[j] = (XT)0;
  p0[j] = (XT)0;
  p1[j] = (XT)0;
}

// ||g||^2 and the initial state of the scalars (single block, fixed order).
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t m, const double* __restrict__ g,
                                                    CgScalars* __restrict__ sc, double rtol,
                                                    double delta) {
  __shared__ double ws[kBlock / kWave];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += kBlock) s += g[j] * g[j];
  s = block_sum(s, ws);
  if (threadIdx.x == 0) {
    sc->gg = s;
    sc->tol2 = rtol * rtol * s;
    sc->delta2 = delta * delta;
    sc->trigger2 = sc->tol2;
    sc->done = 0;
    sc->iter = 0;
    sc->rzh[0] = sc->rzh[1] = 1.0;
    sc->beta = sc->beta_fixed = 0.0;
    sc->alpha = sc->pq = 0.0;
  }
}

template <typename VT, typename XT, typename CT, int L>
void launch_spmv_l(const CgArgs<XT>& a, const CgMatrix& A, int parity, int fixed_beta,
                   hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  if (e0) {
    // the extended launch stamps the events at the kernel's own start and end
    hipExtLaunchKernelGGL((k_cg_spmv<VT, XT, CT, L>), dim3(a.spmv_blocks), dim3(kBlock), 0, s, e0,
                          e1, 0, a.m, A, (const XT*)a.z, (const XT*)a.p[parity], a.p[parity ^ 1],
                          a.q, a.sc, (const double*)a.part_upd, a.update_blocks, a.part_spmv,
                          parity, fixed_beta);
  } else {
    hipLaunchKernelGGL((k_cg_spmv<VT, XT, CT, L>), dim3(a.spmv_blocks), dim3(kBlock), 0, s, a.m,
                       A, (const XT*)a.z, (const XT*)a.p[parity], a.p[parity ^ 1], a.q, a.sc,
                       (const double*)a.part_upd, a.update_blocks, a.part_spmv, parity,
                       fixed_beta);
  }
}

template <typename VT, typename XT, typename CT, int L>
void launch_true_residual_l(const CgArgs<XT>& a, const CgMatrix& A, const double* g,
                            hipStream_t s) {
  hipLaunchKernelGGL((k_true_residual<VT, XT, CT, L>), dim3(a.spmv_blocks), dim3(kBlock), 0, s,
                     a.m, A, (const double*)a.xhi, g, (const XT*)a.dinv, a.r64, a.r, a.z);
}

bool grids_ok(int spmv_blocks, int update_blocks) {
  return spmv_blocks >= 1 && spmv_blocks <= kCgMaxBlocks && update_blocks >= 1 &&
         update_blocks <= kCgMaxBlocks;
}

}  // namespace

int sell_lanes(double mean_row) {
  if (mean_row > 192) return 8;
  if (mean_row > 24) return 4;
  return 2;
}

int cg_grid_blocks(int64_t nslices) {
  const int64_t b = (nslices + kWavesPerBlock - 1) / kWavesPerBlock;
  return (int)(b < 1 ? 1 : (b > kCgMaxBlocks ? kCgMaxBlocks : b));
}

int cg_update_blocks(int64_t m) {
  const int64_t b = (m + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > kCgMaxBlocks ? kCgMaxBlocks : b));
}

namespace {

template <typename VT, typename XT, typename CT>
void spmv_dispatch(const CgArgs<XT>& a, const CgMatrix& A, int parity, int fixed_beta,
                   hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  switch (A.lanes) {
    case 2: launch_spmv_l<VT, XT, CT, 2>(a, A, parity, fixed_beta, e0, e1, s); break;
    case 4: launch_spmv_l<VT, XT, CT, 4>(a, A, parity, fixed_beta, e0, e1, s); break;
    default: launch_spmv_l<VT, XT, CT, 8>(a, A, parity, fixed_beta, e0, e1, s); break;
  }
}

template <typename VT, typename XT, typename CT>
void residual_dispatch(const CgArgs<XT>& a, const CgMatrix& A, const double* g, hipStream_t s) {
  switch (A.lanes) {
    case 2: launch_true_residual_l<VT, XT, CT, 2>(a, A, g, s); break;
    case 4: launch_true_residual_l<VT, XT, CT, 4>(a, A, g, s); break;
    default: launch_true_residual_l<VT, XT, CT, 8>(a, A, g, s); break;
  }
}

}  // namespace

template <typename VT, typename XT>
hipError_t cg_spmv(const CgArgs<XT>& a, const CgMatrix& A, int parity, int fixed_beta,
                   hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  if (!grids_ok(a.spmv_blocks, a.update_blocks)) return hipErrorInvalidValue;
  if (A.col16)
    spmv_dispatch<VT, XT, int16_t>(a, A, parity, fixed_beta, e0, e1, s);
  else
    spmv_dispatch<VT, XT, int32_t>(a, A, parity, fixed_beta, e0, e1, s);
  return hipGetLastError();
}

template <typename XT>
hipError_t cg_update(const CgArgs<XT>& a, int parity, hipStream_t s) {
  if (!grids_ok(a.spmv_blocks, a.update_blocks)) return hipErrorInvalidValue;
  // the direction written by the preceding spmv sits in p[parity ^ 1]
  hipLaunchKernelGGL(k_cg_update<XT>, dim3(a.update_blocks), dim3(kBlock), 0, s, a.m,
                     (const XT*)a.p[parity ^ 1], (const XT*)a.q, a.xlo, a.r, a.z,
                     (const XT*)a.dinv, a.sc, (const double*)a.part_spmv, a.spmv_blocks,
                     a.part_upd, parity);
  return hipGetLastError();
}

template <typename VT, typename XT>
hipError_t cg_true_residual(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int restart,
                            int parity, hipStream_t s) {
  if (!grids_ok(a.spmv_blocks, a.update_blocks)) return hipErrorInvalidValue;
  const int bs = 256;
  const dim3 eg((unsigned)((a.m + bs - 1) / bs));
  hipLaunchKernelGGL(k_fold_solution<XT>, eg, dim3(bs), 0, s, a.m, a.xhi, a.xlo);
  if (A.col16)
    residual_dispatch<VT, XT, int16_t>(a, A, g, s);
  else
    residual_dispatch<VT, XT, int32_t>(a, A, g, s);
  hipLaunchKernelGGL(k_residual_dots<XT>, dim3(a.update_blocks), dim3(kBlock), 0, s, a.m,
                     (const double*)a.r64, (const XT*)a.r, (const XT*)a.z, a.part_upd);
  hipLaunchKernelGGL(k_residual_scalars, dim3(1), dim3(kBlock), 0, s, a.sc,
                     (const double*)a.part_upd, a.update_blocks, restart, parity);
  return hipGetLastError();
}

template <typename XT>
hipError_t cg_setup(const CgArgs<XT>& a, const uint8_t* active, const double* g, double rtol,
                    double delta, hipStream_t s) {
  const int bs = 256;
  const dim3 eg((unsigned)((a.m + bs - 1) / bs));
  hipLaunchKernelGGL(k_zero_inactive<XT>, eg, dim3(bs), 0, s, a.m, active, a.xhi, a.xlo, a.p[0],
                     a.p[1]);
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kBlock), 0, s, a.m, g, a.sc, rtol, delta);
  return hipGetLastError();
}

template hipError_t cg_spmv<double, double>(const CgArgs<double>&, const CgMatrix&, int, int,
                                            hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cg_spmv<float, float>(const CgArgs<float>&, const CgMatrix&, int, int,
                                          hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cg_update<double>(const CgArgs<double>&, int, hipStream_t);
template hipError_t cg_update<float>(const CgArgs<float>&, int, hipStream_t);
template hipError_t cg_true_residual<double, double>(const CgArgs<double>&, const CgMatrix&,
                                                     const double*, int, int, hipStream_t);
template hipError_t cg_true_residual<float, float>(const CgArgs<float>&, const CgMatrix&,
                                                   const double*, int, int, hipStream_t);
template hipError_t cg_setup<double>(const CgArgs<double>&, const uint8_t*, const double*, double,
                                     double, hipStream_t);
template hipError_t cg_setup<float>(const CgArgs<float>&, const uint8_t*, const double*, double,
                                    double, hipStream_t);

}  // namespace rbf
