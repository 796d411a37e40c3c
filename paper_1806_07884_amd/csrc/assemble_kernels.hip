// Numeric assembly of the normal equations (Section 5, eq. 11-12):
//
//     b_jl = sum_{k in supp(j) and supp(l)} phi_kj * phi_kl      (l >= j)
//     g_j  = sum_{k in supp(j)} phi_kj * h_k
//
// One block of kAsmWaves waves owns one row j.  The row's candidate points
// (the hash cells around centre j, in sorted order) are split into kAsmWaves
// contiguous pieces; each wave streams the supported points of its piece
// through its own LDS slab, and every lane owns up to kSlots columns of the
// upper part of the row.  The waves' partial sums are then added in wave
// order.  Each accumulator has exactly one writer (no atomics), so the
// summation order is fixed and the result is deterministic.  The upper
// value is also written to its mirror position (l, j) of the full CSR, which
// the solver reads, so the stored matrix is exactly symmetric.  A is never
// materialised: phi is evaluated on the fly.
//
// Plans whose rows are wider than one wave (more than 64 upper columns on
// average) take a grouped path:
// the staged points are taken 64 at a time (consecutive, so spatially close:
// points are sorted by sub-cell within a hash cell); a group's bounding ball
// selects the columns whose support can reach it; those columns are handed
// to the lanes, and each lane runs through the group's points for its column,
// accumulating into the wave's LDS accumulator of that column.  When few
// columns reach a group, two or four lanes share a column, each summing a
// contiguous part of the group's points, and the parts are added to the
// column's sum in order: every sum has a fixed order, so the result is
// deterministic (its rounding differs from the ungrouped path's order by the
// summation bound).
//
// FP64 variant: float64 phi and float64 accumulation.
// FP32 variant: squared distance and support test in float64 (the pattern is
// fixed in float64), then phi in float32 and float32 Kahan-compensated sums.
#define RBF_CHECK_FILE 2  // place ids of the checked build's device checks
#include <algorithm>

#include "accum.h"
#include "plan_kernels.h"
#include "solver.h"

namespace rbf {
namespace {

constexpr int kAsmChunk = 256;
constexpr int kSlots = 4;  // columns per lane in one pass: 256 per pass
constexpr int kCols = kWave * kSlots;

constexpr int kAsmWaves = 4;

template <int DIM, int PHI, typename T, bool GROUPED>
__global__ __launch_bounds__(kWave* kAsmWaves) void k_assemble(
    PlanView P, const double* __restrict__ hs, const int64_t* __restrict__ row_ptr,
    const int32_t* __restrict__ lower_cnt, const int32_t* __restrict__ col,
    const int64_t* __restrict__ sptr, int lanes, T* __restrict__ val, double* __restrict__ g,
    double* __restrict__ diag) {
  // the grouped path stages half as many points per chunk (its LDS holds the
  // pass's columns and accumulators too)
  constexpr int kChunk = GROUPED ? kAsmChunk / 2 : kAsmChunk;
  __shared__ double sp[kAsmWaves][DIM][kChunk];
  __shared__ int32_t sidx[kAsmWaves][kChunk];
  __shared__ T sphi[kAsmWaves][kChunk];
  __shared__ double red[GROUPED ? 1 : kAsmWaves][GROUPED ? 1 : kCols];
  __shared__ double gred[kAsmWaves];
  // grouped path: the pass's columns, per-wave accumulators and column lists
  __shared__ double cxs[GROUPED ? DIM : 1][GROUPED ? kCols : 1];
  __shared__ double crs[GROUPED ? kCols : 1], cr2s[GROUPED ? kCols : 1], cirs[GROUPED ? kCols : 1];
  __shared__ AccPod<T> cacc[GROUPED ? kAsmWaves : 1][GROUPED ? kCols : 1];
  __shared__ int16_t nlist[GROUPED ? kAsmWaves : 1][GROUPED ? kCols : 1];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = blockIdx.x;
  const uint64_t lt = lanemask_lt();
  if (!P.active[j]) {
    if (threadIdx.x == 0) {
      g[j] = 0.0;
      diag[j] = 0.0;
    }
    return;
  }
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double r2j = P.rho2[j], irj = P.irho[j];
  const int64_t e0 = row_ptr[j] + lower_cnt[j];
  const int64_t e1 = row_ptr[j + 1];
  const int64_t R = e1 - e0;
  Acc<T> gacc;
  for (int64_t cb = 0; cb < R; cb += (int64_t)kWave * kSlots) {
    const int nslot = (int)((R - cb + kWave - 1) / kWave) < kSlots
                          ? (int)((R - cb + kWave - 1) / kWave)
                          : kSlots;
    double xl[kSlots][DIM];
    double r2l[kSlots], irl[kSlots];
    int32_t lcol[kSlots];
    bool ok[kSlots];
    Acc<T> acc[kSlots];
#pragma unroll
    for (int t = 0; t < kSlots; ++t) {
      const int64_t e = e0 + cb + lane + (int64_t)kWave * t;
      ok[t] = t < nslot && e < e1;
      lcol[t] = ok[t] ? col[e] : 0;
      if (ok[t] && !RBF_CHECK(P, (unsigned)lcol[t] < (unsigned)P.m)) {
        ok[t] = false;
        lcol[t] = 0;
      }
      if (!GROUPED) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) xl[t][d] = ok[t] ? P.ctr[d * P.m + lcol[t]] : 0.0;
        r2l[t] = ok[t] ? P.rho2[lcol[t]] : 0.0;
        irl[t] = ok[t] ? P.irho[lcol[t]] : 0.0;
      }
    }
    const bool first = cb == 0;
    const int ncol = (int)(R - cb < kCols ? R - cb : kCols);
    if (GROUPED) {
      for (int t = threadIdx.x; t < ncol; t += kWave * kAsmWaves) {
        const int32_t l0 = col[e0 + cb + t];
        const int32_t l = RBF_CHECK(P, (unsigned)l0 < (unsigned)P.m) ? l0 : 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) cxs[d][t] = P.ctr[d * P.m + l];
        crs[t] = P.rho[l];
        cr2s[t] = P.rho2[l];
        cirs[t] = P.irho[l];
      }
      for (int t = lane; t < ncol; t += kWave) cacc[w][t] = AccPod<T>{(T)0, (T)0};
      __syncthreads();
    }
    T* wphi = sphi[w];
    const int32_t* widx = sidx[w];
    double(*wsp)[kChunk] = sp[w];
    stream_support_part<DIM, kChunk>(P, xj, r2j, w, kAsmWaves, wsp, sidx[w], [&](int np) {
      // phi_kj of the chunk's points, and their share of g_j
      for (int q = lane; q < np; q += kWave) {
        double p[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
        const T phij = wendland<PHI, T>(scaled_r<T>(sqdist<DIM>(p, xj), irj));
        wphi[q] = phij;
        if (first) gacc.add(phij * (T)hs[widx[q]]);
      }
      wave_sync();
      if constexpr (!GROUPED) {
        for (int q = 0; q < np; ++q) {
          double p[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
          const T phij = wphi[q];
#pragma unroll
          for (int t = 0; t < kSlots; ++t) {
            if (t < nslot && ok[t]) {
              const double s = sqdist<DIM>(p, xl[t]);
              if (s < r2l[t]) acc[t].add(phij * wendland<PHI, T>(scaled_r<T>(s, irl[t])));
            }
          }
        }
        return;
      } else {
      for (int g0 = 0; g0 < np; g0 += kWave) {
        const int n = np - g0 < kWave ? np - g0 : kWave;
        // bounding ball of the group: centre its first point, radius the
        // farthest of its points (rounded up)
        double c0[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) c0[d] = wsp[d][g0];
        float rg = 0.f;
        if (lane < n) {
          double p[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) p[d] = wsp[d][g0 + lane];
          rg = (float)__builtin_sqrt(sqdist<DIM>(p, c0)) * 1.0001f + 1e-30f;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) rg = fmaxf(rg, __shfl_xor(rg, off, kWave));
        // the columns whose support can reach the group
        int nn = 0;
        for (int t0 = 0; t0 < ncol; t0 += kWave) {
          const int t = t0 + lane;
          bool need = false;
          if (t < ncol) {
            double xl0[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xl0[d] = cxs[d][t];
            const double reach = (crs[t] + (double)rg) * (1.0 + 1e-9);
            need = sqdist<DIM>(xl0, c0) < reach * reach;
          }
          const uint64_t msk = __ballot(need);
          if (need) nlist[w][nn + __popcll(msk & lt)] = (int16_t)t;
          nn += __popcll(msk);
        }
        wave_sync();
        // lanes per column: when few columns reach the group, P lanes share
        // one, each summing a contiguous part of the group's points; the
        // parts are added to the column's sum in order
        const int P = nn <= 16 ? 4 : (nn <= 32 ? 2 : 1);
        if (P == 1) {
          for (int k0 = 0; k0 < nn; k0 += kWave) {
            const int k = k0 + lane;
            if (k < nn) {
              const int t = nlist[w][k];
              double xt[DIM];
#pragma unroll
              for (int d = 0; d < DIM; ++d) xt[d] = cxs[d][t];
              const double r2t = cr2s[t], irt = cirs[t];
              Acc<T> a = from_pod(cacc[w][t]);
              for (int q = g0; q < g0 + n; ++q) {
                double p[DIM];
#pragma unroll
                for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
                const double s = sqdist<DIM>(p, xt);
                if (s < r2t) a.add(wphi[q] * wendland<PHI, T>(scaled_r<T>(s, irt)));
              }
              cacc[w][t] = to_pod(a);
            }
          }
        } else {
          const int k = lane / P, part = lane - k * P;
          const bool on = k < nn;
          const int t = on ? nlist[w][k] : 0;
          const int len = (n + P - 1) / P;
          const int q0 = g0 + part * len;
          const int q1 = q0 + len < g0 + n ? q0 + len : g0 + n;
          Acc<T> a;
          if (on) {
            if (part == 0) a = from_pod(cacc[w][t]);
            double xt[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xt[d] = cxs[d][t];
            const double r2t = cr2s[t], irt = cirs[t];
            for (int q = q0; q < q1; ++q) {
              double p[DIM];
#pragma unroll
              for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
              const double s = sqdist<DIM>(p, xt);
              if (s < r2t) a.add(wphi[q] * wendland<PHI, T>(scaled_r<T>(s, irt)));
            }
          }
          // the parts of lanes lane+1 .. lane+P-1, added in order by part 0
          const AccPod<T> mine = to_pod(a);
          AccPod<T> nb[3];
#pragma unroll
          for (int j = 1; j < 4; ++j) {
            const int src = lane + j < kWave ? lane + j : lane;
            nb[j - 1].s = __shfl(mine.s, src, kWave);
            nb[j - 1].c = __shfl(mine.c, src, kWave);
          }
          if (on && part == 0) {
            for (int j = 1; j < P; ++j) {
              a.add(nb[j - 1].s);
              a.add(-nb[j - 1].c);
            }
            cacc[w][t] = to_pod(a);
          }
        }
        wave_sync();
      }
      }
    });
    // add the waves' partial sums in wave order (the grouped path's sums are
    // already in LDS)
    if constexpr (!GROUPED) {
#pragma unroll
      for (int t = 0; t < kSlots; ++t) red[w][lane + kWave * t] = partial_value<T>(acc[t]);
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int t = 0; t < kSlots; ++t) {
        if (!ok[t]) continue;
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < kAsmWaves; ++u) {
          if constexpr (GROUPED)
            sum += partial_value<T>(from_pod(cacc[u][lane + kWave * t]));
          else
            sum += red[u][lane + kWave * t];
        }
        const T v = (T)sum;
        const int64_t e = e0 + cb + lane + (int64_t)kWave * t;
        const int64_t pj = sell_pos(sptr, lanes, P.amap[j], e - row_ptr[j]);
        if (RBF_CHECK(P, pj < P.nsell)) val[pj] = v;
        const int32_t l = lcol[t];
        if (l == (int32_t)j) {
          diag[j] = (double)v;
        } else {
          // mirror (l, j): j sits in the lower part of row l, columns ascending
          int64_t lo = row_ptr[l], hi = row_ptr[l] + lower_cnt[l];
          while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col[mid] < (int32_t)j) lo = mid + 1; else hi = mid;
          }
          if (RBF_CHECK(P, lo < P.nnz && col[lo] == (int32_t)j)) {
            const int64_t pl = sell_pos(sptr, lanes, P.amap[l], lo - row_ptr[l]);
            if (RBF_CHECK(P, pl < P.nsell)) val[pl] = v;
          }
        }
      }
    }
    __syncthreads();
  }
  const double gl = wave_sum(partial_value<T>(gacc));
  if (lane == 0) gred[w] = gl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double gs = 0.0;
    for (int u = 0; u < kAsmWaves; ++u) gs += gred[u];
    g[j] = gs;
  }
}

// g = A^T h alone, for new sample values with B kept (vector-valued data):
// the same support stream, chunk size, lane assignment and accumulator as the
// assembly's first column pass, so g is bit for bit what k_assemble gives.
// With kexp, also an exponent k_j with sum_k phi_kj^2 < 2^(k_j - 1) (the
// point tiles' fixed-point scale of row j).
template <int DIM, int PHI, typename T, bool GROUPED>
__global__ __launch_bounds__(kWave* kAsmWaves) void k_rhs(PlanView P,
                                                         const double* __restrict__ hs,
                                                         double* __restrict__ g,
                                                         int32_t* __restrict__ kexp) {
  constexpr int kChunk = GROUPED ? kAsmChunk / 2 : kAsmChunk;
  __shared__ double sp[kAsmWaves][DIM][kChunk];
  __shared__ int32_t sidx[kAsmWaves][kChunk];
  __shared__ double gred[kAsmWaves], dred[kAsmWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = blockIdx.x;
  if (!P.active[j]) {
    if (threadIdx.x == 0) g[j] = 0.0;
    return;
  }
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double r2j = P.rho2[j], irj = P.irho[j];
  Acc<T> gacc;
  double dsum = 0.0;
  double(*wsp)[kChunk] = sp[w];
  const int32_t* widx = sidx[w];
  stream_support_part<DIM, kChunk>(P, xj, r2j, w, kAsmWaves, wsp, sidx[w], [&](int np) {
    for (int q = lane; q < np; q += kWave) {
      double p[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
      const T phij = wendland<PHI, T>(scaled_r<T>(sqdist<DIM>(p, xj), irj));
      gacc.add(phij * (T)hs[widx[q]]);
      if (kexp) dsum += (double)phij * (double)phij;
    }
  });
  const double gl = wave_sum(partial_value<T>(gacc));
  if (lane == 0) gred[w] = gl;
  if (kexp) {
    dsum = wave_sum(dsum);
    if (lane == 0) dred[w] = dsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double gs = 0.0;
    for (int u = 0; u < kAsmWaves; ++u) gs += gred[u];
    g[j] = gs;
    if (kexp) {
      double ds = 0.0;
      for (int u = 0; u < kAsmWaves; ++u) ds += dred[u];
      // 2^(ilogb + 1) > ds; one more power of two covers the rounding of
      // this sum against the tiles' own
      kexp[j] = ds > 0.0 ? ilogb(ds) + 2 : -1000;
    }
  }
}

constexpr int kRed = 256;

// Most blocks of the ridge's first pass (its partials: kRidgeBlocks sums and
// kRidgeBlocks counts).
constexpr int kRidgeBlocks = 512;
static_assert(2 * kRidgeBlocks == kRidgePartDoubles, "ridge partials layout");

// First pass: block b sums diag and counts the active centres over its
// contiguous range of centres.
__global__ __launch_bounds__(kRed) void k_ridge_partial(const double* __restrict__ diag,
                                                        const uint8_t* __restrict__ active,
                                                        int64_t m, double* __restrict__ part) {
  __shared__ double ws[kRed / kWave];
  __shared__ double wc[kRed / kWave];
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < m ? lo + per : m;
  double s = 0.0, c = 0.0;
  for (int64_t j = lo + threadIdx.x; j < hi; j += kRed) {
    if (active[j]) {
      s += diag[j];
      c += 1.0;
    }
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    ws[threadIdx.x / kWave] = s;
    wc[threadIdx.x / kWave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ts = 0.0, tc = 0.0;
    for (int w = 0; w < kRed / kWave; ++w) {
      ts += ws[w];
      tc += wc[w];
    }
    part[blockIdx.x] = ts;
    part[kRidgeBlocks + blockIdx.x] = tc;
  }
}

// lambda = lambda_rel * mean(diag over active centres), written to lam[0],
// from the first pass's nb partials (added in block order).
__global__ __launch_bounds__(kRed) void k_ridge_value(const double* __restrict__ part, int nb,
                                                      double lambda_rel,
                                                      double* __restrict__ lam) {
  __shared__ double ws[kRed / kWave];
  __shared__ int64_t wc[kRed / kWave];
  double s = 0.0;
  int64_t c = 0;
  for (int k = threadIdx.x; k < nb; k += kRed) {
    s += part[k];
    c += (int64_t)part[kRidgeBlocks + k];
  }
  s = wave_sum(s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor((long long)c, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    ws[threadIdx.x / kWave] = s;
    wc[threadIdx.x / kWave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ts = 0.0;
    int64_t tc = 0;
    for (int w = 0; w < kRed / kWave; ++w) {
      ts += ws[w];
      tc += wc[w];
    }
    lam[0] = tc > 0 ? lambda_rel * (ts / (double)tc) : 0.0;
  }
}

// Adds lambda to the stored diagonal and forms the Jacobi inverse diagonal
// from the value actually stored.
template <typename T>
__global__ void k_add_ridge(int64_t ms, const int32_t* __restrict__ srow,
                            const int64_t* __restrict__ sptr, int lanes,
                            const int32_t* __restrict__ lower_cnt, const double* __restrict__ lam,
                            T* __restrict__ val, T* __restrict__ dinv,
                            double* __restrict__ dinv64) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ms) return;
  const int64_t e = sell_pos(sptr, lanes, k, lower_cnt[srow[k]]);
  const T v = (T)((double)val[e] + lam[0]);
  val[e] = v;
  dinv[k] = (T)1 / v;
  dinv64[k] = 1.0 / (double)v;
}

template <int DIM, typename T, bool GROUPED>
void assemble_phi(const PlanView& P, int phi, const double* hs, const int64_t* row_ptr,
                  const int32_t* lower_cnt, const int32_t* col, const int64_t* sptr, int lanes,
                  T* val, double* g, double* diag, hipStream_t s) {
  const dim3 grid((unsigned)P.m), block(kWave * kAsmWaves);
  switch (phi) {
    case 0:
      hipLaunchKernelGGL((k_assemble<DIM, 0, T, GROUPED>), grid, block, 0, s, P, hs, row_ptr,
                         lower_cnt, col, sptr, lanes, val, g, diag);
      break;
    case 1:
      hipLaunchKernelGGL((k_assemble<DIM, 1, T, GROUPED>), grid, block, 0, s, P, hs, row_ptr,
                         lower_cnt, col, sptr, lanes, val, g, diag);
      break;
    case 2:
      hipLaunchKernelGGL((k_assemble<DIM, 2, T, GROUPED>), grid, block, 0, s, P, hs, row_ptr,
                         lower_cnt, col, sptr, lanes, val, g, diag);
      break;
    default:
      hipLaunchKernelGGL((k_assemble<DIM, 3, T, GROUPED>), grid, block, 0, s, P, hs, row_ptr,
                         lower_cnt, col, sptr, lanes, val, g, diag);
      break;
  }
}

template <int DIM, typename T>
hipError_t assemble_dim(const PlanView& P, int phi, bool grouped, const double* hs,
                        const int64_t* row_ptr, const int32_t* lower_cnt, const int32_t* col,
                        const int64_t* sptr, int lanes, T* val, double* g, double* diag,
                        hipStream_t s) {
  if (grouped)
    assemble_phi<DIM, T, true>(P, phi, hs, row_ptr, lower_cnt, col, sptr, lanes, val, g, diag, s);
  else
    assemble_phi<DIM, T, false>(P, phi, hs, row_ptr, lower_cnt, col, sptr, lanes, val, g, diag, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_assemble(const PlanView& P, int phi, bool fp32, bool grouped, const double* hs,
                           const int64_t* row_ptr, const int32_t* lower_cnt, const int32_t* col,
                           const int64_t* sptr, int lanes, void* val, double* g, double* diag,
                           hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  if (P.dim == 2) {
    return fp32 ? assemble_dim<2, float>(P, phi, grouped, hs, row_ptr, lower_cnt, col, sptr,
                                         lanes, (float*)val, g, diag, s)
                : assemble_dim<2, double>(P, phi, grouped, hs, row_ptr, lower_cnt, col, sptr,
                                          lanes, (double*)val, g, diag, s);
  }
  return fp32 ? assemble_dim<3, float>(P, phi, grouped, hs, row_ptr, lower_cnt, col, sptr, lanes,
                                       (float*)val, g, diag, s)
              : assemble_dim<3, double>(P, phi, grouped, hs, row_ptr, lower_cnt, col, sptr, lanes,
                                        (double*)val, g, diag, s);
}

template <int DIM, typename T, bool GROUPED>
void rhs_phi(const PlanView& P, int phi, const double* hs, double* g, int32_t* kexp,
             hipStream_t s) {
  const dim3 grid((unsigned)P.m), block(kWave * kAsmWaves);
  switch (phi) {
    case 0:
      hipLaunchKernelGGL((k_rhs<DIM, 0, T, GROUPED>), grid, block, 0, s, P, hs, g, kexp);
      break;
    case 1:
      hipLaunchKernelGGL((k_rhs<DIM, 1, T, GROUPED>), grid, block, 0, s, P, hs, g, kexp);
      break;
    case 2:
      hipLaunchKernelGGL((k_rhs<DIM, 2, T, GROUPED>), grid, block, 0, s, P, hs, g, kexp);
      break;
    default:
      hipLaunchKernelGGL((k_rhs<DIM, 3, T, GROUPED>), grid, block, 0, s, P, hs, g, kexp);
      break;
  }
}

template <int DIM>
void rhs_dim(const PlanView& P, int phi, bool fp32, bool grouped, const double* hs, double* g,
             int32_t* kexp, hipStream_t s) {
  if (fp32) {
    if (grouped) rhs_phi<DIM, float, true>(P, phi, hs, g, kexp, s);
    else rhs_phi<DIM, float, false>(P, phi, hs, g, kexp, s);
  } else {
    if (grouped) rhs_phi<DIM, double, true>(P, phi, hs, g, kexp, s);
    else rhs_phi<DIM, double, false>(P, phi, hs, g, kexp, s);
  }
}

hipError_t launch_rhs(const PlanView& P, int phi, bool fp32, bool grouped, const double* hs,
                      double* g, hipStream_t s, int32_t* kexp) {
  if (P.m <= 0) return hipSuccess;
  if (P.dim == 2)
    rhs_dim<2>(P, phi, fp32, grouped, hs, g, kexp, s);
  else
    rhs_dim<3>(P, phi, fp32, grouped, hs, g, kexp, s);
  return hipGetLastError();
}

hipError_t launch_finalize(int64_t m, const uint8_t* active, int64_t ms, const int32_t* srow,
                           const int64_t* sptr, int lanes, const int32_t* lower_cnt,
                           const double* diag, double lambda_rel, double* lam, bool fp32,
                           void* val, void* dinv, double* dinv64, double* ridge_part,
                           hipStream_t s) {
  if (m <= 0) return hipSuccess;
  // counts are exact in float64 below 2^53 centres
  const int nb = (int)std::min<int64_t>(kRidgeBlocks, (m + 4 * kRed - 1) / (4 * kRed));
  hipLaunchKernelGGL(k_ridge_partial, dim3(nb), dim3(kRed), 0, s, diag, active, m, ridge_part);
  hipLaunchKernelGGL(k_ridge_value, dim3(1), dim3(kRed), 0, s, (const double*)ridge_part, nb,
                     lambda_rel, lam);
  if (ms <= 0) return hipGetLastError();
  const int bs = 256;
  const dim3 grid((unsigned)((ms + bs - 1) / bs));
  if (fp32)
    hipLaunchKernelGGL(k_add_ridge<float>, grid, dim3(bs), 0, s, ms, srow, sptr, lanes, lower_cnt,
                       (const double*)lam, (float*)val, (float*)dinv, dinv64);
  else
    hipLaunchKernelGGL(k_add_ridge<double>, grid, dim3(bs), 0, s, ms, srow, sptr, lanes,
                       lower_cnt, (const double*)lam, (double*)val, (double*)dinv, dinv64);
  return hipGetLastError();
}

}  // namespace rbf
