// Plan kernels: grid hash of points and centres, support counts and the
// structural sparsity pattern of B = A^T A (Section 5, eq. 11-13).
//
// Support of centre j (Algorithm 1, strict range query; eq. 18):
//     supp(j) = { points x : s(x, xi_j) < rho_j^2 }.
// Pattern of row j of B (both triangles are produced; the stored upper CSR is
// the suffix l >= j of each sorted row):
//     { l active : supp(j) and supp(l) share a point }.
#define RBF_CHECK_FILE 3  // place ids of the checked build's device checks
#include "plan_kernels.h"
#include "solver.h"

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

// Sort key of a point: its cell id, and with sub = 2 DIM, below it the
// Morton code of its sub-cell on a 4^DIM subdivision of the cell, so that
// points of a cell come in a spatially coherent order.  Points outside the box
// get ncell << sub.
template <int DIM>
__global__ void k_cell_keys(Grid G, const double* __restrict__ x, int64_t n, int sub,
                            uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) p[d] = x[d * n + i];
  int c[3];
  const bool in = cell_of<DIM>(G, p, c);
  uint32_t key = in ? (uint32_t)cell_id<DIM>(G, c) : (uint32_t)G.ncell;
  if (sub) {
    uint32_t code = 0;
    if (in) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double f = (p[d] - G.lo[d]) * G.inv_cs - (double)c[d];
        int q = (int)(f * 4.0);
        q = q < 0 ? 0 : (q > 3 ? 3 : q);
        code |= (uint32_t)(q & 1) << d;
        code |= (uint32_t)(q >> 1) << (DIM + d);
      }
    }
    key = (key << sub) | code;
  }
  keys[i] = key;
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

constexpr int kSymWaves = 4;
constexpr int kSymChunk = 128;
constexpr int kCandWords = kMaxCand / 32;
// Candidates whose coordinates and radii the count pass stages in LDS (rows
// with more read them from global memory).
constexpr int kSymStage = 448;

// Pattern of row j (one block of kSymWaves waves per row).
//
// Candidates: active centres whose ball can meet centre j's ball, gathered
// from the centre hash in a fixed order.  Count mode: the row's candidate
// points are split among the waves (as in the assembly); each wave streams
// the supported points of its piece and marks every candidate with one of
// them in its support (LDS bit set, order-independent).  The points are
// taken 64 at a time; a group is scanned only for the unmarked candidates
// whose ball can reach the group's bounding ball, one candidate per lane,
// each stopping at its first hit.  A wave stops once every candidate is
// marked.  The marks are saved as a bitmask per row, and
// the full-row and lower-part sizes and the largest |l - j| are written.
// Fill mode rebuilds the same candidate list, reads the saved marks and
// writes the marked columns in ascending order.
template <int DIM, bool FILL>
__global__ __launch_bounds__(kWave* kSymWaves) void k_symbolic(
    PlanView P, int64_t* __restrict__ full_cnt, int32_t* __restrict__ lower_cnt,
    const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col, int32_t* __restrict__ err,
    int32_t* __restrict__ maxdelta, uint32_t* __restrict__ marks) {
  __shared__ int32_t cand[kMaxCand];
  __shared__ int32_t surv[kMaxCand];
  __shared__ uint32_t word[kCandWords];
  __shared__ double sp[kSymWaves][DIM][kSymChunk];
  __shared__ int16_t glist[kSymWaves][kMaxCand];
  __shared__ double scx[FILL ? 1 : DIM][FILL ? 1 : kSymStage];
  __shared__ double srho[FILL ? 1 : kSymStage];
  __shared__ int nc_s;
  __shared__ int rlo[25], rcnt[25], rpre[26], wcnt[kSymWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = blockIdx.x;
  const uint64_t lt = lanemask_lt();
  if (!P.active[j]) {
    if (!FILL && threadIdx.x == 0) {
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

  {
    // the walk's rows of cells (5 in 2D, 25 in 3D) as ranges of sorted
    // centres, taken as one list over all threads; the candidates keep the
    // walk order (ordered compaction over the block)
    NbrWalk<DIM> walk(P.grid, c, 2);
    const int R = walk.rows();
    if (threadIdx.x < R) {
      int lo_id, hi_id, a = 0, b = 0;
      if (walk.range(threadIdx.x, lo_id, hi_id)) {
        a = P.ccs[lo_id];
        b = P.ccs[hi_id + 1];
      }
      rlo[threadIdx.x] = a;
      rcnt[threadIdx.x] = b - a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < R; ++k) {
        rpre[k] = t;
        t += rcnt[k];
      }
      rpre[R] = t;
    }
    __syncthreads();
    const int T = rpre[R];
    int nc = 0;
    for (int q0 = 0; q0 < T; q0 += kWave * kSymWaves) {
      const int q = q0 + (int)threadIdx.x;
      bool ok = false;
      int l = 0;
      if (q < T) {
        int k = 0;
        while (rpre[k + 1] <= q) ++k;
        const int i = rlo[k] + (q - rpre[k]);
        l = RBF_CHECK(P, (unsigned)i < (unsigned)P.m) ? P.cperm[i] : 0;
        if (RBF_CHECK(P, (unsigned)l < (unsigned)P.m) && P.active[l]) {
          double xl[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) xl[d] = P.ctr_s[d * P.m + i];
          const double reach = (rj + P.rho[l]) * (1.0 + 1e-9);
          ok = sqdist<DIM>(xl, xj) <= reach * reach;
        }
      }
      const uint64_t m = __ballot(ok);
      if (lane == 0) wcnt[w] = __popcll(m);
      __syncthreads();
      int before = 0, all = 0;
#pragma unroll
      for (int u = 0; u < kSymWaves; ++u) {
        before += u < w ? wcnt[u] : 0;
        all += wcnt[u];
      }
      const int pos = nc + before + __popcll(m & lt);
      if (ok && pos < kMaxCand) cand[pos] = l;
      nc += all;
      __syncthreads();
    }
    if (threadIdx.x == 0) nc_s = nc;
  }
  if (threadIdx.x < kCandWords) word[threadIdx.x] = FILL ? marks[j * kCandWords + threadIdx.x] : 0u;
  __syncthreads();
  const int nc = nc_s;
  if (nc > kMaxCand) {
    if (threadIdx.x == 0) {
      atomicExch(err, 1);
      if (!FILL) {
        full_cnt[j] = 0;
        lower_cnt[j] = 0;
      }
    }
    return;
  }

  if (!FILL) {
    // the candidates' coordinates and radii, read for every group below
    const bool staged = nc <= kSymStage;
    if (staged) {
      for (int t = threadIdx.x; t < nc; t += kWave * kSymWaves) {
        const int l = cand[t];
#pragma unroll
        for (int d = 0; d < DIM; ++d) scx[d][t] = P.ctr[d * P.m + l];
        srho[t] = P.rho[l];
      }
      __syncthreads();
    }
    auto cx = [&](int t, int l, int d) -> double {
      return staged ? scx[d][t] : P.ctr[d * P.m + l];
    };
    auto crho = [&](int t, int l) -> double { return staged ? srho[t] : P.rho[l]; };
    // rho^2 as the radius tables form it (one rounded product)
    auto crho2 = [&](int t, int l) -> double {
      if (!staged) return P.rho2[l];
      const double r = srho[t];
      return r * r;
    };
    stream_support_part<DIM, kSymChunk>(P, xj, P.rho2[j], w, kSymWaves, sp[w], nullptr,
                                        [&](int np) {
      // groups of 64 consecutive staged points (spatially close: points are
      // sorted by sub-cell within a hash cell); only the unmarked candidates
      // whose ball can reach a group's bounding ball scan that group
      for (int g0 = 0; g0 < np; g0 += kWave) {
        const int n = np - g0 < kWave ? np - g0 : kWave;
        double c0[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) c0[d] = sp[w][d][g0];
        float rg = 0.f;
        if (lane < n) {
          double p[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) p[d] = sp[w][d][g0 + lane];
          rg = (float)__builtin_sqrt(sqdist<DIM>(p, c0)) * 1.0001f + 1e-30f;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) rg = fmaxf(rg, __shfl_xor(rg, off, kWave));
        int nn = 0;
        for (int t0 = 0; t0 < nc; t0 += kWave) {
          const int t = t0 + lane;
          bool need = false;
          if (t < nc && !((word[t >> 5] >> (t & 31)) & 1u)) {
            const int l = cand[t];
            double xl[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xl[d] = cx(t, l, d);
            const double reach = (crho(t, l) + (double)rg) * (1.0 + 1e-9);
            need = sqdist<DIM>(xl, c0) < reach * reach;
          }
          const uint64_t msk = __ballot(need);
          if (need) glist[w][nn + __popcll(msk & lt)] = (int16_t)t;
          nn += __popcll(msk);
        }
        wave_sync();
        for (int k0 = 0; k0 < nn; k0 += kWave) {
          const int k = k0 + lane;
          if (k < nn) {
            const int t = glist[w][k];
            const int l = cand[t];
            double xl[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xl[d] = cx(t, l, d);
            const double r2l = crho2(t, l);
            // four points per step, stopping after the step with a hit
            const int q1 = g0 + n;
            for (int q = g0; q < q1; q += 4) {
              bool hit = false;
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                if (q + u < q1) {
                  double p[DIM];
#pragma unroll
                  for (int d = 0; d < DIM; ++d) p[d] = sp[w][d][q + u];
                  hit |= sqdist<DIM>(p, xl) < r2l;
                }
              }
              if (hit) {
                atomicOr(&word[t >> 5], 1u << (t & 31));
                break;
              }
            }
          }
        }
        wave_sync();
      }
      int open = 0;
      for (int t = lane; t < nc; t += kWave) open += ((word[t >> 5] >> (t & 31)) & 1u) ? 0 : 1;
      return wave_sum_int(open) == 0;
    });
    __syncthreads();
    if (threadIdx.x < kCandWords) marks[j * kCandWords + threadIdx.x] = word[threadIdx.x];
  }
  if (w != 0) return;

  // compact the marked candidates, keeping candidate order
  int ns = 0, nlow = 0, dmax = 0;
  for (int t0 = 0; t0 < nc; t0 += kWave) {
    const int t = t0 + lane;
    const bool hit = t < nc && ((word[t >> 5] >> (t & 31)) & 1u);
    const int l = hit ? cand[t] : 0;
    const uint64_t m = __ballot(hit);
    const uint64_t ml = __ballot(hit && l < j);
    if (hit) {
      surv[ns + __popcll(m & lt)] = l;
      const int d = l > j ? l - (int)j : (int)j - l;
      dmax = d > dmax ? d : dmax;
    }
    ns += __popcll(m);
    nlow += __popcll(ml);
  }
  wave_sync();
  if (!FILL) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int o = __shfl_xor(dmax, off, kWave);
      dmax = o > dmax ? o : dmax;
    }
    if (lane == 0) {
      full_cnt[j] = ns;
      lower_cnt[j] = nlow;
      // the running maximum is read first: one address shared by every row,
      // so an atomic per row would serialise
      if (dmax > 0 && dmax > *(volatile int32_t*)maxdelta) atomicMax(maxdelta, dmax);
    }
    return;
  }
  // ascending columns: rank of each survivor among the survivors
  const int64_t base = row_ptr[j];
  for (int t = lane; t < ns; t += kWave) {
    const int l = surv[t];
    int rank = 0;
    for (int u = 0; u < ns; ++u) rank += surv[u] < l ? 1 : 0;
    if (RBF_CHECK(P, base + rank < P.nnz)) col[base + rank] = l;
  }
}

// pos[j] = 1 for an active centre, 0 otherwise (pos[m] = 0), scanned next.
__global__ void k_active_flags(const uint8_t* __restrict__ active, int64_t m,
                               int64_t* __restrict__ pos) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  pos[j] = (j < m && active[j]) ? 1 : 0;
}

__global__ void k_solver_rows(const uint8_t* __restrict__ active, const int64_t* __restrict__ pos,
                              int64_t m, int32_t* __restrict__ amap, int32_t* __restrict__ srow) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  if (active[j]) {
    amap[j] = (int32_t)pos[j];
    srow[pos[j]] = (int32_t)j;
  } else {
    amap[j] = -1;
  }
}

// Sliced-ELL geometry over the solver rows: entries per row of every slice
// (longest row of the slice rounded up to a multiple of L) and the slice's
// size S * slen.
__global__ void k_slice_lengths(const int64_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ srow, int64_t ms, int lanes,
                                int64_t nslices, int32_t* __restrict__ slen,
                                int64_t* __restrict__ ssize) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nslices) return;
  if (s == nslices) {
    ssize[s] = 0;
    return;
  }
  const int64_t rows = kWave / lanes;
  int64_t mx = 0;
  for (int64_t i = 0; i < rows; ++i) {
    const int64_t k = s * rows + i;
    if (k < ms) {
      const int64_t j = srow[k];
      const int64_t len = row_ptr[j + 1] - row_ptr[j];
      mx = len > mx ? len : mx;
    }
  }
  mx = (mx + lanes - 1) / lanes * lanes;
  slen[s] = (int32_t)mx;
  ssize[s] = mx * rows;
}

// One block per window of kSortRows solver rows: each row's rank among the
// window's rows by descending length (ties by position) is its new place.
__global__ __launch_bounds__(kSortRows) void k_sort_rows(const int64_t* __restrict__ row_ptr,
                                                         int64_t ms, int32_t* __restrict__ srow,
                                                         int32_t* __restrict__ amap) {
  __shared__ int32_t sj[kSortRows];
  __shared__ int64_t sl[kSortRows];
  const int t = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kSortRows;
  const int n = ms - k0 < kSortRows ? (int)(ms - k0) : kSortRows;
  if (t < n) {
    const int32_t j = srow[k0 + t];
    sj[t] = j;
    sl[t] = row_ptr[j + 1] - row_ptr[j];
  }
  __syncthreads();
  if (t < n) {
    const int64_t lt = sl[t];
    int r = 0;
    for (int u = 0; u < n; ++u) r += (sl[u] > lt || (sl[u] == lt && u < t)) ? 1 : 0;
    srow[k0 + r] = sj[t];
    amap[sj[t]] = (int32_t)(k0 + r);
  }
}

// Column deltas amap[l] - k of every stored entry of solver row k at its
// sliced-ELL position, one wave per row (padding stays 0 from the
// allocation).  Every column of the pattern is an active centre.
template <typename CT>
__global__ __launch_bounds__(256) void k_sell_cols(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ srow,
                                                   const int32_t* __restrict__ amap, int64_t ms,
                                                   const int64_t* __restrict__ sptr, int lanes,
                                                   CT* __restrict__ cols, CheckWord C) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (k >= ms) return;
  const int64_t j = srow[k];
  const int64_t a = row_ptr[j], n = row_ptr[j + 1] - a;
  for (int64_t e = lane; e < n; e += kWave) {
    const int32_t r = amap[col[a + e]];
    // every column is an active centre: a solver row, and the iteration's
    // reads of x at k + delta stay in [0, ms)
    if (RBF_CHECK(C, r >= 0 && (int64_t)r < ms)) cols[sell_pos(sptr, lanes, k, e)] = (CT)(r - (int32_t)k);
  }
}

}  // namespace

hipError_t launch_sort_rows(const int64_t* row_ptr, int64_t ms, int32_t* srow, int32_t* amap,
                            hipStream_t s) {
  if (ms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_rows, dim3((unsigned)((ms + kSortRows - 1) / kSortRows)),
                     dim3(kSortRows), 0, s, row_ptr, ms, srow, amap);
  return hipGetLastError();
}

hipError_t launch_solver_rows(const uint8_t* active, int64_t m, int64_t* pos, void* temp,
                              int32_t* amap, int32_t* srow, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(k_active_flags, dim3((unsigned)((m + 1 + bs - 1) / bs)), dim3(bs), 0, s,
                     active, m, pos);
  hipError_t e = exclusive_scan(pos, pos, m + 1, temp, s);
  if (e != hipSuccess) return e;
  if (m > 0)
    hipLaunchKernelGGL(k_solver_rows, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, active,
                       (const int64_t*)pos, m, amap, srow);
  return hipGetLastError();
}

hipError_t launch_slice_lengths(const int64_t* row_ptr, const int32_t* srow, int64_t ms, int lanes,
                                int64_t nslices, int32_t* slen, int64_t* ssize, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(k_slice_lengths, dim3((unsigned)((nslices + 1 + bs - 1) / bs)), dim3(bs), 0,
                     s, row_ptr, srow, ms, lanes, nslices, slen, ssize);
  return hipGetLastError();
}

hipError_t launch_sell_cols(const int64_t* row_ptr, const int32_t* col, const int32_t* srow,
                            const int32_t* amap, int64_t ms, const int64_t* sptr, int lanes,
                            bool col16, void* cols, int32_t* check, hipStream_t s) {
  if (ms <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ms + 3) / 4));
  if (col16)
    hipLaunchKernelGGL(k_sell_cols<int16_t>, grid, dim3(256), 0, s, row_ptr, col, srow, amap, ms,
                       sptr, lanes, (int16_t*)cols, CheckWord{check});
  else
    hipLaunchKernelGGL(k_sell_cols<int32_t>, grid, dim3(256), 0, s, row_ptr, col, srow, amap, ms,
                       sptr, lanes, (int32_t*)cols, CheckWord{check});
  return hipGetLastError();
}

hipError_t launch_minmax(const double* a, int64_t n, double* partial_min, double* partial_max,
                         int* partial_bad, int nblocks, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_partial, dim3(nblocks), dim3(kRedThreads), 0, s, a, n, partial_min,
                     partial_max, partial_bad);
  hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, s, (const double*)partial_min,
                     (const double*)partial_max, (const int*)partial_bad, nblocks, out3);
  return hipGetLastError();
}

hipError_t launch_cell_keys(int dim, const Grid& G, const double* x, int64_t n, int sub,
                            uint32_t* keys, int32_t* idx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  const dim3 grid((unsigned)((n + bs - 1) / bs));
  if (dim == 2)
    hipLaunchKernelGGL(k_cell_keys<2>, grid, dim3(bs), 0, s, G, x, n, sub, keys, idx);
  else
    hipLaunchKernelGGL(k_cell_keys<3>, grid, dim3(bs), 0, s, G, x, n, sub, keys, idx);
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

// Identical columns of A: an active centre with the same coordinates and radius
// as a centre of lower index (the two share a hash cell).  Every thread that
// finds one stores 1 into *dup.
template <int DIM>
__global__ __launch_bounds__(256) void k_duplicate_centres(PlanView P, int32_t* __restrict__ dup) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P.m || !P.active[j]) return;
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  int c[3];
  if (!cell_of<DIM>(P.grid, xj, c)) return;
  const int id = cell_id<DIM>(P.grid, c);
  const double rj = P.rho[j];
  for (int k = P.ccs[id]; k < P.ccs[id + 1]; ++k) {
    const int32_t o = P.cperm[k];
    if (o >= j) continue;
    bool same = P.rho[o] == rj;
#pragma unroll
    for (int d = 0; d < DIM; ++d) same = same && P.ctr_s[d * P.m + k] == xj[d];
    if (same) {
      *dup = 1;
      return;
    }
  }
}

hipError_t launch_duplicate_centres(const PlanView& P, int32_t* dup, hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.m + 255) / 256)), block(256);
  if (P.dim == 2)
    hipLaunchKernelGGL(k_duplicate_centres<2>, grid, block, 0, s, P, dup);
  else
    hipLaunchKernelGGL(k_duplicate_centres<3>, grid, block, 0, s, P, dup);
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

size_t symbolic_marks_words(int64_t m) { return (size_t)m * kCandWords; }

hipError_t launch_symbolic(const PlanView& P, bool fill, int64_t* full_cnt, int32_t* lower_cnt,
                           const int64_t* row_ptr, int32_t* col, int32_t* err, int32_t* maxdelta,
                           uint32_t* marks, hipStream_t s) {
  const dim3 grid((unsigned)P.m);
  const dim3 block(kWave * kSymWaves);
  if (P.dim == 2) {
    if (fill)
      hipLaunchKernelGGL((k_symbolic<2, true>), grid, block, 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err, maxdelta, marks);
    else
      hipLaunchKernelGGL((k_symbolic<2, false>), grid, block, 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err, maxdelta, marks);
  } else {
    if (fill)
      hipLaunchKernelGGL((k_symbolic<3, true>), grid, block, 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err, maxdelta, marks);
    else
      hipLaunchKernelGGL((k_symbolic<3, false>), grid, block, 0, s, P, full_cnt, lower_cnt,
                         row_ptr, col, err, maxdelta, marks);
  }
  return hipGetLastError();
}

}  // namespace rbf
