// Assembly of the normal equations from point chunks (Section 5, eq. 13-16,
// with the sum over points split instead of the columns of A):
//
//     B = sum_c A_c^T A_c,   g = sum_c A_c^T h_c,   n_j = sum_c n_j^c,
//
// where A_c holds the rows of A of the points of chunk c.  The points never
// have to be resident together: each chunk is hashed on the centres' grid,
// its terms are added to accumulators that live for the whole stream, and the
// pattern, the active set and the solver's layout are formed once the last
// chunk is in.
//
// The accumulators are indexed by the candidate list of every centre j: all
// centres l whose ball can meet j's (|xi_l - xi_j| <= (rho_j + rho_l)(1 + 1e-9)),
// in ascending order, lower part (l < j) then upper part (l >= j).  Every
// structural entry of B is a candidate, whatever the points turn out to be.
// A chunk adds, for every upper candidate (j, l), the sum of phi_pj phi_pl over
// its points p in both supports, and marks the candidate when there is one
// such point (the float64 predicate of the resident pattern, so marks are
// structural even where phi underflows).  One block owns row j: every
// accumulator has one writer, the chunks are added in stream order, and the
// result is deterministic.  Lower entries take the value and mark of their
// mirror (l, j) when the system is formed.
//
// FP64 variant: float64 phi and sums.  FP32 variant: phi in float32 and
// float32 Kahan sums within a chunk (as the resident assembly), the chunk
// partials added in float64 and rounded once when the system is formed.
#include "accum.h"
#include "plan_kernels.h"
#include "solver.h"
#include "stream.h"

namespace rbf {
namespace {

constexpr int kStrWaves = 4;
constexpr int kStrChunk = 256;
constexpr int kStrSlots = 4;
constexpr int kStrCols = kWave * kStrSlots;

// ---- candidate lists ------------------------------------------------------

// Visits the centres whose ball can meet centre j's, in centre-hash order
// (wave-uniform loop; `take(l)` is called by the lanes that hold one).
template <int DIM, typename Take>
__device__ __forceinline__ void walk_candidates(const PlanView& P, int64_t j, Take&& take) {
  const int lane = threadIdx.x & (kWave - 1);
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double rj = P.rho[j];
  int c[3];
  cell_of<DIM>(P.grid, xj, c);  // centres always lie inside the box
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
        double xl[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) xl[d] = P.ctr_s[d * P.m + i];
        const double reach = (rj + P.rho[l]) * (1.0 + 1e-9);
        ok = sqdist<DIM>(xl, xj) <= reach * reach;
      }
      take(ok, l);
    }
  }
}

constexpr int kCandWaves = 4;

// Number of candidates of every centre (one wave per centre); err[0] is set
// when one has more than kMaxCand.
template <int DIM>
__global__ __launch_bounds__(kWave* kCandWaves) void k_cand_count(PlanView P,
                                                                  int64_t* __restrict__ cnt,
                                                                  int32_t* __restrict__ err) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * kCandWaves + threadIdx.x / kWave;
  if (j >= P.m) return;
  int n = 0;
  walk_candidates<DIM>(P, j, [&](bool ok, int) { n += __popcll(__ballot(ok)); });
  if (lane == 0) {
    cnt[j] = n;
    if (n > kMaxCand) atomicOr(err, 1);
  }
}

// The candidates in ascending order (a rank sort in LDS) and the start of the
// upper part of every list.
template <int DIM>
__global__ __launch_bounds__(kWave* kCandWaves) void k_cand_fill(PlanView P,
                                                                 const int64_t* __restrict__ ptr,
                                                                 int64_t* __restrict__ up,
                                                                 int32_t* __restrict__ col) {
  __shared__ int32_t list[kCandWaves][kMaxCand];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = (int64_t)blockIdx.x * kCandWaves + w;
  if (j >= P.m) return;
  const uint64_t lt = lanemask_lt();
  const int64_t base = ptr[j];
  const int nc = (int)(ptr[j + 1] - base);
  if (nc > kMaxCand) return;  // the count pass has flagged it
  int n = 0;
  walk_candidates<DIM>(P, j, [&](bool ok, int l) {
    const uint64_t msk = __ballot(ok);
    if (ok) list[w][n + __popcll(msk & lt)] = l;
    n += __popcll(msk);
  });
  wave_sync();
  int below = 0;
  for (int t = lane; t < nc; t += kWave) {
    const int32_t v = list[w][t];
    int r = 0;
    for (int u = 0; u < nc; ++u) r += list[w][u] < v ? 1 : 0;
    col[base + r] = v;
    below += v < (int32_t)j ? 1 : 0;
  }
  below = wave_sum_int(below);
  if (lane == 0) up[j] = base + below;
}

// ---- one chunk --------------------------------------------------------------

// Non-finite coordinates or values of a chunk set bad[0].
__global__ void k_chunk_check(const double* __restrict__ x, const double* __restrict__ h,
                              int64_t n, int dim, int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool ok = __builtin_isfinite(h[i]);
  for (int d = 0; d < dim; ++d) ok = ok && __builtin_isfinite(x[d * n + i]);
  if (!ok) atomicOr(bad, 1);
}

// The chunk's terms of row j (one block of kStrWaves waves): its points in
// the support of j (the view's point hash is the chunk's) are split among the
// waves.  Ungrouped: lanes own up to kStrSlots upper candidates per pass and
// visit every staged point.  GROUPED (candidate lists longer than one wave on
// average): the staged points are taken 64 at a time (consecutive, so
// spatially close), the candidates whose ball can reach a group's bounding
// ball are listed, and each lane runs through the group's points for one
// listed candidate, adding to the wave's LDS accumulator of that candidate.
// Either way every sum has a fixed order.
template <int DIM, int PHI, typename T, bool GROUPED>
__global__ __launch_bounds__(kWave* kStrWaves) void k_stream_accum(
    PlanView P, const double* __restrict__ hs, const int64_t* __restrict__ cptr,
    const int64_t* __restrict__ cup, const int32_t* __restrict__ ccol, double* __restrict__ acc,
    uint8_t* __restrict__ mark, int64_t* __restrict__ count, double* __restrict__ g) {
  // the grouped path stages half as many points (its LDS holds the pass's
  // candidates and accumulators too)
  constexpr int kChunk = GROUPED ? kStrChunk / 2 : kStrChunk;
  __shared__ double sp[kStrWaves][DIM][kChunk];
  __shared__ int32_t sidx[kStrWaves][kChunk];
  __shared__ T sphi[kStrWaves][kChunk];
  __shared__ double red[GROUPED ? 1 : kStrWaves][GROUPED ? 1 : kStrCols];
  __shared__ uint8_t hit_s[kStrWaves][kStrCols];
  __shared__ double gred[kStrWaves];
  __shared__ int32_t nred[kStrWaves];
  __shared__ double cxs[GROUPED ? DIM : 1][GROUPED ? kStrCols : 1];
  __shared__ double crs[GROUPED ? kStrCols : 1], cr2s[GROUPED ? kStrCols : 1],
      cirs[GROUPED ? kStrCols : 1];
  __shared__ AccPod<T> cacc[GROUPED ? kStrWaves : 1][GROUPED ? kStrCols : 1];
  __shared__ int16_t nlist[GROUPED ? kStrWaves : 1][GROUPED ? kStrCols : 1];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = blockIdx.x;
  const uint64_t lt = lanemask_lt();
  double xj[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) xj[d] = P.ctr[d * P.m + j];
  const double r2j = P.rho2[j], irj = P.irho[j];
  const int64_t e0 = cup[j], e1 = cptr[j + 1];
  const int64_t R = e1 - e0;  // >= 1: j is its own candidate
  Acc<T> gacc;
  int npts = 0;
  for (int64_t cb = 0; cb < R; cb += kStrCols) {
    const bool first = cb == 0;
    const int ncol = (int)(R - cb < kStrCols ? R - cb : kStrCols);
    double xl[GROUPED ? 1 : kStrSlots][DIM];
    double r2l[GROUPED ? 1 : kStrSlots], irl[GROUPED ? 1 : kStrSlots];
    bool hit[GROUPED ? 1 : kStrSlots];
    Acc<T> a[GROUPED ? 1 : kStrSlots];
    if constexpr (!GROUPED) {
#pragma unroll
      for (int t = 0; t < kStrSlots; ++t) {
        const int c = lane + kWave * t;
        const bool ok = c < ncol;
        hit[t] = false;
        const int32_t l = ok ? ccol[e0 + cb + c] : 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) xl[t][d] = ok ? P.ctr[d * P.m + l] : 0.0;
        r2l[t] = ok ? P.rho2[l] : 0.0;  // 0: no point tests inside
        irl[t] = ok ? P.irho[l] : 0.0;
      }
    } else {
      for (int t = threadIdx.x; t < ncol; t += kWave * kStrWaves) {
        const int32_t l = ccol[e0 + cb + t];
#pragma unroll
        for (int d = 0; d < DIM; ++d) cxs[d][t] = P.ctr[d * P.m + l];
        crs[t] = P.rho[l];
        cr2s[t] = P.rho2[l];
        cirs[t] = P.irho[l];
      }
      for (int t = lane; t < ncol; t += kWave) {
        cacc[w][t] = AccPod<T>{(T)0, (T)0};
        hit_s[w][t] = 0;
      }
      __syncthreads();
    }
    T* wphi = sphi[w];
    const int32_t* widx = sidx[w];
    double(*wsp)[kChunk] = sp[w];
    stream_support_part<DIM, kChunk>(P, xj, r2j, w, kStrWaves, wsp, sidx[w], [&](int np) {
      for (int q = lane; q < np; q += kWave) {
        double p[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
        const T phij = wendland<PHI, T>(scaled_r<T>(sqdist<DIM>(p, xj), irj));
        wphi[q] = phij;
        if (first) gacc.add(phij * (T)hs[widx[q]]);
      }
      if (first) npts += np;
      wave_sync();
      if constexpr (!GROUPED) {
        for (int q = 0; q < np; ++q) {
          double p[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
          const T phij = wphi[q];
#pragma unroll
          for (int t = 0; t < kStrSlots; ++t) {
            const double s = sqdist<DIM>(p, xl[t]);
            if (s < r2l[t]) {
              a[t].add(phij * wendland<PHI, T>(scaled_r<T>(s, irl[t])));
              hit[t] = true;
            }
          }
        }
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
          // the candidates whose support can reach the group
          int nn = 0;
          for (int t0 = 0; t0 < ncol; t0 += kWave) {
            const int t = t0 + lane;
            bool need = false;
            if (t < ncol) {
              double xc[DIM];
#pragma unroll
              for (int d = 0; d < DIM; ++d) xc[d] = cxs[d][t];
              const double reach = (crs[t] + (double)rg) * (1.0 + 1e-9);
              need = sqdist<DIM>(xc, c0) < reach * reach;
            }
            const uint64_t msk = __ballot(need);
            if (need) nlist[w][nn + __popcll(msk & lt)] = (int16_t)t;
            nn += __popcll(msk);
          }
          wave_sync();
          for (int k0 = 0; k0 < nn; k0 += kWave) {
            const int k = k0 + lane;
            if (k < nn) {
              const int t = nlist[w][k];
              double xc[DIM];
#pragma unroll
              for (int d = 0; d < DIM; ++d) xc[d] = cxs[d][t];
              const double r2t = cr2s[t], irt = cirs[t];
              Acc<T> at = from_pod(cacc[w][t]);
              bool h = false;
              for (int q = g0; q < g0 + n; ++q) {
                double p[DIM];
#pragma unroll
                for (int d = 0; d < DIM; ++d) p[d] = wsp[d][q];
                const double s = sqdist<DIM>(p, xc);
                if (s < r2t) {
                  at.add(wphi[q] * wendland<PHI, T>(scaled_r<T>(s, irt)));
                  h = true;
                }
              }
              cacc[w][t] = to_pod(at);
              if (h) hit_s[w][t] = 1;
            }
          }
          wave_sync();
        }
      }
    });
    // the waves' partial sums, added in wave order
    if constexpr (!GROUPED) {
#pragma unroll
      for (int t = 0; t < kStrSlots; ++t) {
        red[w][lane + kWave * t] = partial_value<T>(a[t]);
        hit_s[w][lane + kWave * t] = hit[t] ? 1 : 0;
      }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int t = 0; t < kStrSlots; ++t) {
        const int c = lane + kWave * t;
        if (c >= ncol) continue;
        double sum = 0.0;
        int h = 0;
#pragma unroll
        for (int u = 0; u < kStrWaves; ++u) {
          if constexpr (GROUPED)
            sum += partial_value<T>(from_pod(cacc[u][c]));
          else
            sum += red[u][c];
          h |= hit_s[u][c];
        }
        if (h) {
          const int64_t e = e0 + cb + c;
          acc[e] += sum;
          mark[e] = 1;
        }
      }
    }
    __syncthreads();
  }
  const double gl = wave_sum(partial_value<T>(gacc));
  if (lane == 0) {
    gred[w] = gl;
    nred[w] = npts;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double gs = 0.0;
    int64_t ns = 0;
    for (int u = 0; u < kStrWaves; ++u) {
      gs += gred[u];
      ns += nred[u];
    }
    if (ns) {
      g[j] += gs;
      count[j] += ns;
    }
  }
}

// inbox[0] += the chunk's points inside the hash grid (cell start of the
// outside sentinel).
__global__ void k_stream_inbox(const int32_t* __restrict__ sentinel_start,
                               int64_t* __restrict__ inbox) {
  if (threadIdx.x == 0) inbox[0] += sentinel_start[0];
}

// ---- forming the system -----------------------------------------------------

__global__ void k_stream_active(const int64_t* __restrict__ count, int64_t m, int32_t min_support,
                                int32_t* __restrict__ support, uint8_t* __restrict__ active) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t c = count[j];
  support[j] = c > INT32_MAX ? INT32_MAX : (int32_t)c;
  active[j] = c >= (int64_t)min_support ? 1 : 0;
}

// Position of the upper candidate (l, j) in row l (l < j), or -1.
__device__ __forceinline__ int64_t mirror_of(const int64_t* cup, const int64_t* cptr,
                                             const int32_t* ccol, int32_t l, int32_t j) {
  int64_t lo = cup[l], hi = cptr[l + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ccol[mid] < j) lo = mid + 1; else hi = mid;
  }
  return lo < cptr[l + 1] && ccol[lo] == j ? lo : -1;
}

// Entry e of row j's candidates: kept (marked, both ends active) and the
// position of its accumulator.
__device__ __forceinline__ bool kept(const int64_t* cptr, const int64_t* cup, const int32_t* ccol,
                                     const uint8_t* mark, const uint8_t* active, int64_t j,
                                     int64_t e, int64_t* at) {
  const int32_t l = ccol[e];
  if (!active[l]) return false;
  const int64_t a = l >= (int32_t)j ? e : mirror_of(cup, cptr, ccol, l, (int32_t)j);
  *at = a;
  return a >= 0 && mark[a];
}

constexpr int kRowWaves = 4;

// Full-row and lower-part sizes of every row, and the largest |l - j|.
__global__ __launch_bounds__(kWave* kRowWaves) void k_stream_row_count(
    const int64_t* __restrict__ cptr, const int64_t* __restrict__ cup,
    const int32_t* __restrict__ ccol, const uint8_t* __restrict__ mark,
    const uint8_t* __restrict__ active, int64_t m, int64_t* __restrict__ full_cnt,
    int32_t* __restrict__ lower_cnt, int32_t* __restrict__ maxdelta) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * kRowWaves + threadIdx.x / kWave;
  if (j >= m) return;
  if (!active[j]) {
    if (lane == 0) {
      full_cnt[j] = 0;
      lower_cnt[j] = 0;
    }
    return;
  }
  int n = 0, nl = 0, dmax = 0;
  for (int64_t e = cptr[j] + lane; e < cptr[j + 1]; e += kWave) {
    int64_t at;
    if (kept(cptr, cup, ccol, mark, active, j, e, &at)) {
      const int32_t l = ccol[e];
      n += 1;
      nl += l < (int32_t)j ? 1 : 0;
      const int d = l > (int32_t)j ? l - (int32_t)j : (int32_t)j - l;
      dmax = d > dmax ? d : dmax;
    }
  }
  n = wave_sum_int(n);
  nl = wave_sum_int(nl);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(dmax, off, kWave);
    dmax = o > dmax ? o : dmax;
  }
  if (lane == 0) {
    full_cnt[j] = n;
    lower_cnt[j] = nl;
    // the running maximum is read first: one address shared by every row,
    // so an atomic per row would serialise
    if (dmax > *(volatile int32_t*)maxdelta) atomicMax(maxdelta, dmax);
  }
}

// Columns of the full CSR (ascending), and the accumulator of every entry.
__global__ __launch_bounds__(kWave* kRowWaves) void k_stream_row_fill(
    const int64_t* __restrict__ cptr, const int64_t* __restrict__ cup,
    const int32_t* __restrict__ ccol, const uint8_t* __restrict__ mark,
    const uint8_t* __restrict__ active, int64_t m, const int64_t* __restrict__ row_ptr,
    int32_t* __restrict__ col, int64_t* __restrict__ src) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * kRowWaves + threadIdx.x / kWave;
  if (j >= m || !active[j]) return;
  const uint64_t lt = lanemask_lt();
  int64_t pos = row_ptr[j];
  for (int64_t e0 = cptr[j]; e0 < cptr[j + 1]; e0 += kWave) {
    const int64_t e = e0 + lane;
    int64_t at = -1;
    const bool k = e < cptr[j + 1] && kept(cptr, cup, ccol, mark, active, j, e, &at);
    const uint64_t msk = __ballot(k);
    if (k) {
      const int64_t o = pos + __popcll(msk & lt);
      col[o] = ccol[e];
      src[o] = at;
    }
    pos += __popcll(msk);
  }
}

// Values of the full CSR into the solver's layout, diagonals and g of the
// inactive centres.
template <typename T>
__global__ void k_stream_values(const int64_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col, const int64_t* __restrict__ src,
                                const int32_t* __restrict__ amap, const uint8_t* __restrict__ active,
                                const double* __restrict__ acc, const int64_t* __restrict__ sptr,
                                int lanes, int64_t m, T* __restrict__ val,
                                double* __restrict__ diag, double* __restrict__ g) {
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= m) return;
  if (!active[j]) {
    if (lane == 0) {
      diag[j] = 0.0;
      g[j] = 0.0;
    }
    return;
  }
  const int64_t a = row_ptr[j], b = row_ptr[j + 1];
  for (int64_t e = a + lane; e < b; e += kWave) {
    const T v = (T)acc[src[e]];
    val[sell_pos(sptr, lanes, amap[j], e - a)] = v;
    if (col[e] == (int32_t)j) diag[j] = (double)v;
  }
}

template <int DIM, int PHI, typename T>
hipError_t accum_launch(bool grouped, const PlanView& P, const double* hs, const int64_t* cptr,
                        const int64_t* cup, const int32_t* ccol, double* acc, uint8_t* mark,
                        int64_t* count, double* g, hipStream_t s) {
  const dim3 grid((unsigned)P.m), block(kWave * kStrWaves);
  if (grouped)
    hipLaunchKernelGGL((k_stream_accum<DIM, PHI, T, true>), grid, block, 0, s, P, hs, cptr, cup,
                       ccol, acc, mark, count, g);
  else
    hipLaunchKernelGGL((k_stream_accum<DIM, PHI, T, false>), grid, block, 0, s, P, hs, cptr, cup,
                       ccol, acc, mark, count, g);
  return hipGetLastError();
}

template <int DIM, typename T>
hipError_t accum_phi(int phi, bool gr, const PlanView& P, const double* hs, const int64_t* cptr,
                     const int64_t* cup, const int32_t* ccol, double* acc, uint8_t* mark,
                     int64_t* count, double* g, hipStream_t s) {
  switch (phi) {
    case 0: return accum_launch<DIM, 0, T>(gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
    case 1: return accum_launch<DIM, 1, T>(gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
    case 2: return accum_launch<DIM, 2, T>(gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
    default: return accum_launch<DIM, 3, T>(gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
  }
}

}  // namespace

hipError_t launch_cand_count(const PlanView& P, int64_t* cnt, int32_t* err, hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.m + kCandWaves - 1) / kCandWaves));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_cand_count<2>, grid, dim3(kWave * kCandWaves), 0, s, P, cnt, err);
  else
    hipLaunchKernelGGL(k_cand_count<3>, grid, dim3(kWave * kCandWaves), 0, s, P, cnt, err);
  return hipGetLastError();
}

hipError_t launch_cand_fill(const PlanView& P, const int64_t* ptr, int64_t* up, int32_t* col,
                            hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.m + kCandWaves - 1) / kCandWaves));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_cand_fill<2>, grid, dim3(kWave * kCandWaves), 0, s, P, ptr, up, col);
  else
    hipLaunchKernelGGL(k_cand_fill<3>, grid, dim3(kWave * kCandWaves), 0, s, P, ptr, up, col);
  return hipGetLastError();
}

hipError_t launch_chunk_check(const double* x, const double* h, int64_t n, int dim, int32_t* bad,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_chunk_check, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, x, h, n,
                     dim, bad);
  return hipGetLastError();
}

hipError_t launch_stream_inbox(const int32_t* sentinel_start, int64_t* inbox, hipStream_t s) {
  hipLaunchKernelGGL(k_stream_inbox, dim3(1), dim3(kWave), 0, s, sentinel_start, inbox);
  return hipGetLastError();
}

hipError_t launch_stream_accum(const PlanView& P, int phi, bool fp32, bool grouped,
                               const double* hs, const int64_t* cptr, const int64_t* cup,
                               const int32_t* ccol, double* acc, uint8_t* mark, int64_t* count,
                               double* g, hipStream_t s) {
  if (P.m <= 0 || P.n <= 0) return hipSuccess;
  const bool gr = grouped;
  if (P.dim == 2)
    return fp32 ? accum_phi<2, float>(phi, gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s)
                : accum_phi<2, double>(phi, gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
  return fp32 ? accum_phi<3, float>(phi, gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s)
              : accum_phi<3, double>(phi, gr, P, hs, cptr, cup, ccol, acc, mark, count, g, s);
}

hipError_t launch_stream_active(const int64_t* count, int64_t m, int32_t min_support,
                                int32_t* support, uint8_t* active, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_stream_active, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, count,
                     m, min_support, support, active);
  return hipGetLastError();
}

hipError_t launch_stream_rows(const int64_t* cptr, const int64_t* cup, const int32_t* ccol,
                              const uint8_t* mark, const uint8_t* active, int64_t m,
                              int64_t* full_cnt, int32_t* lower_cnt, int32_t* maxdelta,
                              hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kRowWaves - 1) / kRowWaves));
  hipLaunchKernelGGL(k_stream_row_count, grid, dim3(kWave * kRowWaves), 0, s, cptr, cup, ccol,
                     mark, active, m, full_cnt, lower_cnt, maxdelta);
  return hipGetLastError();
}

hipError_t launch_stream_fill(const int64_t* cptr, const int64_t* cup, const int32_t* ccol,
                              const uint8_t* mark, const uint8_t* active, int64_t m,
                              const int64_t* row_ptr, int32_t* col, int64_t* src, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kRowWaves - 1) / kRowWaves));
  hipLaunchKernelGGL(k_stream_row_fill, grid, dim3(kWave * kRowWaves), 0, s, cptr, cup, ccol, mark,
                     active, m, row_ptr, col, src);
  return hipGetLastError();
}

hipError_t launch_stream_values(const int64_t* row_ptr, const int32_t* col, const int64_t* src,
                                const int32_t* amap, const uint8_t* active, const double* acc,
                                const int64_t* sptr, int lanes, int64_t m, bool fp32, void* val,
                                double* diag, double* g, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int wpb = 4;
  const dim3 grid((unsigned)((m + wpb - 1) / wpb)), block(kWave * wpb);
  if (fp32)
    hipLaunchKernelGGL(k_stream_values<float>, grid, block, 0, s, row_ptr, col, src, amap, active,
                       acc, sptr, lanes, m, (float*)val, diag, g);
  else
    hipLaunchKernelGGL(k_stream_values<double>, grid, block, 0, s, row_ptr, col, src, amap,
                       active, acc, sptr, lanes, m, (double*)val, diag, g);
  return hipGetLastError();
}

}  // namespace rbf
