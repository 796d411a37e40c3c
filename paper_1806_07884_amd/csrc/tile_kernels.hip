// Numeric assembly of the normal equations by point tiles (Section 5,
// eq. 11-13: B is a sum over blocks of points of the blocks' own products).
//
// A tile is a piece of one hash cell's points (at most kTilePts, consecutive
// in sorted order).  Its window is the cell's list of active centres whose
// support can reach the cell (widened by 1e-6 of a cell side against the
// rounding of the cell coordinates); every centre whose support holds one of
// the tile's points is in it.  The lists are built once per plan.  With
// Phi[k][a] = phi_a(x_k) for the tile's points k and window centres a, the
// tile's share of B is the dense product
// Phi^T Phi: one evaluation of phi per (point, window centre) pair instead of
// one per (row, point, column) triple, and the products on the matrix cores
// (v_mfma_f64_16x16x4f64, float64 operands and sums; the float32 variant
// evaluates phi in float32, whose products are exact in float64).
//
// Blocks of 16 window centres form the MFMA tiles; each wave of the block
// owns a fixed set of (block a, block b >= a) pairs and keeps their 16 x 16
// sums in registers while the tile's points pass in chunks of kKC.  A tile
// with more pairs than the waves' registers hold runs several passes over
// its points.
//
// The tiles' shares are then added into one 64-bit fixed-point integer per
// stored entry of the full pattern (integer atomics): a share of the pair
// (j, l) goes to entry (j, l) of row j, where j is the pair's first window
// centre, so an entry's value is the sum of its own and its mirror's
// accumulators.  Integer addition is associative, so the sums do not depend
// on the order in which tiles finish: the assembly is deterministic.  The
// scale is per entry: with b_jj < 2^(k_j - 1) (k_j from the right-hand side's
// pass over the same supports), Cauchy-Schwarz gives b_jl <= sqrt(b_jj b_ll)
// < 2^(k - 1) for k = ceil((k_j + k_l) / 2), so the entry in units of
// 2^(k - 63) stays below 2^62.  Every share is >= 0 (phi >= 0); each loses
// less than one unit, i.e. about 1e-19 of sqrt(b_jj b_ll), the scale the
// entry's rounding is judged against.  To place its shares a tile scans the
// stored columns of each window centre's row once (coalesced, the loads of a
// block of 16 rows issued before its shares are laid out) and finds each
// column's window position in an LDS hash of the window; the shares of one
// block of 16 rows wait in LDS meanwhile.  A last pass adds each upper entry's
// two accumulators, converts the sum to float64 once (exactly rescaled),
// rounds it to the stored type and writes it and its mirror into the solver
// layout.
#define RBF_CHECK_FILE 1  // place ids of the checked build's device checks
#include "accum.h"
#include "solver.h"
#include "tiles.h"

namespace rbf {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));


template <int DIM>
struct TileCfg;
template <>
struct TileCfg<2> {
  static constexpr int W = 8;      // waves per block
  static constexpr int MAXP = 5;   // block pairs per wave and pass
  static constexpr int EU = 4;     // waves per SIMD to fit (two blocks per CU)
};
template <>
struct TileCfg<3> {
  static constexpr int W = 8;
  static constexpr int MAXP = 12;
  static constexpr int EU = 2;
};

// Squared distance from x to the box [lo, hi] (0 inside), each operation
// rounded on its own; monotone in the box, so a box holding a point gives a
// value no larger than the point's own squared distance.
template <int DIM>
__device__ __forceinline__ double box_sqdist(const double* x, const double* lo, const double* hi) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double t = x[d] < lo[d] ? lo[d] - x[d] : (x[d] > hi[d] ? x[d] - hi[d] : 0.0);
    s = s + t * t;
  }
  return s;
}

template <int DIM>
__device__ __forceinline__ void cell_coords(const Grid& G, int cell, int* c) {
  c[0] = cell % G.g[0];
  c[1] = (cell / G.g[0]) % G.g[1];
  c[2] = DIM == 3 ? cell / (G.g[0] * G.g[1]) : 0;
}

// Visits the active centres whose ball reaches hash cell `cell` (widened by
// 1e-6 of a cell), in walk order, as f(l) with l the caller's index.
template <int DIM, typename F>
__device__ __forceinline__ void cell_window(const PlanView& P, double cs, int64_t cell, F&& f) {
  int c[3];
  cell_coords<DIM>(P.grid, (int)cell, c);
  double lo[DIM], hi[DIM];
  const double pad = 1e-6 * cs;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    lo[d] = P.grid.lo[d] + (double)c[d] * cs - pad;
    hi[d] = P.grid.lo[d] + (double)(c[d] + 1) * cs + pad;
  }
  NbrWalk<DIM> walk(P.grid, c, 1);
  for (int k = 0; k < walk.rows(); ++k) {
    int lo_id, hi_id;
    if (!walk.range(k, lo_id, hi_id)) continue;
    for (int i = P.ccs[lo_id]; i < P.ccs[hi_id + 1]; ++i) {
      const int l = P.cperm[i];
      if (!P.active[l]) continue;
      double x[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) x[d] = P.ctr_s[d * P.m + i];
      if (box_sqdist<DIM>(x, lo, hi) <= P.rho2[l] * (1.0 + 1e-9)) f(l);
    }
  }
}

template <int DIM>
__global__ void k_tile_count(PlanView P, double cs, uint32_t* __restrict__ cnt,
                             uint32_t* __restrict__ wcnt, int32_t* __restrict__ maxwin) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell > P.grid.ncell) return;
  if (cell == P.grid.ncell) {
    cnt[cell] = 0;
    wcnt[cell] = 0;
    return;
  }
  const int np = P.pcs[cell + 1] - P.pcs[cell];
  cnt[cell] = (uint32_t)((np + kTilePts - 1) / kTilePts);
  int nw = 0;
  if (np > 0) cell_window<DIM>(P, cs, cell, [&](int) { ++nw; });
  wcnt[cell] = (uint32_t)nw;
  if (nw > 0 && nw > *(volatile int32_t*)maxwin) atomicMax(maxwin, nw);
}

template <int DIM>
__global__ void k_tile_fill(PlanView P, double cs, const uint32_t* __restrict__ off,
                            const uint32_t* __restrict__ woff, int4* __restrict__ tiles,
                            int32_t* __restrict__ wids) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= P.grid.ncell) return;
  const int p0 = P.pcs[cell], p1 = P.pcs[cell + 1];
  if (p1 == p0) return;
  const uint32_t w0 = woff[cell], nw = woff[cell + 1] - w0;
  uint32_t t = off[cell];
  for (int a = p0; a < p1; a += kTilePts, ++t)
    tiles[t] = make_int4(a, a + kTilePts < p1 ? a + kTilePts : p1, (int)w0, (int)nw);
  uint32_t k = w0;
  cell_window<DIM>(P, cs, cell, [&](int l) { wids[k++] = l; });
}

// Fixed-point exponent of entry (j, l) from the rows' exponents.
__device__ __forceinline__ int pair_exp(int kj, int kl) { return (kj + kl + 1) >> 1; }

template <int DIM, int PHI, typename T>
__global__ __launch_bounds__(kWave* TileCfg<DIM>::W, TileCfg<DIM>::EU) void k_tile_assemble(
    PlanView P, const int4* __restrict__ tiles, const int32_t* __restrict__ wids,
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ kexp, unsigned long long* __restrict__ acc,
    int32_t* __restrict__ err) {
  constexpr int W = TileCfg<DIM>::W;
  constexpr int MAXP = TileCfg<DIM>::MAXP;
  constexpr int NW = tile_window_max(DIM);
  constexpr int NT = NW / 16;
  constexpr int NTHR = kWave * W;
  constexpr int STRIDE = NW + 16;  // row stride of the LDS tables below
  // points per chunk: Phi of a chunk fills the same LDS as one block row of
  // float64 sums (16 rows): 16 in float64, 32 in float32 (four or eight
  // MFMA K-steps)
  constexpr int kKC = 16 * (int)(sizeof(double) / sizeof(T));
  constexpr int HT = 1024;         // window hash slots (at most 3/8 full)
  static_assert(NW % kWave == 0, "window columns in whole waves");
  static_assert(NTHR >= NW && 2 * NW <= HT, "one evaluation column per thread; sparse hash");
  __shared__ double spt[DIM][kTilePts];
  __shared__ double wx[DIM][NW];
  __shared__ double wr2[NW], wir[NW];
  __shared__ int32_t wid[NW], wke[NW];
  // Phi of a chunk (kKC rows), later one block row of sums (16 rows, float64)
  __shared__ double buf[16 * STRIDE];
  T* phis = reinterpret_cast<T*>(buf);
  __shared__ int32_t hkey[HT];
  __shared__ int16_t hval[HT];
  __shared__ int64_t rbeg[NW];       // window rows' first stored entry
  __shared__ int32_t rlen[NW];       // and their lengths
  __shared__ int32_t rpre[NT][17];   // prefix of the lengths within each block of 16 rows
  __shared__ uint32_t nzmask[2];  // blocks of 16 window centres with a nonzero Phi, by chunk parity
  __shared__ uint16_t pairs[NT * (NT + 1) / 2];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;

  const int4 tl = tiles[blockIdx.x];
  const int p0 = tl.x, npts = tl.y - tl.x, nw = tl.w;
  if (nw > NW) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  if (nw == 0) return;
  const int nt = (nw + 15) / 16;
  const int np = nt * (nt + 1) / 2;

  // the tile's points; the window (coordinates, radii, exponents, rows)
  for (int i = threadIdx.x; i < npts; i += NTHR) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) spt[d][i] = P.ps[d * P.n + p0 + i];
  }
  for (int h = threadIdx.x; h < HT; h += NTHR) hkey[h] = -1;
  if (threadIdx.x < 2) nzmask[threadIdx.x] = 0u;
  if (threadIdx.x < nt * 16) {
    const int a = threadIdx.x;
    if (a < nw) {
      const int l0 = wids[tl.z + a];
      const int l = RBF_CHECK(P, (unsigned)l0 < (unsigned)P.m) ? l0 : 0;
      wid[a] = l;
      wke[a] = kexp[l];
#pragma unroll
      for (int d = 0; d < DIM; ++d) wx[d][a] = P.ctr[d * P.m + l];
      wr2[a] = P.rho2[l];
      wir[a] = P.irho[l];
      const int64_t e0 = row_ptr[l];
      rbeg[a] = e0;
      rlen[a] = (int32_t)(row_ptr[l + 1] - e0);
    } else {
      // the last block's padding: never in support
      wid[a] = -1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) wx[d][a] = 0.0;
      wr2[a] = -1.0;
      wir[a] = 0.0;
      rlen[a] = 0;
    }
  }
  // block pairs (a, b >= a), row by row
  if (threadIdx.x < nt) {
    const int ta = threadIdx.x;
    const int o = ta * nt - ta * (ta - 1) / 2;
    for (int tb = ta; tb < nt; ++tb) pairs[o + tb - ta] = (uint16_t)((ta << 8) | tb);
  }
  __syncthreads();
  // window hash (centre id -> window position); prefix sums of the row
  // lengths within each block of 16 rows
  if (threadIdx.x < nw) {
    const int key = wid[threadIdx.x];
    unsigned h = ((unsigned)key * 2654435761u) >> 22;
    while (atomicCAS(&hkey[h], -1, key) != -1) h = (h + 1) & (HT - 1);
    hval[h] = (int16_t)threadIdx.x;
  }
  if (threadIdx.x < nt * 16) {
    int len = rlen[threadIdx.x];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int t = __shfl_up(len, off, kWave);
      if ((lane & 15) >= off) len += t;
    }
    rpre[threadIdx.x >> 4][(threadIdx.x & 15) + 1] = len;
    if ((threadIdx.x & 15) == 0) rpre[threadIdx.x >> 4][0] = 0;
  }
  __syncthreads();

  // evaluation items (point k, window column c) of a chunk, taken in steps of
  // NTHR: this thread's first item and the step in (k, c)
  const int ncol = nt * 16;
  const int c_first = threadIdx.x % ncol, k_first = threadIdx.x / ncol;
  const int c_step = NTHR % ncol, k_step = NTHR / ncol;
  static_assert(NT <= 32, "one bit per column block");
  int chunk = 0;
  for (int base = 0; base < np; base += W * MAXP) {
    int ta[MAXP], tb[MAXP];
    dbl4 s[MAXP];
#pragma unroll
    for (int sl = 0; sl < MAXP; ++sl) {
      const int k = base + sl * W + w;
      const int pr = k < np ? pairs[k] : 0;
      ta[sl] = k < np ? (pr >> 8) : -1;
      tb[sl] = pr & 255;
      s[sl] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    for (int k0 = 0; k0 < npts; k0 += kKC, ++chunk) {
      // Phi of the chunk's points over all threads; the next chunk's mask
      // (last read before the previous barrier) is cleared meanwhile
      if (threadIdx.x == 0) nzmask[(chunk + 1) & 1] = 0u;
      uint32_t nz = 0u;
      for (int k = k_first, cc = c_first; k < kKC;) {
        T v = (T)0;
        if (k0 + k < npts) {
          double p[DIM], xc[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            p[d] = spt[d][k0 + k];
            xc[d] = wx[d][cc];
          }
          const double q = sqdist<DIM>(p, xc);
          if (q < wr2[cc]) v = wendland<PHI, T>(scaled_r<T>(q, wir[cc]));
        }
        phis[k * STRIDE + cc] = v;
        if (v != (T)0) nz |= 1u << (cc >> 4);
        cc += c_step;
        k += k_step;
        if (cc >= ncol) {
          cc -= ncol;
          ++k;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) nz |= __shfl_xor(nz, off, kWave);
      if (lane == 0 && nz) atomicOr(&nzmask[chunk & 1], nz);
      __syncthreads();
      const uint32_t nzm = nzmask[chunk & 1];
      bool on[MAXP];
#pragma unroll
      for (int sl = 0; sl < MAXP; ++sl)
        on[sl] = ta[sl] >= 0 && ((nzm >> ta[sl]) & 1u) && ((nzm >> tb[sl]) & 1u);
#pragma unroll 1
      for (int ks = 0; ks < kKC; ks += 4) {
        const int row = (ks + (lane >> 4)) * STRIDE + (lane & 15);
        // operands first (unconditional, in bounds), then the products
        double a[MAXP], b[MAXP];
#pragma unroll
        for (int sl = 0; sl < MAXP; ++sl) {
          a[sl] = (double)phis[row + (ta[sl] < 0 ? 0 : ta[sl]) * 16];
          b[sl] = (double)phis[row + tb[sl] * 16];
        }
#pragma unroll
        for (int sl = 0; sl < MAXP; ++sl)
          if (on[sl]) s[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl], b[sl], s[sl], 0, 0, 0);
      }
      __syncthreads();
    }
    // the pass's sums into the fixed-point accumulators, one block row ta of
    // 16 window centres at a time: the waves holding pairs (ta, tb) put their
    // sums into LDS (output (i, j) of a 16 x 16 block sits in lane
    // j + 16 (i % 4), item i / 4); then the stored columns of the 16 rows,
    // taken as one list over all threads, each add the share of their column
    // when this pass formed it
    for (int rt = 0; rt < nt; ++rt) {
      const int o = rt * nt - rt * (rt - 1) / 2;  // pair index of (rt, rt)
      const int* pre = rpre[rt];
      const int L = pre[16];
      constexpr int UB = 4;
      int cc[UB], ii[UB];
      int64_t ee[UB];
      // the first columns of the block's rows, loaded before the sums are laid out
      auto load = [&](int q0) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int q = q0 + u * NTHR;
          ii[u] = -1;
          if (q < L) {
            int i = 0;
#pragma unroll
            for (int step = 8; step > 0; step >>= 1)
              if (pre[i + step] <= q) i += step;
            ee[u] = rbeg[rt * 16 + i] + (q - pre[i]);
            if (RBF_CHECK(P, ee[u] >= 0 && ee[u] < P.nnz)) {
              cc[u] = col[ee[u]];
              ii[u] = i;
            }
          }
        }
      };
      auto place = [&]() {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          if (ii[u] < 0) continue;
          const int a = rt * 16 + ii[u];
          unsigned h = ((unsigned)cc[u] * 2654435761u) >> 22;
          int b = -1;
          for (;;) {
            const int key = hkey[h];
            if (key == cc[u]) {
              b = hval[h];
              break;
            }
            if (key == -1) break;
            h = (h + 1) & (HT - 1);
          }
          if (b < a) continue;  // not in the window, or the pair's share sits in row b
          const int k = o + (b >> 4) - rt;
          if (k < base || k >= base + W * MAXP) continue;  // another pass
          const double x = buf[ii[u] * STRIDE + b];
          if (x != 0.0) {
            const unsigned long long uv =
                (unsigned long long)ldexp(x, 63 - pair_exp(wke[a], wke[b]));
            if (uv) atomicAdd(acc + ee[u], uv);
          }
        }
      };
      load(threadIdx.x);
#pragma unroll
      for (int sl = 0; sl < MAXP; ++sl) {
        if (ta[sl] != rt) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          buf[(4 * v + (lane >> 4)) * STRIDE + tb[sl] * 16 + (lane & 15)] = s[sl][v];
      }
      __syncthreads();
      place();
      for (int q0 = threadIdx.x + UB * NTHR; q0 < L; q0 += UB * NTHR) {
        load(q0);
        place();
      }
      __syncthreads();
    }
  }
}

// ---- the pattern by point tiles ------------------------------------------
//
// Every centre's candidate columns are the centres of the 5^(d-1) rows of
// cells of its cell's walk at radius 2 (all of them, in walk order, sorted
// position within a row); a structural entry (j, l) is a mark bit at l's
// position in that walk of j.  The position follows from a per-cell table of
// the walk's rows (first sorted centre, offset in the walk), so a tile can
// set it with one atomic OR.  A pair (j, l) is structural when some point
// lies in both supports: the tile whose cell holds that point has j and l in
// its window and counts the pair's common points as the MFMA product of the
// 0/1 support indicators (exact small integers in float64).

template <int DIM>
__device__ __forceinline__ int walk_row(const int* cj, const int* cl) {
  return DIM == 2 ? cl[1] - cj[1] + 2 : (cl[1] - cj[1] + 2) + 5 * (cl[2] - cj[2] + 2);
}

// tab[c * (R + 1) + k] = {first sorted centre of row k of cell c's walk,
// offset of the row in the walk}, tab[c * (R + 1) + R] = {0, the walk's
// length}; the longest walk of a cell holding a centre maxed into *maxwalk.
template <int DIM>
__global__ void k_walk_tables(PlanView P, int2* __restrict__ tab, int32_t* __restrict__ maxwalk) {
  constexpr int R = DIM == 2 ? 5 : 25;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= P.grid.ncell) return;
  int c[3];
  cell_coords<DIM>(P.grid, (int)cell, c);
  NbrWalk<DIM> walk(P.grid, c, 2);
  int off = 0;
  for (int k = 0; k < R; ++k) {
    int lo_id, hi_id, a = 0, len = 0;
    if (walk.range(k, lo_id, hi_id)) {
      a = P.ccs[lo_id];
      len = P.ccs[hi_id + 1] - a;
    }
    tab[cell * (R + 1) + k] = make_int2(a, off);
    off += len;
  }
  tab[cell * (R + 1) + R] = make_int2(0, off);
  if (P.ccs[cell + 1] > P.ccs[cell] && off > *(volatile int32_t*)maxwalk) atomicMax(maxwalk, off);
}

// Per centre: its sorted position and its cell id.
template <int DIM>
__global__ void k_centre_slots(PlanView P, int32_t* __restrict__ spos, int32_t* __restrict__ ccell) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.m) return;
  double x[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) x[d] = P.ctr_s[d * P.m + i];
  int c[3];
  cell_of<DIM>(P.grid, x, c);
  const int l = P.cperm[i];
  spos[l] = (int32_t)i;
  ccell[l] = cell_id<DIM>(P.grid, c);
}

template <int DIM>
__global__ __launch_bounds__(kWave* TileCfg<DIM>::W, TileCfg<DIM>::EU) void k_tile_pattern(
    PlanView P, const int4* __restrict__ tiles, const int32_t* __restrict__ wids,
    const int2* __restrict__ tab, const int32_t* __restrict__ spos,
    const int32_t* __restrict__ ccell, int words, int max_nw, uint32_t* __restrict__ marks,
    int32_t* __restrict__ err) {
  constexpr int W = TileCfg<DIM>::W;
  constexpr int MAXP = TileCfg<DIM>::MAXP;
  constexpr int NW = tile_window_max(DIM);
  constexpr int NT = NW / 16;
  constexpr int NTHR = kWave * W;
  constexpr int STRIDE = NW + 16;
  constexpr int kKC = 16;
  constexpr int R = DIM == 2 ? 5 : 25;
  constexpr int NC = DIM == 2 ? 9 : 27;  // cells around the tile's cell
  static_assert(NTHR >= NW && NW % kWave == 0, "one column per thread");
  __shared__ double spt[DIM][kTilePts];
  __shared__ double wx[DIM][NW];
  __shared__ double wr2[NW];
  __shared__ int32_t wid[NW], wpos[NW];
  __shared__ uint8_t wslot[NW];
  __shared__ int8_t wc[NW][3];
  __shared__ double ind[kKC * STRIDE];
  __shared__ int2 ttab[NC][R];
  __shared__ uint32_t nzmask[2];
  __shared__ uint16_t pairs[NT * (NT + 1) / 2];
  // the tile's marks per window row (words per row), sized at launch for the
  // plan's widest window
  extern __shared__ uint32_t lmask[];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;

  const int4 tl = tiles[blockIdx.x];
  const int p0 = tl.x, npts = tl.y - tl.x, nw = tl.w;
  if (nw > NW || nw > max_nw) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  if (nw == 0) return;
  const int nt = (nw + 15) / 16;
  const int np = nt * (nt + 1) / 2;
  for (int t = threadIdx.x; t < nw * words; t += NTHR) lmask[t] = 0u;
  // the tile's cell, from its first point (hashed the same way)
  int tc[3] = {0, 0, 0};
  {
    double x0[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) x0[d] = P.ps[d * P.n + p0];
    cell_of<DIM>(P.grid, x0, tc);
  }
  for (int i = threadIdx.x; i < npts; i += NTHR) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) spt[d][i] = P.ps[d * P.n + p0 + i];
  }
  if (threadIdx.x < 2) nzmask[threadIdx.x] = 0u;
  // walk tables of the cells around the tile's cell (off-grid ones unused)
  for (int t = threadIdx.x; t < NC * R; t += NTHR) {
    const int sl = t / R, k = t - sl * R;
    int c[3] = {tc[0] + sl % 3 - 1, tc[1] + (sl / 3) % 3 - 1, DIM == 3 ? tc[2] + sl / 9 - 1 : 0};
    bool in = c[0] >= 0 && c[0] < P.grid.g[0] && c[1] >= 0 && c[1] < P.grid.g[1];
    if (DIM == 3) in = in && c[2] >= 0 && c[2] < P.grid.g[2];
    ttab[sl][k] = in ? tab[(int64_t)cell_id<DIM>(P.grid, c) * (R + 1) + k] : make_int2(0, 0);
  }
  if (threadIdx.x < nt * 16) {
    const int a = threadIdx.x;
    if (a < nw) {
      const int l0 = wids[tl.z + a];
      const int l = RBF_CHECK(P, (unsigned)l0 < (unsigned)P.m) ? l0 : 0;
      wid[a] = l;
#pragma unroll
      for (int d = 0; d < DIM; ++d) wx[d][a] = P.ctr[d * P.m + l];
      wr2[a] = P.rho2[l];
      wpos[a] = spos[l];
      const int cid = ccell[l];
      const int cx = cid % P.grid.g[0], cy = (cid / P.grid.g[0]) % P.grid.g[1];
      const int cz = DIM == 3 ? cid / (P.grid.g[0] * P.grid.g[1]) : 0;
      wc[a][0] = (int8_t)(cx - tc[0]);
      wc[a][1] = (int8_t)(cy - tc[1]);
      wc[a][2] = (int8_t)(cz - tc[2]);
      // slot of the centre's cell among the tile cell's neighbours (ttab's
      // order: x fastest, then y, then z)
      wslot[a] = (uint8_t)((cx - tc[0] + 1) + 3 * (cy - tc[1] + 1) +
                           (DIM == 3 ? 9 * (cz - tc[2] + 1) : 0));
    } else {
      wid[a] = -1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) wx[d][a] = 0.0;
      wr2[a] = -1.0;
    }
  }
  if (threadIdx.x < nt) {
    const int ta = threadIdx.x;
    const int o = ta * nt - ta * (ta - 1) / 2;
    for (int tb = ta; tb < nt; ++tb) pairs[o + tb - ta] = (uint16_t)((ta << 8) | tb);
  }
  __syncthreads();

  const int ncol = nt * 16;
  const int c_first = threadIdx.x % ncol, k_first = threadIdx.x / ncol;
  const int c_step = NTHR % ncol, k_step = NTHR / ncol;
  int chunk = 0;
  for (int base = 0; base < np; base += W * MAXP) {
    int ta[MAXP], tb[MAXP];
    dbl4 s[MAXP];
#pragma unroll
    for (int sl = 0; sl < MAXP; ++sl) {
      const int k = base + sl * W + w;
      const int pr = k < np ? pairs[k] : 0;
      ta[sl] = k < np ? (pr >> 8) : -1;
      tb[sl] = pr & 255;
      s[sl] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    for (int k0 = 0; k0 < npts; k0 += kKC, ++chunk) {
      if (threadIdx.x == 0) nzmask[(chunk + 1) & 1] = 0u;
      uint32_t nz = 0u;
      for (int k = k_first, cc = c_first; k < kKC;) {
        double v = 0.0;
        if (k0 + k < npts) {
          double p[DIM], xc[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            p[d] = spt[d][k0 + k];
            xc[d] = wx[d][cc];
          }
          v = sqdist<DIM>(p, xc) < wr2[cc] ? 1.0 : 0.0;
        }
        ind[k * STRIDE + cc] = v;
        if (v != 0.0) nz |= 1u << (cc >> 4);
        cc += c_step;
        k += k_step;
        if (cc >= ncol) {
          cc -= ncol;
          ++k;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) nz |= __shfl_xor(nz, off, kWave);
      if (lane == 0 && nz) atomicOr(&nzmask[chunk & 1], nz);
      __syncthreads();
      const uint32_t nzm = nzmask[chunk & 1];
      bool on[MAXP];
#pragma unroll
      for (int sl = 0; sl < MAXP; ++sl)
        on[sl] = ta[sl] >= 0 && ((nzm >> ta[sl]) & 1u) && ((nzm >> tb[sl]) & 1u);
#pragma unroll 1
      for (int ks = 0; ks < kKC; ks += 4) {
        const int row = (ks + (lane >> 4)) * STRIDE + (lane & 15);
        double a[MAXP], b[MAXP];
#pragma unroll
        for (int sl = 0; sl < MAXP; ++sl) {
          a[sl] = ind[row + (ta[sl] < 0 ? 0 : ta[sl]) * 16];
          b[sl] = ind[row + tb[sl] * 16];
        }
#pragma unroll
        for (int sl = 0; sl < MAXP; ++sl)
          if (on[sl]) s[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl], b[sl], s[sl], 0, 0, 0);
      }
      __syncthreads();
    }
    // every pair with a common point marks (j, l) and (l, j); output (i, j)
    // of a 16 x 16 block sits in lane j + 16 (i % 4), item i / 4
#pragma unroll
    for (int sl = 0; sl < MAXP; ++sl) {
      if (ta[sl] < 0) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = ta[sl] * 16 + 4 * v + (lane >> 4);
        const int b = tb[sl] * 16 + (lane & 15);
        if (a >= nw || b >= nw || (ta[sl] == tb[sl] && a > b) || s[sl][v] == 0.0) continue;
        const int ca[3] = {wc[a][0], wc[a][1], wc[a][2]};
        const int cb[3] = {wc[b][0], wc[b][1], wc[b][2]};
        const int2 ra = ttab[wslot[a]][walk_row<DIM>(ca, cb)];
        const int pab = ra.y + (wpos[b] - ra.x);
        // a position outside the row's words would be an internal error:
        // flagged, never written
        if ((unsigned)pab < (unsigned)(32 * words))
          atomicOr(&lmask[a * words + (pab >> 5)], 1u << (pab & 31));
        else
          atomicOr(err, 2);
        if (a != b) {
          const int2 rb = ttab[wslot[b]][walk_row<DIM>(cb, ca)];
          const int pba = rb.y + (wpos[a] - rb.x);
          if ((unsigned)pba < (unsigned)(32 * words))
            atomicOr(&lmask[b * words + (pba >> 5)], 1u << (pba & 31));
          else
            atomicOr(err, 2);
        }
      }
    }
  }
  // the tile's marks, gathered in LDS per window row, go out once per word
  __syncthreads();
  for (int t = threadIdx.x; t < nw * words; t += NTHR) {
    const uint32_t bits = lmask[t];
    const int a = t / words;
    if (bits) atomicOr(&marks[(int64_t)wid[a] * words + (t - a * words)], bits);
  }
}

// Per active centre j (one wave): the marked entries of its walk, i.e. its
// row of the full pattern.  Count mode writes the row's size, the size of
// its part left of the diagonal and maxes the largest |l - j| into
// *maxdelta; fill mode writes the columns in ascending order.  Sets *err
// when a row exceeds kMaxCand entries.
template <int DIM, bool FILL>
__global__ __launch_bounds__(256) void k_mark_rows(
    PlanView P, const int2* __restrict__ tab, const int32_t* __restrict__ ccell, int words,
    const uint32_t* __restrict__ marks, int64_t* __restrict__ full_cnt,
    int32_t* __restrict__ lower_cnt, const int64_t* __restrict__ row_ptr,
    int32_t* __restrict__ col, int32_t* __restrict__ err, int32_t* __restrict__ maxdelta) {
  constexpr int R = DIM == 2 ? 5 : 25;
  constexpr int WPB = 4;
  __shared__ int32_t surv[WPB][kMaxCand];
  __shared__ int2 rt[WPB][R + 1];
  static_assert(R + 1 <= kWave, "one table row per lane");
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t j = (int64_t)blockIdx.x * WPB + w;
  if (j >= P.m) return;
  if (!P.active[j]) {
    if (!FILL && lane == 0) {
      full_cnt[j] = 0;
      lower_cnt[j] = 0;
    }
    return;
  }
  const int cid = ccell[j];
  if (lane <= R) rt[w][lane] = tab[(int64_t)cid * (R + 1) + lane];
  wave_sync();
  const int L = rt[w][R].y;
  const uint64_t lt = lanemask_lt();
  int ns = 0, nlow = 0, dmax = 0;
  const uint32_t* mrow = marks + j * words;
  // positions in batches of UB * 64: the batch's mark words, then the
  // marked entries' centres, are loaded before any is used
  constexpr int UB = 4;
  for (int p0 = 0; p0 < L; p0 += UB * kWave) {
    uint32_t wd[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int p = p0 + u * kWave + lane;
      wd[u] = p < L ? mrow[p >> 5] : 0u;
    }
    int lv[UB];
    bool hv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int p = p0 + u * kWave + lane;
      hv[u] = p < L && ((wd[u] >> (p & 31)) & 1u);
      lv[u] = 0;
      if (hv[u]) {
        int k = 0;
        while (k + 1 < R && rt[w][k + 1].y <= p) ++k;
        const int i = rt[w][k].x + (p - rt[w][k].y);
        lv[u] = RBF_CHECK(P, (unsigned)i < (unsigned)P.m) ? P.cperm[i] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const bool hit = hv[u];
      const int l = lv[u];
      const uint64_t m = __ballot(hit);
      const uint64_t ml = __ballot(hit && l < (int)j);
      if (hit) {
        const int pos = ns + __popcll(m & lt);
        if (pos < kMaxCand) surv[w][pos] = l;
        const int d = l > j ? l - (int)j : (int)j - l;
        dmax = d > dmax ? d : dmax;
      }
      ns += __popcll(m);
      nlow += __popcll(ml);
    }
  }
  if (ns > kMaxCand) {
    if (lane == 0) {
      atomicExch(err, 1);
      if (!FILL) {
        full_cnt[j] = 0;
        lower_cnt[j] = 0;
      }
    }
    return;
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
  const int64_t base = row_ptr[j];
  for (int t = lane; t < ns; t += kWave) {
    const int l = surv[w][t];
    int rank = 0;
    for (int u = 0; u < ns; ++u) rank += surv[w][u] < l ? 1 : 0;
    if (RBF_CHECK(P, base + rank < P.nnz)) col[base + rank] = l;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tile_finish(
    PlanView P, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ lower_cnt,
    const int32_t* __restrict__ col, const int32_t* __restrict__ kexp,
    const unsigned long long* __restrict__ acc, const int64_t* __restrict__ sptr, int lanes,
    T* __restrict__ val, double* __restrict__ diag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (j >= P.m) return;
  if (!P.active[j]) {
    if (lane == 0) diag[j] = 0.0;
    return;
  }
  const int64_t e0 = row_ptr[j] + lower_cnt[j], e1 = row_ptr[j + 1];
  const int kj = kexp[j];
  for (int64_t e = e0 + lane; e < e1; e += kWave) {
    const int32_t l = col[e];
    if (!RBF_CHECK(P, (unsigned)l < (unsigned)P.m)) continue;
    unsigned long long t = acc[e];
    int64_t mirror = -1;
    if (l != (int32_t)j) {
      // mirror (l, j): j sits in the lower part of row l, columns ascending
      int64_t lo = row_ptr[l], hi = row_ptr[l] + lower_cnt[l];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < (int32_t)j) lo = mid + 1; else hi = mid;
      }
      mirror = lo;
      if (!RBF_CHECK(P, mirror < P.nnz && col[mirror] == (int32_t)j)) continue;
      t += acc[mirror];
    }
    const T v = (T)ldexp((double)t, pair_exp(kj, kexp[l]) - 63);
    const int64_t pj = sell_pos(sptr, lanes, P.amap[j], e - row_ptr[j]);
    if (RBF_CHECK(P, pj < P.nsell)) val[pj] = v;
    if (mirror < 0) {
      diag[j] = (double)v;
    } else {
      const int64_t pl = sell_pos(sptr, lanes, P.amap[l], mirror - row_ptr[l]);
      if (RBF_CHECK(P, pl < P.nsell)) val[pl] = v;
    }
  }
}

template <int DIM, typename T>
void tile_phi(const PlanView& P, int phi, const int4* tiles, int64_t ntiles, const int32_t* wids,
              const int64_t* row_ptr, const int32_t* col, const int32_t* kexp,
              unsigned long long* acc, int32_t* err, hipStream_t s) {
  const dim3 grid((unsigned)ntiles), block(kWave * TileCfg<DIM>::W);
  switch (phi) {
    case 0:
      hipLaunchKernelGGL((k_tile_assemble<DIM, 0, T>), grid, block, 0, s, P, tiles, wids,
                         row_ptr, col, kexp, acc, err);
      break;
    case 1:
      hipLaunchKernelGGL((k_tile_assemble<DIM, 1, T>), grid, block, 0, s, P, tiles, wids,
                         row_ptr, col, kexp, acc, err);
      break;
    case 2:
      hipLaunchKernelGGL((k_tile_assemble<DIM, 2, T>), grid, block, 0, s, P, tiles, wids,
                         row_ptr, col, kexp, acc, err);
      break;
    default:
      hipLaunchKernelGGL((k_tile_assemble<DIM, 3, T>), grid, block, 0, s, P, tiles, wids,
                         row_ptr, col, kexp, acc, err);
      break;
  }
}

}  // namespace

hipError_t launch_tile_count(const PlanView& P, double cell_size, uint32_t* cnt, uint32_t* wcnt,
                             int32_t* maxwin, hipStream_t s) {
  const int bs = 256;
  const dim3 grid((unsigned)((P.grid.ncell + 1 + bs - 1) / bs));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_tile_count<2>, grid, dim3(bs), 0, s, P, cell_size, cnt, wcnt, maxwin);
  else
    hipLaunchKernelGGL(k_tile_count<3>, grid, dim3(bs), 0, s, P, cell_size, cnt, wcnt, maxwin);
  return hipGetLastError();
}

hipError_t launch_tile_fill(const PlanView& P, double cell_size, const uint32_t* off,
                            const uint32_t* woff, int4* tiles, int32_t* wids, hipStream_t s) {
  const int bs = 256;
  if (P.grid.ncell <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.grid.ncell + bs - 1) / bs));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_tile_fill<2>, grid, dim3(bs), 0, s, P, cell_size, off, woff, tiles, wids);
  else
    hipLaunchKernelGGL(k_tile_fill<3>, grid, dim3(bs), 0, s, P, cell_size, off, woff, tiles, wids);
  return hipGetLastError();
}

hipError_t launch_tile_assemble(const PlanView& P, int phi, bool fp32, const int4* tiles,
                                int64_t ntiles, const int32_t* wids, const int64_t* row_ptr,
                                const int32_t* col, const int32_t* kexp,
                                unsigned long long* acc, int32_t* err, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (P.dim == 2) {
    if (fp32)
      tile_phi<2, float>(P, phi, tiles, ntiles, wids, row_ptr, col, kexp, acc, err, s);
    else
      tile_phi<2, double>(P, phi, tiles, ntiles, wids, row_ptr, col, kexp, acc, err, s);
  } else {
    if (fp32)
      tile_phi<3, float>(P, phi, tiles, ntiles, wids, row_ptr, col, kexp, acc, err, s);
    else
      tile_phi<3, double>(P, phi, tiles, ntiles, wids, row_ptr, col, kexp, acc, err, s);
  }
  return hipGetLastError();
}

hipError_t launch_tile_finish(const PlanView& P, bool fp32, const int64_t* row_ptr,
                              const int32_t* lower_cnt, const int32_t* col,
                              const int32_t* kexp, const unsigned long long* acc,
                              const int64_t* sptr, int lanes, void* val, double* diag,
                              hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  const int bs = 256;
  const dim3 grid((unsigned)((P.m + bs / kWave - 1) / (bs / kWave)));
  if (fp32)
    hipLaunchKernelGGL(k_tile_finish<float>, grid, dim3(bs), 0, s, P, row_ptr, lower_cnt, col,
                       kexp, acc, sptr, lanes, (float*)val, diag);
  else
    hipLaunchKernelGGL(k_tile_finish<double>, grid, dim3(bs), 0, s, P, row_ptr, lower_cnt, col,
                       kexp, acc, sptr, lanes, (double*)val, diag);
  return hipGetLastError();
}

int walk_rows(int dim) { return dim == 2 ? 5 : 25; }

hipError_t launch_walk_tables(const PlanView& P, int2* tab, int32_t* maxwalk, hipStream_t s) {
  const int bs = 256;
  if (P.grid.ncell <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.grid.ncell + bs - 1) / bs));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_walk_tables<2>, grid, dim3(bs), 0, s, P, tab, maxwalk);
  else
    hipLaunchKernelGGL(k_walk_tables<3>, grid, dim3(bs), 0, s, P, tab, maxwalk);
  return hipGetLastError();
}

hipError_t launch_centre_slots(const PlanView& P, int32_t* spos, int32_t* ccell, hipStream_t s) {
  const int bs = 256;
  if (P.m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.m + bs - 1) / bs));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_centre_slots<2>, grid, dim3(bs), 0, s, P, spos, ccell);
  else
    hipLaunchKernelGGL(k_centre_slots<3>, grid, dim3(bs), 0, s, P, spos, ccell);
  return hipGetLastError();
}

hipError_t launch_tile_pattern(const PlanView& P, const int4* tiles, int64_t ntiles,
                               const int32_t* wids, const int2* tab, const int32_t* spos,
                               const int32_t* ccell, int words, int max_nw, uint32_t* marks,
                               int32_t* err, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = sizeof(uint32_t) * (size_t)max_nw * (size_t)words;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_tile_pattern<2>, dim3((unsigned)ntiles), dim3(kWave * TileCfg<2>::W), lds,
                       s, P, tiles, wids, tab, spos, ccell, words, max_nw, marks, err);
  else
    hipLaunchKernelGGL(k_tile_pattern<3>, dim3((unsigned)ntiles), dim3(kWave * TileCfg<3>::W), lds,
                       s, P, tiles, wids, tab, spos, ccell, words, max_nw, marks, err);
  return hipGetLastError();
}

hipError_t launch_mark_rows(const PlanView& P, bool fill, const int2* tab, const int32_t* ccell,
                            int words, const uint32_t* marks, int64_t* full_cnt,
                            int32_t* lower_cnt, const int64_t* row_ptr, int32_t* col,
                            int32_t* err, int32_t* maxdelta, hipStream_t s) {
  if (P.m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P.m + 3) / 4)), block(256);
  if (P.dim == 2) {
    if (fill)
      hipLaunchKernelGGL((k_mark_rows<2, true>), grid, block, 0, s, P, tab, ccell, words, marks,
                         full_cnt, lower_cnt, row_ptr, col, err, maxdelta);
    else
      hipLaunchKernelGGL((k_mark_rows<2, false>), grid, block, 0, s, P, tab, ccell, words, marks,
                         full_cnt, lower_cnt, row_ptr, col, err, maxdelta);
  } else {
    if (fill)
      hipLaunchKernelGGL((k_mark_rows<3, true>), grid, block, 0, s, P, tab, ccell, words, marks,
                         full_cnt, lower_cnt, row_ptr, col, err, maxdelta);
    else
      hipLaunchKernelGGL((k_mark_rows<3, false>), grid, block, 0, s, P, tab, ccell, words, marks,
                         full_cnt, lower_cnt, row_ptr, col, err, maxdelta);
  }
  return hipGetLastError();
}

}  // namespace rbf
