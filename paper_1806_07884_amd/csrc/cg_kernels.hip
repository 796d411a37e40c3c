// Jacobi-preconditioned conjugate gradients on the assembled normal equations,
// in the single-reduction form of Chronopoulos and Gear (1989), one kernel per
// iteration.
//
// With u = D^-1 r, w = B u, s = B p and gamma = r . u, delta = w . u, the
// iteration i (alpha_i, beta_i known) is
//
//     p_i     = u_i + beta_i p_{i-1}          s_i = w_i + beta_i s_{i-1}
//     x_{i+1} = x_i + alpha_i p_i             r_{i+1} = r_i - alpha_i s_i
//     u_{i+1} = D^-1 r_{i+1}                  w_{i+1} = B u_{i+1}
//     gamma_{i+1} = r_{i+1} . u_{i+1}         delta_{i+1} = w_{i+1} . u_{i+1}
//     beta_{i+1}  = gamma_{i+1} / gamma_i
//     alpha_{i+1} = gamma_{i+1} / (p_{i+1} . s_{i+1}),
//     p_{i+1} . s_{i+1} = delta_{i+1} + beta_{i+1} (u_{i+1} . s_i + p_i . w_{i+1})
//                         + beta_{i+1}^2 p_i . s_i
//
// so both scalars come from dot products of one pass.  (The shorter
// recurrence alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1}
// gamma_{i+1} / alpha_i) leans on orthogonality that float32 iterates lose:
// it broke down on the mixed path, the expanded product does not.)  Kernel i
// reduces the partial sums of gamma_i, delta_i, r_i . r_i and the three
// products left by kernel i - 1 (every block, same fixed order, so all
// blocks agree bit for bit), then streams its
// slices of B once: the u_{i+1} of every column it reads is formed on the fly
// from that neighbour's (r_i, w_i, s_{i-1}, d) record, one vector gather per
// stored entry, and the row's own p_i, x_{i+1}, r_{i+1}, s_i are updated in
// the same pass.  The records are double-buffered (read st[q], write
// st[q ^ 1]); p and x are touched by their own row only.  No device-scope
// fence is ever executed: kernel boundaries make one kernel's partials
// visible to the next on every XCD.
//
// A reliable update (and the start) replaces r by the float64 residual of the
// stored system, recomputes w = B D^-1 r and sets alpha, beta of the next
// iteration from the same expanded product, the direction kept (or reset).
//
// With linear polynomial reproduction (Section 3, eq. 10) the system is
// bordered by Q = A^T P and C = P^T P.  The d + 1 polynomial unknowns are a
// replicated float64 block (PolyState): every block reads its record, a row of
// B adds Q_j u_poly to its w, and Q^T u joins the partial sums, from which the
// next launch forms the polynomial rows' w and their share of every product.
// One extra block per launch writes the block's next state.  Preconditioner:
// D^-1 on B's rows, C^-1 on the polynomial block.
//
// Precision: matrix and iterated vectors are VT / XT (float64, or float32
// for the mixed path); every dot product is a float64 sum of float64
// products; the solution is accumulated in float64 at every reliable update.
#include <hip/hip_ext.h>

#include "plan_kernels.h"
#include "solver.h"

namespace rbf {
namespace {

// Workgroups are dispatched to the 8 XCDs in turn (block b to XCD b mod 8).
// With nb a multiple of 8 xg, this bijection of [0, nb) cuts the logical
// blocks into 8 xg ranges of C = nb / (8 xg) and gives XCD x the ranges
// x, x + 8, ..., so neighbouring slices, which gather largely the same
// records, share an L2, while the xg ranges per XCD spread uneven regions of
// the matrix over all XCDs.  xg = 0 (or nb not such a multiple): identity.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb, int xg) {
  if (xg <= 0 || nb % (kXcds * xg) != 0) return b;
  const int C = nb / (kXcds * xg);
  const int x = b % kXcds, i = b / kXcds;
  const int g = i / C, j = i - g * C;
  return (g * kXcds + x) * C + j;
}

// The scalars as this launch leaves them, copied into the host's snapshot
// slot when the launch ends a chunk (block 0, thread 0, after its own
// updates; the slot is pinned coherent host memory, read by the host once the
// chunk's event has completed).
__device__ __forceinline__ void snapshot(const CgScalars* sc, CgScalars* snap) {
  if (snap) *snap = *sc;
}

// s_i = w_i + beta s_{i-1} and r_{i+1} = r_i - alpha s_i, rounded step by step
// so that a row's own update and every neighbour's on-the-fly copy of it are
// the same numbers.
template <typename XT>
__device__ __forceinline__ XT s_next(XT w, XT s, XT beta) {
#pragma clang fp contract(off)
  return w + beta * s;
}
template <typename XT>
__device__ __forceinline__ XT r_next(XT r, XT sn, XT alpha) {
#pragma clang fp contract(off)
  return r - alpha * sn;
}

// Block-wide sums of N doubles per thread in a fixed order.  ALL: every
// thread gets them (and the call ends with a barrier, so it can be made again
// right away); otherwise only thread 0 does.
template <int N, int W, bool ALL = true>
__device__ __forceinline__ void block_sums(double (&v)[N], double (*ws)[W]) {
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) ws[k][wave] = v[k];
  }
  __syncthreads();
  if (ALL || threadIdx.x == 0) {
    for (int k = 0; k < N; ++k) {
      double t = 0.0;
#pragma unroll 4
      for (int w = 0; w < W; ++w) t += ws[k][w];
      v[k] = t;
    }
  }
  if (ALL) __syncthreads();
}

// The flag is read once per block and broadcast, so that all waves of a block
// take the same branch even if block 0 raises it meanwhile.
__device__ __forceinline__ bool block_done(const CgScalars* sc, int* s_flag) {
  if (threadIdx.x == 0) *s_flag = sc->done;
  __syncthreads();
  return *s_flag != 0;
}

// Row sum over one slice of the wave: acc = sum_e b_e f(col_e), with f the
// gathered quantity of the neighbour, complete in the lane with
// (lane % L) == 0 of every row.  Four independent loads per lane are in
// flight per step; rows past m gather from row m - 1 with value 0.
template <typename VT, typename XT, typename CT, int L, typename F>
__device__ __forceinline__ XT slice_sum(int64_t m, int64_t slice, const CgMatrix& A, F f,
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
  int st = 0;
  for (; st + 3 < steps; st += 4) {
    const int64_t o = base + (int64_t)st * kWave;
    const int32_t l0 = rowc + (int32_t)col[o];
    const int32_t l1 = rowc + (int32_t)col[o + kWave];
    const int32_t l2 = rowc + (int32_t)col[o + 2 * kWave];
    const int32_t l3 = rowc + (int32_t)col[o + 3 * kWave];
    const XT v0 = (XT)val[o], v1 = (XT)val[o + kWave];
    const XT v2 = (XT)val[o + 2 * kWave], v3 = (XT)val[o + 3 * kWave];
    a0 += v0 * f(l0);
    a1 += v1 * f(l1);
    a2 += v2 * f(l2);
    a3 += v3 * f(l3);
  }
  for (; st < steps; ++st) {
    const int64_t o = base + (int64_t)st * kWave;
    const int32_t l0 = rowc + (int32_t)col[o];
    a0 += (XT)val[o] * f(l0);
  }
  XT a = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
  *row_out = row;
  return a;
}

// Steps (of 64 entries per wave) whose column indices and values are loaded
// together; the next batch is in flight while the current one's gathers are.
// Float64 records are twice as wide, so their batches are half as long.
template <typename XT>
constexpr int kBatch = sizeof(XT) == 4 ? 8 : 4;
// Batches of the staged path (longer ones measured no faster: their
// registers cost occupancy).
template <typename XT, bool HALO>
constexpr int kBatchH = kBatch<XT>;

// One batch of a slice: the gathered column index and value of each of its
// steps (index = the row itself and value 0 past the slice's end).
template <typename XT, int U = kBatch<XT>>
struct Batch {
  int32_t l[U];
  XT v[U];
};

// HALO: the entries' LDS slots (hslot) instead of their column deltas.
// raw_batch loads a batch as stored; mask_batch then drops the steps past the
// slice's end (index = the row itself, value 0).  They are apart so that the
// first batch of a slice, loaded before the kernel's reduction, is only waited
// for where it is used.
template <typename VT, typename XT, typename CT, bool HALO = false>
__device__ __forceinline__ void raw_batch(const CgMatrix& A, int64_t base, int st,
                                          Batch<XT, kBatchH<XT, HALO>>& b) {
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const int16_t* __restrict__ slot = A.hslot;
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  // Loads are unconditional: past the slice's end they read the next slice or
  // the zeroed tail of the arrays (kSellTail), and the mask drops them.
#pragma unroll
  for (int t = 0; t < kBatchH<XT, HALO>; ++t) {
    const int64_t o = base + (int64_t)(st + t) * kWave;
    b.l[t] = HALO ? (int32_t)slot[o] : (int32_t)col[o];
    b.v[t] = (XT)val[o];
  }
}
template <typename XT, bool HALO = false>
__device__ __forceinline__ void mask_batch(int32_t rowc, int st, int steps,
                                           Batch<XT, kBatchH<XT, HALO>>& b) {
#pragma unroll
  for (int t = 0; t < kBatchH<XT, HALO>; ++t) {
    const bool in = st + t < steps;
    b.l[t] = HALO ? (in ? b.l[t] : 0) : rowc + (in ? b.l[t] : 0);
    b.v[t] = in ? b.v[t] : (XT)0;
  }
}
template <typename VT, typename XT, typename CT, bool HALO = false>
__device__ __forceinline__ void load_batch(const CgMatrix& A, int64_t base, int32_t rowc, int st,
                                           int steps, Batch<XT, kBatchH<XT, HALO>>& b) {
  raw_batch<VT, XT, CT, HALO>(A, base, st, b);
  mask_batch<XT, HALO>(rowc, st, steps, b);
}

// One slice of a wave: its geometry and its first batch, loaded before the
// kernel's reduction so that their latency overlaps it.
template <typename XT, bool HALO = false>
struct SliceHead {
  int64_t row, base;
  int32_t rowc;
  int steps;
  Batch<XT, kBatchH<XT, HALO>> b;
};

template <typename VT, typename XT, typename CT, int L, bool HALO = false>
__device__ __forceinline__ void open_slice(int64_t m, int64_t slice, const CgMatrix& A,
                                           SliceHead<XT, HALO>& h) {
  constexpr int S = kWave / L;
  const int lane = threadIdx.x & (kWave - 1);
  h.row = slice * S + lane / L;
  h.rowc = (int32_t)(h.row < m ? h.row : m - 1);
  h.base = A.sptr[slice] + lane;
  h.steps = A.slen[slice] / L;
  raw_batch<VT, XT, CT, HALO>(A, h.base, 0, h.b);  // masked in finish_slice
}

// Row sum of an opened slice, complete in the lane with (lane % L) == 0:
// software-pipelined, the next batch's indices and values load while the
// current batch is gathered.
template <typename VT, typename XT, typename CT, int L, bool HALO = false, typename F>
__device__ __forceinline__ XT finish_slice(const SliceHead<XT, HALO>& h, const CgMatrix& A, F f) {
  constexpr int U = kBatchH<XT, HALO>;
  XT acc[U];
#pragma unroll
  for (int t = 0; t < U; ++t) acc[t] = (XT)0;
  Batch<XT, U> cur = h.b;
  mask_batch<XT, HALO>(h.rowc, 0, h.steps, cur);
  for (int st = U;; st += U) {
    const bool more = st < h.steps;
    Batch<XT, U> nxt;
    if (more) load_batch<VT, XT, CT, HALO>(A, h.base, h.rowc, st, h.steps, nxt);
#pragma unroll
    for (int t = 0; t < U; ++t) acc[t] += cur.v[t] * f(cur.l[t]);
    if (!more) break;
    cur = nxt;
  }
#pragma unroll
  for (int w = U / 2; w > 0; w >>= 1) {
#pragma unroll
    for (int t = 0; t < w; ++t) acc[t] += acc[t + w];
  }
  XT a = acc[0];
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
  return a;
}

// The replicated polynomial block of an iteration (see PolySys): from the
// state (r, s_old, p_old) of state buffer q and w, forms u = C^-1 r.
__device__ __forceinline__ void poly_u(const PolySys& S, int np, const double* r, double* u) {
#pragma unroll
  for (int t = 0; t < kMaxPoly; ++t) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxPoly; ++k)
      if (k < np) a += S.Ci[t][k] * r[k];
    u[t] = t < np ? a : 0.0;
  }
}

// w = Q^T u (reduced partials) + C u over the polynomial unknowns.
__device__ __forceinline__ void poly_w(const PolySys& S, int np, const double* qtu,
                                       const double* u, double* w) {
#pragma unroll
  for (int t = 0; t < kMaxPoly; ++t) {
    double a = qtu[t];
#pragma unroll
    for (int k = 0; k < kMaxPoly; ++k)
      if (k < np) a += S.C[t][k] * u[k];
    w[t] = t < np ? a : 0.0;
  }
}

// Writes the polynomial unknowns' state (r, w, s, p, x) and the products an
// iteration's blocks read (see PolyState).
__device__ __forceinline__ void poly_store(const PolySys& S, int np, const double* r,
                                           const double* w, const double* s, const double* p,
                                           const double* x, PolyState* __restrict__ out) {
  double u[kMaxPoly], cis[kMaxPoly], cu[kMaxPoly];
  poly_u(S, np, r, u);
  poly_u(S, np, s, cis);
  const double zero[kMaxPoly] = {0.0, 0.0, 0.0, 0.0};
  poly_w(S, np, zero, u, cu);
  double ru = 0.0, rr = 0.0, us = 0.0, ps = 0.0, ucu = 0.0, pcu = 0.0;
  for (int t = 0; t < kMaxPoly; ++t) {
    out->r[t] = r[t];
    out->w[t] = w[t];
    out->s[t] = s[t];
    out->p[t] = p[t];
    out->x[t] = x[t];
    out->u[t] = u[t];
    out->cis[t] = cis[t];
    out->cu[t] = cu[t];
    ru += r[t] * u[t];
    rr += r[t] * r[t];
    us += u[t] * s[t];
    ps += p[t] * s[t];
    ucu += u[t] * cu[t];
    pcu += p[t] * cu[t];
  }
  out->ru = ru;
  out->rr = rr;
  out->us = us;
  out->ps = ps;
  out->ucu = ucu;
  out->pcu = pcu;
}

// With the polynomial block the grid has one more block than the slice
// kernels' (n_in): it streams no slice and writes no partials, but forms the
// polynomial unknowns' next state from the same scalars as every other block,
// so that the others keep only a few of its values in registers.
// HALO: every slice's neighbourhood is staged in LDS (one u per distinct
// column, computed once) and the entries gather from there (see CgMatrix).
template <typename VT, typename XT, typename CT, int L, int BS, bool POLY, bool HALO = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(POLY ? 4 : 1))) void k_cg_iter(
    int64_t m, CgMatrix A, const CgState<XT>* __restrict__ sin, CgState<XT>* __restrict__ sout,
    XT* __restrict__ p, XT* __restrict__ xlo, CgScalars* __restrict__ sc, CgScalars* snap,
    int32_t* flag, const double* __restrict__ part_in, double* __restrict__ part_out, int n_in,
    int xg, int q,
    int fixed, int np, const XT* __restrict__ Q, const PolySys* __restrict__ psys,
    const PolyState* __restrict__ pin, PolyState* __restrict__ pout) {
  constexpr int W = BS / kWave;
  constexpr int NP = POLY ? kCgParts : 6;
  __shared__ double ws[NP][W];
  __shared__ double ws_out[6][W];
  // the polynomial rows' partials Q^T u, per wave (added slice by slice, so
  // that they hold no registers across the streamed loop)
  __shared__ double ws_poly[POLY ? kMaxPoly : 1][POLY ? W : 1];
  __shared__ XT us[HALO ? W : 1][HALO ? kHaloCap : 1];
  __shared__ int s_flag;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t wstride = (int64_t)(POLY ? n_in : gridDim.x) * W;
  const bool poly_block = POLY && (int)blockIdx.x == n_in;
  // logical block: the slices it streams and its partial sums' slot
  const int blk =
      poly_block ? n_in : xcd_block((int)blockIdx.x, POLY ? n_in : (int)gridDim.x, xg);
  int64_t slice = (int64_t)blk * W + wave;

  // Loads that do not depend on this iteration's scalars go out first: the
  // previous kernel's partials (so that their sum waits for them alone), then
  // the first slice's geometry and first batch, the row's own state and the
  // scalars.  Every partial this thread adds is loaded before the first add
  // (one round trip instead of one per block stride); the loads are
  // unconditional, from a clamped block index, so that no branch separates
  // them, and the surplus ones are dropped by a select.  They are loaded in
  // a launch with fixed scalars too (which ignores them) so that no branch
  // holds their first adds.
  constexpr int KB = (kCgMaxBlocks + BS - 1) / BS;
  double pv[KB][NP];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int k = (int)threadIdx.x + i * BS;
    const int kc = k < n_in ? k : n_in - 1;
#pragma unroll
    for (int t = 0; t < NP; ++t) pv[i][t] = part_in[NP * kc + t];
  }
  // These loads take no branch either (a branch around them would make the
  // partials' sum wait for them too): a wave with no slice (padding or
  // polynomial block) loads the last slice and every lane its clamped row;
  // only the waves with a slice and the rows' owner lanes use them.
  SliceHead<XT, HALO> h;
  const bool have = !poly_block && slice < A.nslices;
  open_slice<VT, XT, CT, L, HALO>(m, have ? slice : A.nslices - 1, A, h);
  CgState<XT> own = sin[h.rowc];
  XT p_old = p[h.rowc], x_old = xlo[h.rowc];
  // the first slice's neighbourhood records (they do not depend on this
  // iteration's scalars): the first rounds go out before the reduction
  constexpr int kStagePre = HALO ? (sizeof(XT) == 4 ? 8 : 4) : 1;
  CgState<XT> srec[kStagePre];
  int st_n = 0;
  int64_t st_off = 0, st_first = 0;
  if constexpr (HALO) {
    if (have) {
      st_n = A.hcount[slice];
      st_off = A.hptr[slice];
      st_first = slice * (kWave / L);
#pragma unroll
      for (int r = 0; r < kStagePre; ++r) {
        const int i = lane + kWave * r;
        if (i < st_n) srec[r] = sin[st_first + A.hrow[st_off + i]];
      }
    }
  }
  // added in block order (also in a launch with fixed scalars, which drops
  // the sum), a surplus load times 0: every load's value is used on every
  // path, so none is made conditional (and the sum waits for no later load)
  double red[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) red[t] = 0.0;
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const double wgt = (int)threadIdx.x + i * BS < n_in ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < NP; ++t) red[t] = __builtin_fma(pv[i][t], wgt, red[t]);
  }
#pragma unroll
  for (int t = 0; t < NP; ++t) red[t] = fixed ? 0.0 : red[t];
  const double gam_prev = sc->gam[q ^ 1];
  const double trigger2 = sc->trigger2;
  const double fgamma = sc->fix_gamma, frr = sc->fix_rr;
  const double falpha = sc->fix_alpha, fbeta = sc->fix_beta;
  // the polynomial record of state buffer q, loaded before the barrier
  double rw[kMaxPoly], ru_[kMaxPoly], rp_[kMaxPoly], rcu[kMaxPoly], rcis[kMaxPoly];
  double rsum[6];
  if constexpr (POLY) {
#pragma unroll
    for (int t = 0; t < kMaxPoly; ++t) {
      rw[t] = pin->w[t];
      ru_[t] = pin->u[t];
      rp_[t] = pin->p[t];
      rcu[t] = pin->cu[t];
      rcis[t] = pin->cis[t];
    }
    rsum[0] = pin->ru;
    rsum[1] = pin->ucu;
    rsum[2] = pin->rr;
    rsum[3] = pin->us;
    rsum[4] = pin->pcu;
    rsum[5] = pin->ps;
  }
  // one barrier publishes both the block's partial sums and the flag
#pragma unroll
  for (int t = 0; t < NP; ++t) red[t] = wave_sum(red[t]);
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < NP; ++t) ws[t][wave] = red[t];
  }
  if (threadIdx.x == 0) s_flag = sc->done;
  __syncthreads();
  if (s_flag) {
    if (blockIdx.x == 0 && threadIdx.x == 0) snapshot(sc, snap);
    return;
  }
  for (int t = 0; t < NP; ++t) {
    double v = 0.0;
#pragma unroll 4
    for (int w = 0; w < W; ++w) v += ws[t][w];
    red[t] = v;
  }
  // polynomial unknowns: w = Q^T u + C u (from the refresh after one) and
  // their share of every product, from the record of state buffer q
  double pw[kMaxPoly];
  if constexpr (POLY) {
    if (fixed) {
#pragma unroll
      for (int t = 0; t < kMaxPoly; ++t) pw[t] = rw[t];
    } else {
      double a1 = 0.0, a4 = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxPoly; ++t) {
        const double qs = red[6 + t];
        pw[t] = qs + rcu[t];
        a1 += qs * ru_[t];
        a4 += rp_[t] * qs;
      }
      red[0] += rsum[0];
      red[1] += a1 + rsum[1];
      red[2] += rsum[2];
      red[3] += rsum[3];
      red[4] += a4 + rsum[4];
      red[5] += rsum[5];
    }
  }
  const double gamma = fixed ? fgamma : red[0];
  const double rr = fixed ? frr : red[2];
  double alpha_d, beta_d;
  if (fixed) {
    alpha_d = falpha;
    beta_d = fbeta;
  } else {
    beta_d = gamma / gam_prev;
    alpha_d = gamma / (red[1] + beta_d * (red[3] + red[4]) + beta_d * beta_d * red[5]);
  }
  if (!__builtin_isfinite(rr) || !__builtin_isfinite(gamma)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->done = 2;
      snapshot(sc, snap);
      if (flag) *flag = 2;
    }
    return;
  }
  if (rr <= trigger2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->rr = rr;
      sc->done = 1;
      snapshot(sc, snap);
      if (flag) *flag = 1;
    }
    return;
  }
  if (!(alpha_d > 0.0) || !__builtin_isfinite(alpha_d) || !__builtin_isfinite(beta_d)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->done = 2;
      snapshot(sc, snap);
      if (flag) *flag = 2;
    }
    return;
  }
  const XT alpha = (XT)alpha_d, beta = (XT)beta_d;
  // the polynomial unknowns' next u for the rows of B:
  // u' = C^-1 (r - alpha (w + beta s)) = u - alpha (C^-1 w + beta C^-1 s)
  XT uq[kMaxPoly];
  if constexpr (POLY) {
    double ciw[kMaxPoly];
    poly_u(*psys, np, pw, ciw);
#pragma unroll
    for (int t = 0; t < kMaxPoly; ++t)
      uq[t] = (XT)(ru_[t] - alpha_d * (ciw[t] + beta_d * rcis[t]));
    if (poly_block) {
      // the state of the next iteration, written by the extra block
      if (threadIdx.x == 0) {
        double rn[kMaxPoly], sn[kMaxPoly], pn[kMaxPoly], xn[kMaxPoly];
        for (int t = 0; t < kMaxPoly; ++t) {
          pn[t] = pin->u[t] + beta_d * pin->p[t];
          sn[t] = pw[t] + beta_d * pin->s[t];
          xn[t] = pin->x[t] + alpha_d * pn[t];
          rn[t] = pin->r[t] - alpha_d * sn[t];
        }
        poly_store(*psys, np, rn, pw, sn, pn, xn, pout);
      }
      return;
    }
  }
  auto u_rec = [&](const CgState<XT>& t) -> XT {
    return t.d * r_next(t.r, s_next(t.w, t.s, beta), alpha);
  };
  auto u_next = [&](int32_t l) -> XT {
    if constexpr (HALO) return us[wave][l];
    else return u_rec(sin[l]);
  };
  // the slice's neighbourhood: u of each distinct column, once (the first
  // slice's first rounds from the records loaded before the barrier)
  auto stage = [&](int64_t sl) {
    if constexpr (HALO) {
      const int n = A.hcount[sl];
      const int64_t off = A.hptr[sl], first = sl * (kWave / L);
      wave_sync();
      int i0 = lane;
      if (sl == (int64_t)blk * W + wave) {
#pragma unroll
        for (int r = 0; r < kStagePre; ++r) {
          const int i = lane + kWave * r;
          if (i < n) us[wave][i] = u_rec(srec[r]);
        }
        i0 = lane + kWave * kStagePre;
      }
      for (int i = i0; i < n; i += kWave) us[wave][i] = u_rec(sin[first + A.hrow[off + i]]);
      wave_sync();
    }
  };
  double part[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if constexpr (POLY) {
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < kMaxPoly; ++k) ws_poly[k][wave] = 0.0;
    }
  }
  double qtu[kMaxPoly];
  auto own_row = [&](int64_t row, XT wn, const CgState<XT>& t, XT po, XT xo) {
    const XT pn = t.d * t.r + beta * po;
    const XT sn = s_next(t.w, t.s, beta);
    const XT rn = r_next(t.r, sn, alpha);
    const XT un = t.d * rn;
    if constexpr (POLY) {
      // w of a row of B takes the polynomial columns Q u; Q^T u is the
      // polynomial unknowns' share of the next w
#pragma unroll
      for (int k = 0; k < kMaxPoly; ++k) {
        if (k < np) {
          const XT qv = Q[k * m + row];
          wn += qv * uq[k];
          qtu[k] = (double)qv * (double)un;
        }
      }
    }
    p[row] = pn;
    xlo[row] = xo + alpha * pn;
    CgState<XT> o;
    o.r = rn;
    o.w = wn;
    o.s = sn;
    o.d = t.d;
    sout[row] = o;
    part[0] += (double)rn * (double)un;
    part[1] += (double)wn * (double)un;
    part[2] += (double)rn * (double)rn;
    part[3] += (double)un * (double)sn;
    part[4] += (double)pn * (double)wn;
    part[5] += (double)pn * (double)sn;
  };
  // the wave's Q^T u of one slice into its LDS slot
  auto poly_slice_sums = [&]() {
    if constexpr (POLY) {
#pragma unroll
      for (int k = 0; k < kMaxPoly; ++k) {
        const double v = wave_sum(qtu[k]);
        if (lane == 0) ws_poly[k][wave] += v;
      }
    }
  };
  if (have) {
#pragma unroll
    for (int k = 0; k < kMaxPoly; ++k) qtu[k] = 0.0;
    stage(slice);
    const XT wn = finish_slice<VT, XT, CT, L, HALO>(h, A, u_next);
    if ((lane & (L - 1)) == 0 && h.row < m) own_row(h.row, wn, own, p_old, x_old);
    poly_slice_sums();
    for (slice += wstride; slice < A.nslices; slice += wstride) {
      open_slice<VT, XT, CT, L, HALO>(m, slice, A, h);
#pragma unroll
      for (int k = 0; k < kMaxPoly; ++k) qtu[k] = 0.0;
      stage(slice);
      const XT wn2 = finish_slice<VT, XT, CT, L, HALO>(h, A, u_next);
      if ((lane & (L - 1)) == 0 && h.row < m)
        own_row(h.row, wn2, sin[h.row], p[h.row], xlo[h.row]);
      poly_slice_sums();
    }
  }
  block_sums<6, W, false>(part, ws_out);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < 6; ++t) part_out[NP * blk + t] = part[t];
    if constexpr (POLY) {
      // block_sums ended with a barrier after every wave's last LDS add
      for (int k = 0; k < kMaxPoly; ++k) {
        double v = 0.0;
        for (int w = 0; w < W; ++w) v += ws_poly[k][w];
        part_out[NP * blk + 6 + k] = v;
      }
    }
    if (blockIdx.x == 0) {
      sc->gam[q] = gamma;
      sc->alp[q] = alpha_d;
      sc->rr = rr;
      sc->iter += 1;
      snapshot(sc, snap);
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

// Float64 residual of the stored system: r64 = g - (B + lambda I) x_hi, and
// r = (XT) r64 into the state record (one wave per slice).  With the
// polynomial block, r64 -= Q x_poly and the block's partials of Q^T x_hi go
// to part_out (kMaxPoly per block).
template <typename VT, typename XT, typename CT, int L, int BS, bool POLY>
__global__ __launch_bounds__(BS) void k_true_residual(int64_t m, CgMatrix A,
                                                            const double* __restrict__ xhi,
                                                            const double* __restrict__ g,
                                                            double* __restrict__ r64,
                                                            CgState<XT>* __restrict__ st, int np,
                                                            const XT* __restrict__ Q,
                                                            const PolyState* __restrict__ pin,
                                                            double* __restrict__ part_out) {
  constexpr int S = kWave / L;
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  const int lane = threadIdx.x & (kWave - 1);
  constexpr int W = BS / kWave;
  __shared__ double ws[kMaxPoly][W];
  double xq[kMaxPoly], qx[kMaxPoly];
#pragma unroll
  for (int t = 0; t < kMaxPoly; ++t) {
    xq[t] = POLY ? pin->x[t] : 0.0;
    qx[t] = 0.0;
  }
  for (int64_t slice = (int64_t)blockIdx.x * W + threadIdx.x / kWave; slice < A.nslices;
       slice += (int64_t)gridDim.x * W) {
    const int64_t row = slice * S + lane / L;
    const int32_t rowc = (int32_t)(row < m ? row : m - 1);
    const int64_t base = A.sptr[slice] + lane;
    const int steps = A.slen[slice] / L;
    double acc = 0.0;
    for (int s = 0; s < steps; ++s) {
      const int64_t o = base + (int64_t)s * kWave;
      acc += (double)val[o] * xhi[rowc + (int32_t)col[o]];
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((lane & (L - 1)) == 0 && row < m) {
      double rv = g[row] - acc;
      if constexpr (POLY) {
        const double xj = xhi[row];
#pragma unroll
        for (int t = 0; t < kMaxPoly; ++t) {
          if (t < np) {
            const double qv = (double)Q[t * m + row];
            rv -= qv * xq[t];
            qx[t] += qv * xj;
          }
        }
      }
      r64[row] = rv;
      st[row].r = (XT)rv;
    }
  }
  if constexpr (POLY) {
    block_sums<kMaxPoly, W, false>(qx, ws);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int t = 0; t < kMaxPoly; ++t) part_out[kMaxPoly * blockIdx.x + t] = qx[t];
    }
  }
}

// The polynomial unknowns' float64 residual e - Q^T x_hi - C x_poly (single
// block; the partials of k_true_residual reduced in a fixed order), into the
// state of buffer q.
__global__ __launch_bounds__(kCgLargeBlock) void k_poly_residual(const PolySys* __restrict__ S,
                                                                 const double* __restrict__ part,
                                                                 int n, PolyState* __restrict__ st) {
  constexpr int W = kCgLargeBlock / kWave;
  __shared__ double ws[kMaxPoly][W];
  double v[kMaxPoly] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += kCgLargeBlock) {
#pragma unroll
    for (int t = 0; t < kMaxPoly; ++t) v[t] += part[kMaxPoly * k + t];
  }
  block_sums<kMaxPoly, W, false>(v, ws);
  if (threadIdx.x == 0) {
    const int np = S->np;
    for (int t = 0; t < kMaxPoly; ++t) {
      double r = 0.0;
      if (t < np) {
        r = S->e[t] - v[t];
        for (int k = 0; k < np; ++k) r -= S->C[t][k] * st->x[k];
      }
      st->r[t] = r;
    }
  }
}

// w = B D^-1 r from the records of st[q] (r just replaced), written with the
// carried s and d into the other buffer; partials of r.u, w.u, r64.r64,
// p.w, u.s and p.s (and, with the polynomial block, of Q^T u; the block's
// own u = C^-1 r feeds w of every row through Q).
template <typename VT, typename XT, typename CT, int L, int BS, bool POLY>
__global__ __launch_bounds__(BS) void k_cg_refresh(int64_t m, CgMatrix A,
                                                         const CgState<XT>* __restrict__ sin,
                                                         CgState<XT>* __restrict__ sout,
                                                         const XT* __restrict__ p,
                                                         const double* __restrict__ r64,
                                                         double* __restrict__ part_out, int np,
                                                         const XT* __restrict__ Q,
                                                         const PolySys* __restrict__ psys,
                                                         const PolyState* __restrict__ pin) {
  constexpr int W = BS / kWave;
  constexpr int NP = POLY ? kCgParts : 6;
  __shared__ double ws[NP][W];
  auto u_of = [&](int32_t l) -> XT {
    const CgState<XT> t = sin[l];
    return t.d * t.r;
  };
  XT uq[kMaxPoly];
  if constexpr (POLY) {
    double pr[kMaxPoly], pu[kMaxPoly];
#pragma unroll
    for (int t = 0; t < kMaxPoly; ++t) pr[t] = pin->r[t];
    poly_u(*psys, np, pr, pu);
#pragma unroll
    for (int t = 0; t < kMaxPoly; ++t) uq[t] = (XT)pu[t];
  }
  const int lane = threadIdx.x & (kWave - 1);
  double part[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) part[t] = 0.0;
  for (int64_t slice = (int64_t)blockIdx.x * W + threadIdx.x / kWave; slice < A.nslices;
       slice += (int64_t)gridDim.x * W) {
    int64_t row;
    XT wn = slice_sum<VT, XT, CT, L>(m, slice, A, u_of, &row);
    if ((lane & (L - 1)) == 0 && row < m) {
      const CgState<XT> t = sin[row];
      const XT u = t.d * t.r;
      if constexpr (POLY) {
#pragma unroll
        for (int k = 0; k < kMaxPoly; ++k) {
          if (k < np) {
            const XT qv = Q[k * m + row];
            wn += qv * uq[k];
            part[6 + k] += (double)qv * (double)u;
          }
        }
      }
      const XT pj = p[row];
      CgState<XT> o;
      o.r = t.r;
      o.w = wn;
      o.s = t.s;
      o.d = t.d;
      sout[row] = o;
      const double r64j = r64[row];
      part[0] += (double)t.r * (double)u;
      part[1] += (double)wn * (double)u;
      part[2] += r64j * r64j;
      part[3] += (double)pj * (double)wn;
      part[4] += (double)u * (double)t.s;
      part[5] += (double)pj * (double)t.s;
    }
  }
  block_sums<NP, W, false>(part, ws);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NP; ++k) part_out[NP * blockIdx.x + k] = part[k];
  }
}

// After a refresh: the true residual norm, the convergence flag, the next
// trigger and the scalars of the next iteration (restart: beta = 0, so
// p = u and s = w; otherwise beta = gamma / gamma_prev with the direction
// kept, and alpha = gamma / (p . s) from the expanded product).  With the
// polynomial block: its w = Q^T u + C u and its share of every product, its
// state carried to buffer q ^ 1, and its solution to xpoly.
template <bool POLY>
__global__ __launch_bounds__(kCgLargeBlock) void k_refresh_scalars(
    CgScalars* __restrict__ sc, const double* __restrict__ part, int n, int q_prev, int restart,
    const PolySys* __restrict__ psys, const PolyState* __restrict__ pin,
    PolyState* __restrict__ pout, double* __restrict__ xpoly) {
  constexpr int W = kCgLargeBlock / kWave;
  constexpr int NP = POLY ? kCgParts : 6;
  __shared__ double ws[NP][W];
  double v[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) v[t] = 0.0;
  for (int k = threadIdx.x; k < n; k += kCgLargeBlock) {
#pragma unroll
    for (int t = 0; t < NP; ++t) v[t] += part[NP * k + t];
  }
  block_sums<NP, W, false>(v, ws);
  if (threadIdx.x == 0) {
    if constexpr (POLY) {
      const int np = psys->np;
      double pr[kMaxPoly], pu[kMaxPoly], pw[kMaxPoly];
      for (int t = 0; t < kMaxPoly; ++t) pr[t] = pin->r[t];
      poly_u(*psys, np, pr, pu);
      poly_w(*psys, np, v + 6, pu, pw);
      double ps[kMaxPoly], pp[kMaxPoly], px[kMaxPoly];
      for (int t = 0; t < kMaxPoly; ++t) {
        pp[t] = pin->p[t];
        ps[t] = pin->s[t];
        px[t] = pin->x[t];
        v[0] += pr[t] * pu[t];
        v[1] += pw[t] * pu[t];
        v[2] += pr[t] * pr[t];
        v[3] += pp[t] * pw[t];
        v[4] += pu[t] * ps[t];
        v[5] += pp[t] * ps[t];
        xpoly[t] = px[t];
      }
      poly_store(*psys, np, pr, pw, ps, pp, px, pout);
    }
    const double gamma = v[0], delta = v[1], rr = v[2];
    const double beta = restart ? 0.0 : gamma / sc->gam[q_prev];
    const double ps = delta + beta * (v[3] + v[4]) + beta * beta * v[5];
    const double alpha = gamma / ps;
    sc->rr_true = rr;
    sc->rr = rr;
    sc->fix_rr = rr;
    sc->fix_gamma = gamma;
    sc->fix_beta = beta;
    sc->fix_alpha = alpha;
    const double trig = sc->delta2 * rr;
    sc->trigger2 = trig > sc->tol2 ? trig : sc->tol2;
    if (!__builtin_isfinite(rr) || !__builtin_isfinite(gamma)) {
      sc->done = 2;
    } else if (rr <= sc->tol2) {
      sc->done = 3;
    } else if (!(ps > 0.0) || !__builtin_isfinite(alpha) || !__builtin_isfinite(beta)) {
      sc->done = 2;
    } else {
      sc->done = 0;
    }
  }
}

// Start of a solve: x_lo, p and both state buffers cleared (s = 0), d = D^-1
// in both; the polynomial unknowns' states cleared likewise, with x from xpoly.
template <typename XT>
__global__ void k_cg_clear(int64_t m, const XT* __restrict__ dinv, XT* __restrict__ xlo,
                           XT* __restrict__ p, CgState<XT>* __restrict__ s0,
                           CgState<XT>* __restrict__ s1, PolyState* __restrict__ p0,
                           PolyState* __restrict__ p1, const double* __restrict__ xpoly) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p0 && j == 0) {
    for (PolyState* st : {p0, p1}) {
      for (int t = 0; t < kMaxPoly; ++t) {
        st->r[t] = st->w[t] = st->s[t] = st->p[t] = 0.0;
        st->u[t] = st->cis[t] = st->cu[t] = 0.0;
        st->x[t] = xpoly[t];
      }
      st->ru = st->rr = st->us = st->ps = st->ucu = st->pcu = 0.0;
    }
  }
  if (j >= m) return;
  xlo[j] = (XT)0;
  p[j] = (XT)0;
  CgState<XT> t;
  t.r = (XT)0;
  t.w = (XT)0;
  t.s = (XT)0;
  t.d = dinv[j];
  s0[j] = t;
  s1[j] = t;
}

// ||g||^2 (with ||e||^2 of the polynomial block) and the initial state of the
// scalars (single block, fixed order).
__global__ __launch_bounds__(kCgLargeBlock) void k_cg_init(int64_t m, const double* __restrict__ g,
                                                      const PolySys* __restrict__ psys,
                                                      CgScalars* __restrict__ sc, double rtol,
                                                      double delta) {
  constexpr int W = kCgLargeBlock / kWave;
  __shared__ double ws[1][W];
  double v[1] = {0.0};
  for (int64_t j = threadIdx.x; j < m; j += kCgLargeBlock) v[0] += g[j] * g[j];
  block_sums<1, W, false>(v, ws);
  if (threadIdx.x == 0) {
    if (psys)
      for (int t = 0; t < psys->np; ++t) v[0] += psys->e[t] * psys->e[t];
    sc->gg = v[0];
    sc->tol2 = rtol * rtol * v[0];
    sc->delta2 = delta * delta;
    sc->trigger2 = sc->tol2;
    sc->done = 0;
    sc->iter = 0;
    sc->gam[0] = sc->gam[1] = 1.0;
    sc->alp[0] = sc->alp[1] = 1.0;
    sc->fix_gamma = sc->fix_alpha = sc->fix_beta = sc->fix_rr = 0.0;
    sc->rr = sc->rr_true = v[0];
  }
}

template <typename VT, typename XT, typename CT, int L, int BS, bool POLY>
void launch_iter_p(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                   hipEvent_t e1, hipStream_t s) {
  const PolyState* pin = POLY ? a.pst[q] : nullptr;
  PolyState* pout = POLY ? a.pst[q ^ 1] : nullptr;
  if (e0) {
    // the extended launch stamps the events at the kernel's own start and end
    hipExtLaunchKernelGGL((k_cg_iter<VT, XT, CT, L, BS, POLY>), dim3(a.blocks + (POLY ? 1 : 0)),
                          dim3(BS), 0, s, e0, e1, 0, a.m, A, (const CgState<XT>*)a.st[q], a.st[q ^ 1], a.p,
                          a.xlo, a.sc, a.snap, a.flag, (const double*)a.part[q ^ 1], a.part[q], a.blocks, a.xg,
                          q, fixed, a.np, a.Q, a.psys, pin, pout);
  } else {
    hipLaunchKernelGGL((k_cg_iter<VT, XT, CT, L, BS, POLY>), dim3(a.blocks + (POLY ? 1 : 0)),
                       dim3(BS), 0, s, a.m,
                       A, (const CgState<XT>*)a.st[q], a.st[q ^ 1], a.p, a.xlo, a.sc, a.snap, a.flag,
                       (const double*)a.part[q ^ 1], a.part[q], a.blocks, a.xg, q, fixed, a.np,
                       a.Q, a.psys, pin, pout);
  }
}

template <typename VT, typename XT, typename CT, int L, int BS>
void launch_iter_b(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                   hipEvent_t e1, hipStream_t s) {
  if (a.np > 0)
    launch_iter_p<VT, XT, CT, L, BS, true>(a, A, q, fixed, e0, e1, s);
  else
    launch_iter_p<VT, XT, CT, L, BS, false>(a, A, q, fixed, e0, e1, s);
}

template <typename VT, typename XT, typename CT, int L>
void launch_iter_l(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                   hipEvent_t e1, hipStream_t s) {
  if (a.threads == kCgSmallBlock)
    launch_iter_b<VT, XT, CT, L, kCgSmallBlock>(a, A, q, fixed, e0, e1, s);
  else
    launch_iter_b<VT, XT, CT, L, kCgLargeBlock>(a, A, q, fixed, e0, e1, s);
}

template <typename VT, typename XT, typename CT, int L, int BS, bool POLY>
void launch_refresh_p(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q,
                      hipStream_t s) {
  const PolyState* pin = POLY ? a.pst[q] : nullptr;
  hipLaunchKernelGGL((k_true_residual<VT, XT, CT, L, BS, POLY>), dim3(a.blocks), dim3(BS), 0, s,
                     a.m, A, (const double*)a.xhi, g, a.r64, a.st[q], a.np, a.Q, pin, a.part_ref);
  if (POLY)
    hipLaunchKernelGGL(k_poly_residual, dim3(1), dim3(kCgLargeBlock), 0, s, a.psys,
                       (const double*)a.part_ref, a.blocks, a.pst[q]);
  hipLaunchKernelGGL((k_cg_refresh<VT, XT, CT, L, BS, POLY>), dim3(a.blocks), dim3(BS), 0, s, a.m,
                     A, (const CgState<XT>*)a.st[q], a.st[q ^ 1], (const XT*)a.p,
                     (const double*)a.r64, a.part_ref, a.np, a.Q, a.psys, pin);
}

template <typename VT, typename XT, typename CT, int L, int BS>
void launch_refresh_b(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q,
                      hipStream_t s) {
  if (a.np > 0)
    launch_refresh_p<VT, XT, CT, L, BS, true>(a, A, g, q, s);
  else
    launch_refresh_p<VT, XT, CT, L, BS, false>(a, A, g, q, s);
}

template <typename VT, typename XT, typename CT, int L>
void launch_refresh_l(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q,
                      hipStream_t s) {
  if (a.threads == kCgSmallBlock)
    launch_refresh_b<VT, XT, CT, L, kCgSmallBlock>(a, A, g, q, s);
  else
    launch_refresh_b<VT, XT, CT, L, kCgLargeBlock>(a, A, g, q, s);
}

template <typename VT, typename XT, int L>
void launch_iter_halo(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                      hipEvent_t e1, hipStream_t s) {
  constexpr int BS = kCgSmallBlock;
  if (e0) {
    hipExtLaunchKernelGGL((k_cg_iter<VT, XT, int16_t, L, BS, false, true>), dim3(a.blocks),
                          dim3(BS), 0, s, e0, e1, 0, a.m, A, (const CgState<XT>*)a.st[q],
                          a.st[q ^ 1], a.p, a.xlo, a.sc, a.snap, a.flag, (const double*)a.part[q ^ 1], a.part[q],
                          a.blocks, a.xg, q, fixed, 0, (const XT*)nullptr,
                          (const PolySys*)nullptr, (const PolyState*)nullptr, (PolyState*)nullptr);
  } else {
    hipLaunchKernelGGL((k_cg_iter<VT, XT, int16_t, L, BS, false, true>), dim3(a.blocks), dim3(BS),
                       0, s, a.m, A, (const CgState<XT>*)a.st[q], a.st[q ^ 1], a.p, a.xlo, a.sc, a.snap, a.flag,
                       (const double*)a.part[q ^ 1], a.part[q], a.blocks, a.xg, q, fixed, 0,
                       (const XT*)nullptr, (const PolySys*)nullptr, (const PolyState*)nullptr,
                       (PolyState*)nullptr);
  }
}

template <typename VT, typename XT, typename CT>
void iter_dispatch(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                   hipEvent_t e1, hipStream_t s) {
  // staged neighbourhoods: float64 single solve without the polynomial
  // block, one slice per wave
  if constexpr (sizeof(XT) == 8) {
    if (A.hslot && a.np == 0 && a.threads == kCgSmallBlock) {
      switch (A.lanes) {
        case 2: launch_iter_halo<VT, XT, 2>(a, A, q, fixed, e0, e1, s); return;
        case 4: launch_iter_halo<VT, XT, 4>(a, A, q, fixed, e0, e1, s); return;
        default: launch_iter_halo<VT, XT, 8>(a, A, q, fixed, e0, e1, s); return;
      }
    }
  }
  switch (A.lanes) {
    case 2: launch_iter_l<VT, XT, CT, 2>(a, A, q, fixed, e0, e1, s); break;
    case 4: launch_iter_l<VT, XT, CT, 4>(a, A, q, fixed, e0, e1, s); break;
    default: launch_iter_l<VT, XT, CT, 8>(a, A, q, fixed, e0, e1, s); break;
  }
}

template <typename VT, typename XT, typename CT>
void refresh_dispatch(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q,
                      hipStream_t s) {
  switch (A.lanes) {
    case 2: launch_refresh_l<VT, XT, CT, 2>(a, A, g, q, s); break;
    case 4: launch_refresh_l<VT, XT, CT, 4>(a, A, g, q, s); break;
    default: launch_refresh_l<VT, XT, CT, 8>(a, A, g, q, s); break;
  }
}

template <typename XT>
bool args_ok(const CgArgs<XT>& a, const CgMatrix& A) {
  const bool poly_ok = a.np == 0 || (a.np >= 3 && a.np <= kMaxPoly && a.Q && a.psys &&
                                     a.pst[0] && a.pst[1] && a.xpoly);
  return a.blocks >= 1 && a.blocks <= kCgMaxBlocks && A.nslices >= 1 &&
         (a.threads == kCgSmallBlock || a.threads == kCgLargeBlock) &&
         (A.lanes == 2 || A.lanes == 4 || A.lanes == 8) && poly_ok;
}

}  // namespace

int sell_lanes(double mean_row) {
  if (mean_row > 192) return 8;
  if (mean_row > 24) return 4;
  return 2;
}

// Grids of one slice per wave stream each slice once, and XCD locality pays:
// two ranges per XCD measured 17.7 us per float32 terrain2d iteration against
// 18.8 in dispatch order and 18.3 with one range (one range leaves the XCD
// that holds the densest region with up to 12 % more work on clustered 3D
// data).  Grids of large blocks stride over the slices and keep the dispatch
// order (two ranges measured 3-5 % slower on a 1M-row matrix).
constexpr int kXcdChunks = 2;

void cg_grid(int64_t nslices, int* blocks, int* threads, int* xcd_chunks) {
  const int64_t ws = kCgSmallBlock / kWave, wl = kCgLargeBlock / kWave;
  const int64_t bs = (nslices + ws - 1) / ws;
  if (bs <= kCgMaxBlocks) {
    int64_t b = bs < 1 ? 1 : bs;
    constexpr int64_t q = (int64_t)kXcds * kXcdChunks;
    static_assert(kCgMaxBlocks % q == 0, "the rounded grid must stay within kCgMaxBlocks");
    int g = 0;
    if (b >= q) {
      // padding blocks find no slice and contribute zero partial sums
      b = (b + q - 1) / q * q;
      g = kXcdChunks;
    }
    *blocks = (int)b;
    *threads = kCgSmallBlock;
    *xcd_chunks = g;
    return;
  }
  const int64_t bl = (nslices + wl - 1) / wl;
  *blocks = (int)(bl > kCgMaxBlocks ? kCgMaxBlocks : bl);
  *threads = kCgLargeBlock;
  *xcd_chunks = 0;
}

template <typename VT, typename XT>
hipError_t cg_iterate(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                      hipEvent_t e1, hipStream_t s) {
  if (!args_ok(a, A) || (q != 0 && q != 1)) return hipErrorInvalidValue;
  if (A.col16)
    iter_dispatch<VT, XT, int16_t>(a, A, q, fixed, e0, e1, s);
  else
    iter_dispatch<VT, XT, int32_t>(a, A, q, fixed, e0, e1, s);
  return hipGetLastError();
}

template <typename VT, typename XT>
hipError_t cg_refresh(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q, int q_prev,
                      int restart, hipStream_t s) {
  if (!args_ok(a, A) || (q != 0 && q != 1) || (q_prev != 0 && q_prev != 1))
    return hipErrorInvalidValue;
  const int bs = 256;
  const dim3 eg((unsigned)((a.m + bs - 1) / bs));
  hipLaunchKernelGGL(k_fold_solution<XT>, eg, dim3(bs), 0, s, a.m, a.xhi, a.xlo);
  if (A.col16)
    refresh_dispatch<VT, XT, int16_t>(a, A, g, q, s);
  else
    refresh_dispatch<VT, XT, int32_t>(a, A, g, q, s);
  if (a.np > 0)
    hipLaunchKernelGGL(k_refresh_scalars<true>, dim3(1), dim3(kCgLargeBlock), 0, s, a.sc,
                       (const double*)a.part_ref, a.blocks, q_prev, restart, a.psys,
                       (const PolyState*)a.pst[q], a.pst[q ^ 1], a.xpoly);
  else
    hipLaunchKernelGGL(k_refresh_scalars<false>, dim3(1), dim3(kCgLargeBlock), 0, s, a.sc,
                       (const double*)a.part_ref, a.blocks, q_prev, restart, nullptr, nullptr,
                       nullptr, nullptr);
  return hipGetLastError();
}

template <typename XT>
hipError_t cg_setup(const CgArgs<XT>& a, const double* g, double rtol, double delta,
                    hipStream_t s) {
  const int bs = 256;
  const dim3 eg((unsigned)((a.m + bs - 1) / bs));
  hipLaunchKernelGGL(k_cg_clear<XT>, eg, dim3(bs), 0, s, a.m, a.dinv, a.xlo, a.p, a.st[0],
                     a.st[1], a.np ? a.pst[0] : nullptr, a.np ? a.pst[1] : nullptr,
                     (const double*)a.xpoly);
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kCgLargeBlock), 0, s, a.m, g,
                     a.np ? a.psys : nullptr, a.sc, rtol, delta);
  return hipGetLastError();
}

template hipError_t cg_iterate<double, double>(const CgArgs<double>&, const CgMatrix&, int, int,
                                               hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cg_iterate<float, float>(const CgArgs<float>&, const CgMatrix&, int, int,
                                             hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cg_refresh<double, double>(const CgArgs<double>&, const CgMatrix&,
                                               const double*, int, int, int, hipStream_t);
template hipError_t cg_refresh<float, float>(const CgArgs<float>&, const CgMatrix&, const double*,
                                             int, int, int, hipStream_t);
template hipError_t cg_setup<double>(const CgArgs<double>&, const double*, double, double,
                                     hipStream_t);
template hipError_t cg_setup<float>(const CgArgs<float>&, const double*, double, double,
                                    hipStream_t);

// ---------------------------------------------------------------------------
// Several right-hand sides (vector-valued data): NR independent solves of the
// same system in one kernel per iteration, each exactly the iteration above
// with its own scalars.  The matrix is streamed once for all of them; a
// neighbour's record holds its d and the (r, w, s) of every right-hand side,
// so it is gathered once per stored entry.
namespace {

// Steps per batch: the gathered records are (1 + 3 NR) values wide, so the
// batches are shorter than the single solve's to keep the same registers.
template <typename XT, int NR>
constexpr int kBatchN = sizeof(XT) == 4 ? (NR <= 2 ? 8 : 4) : (NR <= 2 ? 4 : 2);

template <typename XT, int U>
struct SliceHeadU {
  int64_t row, base;
  int32_t rowc;
  int steps;
  int32_t l[U];
  XT v[U];
};

template <typename VT, typename XT, typename CT, int U, bool HALO = false>
__device__ __forceinline__ void load_batch_u(const CgMatrix& A, int64_t base, int32_t rowc, int st,
                                             int steps, int32_t* l, XT* v) {
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const int16_t* __restrict__ slot = A.hslot;
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  // unconditional loads (at most 7 steps past a slice, inside the zeroed tail)
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const int64_t o = base + (int64_t)(st + t) * kWave;
    const int32_t c = HALO ? (int32_t)slot[o] : (int32_t)col[o];
    const XT x = (XT)val[o];
    const bool in = st + t < steps;
    l[t] = HALO ? (in ? c : 0) : rowc + (in ? c : 0);
    v[t] = in ? x : (XT)0;
  }
}

template <typename VT, typename XT, typename CT, int L, int U, bool HALO = false>
__device__ __forceinline__ void open_slice_u(int64_t m, int64_t slice, const CgMatrix& A,
                                             SliceHeadU<XT, U>& h) {
  constexpr int S = kWave / L;
  const int lane = threadIdx.x & (kWave - 1);
  h.row = slice * S + lane / L;
  h.rowc = (int32_t)(h.row < m ? h.row : m - 1);
  h.base = A.sptr[slice] + lane;
  h.steps = A.slen[slice] / L;
  load_batch_u<VT, XT, CT, U, HALO>(A, h.base, h.rowc, 0, h.steps, h.l, h.v);
}

// Row sums of an opened slice for every right-hand side: wn[k] =
// sum_e b_e u_k(col_e), complete in the lane with (lane % L) == 0.
// HALO: us[slot] holds u of every right-hand side for the slice's staged
// columns (interleaved, padded to kRhsPad).
template <typename XT, int NR>
struct alignas(kRhsPad<NR> * sizeof(XT)) URec {
  XT u[kRhsPad<NR>];
};
template <typename VT, typename XT, typename CT, int L, int U, int NR, bool HALO = false>
__device__ __forceinline__ void finish_slice_n(const SliceHeadU<XT, U>& h, const CgMatrix& A,
                                               const CgStateN<XT, NR>* __restrict__ sin,
                                               const XT* alpha, const XT* beta, XT* wn,
                                               const URec<XT, NR>* us = nullptr) {
  XT acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = (XT)0;
  int32_t cl[U], nl[U];
  XT cv[U], nv[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    cl[t] = h.l[t];
    cv[t] = h.v[t];
  }
  for (int st = U;; st += U) {
    const bool more = st < h.steps;
    if (more) load_batch_u<VT, XT, CT, U, HALO>(A, h.base, h.rowc, st, h.steps, nl, nv);
#pragma unroll
    for (int t = 0; t < U; ++t) {
      if constexpr (HALO) {
        const URec<XT, NR> r = us[cl[t]];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] += cv[t] * r.u[k];
      } else {
        const CgStateN<XT, NR> r = sin[cl[t]];
#pragma unroll
        for (int k = 0; k < NR; ++k)
          acc[k] += cv[t] * (r.d * r_next(r.r[k], s_next(r.w[k], r.s[k], beta[k]), alpha[k]));
      }
    }
    if (!more) break;
#pragma unroll
    for (int t = 0; t < U; ++t) {
      cl[t] = nl[t];
      cv[t] = nv[t];
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    XT a = acc[k];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
    wn[k] = a;
  }
}

template <typename VT, typename XT, typename CT, int L, int BS, int NR, bool HALO = false>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_cgn_iter(
    int64_t m, CgMatrix A, const CgStateN<XT, NR>* __restrict__ sin,
    CgStateN<XT, NR>* __restrict__ sout, XT* __restrict__ p, XT* __restrict__ xlo,
    CgScalarsN* __restrict__ sc, CgScalarsN* snap, int32_t* hflag,
    const double* __restrict__ part_in, double* __restrict__ part_out, int n_in, int xg, int q,
    int fixed) {
  constexpr int W = BS / kWave;
  constexpr int NPT = 6 * NR;
  constexpr int U = kBatchN<XT, NR>;
  __shared__ double ws[NPT][W];
  // this iteration's partials, per wave (added slice by slice, so that they
  // hold no registers across the streamed loop)
  __shared__ double ws_acc[NPT][W];
  __shared__ URec<XT, NR> us[HALO ? W : 1][HALO ? kHaloCapN<XT, NR> : 1];
  __shared__ int s_flag;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t wstride = (int64_t)gridDim.x * W;
  const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x, xg);
  int64_t slice = (int64_t)blk * W + wave;
  SliceHeadU<XT, U> h;
  const bool have = slice < A.nslices;
  if (have) open_slice_u<VT, XT, CT, L, U, HALO>(m, slice, A, h);
  // the previous kernel's partials, one right-hand side at a time
  if (!fixed) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      double r6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int b = threadIdx.x; b < n_in; b += BS) {
#pragma unroll
        for (int t = 0; t < 6; ++t) r6[t] += part_in[(int64_t)b * NPT + 6 * k + t];
      }
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const double v = wave_sum(r6[t]);
        if (lane == 0) ws[6 * k + t][wave] = v;
      }
    }
  }
  if (threadIdx.x == 0) s_flag = sc->done;
  __syncthreads();
  if (s_flag) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && snap) *snap = *sc;
    return;
  }
  XT alpha[NR], beta[NR];
  double alpha_d[NR], gamma_d[NR], rr_d[NR];
  bool act[NR];
  int flag = 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    act[k] = sc->active[k] != 0;
    double gamma, rr, a, b;
    if (fixed) {
      gamma = sc->fix_gamma[k];
      rr = sc->fix_rr[k];
      a = sc->fix_alpha[k];
      b = sc->fix_beta[k];
    } else {
      double v[6];
      for (int t = 0; t < 6; ++t) {
        double x = 0.0;
#pragma unroll 4
        for (int w = 0; w < W; ++w) x += ws[6 * k + t][w];
        v[t] = x;
      }
      gamma = v[0];
      rr = v[2];
      b = gamma / sc->gam[q ^ 1][k];
      a = gamma / (v[1] + b * (v[3] + v[4]) + b * b * v[5]);
    }
    if (act[k]) {
      if (!__builtin_isfinite(rr) || !__builtin_isfinite(gamma)) {
        flag = 2;
      } else if (rr <= sc->trigger2[k]) {
        flag = flag > 1 ? flag : 1;
      } else if (!(a > 0.0) || !__builtin_isfinite(a) || !__builtin_isfinite(b)) {
        flag = 2;
      }
    } else {
      a = 0.0;
      b = 0.0;
    }
    alpha_d[k] = a;
    gamma_d[k] = gamma;
    rr_d[k] = rr;
    alpha[k] = (XT)a;
    beta[k] = (XT)b;
  }
  if (flag) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      for (int k = 0; k < NR; ++k) sc->rr[k] = rr_d[k];
      sc->done = flag;
      if (snap) *snap = *sc;
      if (hflag) *hflag = flag;
    }
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < NPT; ++t) ws_acc[t][wave] = 0.0;
  }
  for (; have && slice < A.nslices; slice += wstride) {
    if (slice != (int64_t)blk * W + wave)
      open_slice_u<VT, XT, CT, L, U, HALO>(m, slice, A, h);
    XT wn[NR];
    if constexpr (HALO) {
      // u of every right-hand side, once per distinct column of the slice
      const int n = A.hcount[slice];
      const int64_t off = A.hptr[slice], first = slice * (kWave / L);
      wave_sync();
      for (int i = lane; i < n; i += kWave) {
        const CgStateN<XT, NR> r = sin[first + A.hrow[off + i]];
        URec<XT, NR> o;
#pragma unroll
        for (int k = 0; k < kRhsPad<NR>; ++k)
          o.u[k] = k < NR ? r.d * r_next(r.r[k], s_next(r.w[k], r.s[k], beta[k]), alpha[k])
                          : (XT)0;
        us[wave][i] = o;
      }
      wave_sync();
      finish_slice_n<VT, XT, CT, L, U, NR, true>(h, A, sin, alpha, beta, wn, us[wave]);
    } else {
      finish_slice_n<VT, XT, CT, L, U, NR>(h, A, sin, alpha, beta, wn);
    }
    double part[NPT];
#pragma unroll
    for (int t = 0; t < NPT; ++t) part[t] = 0.0;
    if ((lane & (L - 1)) == 0 && h.row < m) {
      const int64_t row = h.row;
      const CgStateN<XT, NR> t = sin[row];
      CgStateN<XT, NR> o;
      o.d = t.d;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if (act[k]) {
          const XT pn = t.d * t.r[k] + beta[k] * p[k * m + row];
          const XT sn = s_next(t.w[k], t.s[k], beta[k]);
          const XT rn = r_next(t.r[k], sn, alpha[k]);
          const XT un = t.d * rn;
          p[k * m + row] = pn;
          xlo[k * m + row] = xlo[k * m + row] + alpha[k] * pn;
          o.r[k] = rn;
          o.w[k] = wn[k];
          o.s[k] = sn;
          part[6 * k + 0] += (double)rn * (double)un;
          part[6 * k + 1] += (double)wn[k] * (double)un;
          part[6 * k + 2] += (double)rn * (double)rn;
          part[6 * k + 3] += (double)un * (double)sn;
          part[6 * k + 4] += (double)pn * (double)wn[k];
          part[6 * k + 5] += (double)pn * (double)sn;
        } else {
          o.r[k] = t.r[k];
          o.w[k] = t.w[k];
          o.s[k] = t.s[k];
        }
      }
      sout[row] = o;
    }
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      const double v = wave_sum(part[t]);
      if (lane == 0) ws_acc[t][wave] += v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 0; t < NPT; ++t) {
      double v = 0.0;
      for (int w = 0; w < W; ++w) v += ws_acc[t][w];
      part_out[(int64_t)blk * NPT + t] = v;
    }
    if (blockIdx.x == 0) {
      for (int k = 0; k < NR; ++k) {
        sc->gam[q][k] = gamma_d[k];
        sc->rr[k] = rr_d[k];
      }
      sc->iter += 1;
      if (snap) *snap = *sc;  // the chunk's last launch: the host's slot
    }
  }
  (void)alpha_d;
}

// x_hi += x_lo and x_lo = 0 for every right-hand side ([nr][m]).
template <typename XT>
__global__ void k_cgn_fold(int64_t n, double* __restrict__ xhi, XT* __restrict__ xlo) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  xhi[j] += (double)xlo[j];
  xlo[j] = (XT)0;
}

// Float64 residuals r64_k = g_k - (B + lambda I) x_hi,k, and r_k = (XT) r64_k
// into the records of st.
template <typename VT, typename XT, typename CT, int L, int BS, int NR>
__global__ __launch_bounds__(BS) void k_cgn_true_residual(int64_t m, CgMatrix A,
                                                          const double* __restrict__ xhi,
                                                          const double* __restrict__ g,
                                                          double* __restrict__ r64,
                                                          CgStateN<XT, NR>* __restrict__ st) {
  constexpr int S = kWave / L;
  constexpr int W = BS / kWave;
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  const int lane = threadIdx.x & (kWave - 1);
  for (int64_t slice = (int64_t)blockIdx.x * W + threadIdx.x / kWave; slice < A.nslices;
       slice += (int64_t)gridDim.x * W) {
    const int64_t row = slice * S + lane / L;
    const int32_t rowc = (int32_t)(row < m ? row : m - 1);
    const int64_t base = A.sptr[slice] + lane;
    const int steps = A.slen[slice] / L;
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    for (int s = 0; s < steps; ++s) {
      const int64_t o = base + (int64_t)s * kWave;
      const double b = (double)val[o];
      const int32_t l = rowc + (int32_t)col[o];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] += b * xhi[k * m + l];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, kWave);
    }
    if ((lane & (L - 1)) == 0 && row < m) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const double rv = g[k * m + row] - acc[k];
        r64[k * m + row] = rv;
        st[row].r[k] = (XT)rv;
      }
    }
  }
}

// w_k = B D^-1 r_k from the records of sin, written with the carried s and d
// to sout; partials of r.u, w.u, r64.r64, p.w, u.s, p.s per right-hand side.
template <typename VT, typename XT, typename CT, int L, int BS, int NR>
__global__ __launch_bounds__(BS) void k_cgn_refresh(int64_t m, CgMatrix A,
                                                    const CgStateN<XT, NR>* __restrict__ sin,
                                                    CgStateN<XT, NR>* __restrict__ sout,
                                                    const XT* __restrict__ p,
                                                    const double* __restrict__ r64,
                                                    double* __restrict__ part_out) {
  constexpr int S = kWave / L;
  constexpr int W = BS / kWave;
  constexpr int NPT = 6 * NR;
  __shared__ double ws[NPT][W];
  const CT* __restrict__ col = static_cast<const CT*>(A.col);
  const VT* __restrict__ val = static_cast<const VT*>(A.val);
  const int lane = threadIdx.x & (kWave - 1);
  double part[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) part[t] = 0.0;
  for (int64_t slice = (int64_t)blockIdx.x * W + threadIdx.x / kWave; slice < A.nslices;
       slice += (int64_t)gridDim.x * W) {
    const int64_t row = slice * S + lane / L;
    const int32_t rowc = (int32_t)(row < m ? row : m - 1);
    const int64_t base = A.sptr[slice] + lane;
    const int steps = A.slen[slice] / L;
    XT acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = (XT)0;
    for (int s = 0; s < steps; ++s) {
      const int64_t o = base + (int64_t)s * kWave;
      const XT b = (XT)val[o];
      const CgStateN<XT, NR> r = sin[rowc + (int32_t)col[o]];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] += b * (r.d * r.r[k]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, kWave);
    }
    if ((lane & (L - 1)) == 0 && row < m) {
      const CgStateN<XT, NR> t = sin[row];
      CgStateN<XT, NR> o = t;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const XT u = t.d * t.r[k];
        const XT pj = p[k * m + row];
        o.w[k] = acc[k];
        const double r64j = r64[k * m + row];
        part[6 * k + 0] += (double)t.r[k] * (double)u;
        part[6 * k + 1] += (double)acc[k] * (double)u;
        part[6 * k + 2] += r64j * r64j;
        part[6 * k + 3] += (double)pj * (double)acc[k];
        part[6 * k + 4] += (double)u * (double)t.s[k];
        part[6 * k + 5] += (double)pj * (double)t.s[k];
      }
      sout[row] = o;
    }
  }
  block_sums<NPT, W, false>(part, ws);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < NPT; ++t) part_out[(int64_t)blockIdx.x * NPT + t] = part[t];
  }
}

// After a refresh, per right-hand side: the true residual, convergence
// (a converged solve is frozen), the next trigger and the scalars of the next
// iteration (as k_refresh_scalars); done for the batch.
template <int NR>
__global__ __launch_bounds__(kCgLargeBlock) void k_cgn_refresh_scalars(
    CgScalarsN* __restrict__ sc, const double* __restrict__ part, int n, int q_prev,
    int restart) {
  constexpr int W = kCgLargeBlock / kWave;
  constexpr int NPT = 6 * NR;
  __shared__ double ws[NPT][W];
  double v[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) v[t] = 0.0;
  for (int b = threadIdx.x; b < n; b += kCgLargeBlock) {
#pragma unroll
    for (int t = 0; t < NPT; ++t) v[t] += part[(int64_t)b * NPT + t];
  }
  block_sums<NPT, W, false>(v, ws);
  if (threadIdx.x != 0) return;
  int bad = 0, left = 0;
  for (int k = 0; k < NR; ++k) {
    if (!sc->active[k]) {
      sc->fix_gamma[k] = sc->fix_alpha[k] = sc->fix_beta[k] = sc->fix_rr[k] = 0.0;
      continue;
    }
    const double gamma = v[6 * k], delta = v[6 * k + 1], rr = v[6 * k + 2];
    const double beta = restart ? 0.0 : gamma / sc->gam[q_prev][k];
    const double ps = delta + beta * (v[6 * k + 3] + v[6 * k + 4]) + beta * beta * v[6 * k + 5];
    const double alpha = gamma / ps;
    sc->rr_true[k] = rr;
    sc->rr[k] = rr;
    sc->fix_rr[k] = rr;
    sc->fix_gamma[k] = gamma;
    sc->fix_beta[k] = beta;
    sc->fix_alpha[k] = alpha;
    const double trig = sc->delta2 * rr;
    sc->trigger2[k] = trig > sc->tol2[k] ? trig : sc->tol2[k];
    if (!__builtin_isfinite(rr) || !__builtin_isfinite(gamma)) {
      bad = 1;
    } else if (rr <= sc->tol2[k]) {
      sc->active[k] = 0;
      sc->conv_iter[k] = sc->iter;
      sc->fix_alpha[k] = sc->fix_beta[k] = 0.0;
    } else if (!(ps > 0.0) || !__builtin_isfinite(alpha) || !__builtin_isfinite(beta)) {
      bad = 1;
    } else {
      ++left;
    }
  }
  sc->done = bad ? 2 : (left == 0 ? 3 : 0);
}

template <typename XT, int NR>
__global__ void k_cgn_clear(int64_t m, const XT* __restrict__ dinv, XT* __restrict__ xlo,
                            XT* __restrict__ p, CgStateN<XT, NR>* __restrict__ s0,
                            CgStateN<XT, NR>* __restrict__ s1) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  CgStateN<XT, NR> t;
  t.d = dinv[j];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    xlo[k * m + j] = (XT)0;
    p[k * m + j] = (XT)0;
    t.r[k] = t.w[k] = t.s[k] = (XT)0;
  }
  s0[j] = t;
  s1[j] = t;
}

// ||g_k||^2 and the initial scalars (single block, fixed order).
__global__ __launch_bounds__(kCgLargeBlock) void k_cgn_init(int64_t m, int nr,
                                                           const double* __restrict__ g,
                                                           CgScalarsN* __restrict__ sc,
                                                           double rtol, double delta) {
  constexpr int W = kCgLargeBlock / kWave;
  __shared__ double ws[1][W];
  for (int k = 0; k < nr; ++k) {
    double v[1] = {0.0};
    for (int64_t j = threadIdx.x; j < m; j += kCgLargeBlock) v[0] += g[k * m + j] * g[k * m + j];
    block_sums<1, W, true>(v, ws);
    if (threadIdx.x == 0) {
      sc->gg[k] = v[0];
      sc->tol2[k] = rtol * rtol * v[0];
      sc->trigger2[k] = sc->tol2[k];
      sc->rr[k] = sc->rr_true[k] = v[0];
      sc->gam[0][k] = sc->gam[1][k] = 1.0;
      sc->fix_gamma[k] = sc->fix_alpha[k] = sc->fix_beta[k] = sc->fix_rr[k] = 0.0;
      sc->active[k] = 1;
      sc->conv_iter[k] = -1;
    }
  }
  if (threadIdx.x == 0) {
    for (int k = nr; k < kMaxRhs; ++k) sc->active[k] = 0;
    sc->delta2 = delta * delta;
    sc->done = 0;
    sc->iter = 0;
  }
}

template <typename VT, typename XT, typename CT, int L, int BS, int NR, bool HALO>
void cgn_iter_launch_h(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                       hipEvent_t e1, hipStream_t s) {
  using St = CgStateN<XT, NR>;
  if (e0) {
    hipExtLaunchKernelGGL((k_cgn_iter<VT, XT, CT, L, BS, NR, HALO>), dim3(a.blocks), dim3(BS), 0,
                          s, e0, e1, 0, a.m, A, (const St*)a.st[q], (St*)a.st[q ^ 1], a.p, a.xlo,
                          a.sc, a.snap, a.flag, (const double*)a.part[q ^ 1], a.part[q], a.blocks,
                          a.xg, q, fixed);
  } else {
    hipLaunchKernelGGL((k_cgn_iter<VT, XT, CT, L, BS, NR, HALO>), dim3(a.blocks), dim3(BS), 0, s,
                       a.m, A, (const St*)a.st[q], (St*)a.st[q ^ 1], a.p, a.xlo, a.sc, a.snap,
                       a.flag, (const double*)a.part[q ^ 1], a.part[q], a.blocks, a.xg, q, fixed);
  }
}

// Staged neighbourhoods when the layout carries them (one slice per wave).
template <typename VT, typename XT, typename CT, int L, int BS, int NR>
void cgn_iter_launch(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                     hipEvent_t e1, hipStream_t s) {
  if constexpr (BS == kCgSmallBlock) {
    if (A.hslot) {
      cgn_iter_launch_h<VT, XT, CT, L, BS, NR, true>(a, A, q, fixed, e0, e1, s);
      return;
    }
  }
  cgn_iter_launch_h<VT, XT, CT, L, BS, NR, false>(a, A, q, fixed, e0, e1, s);
}

template <typename VT, typename XT, typename CT, int L, int BS, int NR>
void cgn_refresh_launch(const CgArgsN<XT>& a, const CgMatrix& A, const double* g, int q,
                        hipStream_t s) {
  using St = CgStateN<XT, NR>;
  hipLaunchKernelGGL((k_cgn_true_residual<VT, XT, CT, L, BS, NR>), dim3(a.blocks), dim3(BS), 0,
                     s, a.m, A, (const double*)a.xhi, g, a.r64, (St*)a.st[q]);
  hipLaunchKernelGGL((k_cgn_refresh<VT, XT, CT, L, BS, NR>), dim3(a.blocks), dim3(BS), 0, s, a.m,
                     A, (const St*)a.st[q], (St*)a.st[q ^ 1], (const XT*)a.p,
                     (const double*)a.r64, a.part_ref);
}

// Dispatch over (lanes, block size, right-hand sides); `Op` is one of the two
// launchers above.
template <typename VT, typename XT, typename CT, int L, int BS, typename F>
void cgn_nr(int nr, F&& f) {
  switch (nr) {
    case 2: f(std::integral_constant<int, 2>()); break;
    case 3: f(std::integral_constant<int, 3>()); break;
    default: f(std::integral_constant<int, 4>()); break;
  }
}

template <typename XT>
bool argsn_ok(const CgArgsN<XT>& a, const CgMatrix& A) {
  return a.blocks >= 1 && a.blocks <= kCgMaxBlocks && A.nslices >= 1 && a.nr >= 2 &&
         a.nr <= kMaxRhs && (a.threads == kCgSmallBlock || a.threads == kCgLargeBlock) &&
         (A.lanes == 2 || A.lanes == 4 || A.lanes == 8);
}

template <typename VT, typename XT, typename CT, int L>
void cgn_iter_l(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                hipEvent_t e1, hipStream_t s) {
  auto go = [&](auto nr) {
    if (a.threads == kCgSmallBlock)
      cgn_iter_launch<VT, XT, CT, L, kCgSmallBlock, decltype(nr)::value>(a, A, q, fixed, e0, e1,
                                                                        s);
    else
      cgn_iter_launch<VT, XT, CT, L, kCgLargeBlock, decltype(nr)::value>(a, A, q, fixed, e0, e1,
                                                                        s);
  };
  cgn_nr<VT, XT, CT, L, 0>(a.nr, go);
}

template <typename VT, typename XT, typename CT, int L>
void cgn_refresh_l(const CgArgsN<XT>& a, const CgMatrix& A, const double* g, int q,
                   hipStream_t s) {
  auto go = [&](auto nr) {
    if (a.threads == kCgSmallBlock)
      cgn_refresh_launch<VT, XT, CT, L, kCgSmallBlock, decltype(nr)::value>(a, A, g, q, s);
    else
      cgn_refresh_launch<VT, XT, CT, L, kCgLargeBlock, decltype(nr)::value>(a, A, g, q, s);
  };
  cgn_nr<VT, XT, CT, L, 0>(a.nr, go);
}

template <typename VT, typename XT, typename CT>
void cgn_iter_c(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                hipEvent_t e1, hipStream_t s) {
  switch (A.lanes) {
    case 2: cgn_iter_l<VT, XT, CT, 2>(a, A, q, fixed, e0, e1, s); break;
    case 4: cgn_iter_l<VT, XT, CT, 4>(a, A, q, fixed, e0, e1, s); break;
    default: cgn_iter_l<VT, XT, CT, 8>(a, A, q, fixed, e0, e1, s); break;
  }
}

template <typename VT, typename XT, typename CT>
void cgn_refresh_c(const CgArgsN<XT>& a, const CgMatrix& A, const double* g, int q,
                   hipStream_t s) {
  switch (A.lanes) {
    case 2: cgn_refresh_l<VT, XT, CT, 2>(a, A, g, q, s); break;
    case 4: cgn_refresh_l<VT, XT, CT, 4>(a, A, g, q, s); break;
    default: cgn_refresh_l<VT, XT, CT, 8>(a, A, g, q, s); break;
  }
}

}  // namespace

template <typename VT, typename XT>
hipError_t cgn_iterate(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed,
                       hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  if (!argsn_ok(a, A) || (q != 0 && q != 1)) return hipErrorInvalidValue;
  if (A.col16)
    cgn_iter_c<VT, XT, int16_t>(a, A, q, fixed, e0, e1, s);
  else
    cgn_iter_c<VT, XT, int32_t>(a, A, q, fixed, e0, e1, s);
  return hipGetLastError();
}

template <typename VT, typename XT>
hipError_t cgn_refresh(const CgArgsN<XT>& a, const CgMatrix& A, const double* g, int q,
                       int q_prev, int restart, hipStream_t s) {
  if (!argsn_ok(a, A) || (q != 0 && q != 1) || (q_prev != 0 && q_prev != 1))
    return hipErrorInvalidValue;
  const int bs = 256;
  const int64_t n = (int64_t)a.nr * a.m;
  hipLaunchKernelGGL(k_cgn_fold<XT>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, n,
                     a.xhi, a.xlo);
  if (A.col16)
    cgn_refresh_c<VT, XT, int16_t>(a, A, g, q, s);
  else
    cgn_refresh_c<VT, XT, int32_t>(a, A, g, q, s);
  switch (a.nr) {
    case 2:
      hipLaunchKernelGGL(k_cgn_refresh_scalars<2>, dim3(1), dim3(kCgLargeBlock), 0, s, a.sc,
                         (const double*)a.part_ref, a.blocks, q_prev, restart);
      break;
    case 3:
      hipLaunchKernelGGL(k_cgn_refresh_scalars<3>, dim3(1), dim3(kCgLargeBlock), 0, s, a.sc,
                         (const double*)a.part_ref, a.blocks, q_prev, restart);
      break;
    default:
      hipLaunchKernelGGL(k_cgn_refresh_scalars<4>, dim3(1), dim3(kCgLargeBlock), 0, s, a.sc,
                         (const double*)a.part_ref, a.blocks, q_prev, restart);
      break;
  }
  return hipGetLastError();
}

template <typename XT>
hipError_t cgn_setup(const CgArgsN<XT>& a, const double* g, double rtol, double delta,
                     hipStream_t s) {
  if (a.nr < 2 || a.nr > kMaxRhs) return hipErrorInvalidValue;
  const int bs = 256;
  const dim3 eg((unsigned)((a.m + bs - 1) / bs));
  switch (a.nr) {
    case 2:
      hipLaunchKernelGGL((k_cgn_clear<XT, 2>), eg, dim3(bs), 0, s, a.m, a.dinv, a.xlo, a.p,
                         (CgStateN<XT, 2>*)a.st[0], (CgStateN<XT, 2>*)a.st[1]);
      break;
    case 3:
      hipLaunchKernelGGL((k_cgn_clear<XT, 3>), eg, dim3(bs), 0, s, a.m, a.dinv, a.xlo, a.p,
                         (CgStateN<XT, 3>*)a.st[0], (CgStateN<XT, 3>*)a.st[1]);
      break;
    default:
      hipLaunchKernelGGL((k_cgn_clear<XT, 4>), eg, dim3(bs), 0, s, a.m, a.dinv, a.xlo, a.p,
                         (CgStateN<XT, 4>*)a.st[0], (CgStateN<XT, 4>*)a.st[1]);
      break;
  }
  hipLaunchKernelGGL(k_cgn_init, dim3(1), dim3(kCgLargeBlock), 0, s, a.m, a.nr, g, a.sc, rtol,
                     delta);
  return hipGetLastError();
}

template hipError_t cgn_iterate<double, double>(const CgArgsN<double>&, const CgMatrix&, int, int,
                                                hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cgn_iterate<float, float>(const CgArgsN<float>&, const CgMatrix&, int, int,
                                              hipEvent_t, hipEvent_t, hipStream_t);
template hipError_t cgn_refresh<double, double>(const CgArgsN<double>&, const CgMatrix&,
                                                const double*, int, int, int, hipStream_t);
template hipError_t cgn_refresh<float, float>(const CgArgsN<float>&, const CgMatrix&,
                                              const double*, int, int, int, hipStream_t);
template hipError_t cgn_setup<double>(const CgArgsN<double>&, const double*, double, double,
                                      hipStream_t);
template hipError_t cgn_setup<float>(const CgArgsN<float>&, const double*, double, double,
                                     hipStream_t);

}  // namespace rbf
