// Device scalars, per-row state and argument bundles of the conjugate-gradient kernels.
#pragma once

#include "internal.h"

namespace rbf {

// CG blocks hold 256 threads (4 waves) while a grid of one slice per wave has
// at most kCgMaxBlocks blocks, else 1024 threads (16 waves).  Every block of a
// kernel reduces all partial sums of the previous kernel, a cost quadratic in
// the block count that kCgMaxBlocks bounds; small blocks keep the waves of a
// block from waiting on one another at its barriers.
constexpr int kCgSmallBlock = 256;
constexpr int kCgLargeBlock = 1024;
constexpr int kCgMaxBlocks = 1024;
// Entries past the last slice that every stored-matrix array (columns and
// values) carries, zeroed: a CG kernel loads whole batches of 8 steps of 64
// entries, so a batch may run up to 7 steps past the end of its slice.
constexpr int64_t kSellTail = 8 * 64;

// Scalars of one CG solve, kept in device memory.  Each is written by block 0
// of one kernel and read by later kernels (or the host) only; the per-parity
// pairs let an iteration read its predecessor's value while writing its own.
struct CgScalars {
  double gam[2];     // gamma = r . u of the iteration run on state buffer q, at [q]
  double alp[2];     // alpha of that iteration, at [q] (reported only)
  double fix_gamma;  // gamma, alpha, beta, ||r||^2 of the first iteration after a
  double fix_alpha;  // float64 residual (set by the refresh)
  double fix_beta;
  double fix_rr;
  double rr;         // ||r||^2 of the iterated residual (last seen)
  double rr_true;    // ||g - (B + lambda I) x||^2 at the last float64 recomputation
  double gg;         // ||g||^2
  double tol2;       // rtol^2 * gg
  double delta2;     // reliable-update factor squared
  double trigger2;   // iterated ||r||^2 at which an iteration raises the flag
  int64_t iter;      // executed iterations
  int32_t done;      // 0 running, 1 trigger reached, 2 breakdown, 3 converged
  int32_t pad_;
};

// Per-row state read by neighbouring rows: residual r, w = B D^-1 r, the
// recurrence s = B p, and the Jacobi scale d = 1 / (b_jj + lambda).  One
// aligned record per row, so a neighbour's whole state is one vector load.
template <typename XT>
struct alignas(4 * sizeof(XT)) CgState {
  XT r, w, s, d;
};

// Linear polynomial reproduction (Section 3, eq. 10) borders B with the
// blocks Q = A^T P (one column per basis function, per solver row),
// C = P^T P and e = P^T h, in the scaled basis P_i = ((x_i - o) / s, 1) with
// o and s the centre and half-extent of the points' bounding box.  Those d + 1
// unknowns are few, so every CG block keeps and updates them itself, in
// float64, from the same inputs in the same order: a replicated block of the
// iteration.  Their preconditioner block is C^-1 (block Jacobi), the rows of B
// keep D^-1.
constexpr int kMaxPoly = 4;
struct PolySys {
  double C[kMaxPoly][kMaxPoly];   // P^T P, zero past np
  double Ci[kMaxPoly][kMaxPoly];  // its inverse, zero past np
  double e[kMaxPoly];             // P^T h
  int32_t np;                     // d + 1
  int32_t bad;                    // P^T P is not positive definite
};
// The polynomial unknowns' share of the CG state (see CgState), with the
// search direction p and the solution x, which the rows of B keep apart,
// and what an iteration's blocks need of it, formed once by the launch that
// writes the state: u = C^-1 r, C^-1 s, C u and the products r.u, r.r, u.s,
// p.s, u.C u, p.C u.
struct PolyState {
  double r[kMaxPoly], w[kMaxPoly], s[kMaxPoly], p[kMaxPoly], x[kMaxPoly];
  double u[kMaxPoly], cis[kMaxPoly], cu[kMaxPoly];
  double ru, rr, us, ps, ucu, pcu;
};
// Partial sums per block: the six dot products, then Q^T u (or Q^T x).
constexpr int kCgParts = 6 + kMaxPoly;
// The scaled basis: coordinate d enters as (x_d - o[d]) / s[d].
struct PolyBasis {
  double o[3], s[3];
};

template <typename XT>
struct CgArgs {
  int64_t m;
  CgState<XT>* st[2];  // state, double-buffered: an iteration reads one, writes the other
  XT* p;               // search direction (read and written by its own row only)
  XT* xlo;             // iterated correction of the solution
  const XT* dinv;
  double* xhi;         // float64 solution
  double* r64;         // float64 true residual
  CgScalars* sc;
  // host snapshot slot (device address of pinned, coherent host memory) that
  // the launch copies the scalars into when it ends a chunk; NULL otherwise
  CgScalars* snap;
  // a pinned, coherent host word that the iteration raising a flag (1
  // reliable-update trigger, 2 breakdown) also sets, so that the host stops
  // queueing launches that would return at entry; NULL: none
  int32_t* flag;
  double* part[2];     // [kCgParts * blocks] partials of an iteration, by state buffer
  double* part_ref;    // [kCgParts * blocks] partials of a refresh
  int blocks;          // grid of every slice kernel
  int threads;         // its block size: kCgSmallBlock or kCgLargeBlock
  int xg;              // XCD chunks of the iteration kernel (see cg_grid)
  // polynomial block (np = 0: none)
  int np;
  const XT* Q;            // [np][m], Q[t * m + row]
  const PolySys* psys;
  PolyState* pst[2];      // by state buffer, as st
  double* xpoly;          // [kMaxPoly] solution at the last refresh (start value on entry)
};

// The stored matrix in the solver's sliced-ELL layout.  Rows are taken in
// slices of S = 64 / L consecutive rows; each row of a slice gets L lanes of a
// wave.  Slice s starts at sptr[s] and holds slen[s] entries per row (the
// longest row of the slice, rounded up to a multiple of L); entry k of row
// i = j - s S sits at sptr[s] + (k / L) * 64 + i * L + (k % L), so every
// wave-wide load is one contiguous 64-entry run.  Columns are stored as
// l - j (int16 when every |l - j| fits, else int32); padding entries have
// delta 0 and value 0.
struct CgMatrix {
  const int64_t* sptr;
  const int32_t* slen;
  int64_t nslices;
  const void* col;
  bool col16;
  const void* val;  // VT
  int lanes;        // L: lanes per row (2, 4 or 8)
  // Neighbourhoods for the LDS-staged iteration (null when not built): per
  // slice the sorted distinct columns its entries reference (hrow: offsets
  // from the slice's first row, at hptr[s]; hcount[s] of them), and per
  // stored entry the rank of its column among them (hslot).
  const int16_t* hslot;
  const int16_t* hrow;
  const int64_t* hptr;
  const int32_t* hcount;
};
// Column range (bits of a wave's bitmap) a slice may span to be staged, and
// the most distinct columns one wave stages (its LDS holds one float64 u per
// column).  Staging serves the float64 iteration only: with float32 records
// the global gathers measured as fast.
constexpr int kHaloSpan = 16384;
constexpr int kHaloCap = 1024;
// ... and for the batched iteration, which stages one u per right-hand side
// in 8 KB of LDS per wave.
// The u values of a column are interleaved (NR rounded up to a power of two),
// so one LDS load serves every right-hand side.
template <int NR>
constexpr int kRhsPad = NR == 3 ? 4 : NR;
template <typename XT, int NR>
constexpr int kHaloCapN = 8192 / (kRhsPad<NR> * (int)sizeof(XT));
inline int halo_cap_n(int nr, int xt_bytes) { return 8192 / ((nr == 3 ? 4 : nr) * xt_bytes); }
hipError_t launch_halo_count(const CgMatrix& A, int64_t ms, int cap, int32_t* hcount,
                             hipStream_t s);
hipError_t launch_halo_fill(const CgMatrix& A, int64_t ms, const int32_t* hcount,
                            const int64_t* hptr, int16_t* hrow, int16_t* hslot, hipStream_t s);

__host__ __device__ inline int64_t sell_pos(const int64_t* sptr, int lanes, int64_t j, int64_t k) {
  const int64_t rows = 64 / lanes;
  const int64_t s = j / rows, i = j - s * rows;
  return sptr[s] + (k / lanes) * 64 + i * lanes + (k % lanes);
}

int sell_lanes(double mean_row);
// Grid (blocks, threads per block) of the slice kernels for nslices slices,
// and the XCD chunking of the iteration kernels: with xcd_chunks = G > 0 the
// block count is a multiple of 8 G and each XCD streams G contiguous ranges
// of slices (0: blocks in dispatch order).
void cg_grid(int64_t nslices, int* blocks, int* threads, int* xcd_chunks);

// One CG iteration on state buffer q (reads st[q], writes st[q ^ 1]).  fixed:
// the first iteration after a refresh, which takes its scalars from the
// refresh instead of from partial sums.  With e0/e1 (may be null) the launch
// stamps the two events at the kernel's start and end.
template <typename VT, typename XT>
hipError_t cg_iterate(const CgArgs<XT>& a, const CgMatrix& A, int q, int fixed, hipEvent_t e0,
                      hipEvent_t e1, hipStream_t s);
// Reliable update on state buffer q: x_hi += x_lo, float64 residual
// r64 = g - (B + lambda I) x_hi, r = (XT) r64, w = B D^-1 r written to
// st[q ^ 1] (with s, d carried over), then the scalars of the next iteration
// (restart: beta = 0; otherwise the direction is kept).  q_prev is the state
// buffer of the last executed iteration (its gamma is the previous one).
template <typename VT, typename XT>
hipError_t cg_refresh(const CgArgs<XT>& a, const CgMatrix& A, const double* g, int q, int q_prev,
                      int restart, hipStream_t s);
// x_lo, p and both state buffers cleared (s = 0, d = D^-1); scalars from g.
template <typename XT>
hipError_t cg_setup(const CgArgs<XT>& a, const double* g, double rtol, double delta,
                    hipStream_t s);

// ---- several right-hand sides (vector-valued data) ------------------------
// nr independent CG solves of the same B in one kernel per iteration: the
// matrix is streamed once for all of them, and the state of a row for all
// right-hand sides is one record, gathered together.
constexpr int kMaxRhs = 4;

template <typename XT, int NR>
struct alignas(16) CgStateN {
  XT d;
  XT r[NR], w[NR], s[NR];
};

// Scalars of a batched solve: as CgScalars, per right-hand side.  A solve
// whose float64 residual met its tolerance at a refresh is frozen (active 0):
// its state is carried unchanged.  done: 0 running, 1 some trigger reached
// (every right-hand side is refreshed), 2 breakdown, 3 all converged.
struct CgScalarsN {
  double gam[2][kMaxRhs];
  double fix_gamma[kMaxRhs], fix_alpha[kMaxRhs], fix_beta[kMaxRhs], fix_rr[kMaxRhs];
  double rr[kMaxRhs], rr_true[kMaxRhs], gg[kMaxRhs], tol2[kMaxRhs], trigger2[kMaxRhs];
  double delta2;
  int64_t iter;
  int64_t conv_iter[kMaxRhs];  // iterations when the right-hand side converged
  int32_t active[kMaxRhs];
  int32_t done;
  int32_t pad_;
};

template <typename XT>
struct CgArgsN {
  int64_t m;
  int nr;
  void* st[2];      // CgStateN<XT, nr> [m], double-buffered
  XT* p;            // [nr][m]
  XT* xlo;          // [nr][m]
  const XT* dinv;   // [m]
  double* xhi;      // [nr][m]
  double* r64;      // [nr][m]
  CgScalarsN* sc;
  CgScalarsN* snap;  // host snapshot slot written by a chunk's last launch, or NULL
  int32_t* flag;     // pinned host word set by the iteration raising a flag (see CgArgs)
  double* part[2];  // [blocks][6 nr] partials of an iteration, by state buffer
  double* part_ref; // [blocks][6 nr] partials of a refresh
  int blocks;
  int threads;
  int xg;           // XCD chunks of the iteration kernel (see cg_grid)
};
template <typename VT, typename XT>
hipError_t cgn_iterate(const CgArgsN<XT>& a, const CgMatrix& A, int q, int fixed,
                       hipEvent_t e0, hipEvent_t e1, hipStream_t s);
// g: [nr][m]
template <typename VT, typename XT>
hipError_t cgn_refresh(const CgArgsN<XT>& a, const CgMatrix& A, const double* g, int q,
                       int q_prev, int restart, hipStream_t s);
template <typename XT>
hipError_t cgn_setup(const CgArgsN<XT>& a, const double* g, double rtol, double delta,
                     hipStream_t s);

}  // namespace rbf
