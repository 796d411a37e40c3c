// Plan data shared by the plan, assembly, solve and evaluation kernels.
#pragma once

#include <type_traits>

#include "checks.h"
#include "internal.h"

namespace rbf {

// Most candidate columns one row of B may test (centres whose balls can meet).
constexpr int kMaxCand = 1024;

// Device view of a plan (passed by value to kernels).
struct PlanView {
  int32_t dim;
  int64_t n, m;
  Grid grid;
  const double* ps;       // points sorted by cell, SoA [dim][n]
  const int32_t* pcs;     // point cell starts [ncell + 2]
  const int32_t* pperm;   // sorted position -> caller's point index
  const double* ctr;      // centres, caller order, SoA [dim][m]
  const double* ctr_s;    // centres sorted by cell, SoA [dim][m]
  const int32_t* cperm;   // sorted position -> caller's centre index
  const int32_t* ccs;     // centre cell starts [ncell + 2]
  const double* rho;      // per-centre radius, caller order [m]
  const double* rho2;     // rho * rho
  const double* irho;     // 1 / rho
  const uint8_t* active;  // centre has >= min_support points
  const int32_t* amap;    // centre -> row of the solver's system (active centres in order), -1 if inactive
  int64_t nnz;            // entries of the full pattern (0 before it is built)
  int64_t nsell;          // stored entries of the solver layout (0 before it is built)
  int32_t* check;         // check word of the checked build (see checks.h), else NULL
};

// Orders LDS traffic among the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Streams part `part` of `nparts` of the support of centre j through this
// wave's LDS slab in chunks of kChunk points.  The candidate points (the cells
// around the centre's cell, in sorted order) are split into nparts contiguous
// pieces; the points of this piece that lie in the support are compacted in
// sorted order (coordinates in sp, sorted positions in sidx unless it is
// null) and handed to
// `consume(np)`.  A consumer that returns bool stops the stream by returning
// true (the value must be uniform over the wave).  Only wave-level
// synchronisation is used, so the waves of a block may take different
// numbers of chunks.
template <int DIM, int kChunk, typename Consume>
__device__ __forceinline__ void stream_support_part(const PlanView& P, const double* xj, double r2,
                                                    int part, int nparts,
                                                    double (*sp)[kChunk], int32_t* sidx,
                                                    Consume&& consume) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t lt = lanemask_lt();
  int c[3];
  if (!cell_of<DIM>(P.grid, xj, c)) return;
  NbrWalk<DIM> walk(P.grid, c, 1);
  int64_t total = 0;
  for (int k = 0; k < walk.rows(); ++k) {
    int lo_id, hi_id;
    if (walk.range(k, lo_id, hi_id)) total += P.pcs[hi_id + 1] - P.pcs[lo_id];
  }
  const int64_t my0 = total * part / nparts, my1 = total * (part + 1) / nparts;
  int64_t off = 0;
  int np = 0;
  for (int k = 0; k < walk.rows(); ++k) {
    int lo_id, hi_id;
    if (!walk.range(k, lo_id, hi_id)) continue;
    const int lo = P.pcs[lo_id], hi = P.pcs[hi_id + 1];
    // this row's slice of the wave's piece [my0, my1) of the virtual range
    const int64_t a = my0 > off ? my0 - off : 0;
    const int64_t b = (my1 - off) < (int64_t)(hi - lo) ? (my1 - off) : (int64_t)(hi - lo);
    off += hi - lo;
    if (b <= a) continue;
    const int s0 = lo + (int)a, s1 = lo + (int)b;
    for (int i0 = s0; i0 < s1; i0 += kWave) {
      if (np > kChunk - kWave) {
        wave_sync();
        if constexpr (std::is_same<decltype(consume(np)), bool>::value) {
          if (consume(np)) return;
        } else {
          consume(np);
        }
        wave_sync();
        np = 0;
      }
      const int i = i0 + lane;
      double p[DIM];
      bool in = false;
      if (i < s1) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) p[d] = P.ps[d * P.n + i];
        in = sqdist<DIM>(p, xj) < r2;
      }
      const uint64_t m = __ballot(in);
      if (in) {
        const int pos = np + __popcll(m & lt);
#pragma unroll
        for (int d = 0; d < DIM; ++d) sp[d][pos] = p[d];
        if (sidx) sidx[pos] = i;
      }
      np += __popcll(m);
    }
  }
  if (np > 0) {
    wave_sync();
    consume(np);
    wave_sync();
  }
}

hipError_t launch_minmax(const double* a, int64_t n, double* partial_min, double* partial_max,
                         int* partial_bad, int nblocks, double* out3, hipStream_t s);
// Cell keys (shifted left by `sub` bits with the sub-cell Morton code below,
// see k_cell_keys) and identity indices.
hipError_t launch_cell_keys(int dim, const Grid& G, const double* x, int64_t n, int sub,
                            uint32_t* keys, int32_t* idx, hipStream_t s);
hipError_t launch_gather_soa(const double* src, const int32_t* perm, int64_t n, int dim,
                             double* dst, hipStream_t s);
hipError_t launch_radius_tables(const double* rho_in, double rho, int64_t m, double* rho_c,
                                double* rho2_c, double* irho_c, hipStream_t s);
hipError_t launch_support_count(const PlanView& P, int32_t min_support, int32_t* count,
                                uint8_t* active, hipStream_t s);
// *dup = 1 if two active centres have the same coordinates and radius
// (identical columns of A); needs the centre hash and the active marks.
hipError_t launch_duplicate_centres(const PlanView& P, int32_t* dup, hipStream_t s);
// Count pass (fill = false) then fill pass; `marks` (symbolic_marks_words(m)
// words) carries the candidate marks from the first to the second.
size_t symbolic_marks_words(int64_t m);
hipError_t launch_symbolic(const PlanView& P, bool fill, int64_t* full_cnt, int32_t* lower_cnt,
                           const int64_t* row_ptr, int32_t* col, int32_t* err, int32_t* maxdelta,
                           uint32_t* marks, hipStream_t s);
// Rows of the solver's system: the active centres in order.  pos (m + 1
// int64, scratch of a scan with `temp` of scan_temp_bytes(m + 1) bytes) ends
// with pos[m] = number of solver rows; amap[j] = row of centre j or -1;
// srow[k] = centre of row k (room for m entries).
// launch_sort_rows then reorders the ms rows within windows of kSortRows
// consecutive rows, longest first (ties in order), updating srow and amap,
// so that the rows of a slice of the solver's layout have similar lengths.
// A row moves by less than kSortRows.
constexpr int kSortRows = 64;
hipError_t launch_sort_rows(const int64_t* row_ptr, int64_t ms, int32_t* srow, int32_t* amap,
                            hipStream_t s);
hipError_t launch_solver_rows(const uint8_t* active, int64_t m, int64_t* pos, void* temp,
                              int32_t* amap, int32_t* srow, hipStream_t s);
// Sliced-ELL layout of the solver (see CgMatrix) over its ms rows: slice
// lengths and sizes, then the column deltas (in solver rows) at their
// positions (check: the checked build's check word, or null).
hipError_t launch_slice_lengths(const int64_t* row_ptr, const int32_t* srow, int64_t ms, int lanes,
                                int64_t nslices, int32_t* slen, int64_t* ssize, hipStream_t s);
hipError_t launch_sell_cols(const int64_t* row_ptr, const int32_t* col, const int32_t* srow,
                            const int32_t* amap, int64_t ms, const int64_t* sptr, int lanes,
                            bool col16, void* cols, int32_t* check, hipStream_t s);

}  // namespace rbf

namespace rbf {
// assemble_kernels.hip
// Values go to the solver's sliced-ELL layout (sptr, lanes): entry e of row j
// of the CSR pattern sits at sell_pos(sptr, lanes, P.amap[j], e - row_ptr[j]).
// grouped: the grouped path (rows wider than one wave on average).
hipError_t launch_assemble(const PlanView& P, int phi, bool fp32, bool grouped, const double* hs,
                           const int64_t* row_ptr, const int32_t* lower_cnt, const int32_t* col,
                           const int64_t* sptr, int lanes, void* val, double* g, double* diag,
                           hipStream_t s);
// g = A^T h alone (same sums as launch_assemble's g for the same fp32/grouped);
// with kexp, also per active centre an exponent k_j with
// sum_k phi_kj^2 < 2^(k_j - 1) (phi in the same precision).
hipError_t launch_rhs(const PlanView& P, int phi, bool fp32, bool grouped, const double* hs,
                      double* g, hipStream_t s, int32_t* kexp = nullptr);
// lambda from the diagonals of the m centres, then, over the ms solver rows,
// the diagonal entries + lambda and the Jacobi scales dinv[k] (in solver rows).
hipError_t launch_finalize(int64_t m, const uint8_t* active, int64_t ms, const int32_t* srow,
                           const int64_t* sptr, int lanes, const int32_t* lower_cnt,
                           const double* diag, double lambda_rel, double* lam, bool fp32,
                           void* val, void* dinv, double* dinv64, double* ridge_part,
                           hipStream_t s);
// Doubles of the ridge's partial sums (launch_finalize's ridge_part).
constexpr int64_t kRidgePartDoubles = 2 * 512;
// eval_kernels.hip
hipError_t launch_gather(const double* src, const int32_t* perm, int64_t n, double* dst,
                         hipStream_t s);
// dst[j] = amap[j] >= 0 ? src[amap[j]] : 0 for j < m.
hipError_t launch_scatter_rows(const double* src, const int32_t* amap, int64_t m, double* dst,
                               hipStream_t s);
// kpoly: NULL, or device [dim + 1] coefficients (a, a_0) of the linear
// polynomial (eq. 7) added to every value.
hipError_t launch_eval(const PlanView& P, int phi, int64_t nq, const double* y, const double* cs,
                       const double* rho2_s, const double* irho_s, const double* kpoly,
                       double* out, hipStream_t s);
int sq_err_blocks(int64_t n);
hipError_t launch_sq_err(const double* f, const double* h, int64_t n, double* part, int nb,
                         double* out, hipStream_t s);
// poly_kernels.hip (PolySys and PolyBasis in solver.h)
struct PolySys;
struct PolyBasis;
int poly_gram_blocks(int64_t n);
// Q (float64 [dim+1][ms] by solver row, and its float32 copy when q32 is not
// NULL: then phi is evaluated in float32, as the mixed assembly does), C, e
// and C^-1 into S, for basis `phi` and sorted values hs; part holds
// poly_gram_blocks(n) * 14 doubles.
hipError_t launch_poly_system(const PlanView& P, int phi, const PolyBasis& B, int64_t ms,
                              const double* hs, double* q64, float* q32, double* part, int nb,
                              PolySys* S, hipStream_t s);
// out = the coefficients of `in` in the paper's basis (to_paper) or in the
// scaled basis (dim + 1 values each); in and out may not alias.
hipError_t launch_poly_coeffs(const double* in, const PolyBasis& B, int dim, bool to_paper,
                              double* out, hipStream_t s);
// C, e and C^-1 alone (new sample values, Q kept).
hipError_t launch_poly_gram(const PlanView& P, const PolyBasis& B, const double* hs, double* part,
                            int nb, PolySys* S, hipStream_t s);
// x = C^-1 e (the fit when no centre is active).
hipError_t launch_poly_only(const PolySys* S, double* x, hipStream_t s);
}  // namespace rbf
