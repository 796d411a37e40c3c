// Plan data shared by the plan, assembly, solve and evaluation kernels.
#pragma once

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
};

// Streams the support of centre j through LDS in chunks of kChunk points,
// keeping the sorted point order (coordinates in sp, sorted positions in sidx
// when it is not null), and hands each chunk to `consume(np)`.  One wave per
// block; every branch around the barriers is wave-uniform.
template <int DIM, int kChunk, typename Consume>
__device__ __forceinline__ void stream_support(const PlanView& P, const double* xj, double r2,
                                               double (*sp)[kChunk], int32_t* sidx,
                                               Consume&& consume) {
  const int lane = threadIdx.x;
  const uint64_t lt = lanemask_lt();
  int c[3];
  if (!cell_of<DIM>(P.grid, xj, c)) return;
  NbrWalk<DIM> walk(P.grid, c, 1);
  int np = 0;
  for (int k = 0; k < walk.rows(); ++k) {
    int lo_id, hi_id;
    if (!walk.range(k, lo_id, hi_id)) continue;
    const int lo = P.pcs[lo_id], hi = P.pcs[hi_id + 1];
    for (int i0 = lo; i0 < hi; i0 += kWave) {
      if (np > kChunk - kWave) {
        __syncthreads();
        consume(np);
        __syncthreads();
        np = 0;
      }
      const int i = i0 + lane;
      double p[DIM];
      bool in = false;
      if (i < hi) {
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
    __syncthreads();
    consume(np);
    __syncthreads();
  }
}


hipError_t launch_minmax(const double* a, int64_t n, double* partial_min, double* partial_max,
                         int* partial_bad, int nblocks, double* out3, hipStream_t s);
hipError_t launch_cell_keys(int dim, const Grid& G, const double* x, int64_t n, uint32_t* keys,
                            int32_t* idx, hipStream_t s);
hipError_t launch_gather_soa(const double* src, const int32_t* perm, int64_t n, int dim,
                             double* dst, hipStream_t s);
hipError_t launch_radius_tables(const double* rho_in, double rho, int64_t m, double* rho_c,
                                double* rho2_c, double* irho_c, hipStream_t s);
hipError_t launch_support_count(const PlanView& P, int32_t min_support, int32_t* count,
                                uint8_t* active, hipStream_t s);
hipError_t launch_symbolic(const PlanView& P, bool fill, int64_t* full_cnt, int32_t* lower_cnt,
                           const int64_t* row_ptr, int32_t* col, int32_t* err, hipStream_t s);

}  // namespace rbf

namespace rbf {
// assemble_kernels.hip
hipError_t launch_assemble(const PlanView& P, int phi, bool fp32, const double* hs,
                           const int64_t* row_ptr, const int32_t* lower_cnt, const int32_t* col,
                           void* val, double* g, double* diag, hipStream_t s);
hipError_t launch_finalize(int64_t m, const uint8_t* active, const int64_t* row_ptr,
                           const int32_t* lower_cnt, const double* diag, double lambda_rel,
                           double* lam, bool fp32, void* val, void* dinv, double* dinv64,
                           hipStream_t s);
// eval_kernels.hip
hipError_t launch_gather(const double* src, const int32_t* perm, int64_t n, double* dst,
                         hipStream_t s);
hipError_t launch_eval(const PlanView& P, int phi, int64_t nq, const double* y, const double* cs,
                       const double* rho2_s, const double* irho_s, double* out, hipStream_t s);
int sq_err_blocks(int64_t n);
hipError_t launch_sq_err(const double* f, const double* h, int64_t n, double* part, int nb,
                         double* out, hipStream_t s);
}  // namespace rbf
