/*
 * librbf -- compactly-supported RBF least-squares approximation on one MI355X.
 *
 * The library fits f(x) = sum_j c_j phi(||x - xi_j|| / rho_j) (Majdisova & Skala,
 * "Big Geo Data Surface Approximation using Radial Basis Functions", Section 2,
 * eq. 3) to N scattered samples (x_i, h_i) with M << N reference points xi_j,
 * by forming the normal equations of the overdetermined system A c = h
 * (Section 2, eq. 4-5):
 *
 *     B = A^T A  (sparse, symmetric; Section 5, eq. 11-12)      g = A^T h
 *
 * with A_ij = phi(||x_i - xi_j|| / rho_j) a Wendland CS-RBF (Table 2), and
 * solving (B + lambda I) c = g by Jacobi-preconditioned conjugate gradients.
 * Optionally the approximant carries a linear polynomial a^T x + a_0
 * (Section 3, eq. 6-7) and the solved system is the bordered one of eq. 10,
 *
 *     [ B + lambda I   A^T P ] [ c ]   [ A^T h ]
 *     [ P^T A          P^T P ] [ k ] = [ P^T h ],   P_i = (x_i^T, 1), k = (a, a_0).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers documented "device" are HIP device allocations owned by the
 *    caller; the library only reads or writes them on the plan's stream and
 *    keeps no reference after the call returns unless stated.  "_h" pointers
 *    are host memory owned by the caller.
 *  - Coordinates are SoA float64: component d of point i at ptr[d * n + i].
 *  - Indices of reference points ("centres") are the caller's order 0..M-1.
 *  - Every call returns an int status: 0 (RBF_OK), a negative error or a
 *    positive warning.  No call aborts or throws; rbf_last_error() gives the
 *    text of the last failure on the calling thread.
 *  - A plan is not thread-safe; distinct plans are independent.  All GPU work
 *    of a plan is ordered on the stream passed to rbf_fit_plan.  Calls block
 *    the host only where stated.
 *  - The support predicate is the strict range query of Algorithm 1:
 *    point x is in the support of centre j iff s < rho_j * rho_j, where
 *    s = (dx*dx + dy*dy) [+ dz*dz] with dx = x - xi in float64 and every
 *    operation rounded separately (no fused multiply-add).  The sparsity
 *    pattern is therefore reproducible bit for bit on any IEEE-754 machine.
 *  - Limits: dim in {2, 3}; 1 <= N < 2^31; 1 <= M < 2^31.
 *  - The checked build (librbf_checked.so, the same entry points) bounds-checks
 *    the data-dependent indices of the plan, assembly and evaluation kernels
 *    on the device: an index outside its buffer skips its access, and
 *    rbf_fit_plan, rbf_assemble, rbf_eval, rbf_eval_noalloc and
 *    rbf_stream_finish then return RBF_ERR_HIP naming the check's source file
 *    and line (rbf_fit_plan releases the plan).  Those calls then block the
 *    host.  A correct plan never trips a check.
 */
#ifndef RBF_H_
#define RBF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define RBF_OK 0
#define RBF_WARN_MAXITER 1   /* solver stopped at max_iter; best iterate returned */
#define RBF_WARN_FALLBACK 2  /* mixed-precision solve gave up; finished in FP64 */
#define RBF_ERR_INVALID (-1)     /* bad argument, size or call order */
#define RBF_ERR_NONFINITE (-2)   /* NaN/Inf in coordinates, radii or values */
#define RBF_ERR_SINGULAR (-3)    /* system not positive definite at set-up */
#define RBF_ERR_BREAKDOWN (-4)   /* CG breakdown: p^T B p <= 0 or NaN */
#define RBF_ERR_HIP (-5)         /* a HIP runtime call failed */
#define RBF_ERR_OOM (-6)         /* device allocation failed */

/* Wendland CS-RBFs phi_{3,s}, Table 2 (s = 0, 1, 3) and the same family's s = 2:
 *   W30 (1-r)^2_+   W31 (1-r)^4_+(4r+1)   W32 (1-r)^6_+(35r^2+18r+3)
 *   W33 (1-r)^8_+(32r^3+25r^2+8r+1)       with r = ||x - xi|| / rho.        */
typedef enum { RBF_PHI_W30 = 0, RBF_PHI_W31 = 1, RBF_PHI_W32 = 2, RBF_PHI_W33 = 3 } rbf_phi;

/* FP64: float64 basis values, assembly, matrix and CG.
 * FP32_REFINE: float32 basis values with compensated (Kahan) assembly, a
 * float32 matrix and float32 CG vectors; float64 dot products, float64
 * residual recomputation and float64 solution updates (reliable updates). */
typedef enum { RBF_PREC_FP64 = 0, RBF_PREC_FP32_REFINE = 1 } rbf_precision;

typedef struct rbf_plan rbf_plan;

/* Optional device allocator for every buffer the plan owns.  alloc returns a
 * device pointer (NULL on failure); release gives it back.  NULL allocator:
 * hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, size_t bytes, void* ctx);
  void* ctx;
} rbf_allocator;

typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int64_t n_points;             /* N */
  int64_t n_centers;            /* M */
  const double* points;         /* device, SoA [dim][N]; read during the call */
  const double* centers;        /* device, SoA [dim][M]; copied into the plan */
  double rho;                   /* support radius (= 1/alpha of eq. 18), > 0,
                                   used when rho_per_center is NULL */
  const double* rho_per_center; /* device [M] radii > 0, or NULL; copied */
  int32_t min_support;          /* centres with fewer supported points are
                                   inactive: no row/column, c_j = 0 (>= 1) */
  double lambda_rel;            /* ridge: lambda = lambda_rel * mean diag(B) over
                                   active centres, added to the diagonal of B only
                                   (>= 0) */
  int32_t polynomial;           /* 0: none; 1: linear polynomial reproduction
                                   (Section 3): dim + 1 more unknowns k */
  uint32_t flags;               /* RBF_PLAN_* bits, 0 by default */
} rbf_plan_desc;

/* rbf_plan_desc.flags: the float64 CG iteration gathers every neighbour from
 * global memory instead of staging the slices' neighbourhoods in LDS (same
 * results bit for bit; for comparisons). */
#define RBF_PLAN_NO_STAGING 1u
/* rbf_plan_desc.flags: form the pattern and assemble B row by row (one
 * workgroup per centre, the supported points streamed per row) instead of by
 * point tiles (each hash cell's points against the centres that reach the
 * cell, products on the matrix cores); the same pattern, and the same values
 * up to the order of the float64 sums, for comparisons. */
#define RBF_PLAN_ROW_ASSEMBLY 2u

typedef struct {
  int32_t dim;
  int32_t grid[3];              /* hash grid cells per dimension */
  int64_t n_points, n_centers;
  int64_t n_points_in_box;      /* points within reach of some centre's cell */
  int64_t n_active;             /* centres with >= min_support points */
  int64_t nnz_upper;            /* stored entries of B, diagonal and above */
  int64_t nnz_full;             /* entries of the full symmetric B */
  double density;               /* nnz_full / M^2 (Table 4 "density of LSE matrix") */
  int64_t support_total;        /* sum_j n_j = nonzeros of A */
  int32_t support_max;          /* max_j n_j */
  int32_t row_max;              /* max entries in a full row of B */
  double cell_size;
  int64_t solver_entries;       /* stored entries of the solver layout (with padding) */
  int32_t solver_col_bytes;     /* bytes per stored column index (2 or 4) */
  int32_t solver_lanes;         /* lanes per row of the solver layout */
  int32_t n_poly;               /* dim + 1 with a linear polynomial, else 0 */
  int32_t solver_staged;        /* most distinct columns one slice stages in LDS
                                   for the float64 CG iteration (0: not staged;
                                   built at the plan's first float64 solve) */
  int32_t assembly_tiles;       /* 1: the last assembly went by point tiles,
                                   0: by rows (or none yet) */
  int32_t tile_window;          /* most active centres within reach of one hash
                                   cell (0 with RBF_PLAN_ROW_ASSEMBLY; point
                                   tiles need at most 256 in 2D, 384 in 3D) */
  int32_t solver_rows_sorted;   /* 1: the solver's rows were reordered within
                                   windows of 64, longest first, because the
                                   layout padded the rows to more than 1.3
                                   times the nonzeros; 0: centre order */
  int32_t pad_;
} rbf_plan_stats;

typedef struct {
  double rtol;          /* stop when ||g - (B + lambda I) c||_2 <= rtol ||g||_2 */
  int64_t max_iter;     /* CG iteration cap (> 0) */
  int32_t warm_start;   /* nonzero: coeffs holds the initial guess on entry */
  int32_t check_every;  /* iterations between host reads of the residual (>= 1) */
  double reliable_delta;/* FP32_REFINE: float64 residual recomputation when the
                           iterated residual fell by this factor (0 < d < 1) */
  int32_t stall_limit;  /* FP32_REFINE: consecutive reliable updates whose float64
                           residual fell by less than 2x before the solve gives up
                           on float32 (>= 0; 0 = the default, 8) */
} rbf_solve_opts;

typedef struct {
  int64_t iterations;        /* CG iterations performed */
  int64_t reliable_updates;  /* float64 residual recomputations */
  double rel_residual;       /* final ||g - (B+lambda I)c|| / ||g||, recomputed in FP64 */
  double lambda;             /* ridge on the diagonal */
  int32_t precision;         /* rbf_precision actually used */
  int32_t status;            /* same as the return value */
} rbf_solve_info;

/* Build the neighbour structure and the sparsity pattern of B (Section 5:
 * upper triangle of the symmetric matrix; Algorithm 1: strict range query).
 * Hashes points and centres into a uniform grid of cell size >= max rho,
 * counts each centre's supported points, marks active centres and builds the
 * structural pattern: (j, l) is stored iff some point lies in both supports.
 * stream: a hipStream_t (NULL = default stream).  Blocks the host to read the
 * pattern size.  Errors: INVALID (sizes, dim, rho <= 0, min_support < 1,
 * lambda_rel < 0, NULL pointers), NONFINITE (NaN/Inf coordinates or radii),
 * OOM, HIP.  On error *out is NULL. */
int rbf_fit_plan(const rbf_plan_desc* desc, const rbf_allocator* allocator, void* stream,
                 rbf_plan** out);

/* Sizes of the plan (host struct); reads the per-centre counts back, so it
 * blocks the host. */
int rbf_plan_info(const rbf_plan* plan, rbf_plan_stats* out);

/* Copy the upper-triangular CSR pattern of B (diagonal included, columns
 * ascending, caller's centre numbering) and the support counts n_j to host
 * arrays of sizes M+1, nnz_upper and M.  Any pointer may be NULL to skip it.
 * Blocks the host. */
int rbf_plan_pattern(const rbf_plan* plan, int64_t* row_ptr_h, int32_t* col_h,
                     int32_t* support_count_h);

/* Assemble the values of B and g = A^T h for samples `values` (device [N],
 * caller's point order) with basis `phi` in precision `prec` (Section 5,
 * eq. 11-12: b_jl = sum_k phi_kj phi_kl over the points in both supports),
 * then add the ridge and form the Jacobi preconditioner.  With a polynomial
 * also A^T P, P^T P and P^T h of eq. 10 (float64; internally in the basis
 * ((x - o) / s, 1), o and s the centre and half-extent of the points'
 * bounding box, which spans the same functions).  Stream-ordered, does not
 * block.  Errors: INVALID (bad phi/prec, NULL values), HIP. */
int rbf_assemble(rbf_plan* plan, rbf_phi phi, rbf_precision prec, const double* values);

/* New sample values (device [N], caller's point order) for the assembled
 * system: g = A^T h (and P^T h with a polynomial) recomputed, B, lambda and
 * the preconditioner kept.  g is bit for bit what rbf_assemble computes for
 * the same values and precision.  Vector-valued data (h_i in E^p, Section 2)
 * share A and B across components: assemble once, then per component
 * rbf_set_values and rbf_solve.  Stream-ordered.  Errors: INVALID (nothing
 * assembled, NULL values), HIP. */
int rbf_set_values(rbf_plan* plan, const double* values);

/* Copy the polynomial blocks of eq. 10 to host memory, in the paper's basis
 * P_i = (x_i^T, 1): q_h [M][n_poly] row-major = A^T P (rows of inactive
 * centres 0), c_h [n_poly][n_poly] = P^T P, e_h [n_poly] = P^T h; float64 as
 * assembled (a float32 solve uses A^T P rounded to float32).  Any pointer may
 * be NULL.  Blocks the host.  Errors: INVALID (no polynomial, nothing
 * assembled). */
int rbf_poly_export(const rbf_plan* plan, double* q_h, double* c_h, double* e_h);

/* Copy the assembled system to host memory: the upper-CSR values of
 * B + lambda I in the pattern's order (nnz_upper; float32 values widened when
 * assembled in FP32_REFINE), g (M) and lambda (scalar).  Any pointer may be
 * NULL.  Blocks the host.  Errors: INVALID if nothing was assembled. */
int rbf_system_export(const rbf_plan* plan, double* val_upper_h, double* g_h, double* lambda_h);

/* Solve (B + lambda I) c = g by Jacobi-preconditioned CG in the precision of
 * the last rbf_assemble; with a polynomial, the bordered system of eq. 10 by
 * the same CG, the polynomial unknowns preconditioned by (P^T P)^-1 and
 * iterated in float64.  coeffs: device [M + n_poly] float64 output (input too
 * when opts->warm_start): c in the caller's centre order, then k = (a, a_0)
 * in the paper's basis (x^T, 1); inactive centres get 0.  The residual
 * ||.|| and ||g|| of the stopping test cover the whole bordered system.  opts NULL: rtol 1e-10,
 * max_iter 100000, check_every 32, reliable_delta 0.1.  Iterations are queued
 * in chunks of at most check_every, shorter as the residual nears the next
 * reliable-update trigger (sized from its decay); the last launch of a chunk
 * writes the residual and flags into pinned host memory, and the host waits
 * on a chunk only after the next chunk is queued, so launches queued past a
 * trigger or convergence return at entry.  A float32 (FP32_REFINE) solve
 * that stalls (opts->stall_limit) or breaks down while iterations remain goes
 * on in float64 from its current solution, within the same max_iter: a plan
 * holding its points assembles B, g, lambda and the preconditioner again in
 * float64; a chunked plan (rbf_stream_*) takes its float64 accumulators (the
 * sums as added, from float32 basis values) as the float64 matrix.  Either way
 * the plan is a float64 plan afterwards (later solves, rbf_set_values and
 * rbf_system_export use the float64 system).  A float32 solve that reaches
 * max_iter, or stalls with no iteration left, returns WARN_MAXITER with the
 * float32 system untouched.  Returns OK, WARN_MAXITER (best iterate kept),
 * WARN_FALLBACK (mixed precision stalled or broke down and float64 finished
 * the solve), ERR_BREAKDOWN, ERR_INVALID (not assembled, bad options),
 * ERR_HIP, ERR_OOM.  info may be NULL. */
int rbf_solve(rbf_plan* plan, const rbf_solve_opts* opts, double* coeffs, rbf_solve_info* info);

/* Solve for nrhs right-hand sides at once (vector-valued data, h_i in E^p,
 * Section 2): component k of the samples at values + k N (device [nrhs][N],
 * caller's point order), its coefficients at coeffs + k M (device
 * [nrhs][M]; input too when opts->warm_start); info: host [nrhs] or NULL.
 * Uses B and the precision of the last rbf_assemble; each component's g is
 * formed as rbf_set_values forms it (the plan is left holding the last
 * component's values).  One CG kernel per iteration serves every component,
 * so B is streamed once per iteration for all of them; a reliable update of
 * one refreshes all, and a component whose float64 residual meets rtol at a
 * refresh stops while the others go on (info[k].iterations: the iteration at
 * which it did).  2 <= nrhs <= 4; no polynomial block (call rbf_set_values and
 * rbf_solve per component instead); no float64 fallback: a stalled mixed
 * solve ends at max_iter with WARN_MAXITER.  Blocks the host as rbf_solve.
 * Errors: INVALID, BREAKDOWN, HIP, OOM. */
int rbf_solve_batch(rbf_plan* plan, int32_t nrhs, const double* values,
                    const rbf_solve_opts* opts, double* coeffs, rbf_solve_info* info);

/* The same least-squares fit as rbf_solve -- min ||A c + P k - h||^2 +
 * lambda ||c||^2 (Section 2, eq. 4-5; with a polynomial, the columns of P of
 * Section 3, eq. 9) -- by LSQR (Paige & Saunders, ACM TOMS 8, 1982) on the
 * design matrix itself instead of CG on the normal equations: A v is an
 * evaluation at the data points (eq. 3) and A^T u the assembly's g = A^T h
 * pass, so the iteration sees the conditioning of A, not its square.  For
 * dense or nearly dense A (large supports, as the paper's synthetic
 * experiment has: Table 3) where kappa(A^T A) is beyond float64.  All in
 * float64 with the basis of the last rbf_assemble and the values it (or
 * rbf_set_values) gave; B itself is not used.  lambda is the plan's ridge.
 * opts->rtol: LSQR's stopping test ||[A P]^T r - lambda c|| <= rtol ||[A P]||
 * ||r|| (the norms estimated by the bidiagonalisation); max_iter, warm_start
 * as rbf_solve (check_every, reliable_delta, stall_limit unused).  opts NULL:
 * rtol 1e-12, max_iter 100000.  coeffs as rbf_solve.  info->rel_residual: the
 * normal-equation residual ||[A P]^T (h - A c - P k) - lambda c|| / ||[A P]^T
 * h||, recomputed at the end.  Blocks the host at every iteration (two norm
 * reads).  Returns OK, WARN_MAXITER, ERR_BREAKDOWN (non-finite recurrence),
 * ERR_INVALID (not assembled, a plan made from point chunks, bad options),
 * ERR_HIP, ERR_OOM. */
int rbf_solve_lsqr(rbf_plan* plan, const rbf_solve_opts* opts, double* coeffs,
                   rbf_solve_info* info);

/* Evaluate the approximant (eq. 3) at n_query points: out[q] =
 * sum_j coeffs[j] phi(||y_q - xi_j|| / rho_j) over centres with y_q in their
 * support (plus a^T y_q + a_0 with a polynomial, eq. 6), basis of the last
 * rbf_assemble (or W31 if none).  queries: device SoA [dim][n_query]; coeffs:
 * device [M + n_poly] as rbf_solve writes them; out: device [n_query].  When
 * values is not NULL (device [n_query]) the root-mean-square of out - values
 * is written to *rmse_h (blocks the host); otherwise stream-ordered. */
int rbf_eval(const rbf_plan* plan, int64_t n_query, const double* queries,
             const double* coeffs, double* out, const double* values, double* rmse_h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rbf_eval
 * with every workspace in a static device array of the library instead of
 * memory the plan allocates -- the coefficients gathered into centre-hash
 * order (n_centers doubles) and the squared-error partial sums.  Same
 * arguments, kernels and results (bit for bit) as rbf_eval; calls no
 * allocating routine.  The array holds RBF_NOALLOC_MAX_CENTERS + 1025
 * doubles (8.4 MB) per GPU, for the life of the process; its device address
 * is taken at the first call on each GPU (that GPU current).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (from several
 * threads or streams) race and must be serialised by the caller.  Errors: as
 * rbf_eval, and INVALID for a plan with more than RBF_NOALLOC_MAX_CENTERS
 * centres. */
#define RBF_NOALLOC_MAX_CENTERS 1048576
int rbf_eval_noalloc(const rbf_plan* plan, int64_t n_query, const double* queries,
                     const double* coeffs, double* out, const double* values, double* rmse_h);

/* ---- points streamed through the GPU in chunks -------------------------- *
 * B = A^T A and g = A^T h are sums over the points: with A_c the rows of A of
 * the points of chunk c, B = sum_c A_c^T A_c and g = sum_c A_c^T h_c (the
 * block decomposition of Section 5, eq. 13-16, taken over point blocks rather
 * than column blocks).  A fit therefore need not hold its points in HBM: a
 * stream plan is made from the centres alone, chunks of points and values are
 * added one at a time (from device or host memory), and rbf_stream_finish
 * forms what rbf_fit_plan and rbf_assemble form for the union of the chunks:
 * the support counts, the active set and the structural pattern are the same
 * bit for bit; the values of B and g are summed per chunk in the precision of
 * the assembly (float32 Kahan sums of float32 phi, or float64) and across
 * chunks in float64, so they agree with a resident assembly to within the
 * rounding of the sums.  The finished plan serves rbf_solve, rbf_eval,
 * rbf_plan_info, rbf_plan_pattern, rbf_system_export, rbf_block_sq_err and
 * rbf_radius_broadcast; calls that need the points (rbf_assemble,
 * rbf_set_values, rbf_solve_batch, rbf_density_features) fail with INVALID,
 * and so do rbf_plan_info and rbf_plan_pattern before the finish.  No
 * polynomial block. */
typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int64_t n_centers;            /* M */
  const double* centers;        /* device, SoA [dim][M]; copied */
  double rho;                   /* support radius (> 0) when rho_per_center is NULL */
  const double* rho_per_center; /* device [M] radii > 0, or NULL; copied */
  int32_t min_support;          /* as rbf_plan_desc, applied at the finish (>= 1) */
  double lambda_rel;            /* as rbf_plan_desc (>= 0) */
  rbf_phi phi;                  /* basis of the assembly */
  rbf_precision precision;      /* precision of the assembly and of rbf_solve */
  int64_t max_chunk;            /* most points one rbf_stream_add takes, [1, 2^31);
                                   the plan holds one chunk's hash workspace (and,
                                   for host chunks, two staging slots) of this size */
  uint32_t flags;               /* RBF_PLAN_* bits, 0 by default */
} rbf_stream_desc;

/* Make a stream plan: centre hash, the candidate list of every centre (the
 * centres whose ball can meet its own) and zeroed accumulators over them.
 * Blocks the host to size the lists.  Errors: INVALID (as rbf_fit_plan, bad
 * phi/precision/max_chunk, a centre with more than 1024 candidates),
 * NONFINITE, OOM, HIP.  On error *out is NULL. */
int rbf_stream_begin(const rbf_stream_desc* desc, const rbf_allocator* allocator, void* stream,
                     rbf_plan** out);

/* Add a chunk of n points (0 <= n <= max_chunk): coordinates SoA [dim][n]
 * (component d of point i at points[d * n + i]) and values [n], both on the
 * device (on_host = 0: read on the plan's stream, stream-ordered) or both in
 * host memory (on_host != 0: copied into a staging slot on the plan's own copy
 * stream, so the copy of one chunk overlaps the accumulation of the one
 * before; pinned memory makes the copy asynchronous).  A host chunk's memory
 * may be reused once the next rbf_stream_add or rbf_stream_finish has
 * returned.  Chunks may come in any order and sizes; the sums are added in the
 * order of the calls, so the same chunks in the same order give the same bits.
 * Non-finite coordinates or values are reported by rbf_stream_finish.  Errors:
 * INVALID (not an open stream plan, n out of range, NULL pointers), HIP, OOM. */
int rbf_stream_add(rbf_plan* plan, int64_t n, const double* points, const double* values,
                   int32_t on_host);

/* Form the system of all chunks added: active centres (support count >=
 * min_support), the structural pattern (upper and full CSR, columns ascending),
 * the solver layout, the values of B and g, the ridge and the Jacobi
 * preconditioner; the plan then solves as an assembled one.  Blocks the host.
 * Errors: INVALID (not an open stream plan, pattern over 2^31 entries),
 * NONFINITE (a chunk held NaN/Inf), OOM, HIP. */
int rbf_stream_finish(rbf_plan* plan);

/* Kernel timing for measurement.  rbf_profile(plan, 1) resets the counters and
 * starts timing, with HIP events on the plan's stream, the assembly launch
 * (events recorded around it) and one CG iteration launch in 128
 * (events stamped at the kernel's own start and end by the extended launch;
 * launches that returned at entry after convergence are not counted);
 * rbf_profile(plan, 0) stops.
 * rbf_profile_read returns the number of timed launches of `kernel` and their
 * summed duration in milliseconds.  Both block the host (stream sync).
 * Kernel ids: */
#define RBF_KERNEL_CG_ITER 0   /* one CG iteration: vector updates, w = B D^-1 r, dot products */
#define RBF_KERNEL_CG_ITER_BATCH 1  /* one iteration of rbf_solve_batch (all right-hand sides) */
#define RBF_KERNEL_ASSEMBLE 2  /* numeric assembly of B and g */
int rbf_profile(rbf_plan* plan, int32_t enable);
int rbf_profile_read(rbf_plan* plan, int32_t kernel, int64_t* launches, double* total_ms);

/* ---- learned support radius -------------------------------------------- *
 * The paper observes that CS-RBF approximation is sensitive to data density
 * and to the shape parameter, chooses alpha = 1/rho experimentally (Section 6,
 * Table 3) and leaves optimal shape parameters to future work (Section 7).
 * These calls predict a radius per block of centres from the local density:
 * density features -> MLP 16-64-64-1 (tanh) -> log(rho / spacing) -> rho_j.
 * Blocks: a uniform blocks_per_dim^dim partition of the centres' bounding box,
 * t = (xi - min) / (max - min), b = min(nb - 1, floor(t nb)) per dimension,
 * first coordinate fastest (queries outside the box go to the nearest block). */
#define RBF_MLP_INPUTS 16
#define RBF_MLP_PARAMS 5313  /* W1[16][64] input-major, b1[64], W2[64][64], b2[64], W3[64], b3 */
#define RBF_MAX_RADII 8

typedef struct rbf_mlp rbf_mlp;

/* feats (device float32 [nblocks][2 n_radii]): for block b and radius s, the
 * mean and the population standard deviation over the block's centres of
 * log(1 + n_j(radii_h[s])), n_j = points in the support of centre j at that
 * radius (strict predicate as above).  1 <= n_radii <= 8; every radius at
 * most four hash cells (build the plan with rho = the largest radius).
 * Blocks the host.  Errors: INVALID. */
int rbf_density_features(rbf_plan* plan, int32_t n_radii, const double* radii_h,
                         int32_t blocks_per_dim, float* feats);

/* Per block: sums_h[b] = sum of (f - h)^2 and counts_h[b] = number of the
 * n_query points (device SoA [dim][n_query]; f, h device [n_query]) in block
 * b; for held-out scoring of radius sweeps.  Blocks the host. */
int rbf_block_sq_err(rbf_plan* plan, int64_t n_query, const double* queries, const double* f,
                     const double* h, int32_t blocks_per_dim, double* sums_h, int64_t* counts_h);

/* rho_out[j] (device [M]) = clamp(spacing exp(pred_log[block(j)]), rho_min,
 * rho_max), or rho_fallback where the prediction is not finite; pred_log is
 * device float32 [nblocks].  Blocks the host. */
int rbf_radius_broadcast(rbf_plan* plan, const float* pred_log, int32_t blocks_per_dim,
                         double spacing, double rho_min, double rho_max, double rho_fallback,
                         double* rho_out);

/* An MLP with the given float32 parameters (host [RBF_MLP_PARAMS]) and zero
 * Adam moments; its work runs on `stream`.  The object owns its device
 * memory.  Blocks the host. */
int rbf_mlp_create(const float* params_h, void* stream, rbf_mlp** out);
int rbf_mlp_params(const rbf_mlp* mlp, float* params_h);  /* copy out; blocks */

/* Gradient (host [RBF_MLP_PARAMS]) and value (host scalar) of the mean
 * squared error of the float32 network over n rows x (device [n][16]) with
 * targets y (device [n]).  Blocks the host. */
int rbf_mlp_grad(rbf_mlp* mlp, const float* x, const float* y, int64_t n, float* grad_h,
                 float* loss_h);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * mini-batches of `batch` rows: step k uses rows order[k*batch .. ) (device
 * int32 [steps*batch], each in [0, n_rows)), float32 forward and backward in
 * one workgroup.  losses_h (host [steps], may be NULL) gets every batch loss.
 * The row indices are checked on the host first.  Blocks the host. */
int rbf_mlp_train(rbf_mlp* mlp, const float* x, const float* y, int64_t n_rows,
                  const int32_t* order, int32_t steps, int32_t batch, float lr, float* losses_h);

/* out (device float32 [n]) = network(x) with weights, inputs and hidden
 * activations rounded to bfloat16 (nearest even) and float32 accumulation.
 * Stream-ordered. */
int rbf_mlp_infer_bf16(const rbf_mlp* mlp, const float* x, int64_t n, float* out);

/* Input standardisation used by rbf_mlp_grad, rbf_mlp_train and
 * rbf_mlp_infer_bf16: every input x_i is replaced by (x_i - mean_h[i]) /
 * std_h[i] (float32) as the kernels load it; host [16] each, std > 0.  A new
 * MLP has mean 0 and std 1 (inputs as given).  Blocks the host.  Errors:
 * INVALID (NULL, non-finite, std <= 0). */
int rbf_mlp_set_input_scaling(rbf_mlp* mlp, const float* mean_h, const float* std_h);

/* Checkpoint of everything training continues from: parameters (host
 * [RBF_MLP_PARAMS]), Adam first and second moments (host [RBF_MLP_PARAMS]
 * each), Adam steps taken (host scalar) and the input standardisation (host
 * [16] each).  Any pointer may be NULL.  Training resumed from a checkpoint
 * (rbf_mlp_load_state into any MLP, then rbf_mlp_train on the remaining
 * batches) gives the same bits as training without the interruption.  Both
 * block the host.  Errors: INVALID (NULL MLP; for the load, any NULL array, a
 * step count outside [0, 2^30], bad scaling). */
int rbf_mlp_state(const rbf_mlp* mlp, float* params_h, float* m1_h, float* m2_h,
                  int64_t* step_h, float* mean_h, float* std_h);
int rbf_mlp_load_state(rbf_mlp* mlp, const float* params_h, const float* m1_h,
                       const float* m2_h, int64_t step, const float* mean_h, const float* std_h);
void rbf_mlp_destroy(rbf_mlp* mlp);

/* Release every buffer of the plan (after the plan's stream work finished). */
void rbf_plan_destroy(rbf_plan* plan);

const char* rbf_status_string(int status);
const char* rbf_last_error(void);
/* 1 in the checked build (device index checks, see the conventions above),
 * 0 otherwise. */
int rbf_build_checked(void);

#ifdef __cplusplus
}
#endif
#endif /* RBF_H_ */
