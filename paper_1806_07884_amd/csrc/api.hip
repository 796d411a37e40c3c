// Host side of the C-ABI: plan object, device workspace, and the call
// sequences of set-up, assembly, solve and evaluation.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <mutex>
#include <vector>

#include "mlp_kernels.h"
#include "plan_kernels.h"
#include "rbf.h"
#include "chunk_planner.h"
#include "solve_policy.h"
#include "lsqr.h"
#include "solver.h"
#include "stream.h"
#include "tiles.h"

namespace {

thread_local std::string g_last_error;

// With timing on, one CG iteration launch in kProfPeriod carries start/stop
// events.  Stamped launches cost extra time on the stream (one in 32 added
// 0.8 ms to a 89 ms terrain2d fit), so the sample is kept sparse (a terrain2d
// fit still times ~40).
constexpr int64_t kProfPeriod = 128;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIPCHK(...)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (__VA_ARGS__);                                                     \
    if (e_ != hipSuccess)                                                              \
      return fail(RBF_ERR_HIP, "%s failed: %s", #__VA_ARGS__, hipGetErrorString(e_));  \
  } while (0)

constexpr int64_t kMaxCells = int64_t(1) << 26;
static_assert(rbf::kPlanMaxRhs == rbf::kMaxRhs, "the chunk planner tracks every right-hand side");

}  // namespace

// Pinned host slots for the solver's scalar snapshots, kept for the life of
// the process and handed from plan to plan (page-locking memory is slow, and
// a plan is often made per fit).
std::mutex g_pinned_mu;
std::vector<rbf::CgScalars*> g_pinned_free;

rbf::CgScalars* pinned_acquire() {
  {
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      rbf::CgScalars* p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  // mapped and coherent: the CG kernel that ends a chunk writes its slot; the
  // third slot's `done` is the word an iteration raising a flag sets
  if (hipHostMalloc(&p, 3 * sizeof(rbf::CgScalars), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return static_cast<rbf::CgScalars*>(p);
}

void pinned_release(rbf::CgScalars* p) {
  std::lock_guard<std::mutex> lock(g_pinned_mu);
  g_pinned_free.push_back(p);
}

struct rbf_plan {
  rbf_allocator alloc{};
  bool custom_alloc = false;
  hipStream_t stream = nullptr;
  struct Buf {
    void* p;
    size_t bytes;
  };
  std::vector<Buf> bufs;

  int32_t dim = 2;
  int64_t n = 0, m = 0;
  int32_t min_support = 1;
  double lambda_rel = 0.0;
  int32_t npoly = 0;       // d + 1 with linear polynomial reproduction, else 0
  rbf::PolyBasis pbasis{};  // its scaled basis (centre and half-extent of the points' box)
  rbf::Grid grid{};
  double cell_size = 0.0;
  double cbox[6] = {0, 0, 0, 0, 0, 0};  // centres' bounding box {min_0, max_0, ...}
  double* cbox_dev = nullptr;

  // hash of points and centres
  double* ps = nullptr;
  int32_t* pperm = nullptr;
  int32_t* pcs = nullptr;
  double* ctr = nullptr;
  double* ctr_s = nullptr;
  int32_t* cperm = nullptr;
  int32_t* ccs = nullptr;
  double* rho = nullptr;
  double* rho2 = nullptr;
  double* irho = nullptr;
  double* rho2_s = nullptr;
  double* irho_s = nullptr;
  // pattern
  int32_t* support = nullptr;
  uint8_t* active = nullptr;
  int32_t* amap = nullptr;  // centre -> solver row (active centres in order) or -1
  int32_t* srow = nullptr;  // solver row -> centre
  int64_t ms = 0;           // solver rows
  int64_t* row_ptr = nullptr;
  int32_t* lower_cnt = nullptr;
  int32_t* col = nullptr;
  int64_t nnz_full = 0;
  // solver layout (sliced ELL, column deltas; see CgMatrix)
  int64_t* sptr = nullptr;
  int32_t* slen = nullptr;
  int64_t nslices = 0;
  int32_t lanes = 4;
  void* scol = nullptr;
  bool col16 = false;
  int64_t nsell = 0;
  // neighbourhoods for the LDS-staged iteration (see CgMatrix); hslot null
  // when the layout does not qualify
  int16_t* hslot = nullptr;
  int16_t* hrow = nullptr;
  int64_t* hptr = nullptr;
  int32_t* hcount = nullptr;
  int32_t halo_max = 0;  // most distinct columns of a slice
  bool staging = true;   // build them (RBF_PLAN_NO_STAGING clears it)
  bool halo_tried = false;
  // system
  double* hs = nullptr;
  double* g = nullptr;
  double* g_s = nullptr;  // g over the solver rows
  double* diag = nullptr;
  double* lam = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  int phi = -1;
  int prec = -1;
  bool grouped = false;  // the row assembly took the grouped path (and g's sums follow it)
  // assembly by point tiles (tile_kernels.hip), set up at the first assembly
  bool row_assembly = false;  // RBF_PLAN_ROW_ASSEMBLY: always assemble by rows
  int tile_state = 0;         // 0 not set up, 1 usable, 2 a window exceeds the limit
  bool tiled = false;         // the last assembly took the tiles
  int4* tiles = nullptr;
  int64_t ntiles = 0;
  int32_t* wids = nullptr;    // the cells' windows (caller indices), tiles point into it
  int32_t tile_window = 0;    // most active centres within reach of one cell
  bool rows_sorted = false;   // solver rows reordered within windows (build_layout)
  unsigned long long* tacc = nullptr;  // [nnz_full] fixed-point sums
  int32_t* kexp = nullptr;             // [m] their per-row exponents
  int32_t* tile_err = nullptr;
  int32_t* check = nullptr;   // the checked build's check word (see checks.h)
  // solver workspace
  double* xhi = nullptr;
  double* r64 = nullptr;
  rbf::CgScalars* sc = nullptr;
  double* part_it = nullptr;   // [2][kCgParts * kCgMaxBlocks] partials of the iterations
  double* part_ref = nullptr;  // [kCgParts * kCgMaxBlocks] partials of a refresh
  // polynomial block (npoly > 0)
  double* q64 = nullptr;  // Q = A^T P, [npoly][ms] by solver row
  float* q32 = nullptr;   // its float32 copy for the mixed solve
  double* gram_part = nullptr;
  rbf::PolySys* psys = nullptr;
  rbf::PolyState* pst = nullptr;  // [2], by state buffer
  double* xpoly = nullptr;        // [kMaxPoly] polynomial unknowns in the scaled basis
  // batched solve (several right-hand sides; sized for kMaxRhs)
  void* bst[2][2] = {};           // [precision: 0 float64, 1 float32][state buffer]
  void* bvec[2][2] = {};          // [precision][p, x_lo], [kMaxRhs][ms]
  double* bxhi = nullptr;         // [kMaxRhs][ms]
  double* br64 = nullptr;
  double* bg = nullptr;
  double* bpart_it = nullptr;     // [2][6 kMaxRhs kCgMaxBlocks]
  double* bpart_ref = nullptr;
  rbf::CgScalarsN* bsc = nullptr;
  rbf::CgScalarsN* host_bsc = nullptr;  // pinned, two snapshot slots and a flag slot
  rbf::CgScalarsN* host_bsc_dev = nullptr;  // their device address
  void* vec64[4] = {};         // state buffers 0 and 1 (4 per row), p, x_lo
  void* vec32[4] = {};
  double* cs_sorted = nullptr;
  double* eval_part = nullptr;
  double* ridge_part = nullptr;  // partial sums of the ridge value
  // LSQR solve: u [n], u_d [m] (damping rows), v, w, x, t [m + 4], t_n [n],
  // reduction partials and scalars
  double *lq_u = nullptr, *lq_ud = nullptr, *lq_v = nullptr, *lq_w = nullptr, *lq_x = nullptr;
  double *lq_t = nullptr, *lq_tn = nullptr, *lq_part = nullptr, *lq_sc = nullptr;
  rbf::CgScalars* host_sc = nullptr;  // pinned, two snapshot slots and a flag slot (pinned pool)
  rbf::CgScalars* host_sc_dev = nullptr;  // their device address
  hipEvent_t snap_ev[2] = {nullptr, nullptr};

  // chunked assembly (rbf_stream_*): 0 = not a stream plan, 1 = taking
  // chunks, 2 = finished
  int stream_state = 0;
  int stream_prec = -1;  // precision of the chunks' sums (rbf_precision)
  bool stream_grouped = false;  // upper candidate lists longer than one wave on average
  int64_t max_chunk = 0;
  int64_t* cptr = nullptr;   // candidate lists: [m + 1] offsets, ascending columns
  int64_t* cup = nullptr;    // [m] start of each list's upper part
  int32_t* ccol = nullptr;
  double* sacc = nullptr;    // per upper candidate: float64 sum over the chunks so far
  uint8_t* smark = nullptr;  // per upper candidate: a point in both supports seen
  int64_t* scount = nullptr; // per centre: supported points so far
  int64_t* sinbox = nullptr; // points inside the hash grid so far
  int32_t* sbad = nullptr;   // a non-finite coordinate or value seen
  // one chunk's hash (max_chunk points) and the two staging slots of host chunks
  uint32_t *ckey[2] = {nullptr, nullptr};
  int32_t* cval[2] = {nullptr, nullptr};
  void* crtmp = nullptr;
  double* cps = nullptr;
  int32_t* cpp = nullptr;
  int32_t* cpcs = nullptr;
  double* chs = nullptr;
  double* stage_x[2] = {nullptr, nullptr};
  double* stage_h[2] = {nullptr, nullptr};
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_copied[2] = {nullptr, nullptr};
  hipEvent_t ev_used[2] = {nullptr, nullptr};
  int stage_next = 0;
  bool stage_pending[2] = {false, false};

  // optional kernel timing: HIP events bracketing sampled launches
  struct Pending {
    int kernel;
    int64_t iter;  // CG iteration index of the launch, -1 outside CG
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<Pending> pending;
  int64_t prof_launches[3] = {0, 0, 0};
  double prof_ms[3] = {0.0, 0.0, 0.0};

  hipEvent_t event() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Folds the pairs of executed launches (CG launches below `cg_done`
  // iterations, every other launch) into the totals.  CG launches at or
  // beyond it either returned at entry, when `settled` (dropped), or are
  // still queued (kept for a later call).
  void resolve(int64_t cg_done, bool settled) {
    std::vector<Pending> keep;
    for (const Pending& q : pending) {
      const bool ran = q.iter < 0 || q.iter < cg_done;
      if (!ran && !settled) {
        keep.push_back(q);
        continue;
      }
      float ms = 0.f;
      if (ran && hipEventSynchronize(q.b) == hipSuccess &&
          hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
        prof_launches[q.kernel] += 1;
        prof_ms[q.kernel] += ms;
      }
      ev_free.push_back(q.a);
      ev_free.push_back(q.b);
    }
    pending.swap(keep);
  }

  void* alloc_bytes(size_t bytes) {
    if (bytes == 0) bytes = 8;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (custom_alloc) {
      p = alloc.alloc(bytes, alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) bufs.push_back({p, bytes});
    return p;
  }
  void release(void* p) {
    if (!p) return;
    for (size_t i = 0; i < bufs.size(); ++i) {
      if (bufs[i].p == p) {
        if (custom_alloc)
          alloc.release(p, bufs[i].bytes, alloc.ctx);
        else
          (void)hipFree(p);
        bufs.erase(bufs.begin() + (long)i);
        return;
      }
    }
  }
  template <typename T>
  bool get(T** out, int64_t count) {
    *out = static_cast<T*>(alloc_bytes((size_t)std::max<int64_t>(count, 1) * sizeof(T)));
    return *out != nullptr;
  }
  rbf::PlanView view() const {
    rbf::PlanView v;
    v.dim = dim;
    v.n = n;
    v.m = m;
    v.grid = grid;
    v.ps = ps;
    v.pcs = pcs;
    v.pperm = pperm;
    v.ctr = ctr;
    v.ctr_s = ctr_s;
    v.cperm = cperm;
    v.ccs = ccs;
    v.rho = rho;
    v.rho2 = rho2;
    v.irho = irho;
    v.active = active;
    v.amap = amap;
    v.nnz = nnz_full;
    v.nsell = nsell;
    v.check = check;
    return v;
  }
  // The solver layout with values `val`; staged neighbourhoods when built and
  // the iterates are float64 (xt_bytes 8), or for a batched iteration of nr
  // right-hand sides when every slice fits its LDS.
  rbf::CgMatrix matrix(const void* val, int xt_bytes, int nr = 1) const {
    rbf::CgMatrix A;
    A.sptr = sptr;
    A.slen = slen;
    A.nslices = nslices;
    A.col = scol;
    A.col16 = col16;
    A.val = val;
    A.lanes = lanes;
    const bool staged =
        hslot && ((nr == 1 && xt_bytes == 8 && halo_max <= rbf::kHaloCap) ||
                  (nr > 1 && halo_max <= rbf::halo_cap_n(nr, xt_bytes)));
    A.hslot = staged ? hslot : nullptr;
    A.hrow = staged ? hrow : nullptr;
    A.hptr = staged ? hptr : nullptr;
    A.hcount = staged ? hcount : nullptr;
    return A;
  }
  ~rbf_plan() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (copy_stream) {
      (void)hipStreamSynchronize(copy_stream);
      (void)hipStreamDestroy(copy_stream);
    }
    for (int k = 0; k < 2; ++k) {
      if (ev_copied[k]) (void)hipEventDestroy(ev_copied[k]);
      if (ev_used[k]) (void)hipEventDestroy(ev_used[k]);
    }
    while (!bufs.empty()) release(bufs.back().p);
    if (host_sc) pinned_release(host_sc);
    if (host_bsc) (void)hipHostFree(host_bsc);
    for (hipEvent_t e : snap_ev)
      if (e) (void)hipEventDestroy(e);
    for (const Pending& q : pending) {
      (void)hipEventDestroy(q.a);
      (void)hipEventDestroy(q.b);
    }
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
  }
};

#define GET(ptr, count)                                                                        \
  do {                                                                                         \
    if (!P->get(&(ptr), (count)))                                                              \
      return fail(RBF_ERR_OOM, "device allocation of %lld elements for " #ptr " failed",       \
                  (long long)(count));                                                         \
  } while (0)

namespace {

// Grid hash of `count` points into caller workspace (keys/values twice
// `count`, radix temporaries of radix_temp_bytes(count) bytes): sorted by
// cell (with sub_order, by sub-cell within a cell as well), sorted copy,
// permutation and cell starts.  Stream-ordered.
int hash_core(rbf_plan* P, const double* coords, int64_t count, uint32_t* ka, uint32_t* kb,
              int32_t* va, int32_t* vb, void* tmp, double* sorted, int32_t* perm,
              int32_t* cell_start, bool sub_order) {
  hipStream_t s = P->stream;
  // sub-cell bits below the cell id while the shifted ids still fit 32 bits
  int sub = sub_order ? 2 * P->dim : 0;
  if ((((int64_t)P->grid.ncell + 1) << sub) > (int64_t)UINT32_MAX) sub = 0;
  HIPCHK(rbf::launch_cell_keys(P->dim, P->grid, coords, count, sub, ka, va, s));
  int bits = 1;
  while ((int64_t(1) << bits) <= ((int64_t)P->grid.ncell << sub) + ((int64_t(1) << sub) - 1)) ++bits;
  bool in_alt = false;
  HIPCHK(rbf::radix_sort_pairs(ka, va, kb, vb, count, bits, tmp, s, &in_alt));
  const uint32_t* keys = in_alt ? kb : ka;
  const int32_t* vals = in_alt ? vb : va;
  HIPCHK(rbf::cell_starts(keys, count, P->grid.ncell, sub, cell_start, s));
  HIPCHK(hipMemcpyAsync(perm, vals, (size_t)count * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  HIPCHK(rbf::launch_gather_soa(coords, perm, count, P->dim, sorted, s));
  return RBF_OK;
}

// hash_core with temporaries taken from the allocator and given back once
// the stream has consumed them (synchronises the stream).
int hash_into(rbf_plan* P, const double* coords, int64_t count, double* sorted, int32_t* perm,
              int32_t* cell_start, bool sub_order) {
  uint32_t *ka, *kb;
  int32_t *va, *vb;
  void* tmp;
  const size_t tb = rbf::radix_temp_bytes(count);
  if (!P->get(&ka, count) || !P->get(&kb, count) || !P->get(&va, count) || !P->get(&vb, count) ||
      !(tmp = P->alloc_bytes(tb)))
    return fail(RBF_ERR_OOM, "hash workspace allocation failed");
  const int rc = hash_core(P, coords, count, ka, kb, va, vb, tmp, sorted, perm, cell_start,
                           sub_order);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(P->stream));
  P->release(tmp);
  P->release(vb);
  P->release(va);
  P->release(kb);
  P->release(ka);
  return RBF_OK;
}

// Neighbourhoods of the solver's slices (see CgMatrix).  A layout with a slice
// that does not qualify keeps hslot null: the iteration then gathers from
// global memory.
int build_halo(rbf_plan* P) {
  hipStream_t s = P->stream;
  // once per plan, for grids of one slice per wave
  if (P->halo_tried || !P->staging || P->ms <= 0) return RBF_OK;
  P->halo_tried = true;
  int blocks = 0, threads = 0, xg = 0;
  rbf::cg_grid(P->nslices, &blocks, &threads, &xg);
  if (threads != rbf::kCgSmallBlock) return RBF_OK;
  const int64_t ns = P->nslices;
  const rbf::CgMatrix A = P->matrix(nullptr, 0);
  int32_t* hc;
  GET(hc, ns);
  HIPCHK(rbf::launch_halo_count(A, P->ms, rbf::kHaloCap, hc, s));
  std::vector<int32_t> cnt(ns);
  std::vector<int64_t> ptr(ns + 1);
  HIPCHK(hipMemcpyAsync(cnt.data(), hc, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t total = 0;
  int32_t mx = 0;
  for (int64_t k = 0; k < ns; ++k) {
    if (cnt[k] < 0) {
      P->release(hc);
      return RBF_OK;
    }
    ptr[k] = total;
    total += cnt[k];
    mx = std::max(mx, cnt[k]);
  }
  ptr[ns] = total;
  int64_t* hp;
  int16_t *hr, *hs;
  GET(hp, ns + 1);
  GET(hr, std::max<int64_t>(total, 1));
  GET(hs, P->nsell + rbf::kSellTail);
  HIPCHK(hipMemcpyAsync(hp, ptr.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(hs, 0, sizeof(int16_t) * (P->nsell + rbf::kSellTail), s));
  HIPCHK(rbf::launch_halo_fill(A, P->ms, hc, hp, hr, hs, s));
  HIPCHK(hipStreamSynchronize(s));  // ptr is read by the copy above
  P->hcount = hc;
  P->hptr = hp;
  P->hrow = hr;
  P->hslot = hs;
  P->halo_max = mx;
  return RBF_OK;
}

// The solver layout over the plan's full CSR (row_ptr, col, ms solver rows,
// nnz_full entries, col16): sliced ELL with L lanes per row.  Reads its size
// back, so it synchronises the plan's stream.
//
// When the slices pad the rows to more than kSortPad times the nonzeros, the
// rows are first reordered within windows of rbf::kSortRows, longest first,
// so that a slice's rows have similar lengths.  A slice's rows are then no
// longer consecutive centres, and its gathers touch more lines: on
// terrain2d (padding 1.13) the reordered iteration took 18.0 against 16.9 us,
// on the clustered 3D field (padding 1.53, 1.18 reordered) 23.4 against 24.6.
constexpr double kSortPad = 1.3;
int build_layout(rbf_plan* P) {
  hipStream_t s = P->stream;
  const int64_t ms = P->ms;
  P->lanes = rbf::sell_lanes((double)P->nnz_full / (double)std::max<int64_t>(ms, 1));
  const int64_t rows_per_slice = 64 / P->lanes;
  P->nslices = (ms + rows_per_slice - 1) / rows_per_slice;
  int64_t* ssize;
  GET(P->slen, P->nslices);
  GET(P->sptr, P->nslices + 1);
  GET(ssize, P->nslices + 1);
  void* stmp2 = P->alloc_bytes(rbf::scan_temp_bytes(P->nslices + 1));
  if (!stmp2) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  int64_t total = 0;
  for (int pass = 0; pass < 2; ++pass) {
    HIPCHK(rbf::launch_slice_lengths(P->row_ptr, P->srow, ms, P->lanes, P->nslices, P->slen,
                                     ssize, s));
    HIPCHK(rbf::exclusive_scan(ssize, P->sptr, P->nslices + 1, stmp2, s));
    HIPCHK(hipMemcpyAsync(&total, P->sptr + P->nslices, sizeof(int64_t), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    if (pass == 1 || (double)total <= kSortPad * (double)P->nnz_full) break;
    // rows of similar length share a slice (the slices pad to their longest)
    HIPCHK(rbf::launch_sort_rows(P->row_ptr, ms, P->srow, P->amap, s));
    P->rows_sorted = true;
  }
  P->release(stmp2);
  P->release(ssize);
  if (total >= (int64_t(1) << 31)) return fail(RBF_ERR_INVALID, "solver layout exceeds 2^31 entries");
  P->nsell = total;
  const size_t cbytes = (size_t)(total + rbf::kSellTail) * (P->col16 ? 2 : 4);
  P->scol = P->alloc_bytes(cbytes);
  if (!P->scol) return fail(RBF_ERR_OOM, "device allocation of the solver columns failed");
  HIPCHK(hipMemsetAsync(P->scol, 0, cbytes, s));
  HIPCHK(rbf::launch_sell_cols(P->row_ptr, P->col, P->srow, P->amap, ms, P->sptr, P->lanes,
                               P->col16, P->scol, P->check, s));
  return RBF_OK;
}

// Centres, radii, hash grid and centre hash of a plan.  points (device SoA
// [dim][P->n]) may be NULL (a stream plan); when given, their ranges set the
// polynomial basis and their finiteness is checked in the same host read.
int setup_centres(rbf_plan* P, const double* centers, const double* rho_per_center, double rho,
                  const double* points) {
  const int64_t n = points ? P->n : 0, m = P->m;
  const int dim = P->dim;
  hipStream_t s = P->stream;
  if (RBF_CHECKED_BUILD) {
    GET(P->check, 1);
    HIPCHK(hipMemsetAsync(P->check, 0, sizeof(int32_t), s));
  }
  GET(P->ctr, dim * m);
  HIPCHK(hipMemcpyAsync(P->ctr, centers, sizeof(double) * dim * m, hipMemcpyDeviceToDevice, s));
  GET(P->rho, m);
  GET(P->rho2, m);
  GET(P->irho, m);
  HIPCHK(rbf::launch_radius_tables(rho_per_center, rho, m, P->rho, P->rho2, P->irho, s));

  // ranges and finiteness of centres, points and radii: one host read
  const int nred = 2 * dim + 1;
  const int nb = 256;
  double *pmin, *pmax, *res;
  int* pbad;
  GET(pmin, nb);
  GET(pmax, nb);
  GET(pbad, nb);
  GET(res, 3 * nred);
  HIPCHK(hipMemsetAsync(res, 0, sizeof(double) * 3 * nred, s));
  for (int k = 0; k < dim; ++k) {
    HIPCHK(rbf::launch_minmax(P->ctr + k * m, m, pmin, pmax, pbad, nb, res + 3 * k, s));
    if (points)
      HIPCHK(rbf::launch_minmax(points + k * n, n, pmin, pmax, pbad, nb, res + 3 * (dim + k), s));
  }
  HIPCHK(rbf::launch_minmax(P->rho, m, pmin, pmax, pbad, nb, res + 3 * (2 * dim), s));
  double host[3 * 7];
  HIPCHK(hipMemcpyAsync(host, res, sizeof(double) * 3 * nred, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(res);
  P->release(pbad);
  P->release(pmax);
  P->release(pmin);
  for (int k = 0; k < nred; ++k)
    if (host[3 * k + 2] != 0.0)
      return fail(RBF_ERR_NONFINITE, "non-finite %s", k < dim ? "centre coordinate"
                                                      : k < 2 * dim ? "point coordinate"
                                                                    : "support radius");
  const double rho_min = host[3 * 2 * dim], rho_max = host[3 * 2 * dim + 1];
  for (int k = 0; k < 3; ++k) {
    const double lo = k < dim ? host[3 * (dim + k)] : 0.0, hi = k < dim ? host[3 * (dim + k) + 1] : 0.0;
    const double half = 0.5 * (hi - lo);
    P->pbasis.o[k] = 0.5 * (lo + hi);
    P->pbasis.s[k] = half > 0.0 ? half : 1.0;
  }
  if (!(rho_min > 0.0)) return fail(RBF_ERR_INVALID, "support radius must be > 0");

  // grid: cells of size >= max radius over the centres' box widened by 1.5 cells
  double cs = rho_max * (1.0 + 1e-6);
  for (int it = 0; it < 64; ++it) {
    int64_t cells = 1;
    for (int k = 0; k < dim; ++k) {
      const double ext = (host[3 * k + 1] - host[3 * k]) + 3.0 * cs;
      cells *= (int64_t)ceil(ext / cs) + 1;
    }
    if (cells <= kMaxCells) break;
    cs *= 1.25;
  }
  P->cell_size = cs;
  for (int k = 0; k < dim; ++k) {
    P->cbox[2 * k] = host[3 * k];
    P->cbox[2 * k + 1] = host[3 * k + 1];
  }
  P->grid.inv_cs = 1.0 / cs;
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < dim) {
      P->grid.lo[k] = host[3 * k] - 1.5 * cs;
      const double ext = (host[3 * k + 1] - host[3 * k]) + 3.0 * cs;
      P->grid.g[k] = (int32_t)ceil(ext / cs) + 1;
    } else {
      P->grid.lo[k] = 0.0;
      P->grid.g[k] = 1;
    }
    ncell *= P->grid.g[k];
  }
  if (ncell > kMaxCells) return fail(RBF_ERR_INVALID, "hash grid too large");
  P->grid.ncell = (int32_t)ncell;

  GET(P->ctr_s, dim * m);
  GET(P->cperm, m);
  GET(P->ccs, ncell + 2);
  const int rc = hash_into(P, P->ctr, m, P->ctr_s, P->cperm, P->ccs, false);
  if (rc) return rc;
  GET(P->rho2_s, m);
  GET(P->irho_s, m);
  HIPCHK(rbf::launch_gather(P->rho2, P->cperm, m, P->rho2_s, s));
  HIPCHK(rbf::launch_gather(P->irho, P->cperm, m, P->irho_s, s));
  return RBF_OK;
}

// The check word of a checked build (checks.h), read after an entry point's
// kernels: a failed device check becomes RBF_ERR_HIP naming its place.  A
// normal build holds no check word and passes rc on.
int device_checks(const rbf_plan* P, int rc) {
  if (!RBF_CHECKED_BUILD || !P || !P->check) return rc;
  int32_t w = 0;
  HIPCHK(hipMemcpyAsync(&w, P->check, sizeof(int32_t), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  if (w == 0) return rc;
  static const char* const files[] = {"?", "tile_kernels.hip", "assemble_kernels.hip",
                                      "plan_kernels.hip", "eval_kernels.hip"};
  const int f = w / 100000;
  return fail(RBF_ERR_HIP, "device check failed: %s line %d",
              f >= 1 && f <= 4 ? files[f] : files[0], w % 100000);
}

int tile_setup(rbf_plan* P);

int build_plan(rbf_plan* P, const rbf_plan_desc* d) {
  const int64_t n = P->n, m = P->m;
  const int dim = P->dim;
  hipStream_t s = P->stream;
  int rc = setup_centres(P, d->centers, d->rho_per_center, d->rho, d->points);
  if (rc) return rc;
  GET(P->ps, dim * n);
  GET(P->pperm, n);
  GET(P->pcs, P->grid.ncell + 2);
  rc = hash_into(P, d->points, n, P->ps, P->pperm, P->pcs, true);
  if (rc) return rc;

  GET(P->support, m);
  GET(P->active, m);
  rbf::PlanView v = P->view();
  HIPCHK(rbf::launch_support_count(v, P->min_support, P->support, P->active, s));

  // rows of the solver's system: the active centres in order
  int64_t* apos;
  GET(P->amap, m);
  GET(P->srow, m);
  GET(apos, m + 1);
  void* atmp = P->alloc_bytes(rbf::scan_temp_bytes(m + 1));
  if (!atmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(rbf::launch_solver_rows(P->active, m, apos, atmp, P->amap, P->srow, s));

  int64_t* cnt;
  int32_t *err, *maxd;
  GET(cnt, m + 1);
  GET(P->lower_cnt, m);
  GET(P->row_ptr, m + 1);
  GET(err, 4);
  maxd = err + 1;
  HIPCHK(hipMemsetAsync(err, 0, 4 * sizeof(int32_t), s));
  // without a ridge, identical columns of A make B singular
  if (P->lambda_rel == 0.0) HIPCHK(rbf::launch_duplicate_centres(v, err + 2, s));
  HIPCHK(hipMemsetAsync(cnt + m, 0, sizeof(int64_t), s));
  // the pattern: by point tiles (marks over each row's walk of cells) when
  // the windows fit, else row by row (marks over each row's candidates)
  if (!P->row_assembly) {
    rc = tile_setup(P);
    if (rc) return rc;
  }
  bool tiled = !P->row_assembly && P->tile_state == 1;
  uint32_t* marks = nullptr;
  int2* wtab = nullptr;
  int32_t *spos = nullptr, *ccell = nullptr;
  int words = 0;
  if (tiled) {
    const int R = rbf::walk_rows(dim);
    int32_t* maxwalk;
    GET(wtab, (int64_t)P->grid.ncell * (R + 1));
    GET(spos, m);
    GET(ccell, m);
    GET(maxwalk, 1);
    HIPCHK(hipMemsetAsync(maxwalk, 0, sizeof(int32_t), s));
    HIPCHK(rbf::launch_walk_tables(v, wtab, maxwalk, s));
    HIPCHK(rbf::launch_centre_slots(v, spos, ccell, s));
    int32_t mwalk = 0;
    HIPCHK(hipMemcpyAsync(&mwalk, maxwalk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    P->release(maxwalk);
    words = std::max(1, (mwalk + 31) / 32);
    // a tile's marks must fit its LDS: otherwise the rows path
    if (sizeof(uint32_t) * (size_t)P->tile_window * (size_t)words > rbf::tile_pattern_lds_max(dim))
      tiled = false;
  }
  if (tiled) {
    GET(marks, m * (int64_t)words);
    HIPCHK(hipMemsetAsync(marks, 0, sizeof(uint32_t) * m * words, s));
    HIPCHK(rbf::launch_tile_pattern(v, P->tiles, P->ntiles, P->wids, wtab, spos, ccell, words,
                                    P->tile_window, marks, err + 3, s));
    HIPCHK(rbf::launch_mark_rows(v, false, wtab, ccell, words, marks, cnt, P->lower_cnt, nullptr,
                                 nullptr, err, maxd, s));
  } else {
    GET(marks, (int64_t)rbf::symbolic_marks_words(m));
    HIPCHK(rbf::launch_symbolic(v, false, cnt, P->lower_cnt, nullptr, nullptr, err, maxd, marks,
                                s));
  }
  void* stmp = P->alloc_bytes(rbf::scan_temp_bytes(m + 1));
  if (!stmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(rbf::exclusive_scan(cnt, P->row_ptr, m + 1, stmp, s));
  int64_t nnz = 0, ms = 0;
  int32_t flags[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(&nnz, P->row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&ms, apos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(flags, err, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(cnt);
  P->release(apos);
  P->release(atmp);
  P->ms = ms;
  if (flags[3])
    return fail(RBF_ERR_HIP, "internal error in the tile pattern (%s)",
                (flags[3] & 1) ? "window overflow" : "mark outside its row");
  if (flags[0])
    return fail(RBF_ERR_INVALID,
                "a centre has more than %d neighbouring centres within two support radii",
                rbf::kMaxCand);
  if (flags[2])
    return fail(RBF_ERR_SINGULAR,
                "two active centres have the same coordinates and radius and lambda_rel is 0: "
                "B is singular");
  if (nnz >= (int64_t(1) << 31)) return fail(RBF_ERR_INVALID, "pattern exceeds 2^31 entries");
  P->nnz_full = nnz;
  v.nnz = nnz;
  // a column delta grows by less than kSortRows when the rows are sorted
  P->col16 = flags[1] + rbf::kSortRows <= 32767;
  GET(P->col, nnz);
  if (tiled)
    HIPCHK(rbf::launch_mark_rows(v, true, wtab, ccell, words, marks, nullptr, P->lower_cnt,
                                 P->row_ptr, P->col, err, maxd, s));
  else
    HIPCHK(rbf::launch_symbolic(v, true, nullptr, P->lower_cnt, P->row_ptr, P->col, err, maxd,
                                marks, s));
  rc = build_layout(P);  // synchronises the stream
  P->release(stmp);
  P->release(err);
  P->release(marks);
  P->release(wtab);
  P->release(spos);
  P->release(ccell);
  return rc;
}

// ---- chunked assembly --------------------------------------------------------

// Candidate lists, accumulators and the chunk workspace of a stream plan.
int build_stream(rbf_plan* P) {
  const int64_t m = P->m, mc = P->max_chunk;
  const int dim = P->dim;
  hipStream_t s = P->stream;
  int64_t* cnt;
  int32_t* err;
  GET(cnt, m + 1);
  GET(err, 1);
  GET(P->cptr, m + 1);
  GET(P->cup, m);
  HIPCHK(hipMemsetAsync(err, 0, sizeof(int32_t), s));
  HIPCHK(hipMemsetAsync(cnt + m, 0, sizeof(int64_t), s));
  const rbf::PlanView v = P->view();
  HIPCHK(rbf::launch_cand_count(v, cnt, err, s));
  void* stmp = P->alloc_bytes(rbf::scan_temp_bytes(m + 1));
  if (!stmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(rbf::exclusive_scan(cnt, P->cptr, m + 1, stmp, s));
  int64_t nc = 0;
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(&nc, P->cptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&bad, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(stmp);
  P->release(err);
  P->release(cnt);
  if (bad)
    return fail(RBF_ERR_INVALID,
                "a centre has more than %d neighbouring centres within two support radii",
                rbf::kMaxCand);
  GET(P->ccol, nc);
  HIPCHK(rbf::launch_cand_fill(v, P->cptr, P->cup, P->ccol, s));
  // the candidate relation is symmetric and holds every centre's own index:
  // the upper lists hold (nc + m) / 2 entries in all
  P->stream_grouped = (double)(nc + m) / (2.0 * (double)std::max<int64_t>(m, 1)) > 64.0;
  // accumulators over the candidates (the upper parts are used) and centres
  GET(P->sacc, nc);
  GET(P->smark, nc);
  GET(P->scount, m);
  GET(P->sinbox, 1);
  GET(P->sbad, 1);
  GET(P->g, m);
  GET(P->diag, m);
  GET(P->lam, 1);
  GET(P->dinv64, m);
  HIPCHK(hipMemsetAsync(P->sacc, 0, sizeof(double) * nc, s));
  HIPCHK(hipMemsetAsync(P->smark, 0, (size_t)nc, s));
  HIPCHK(hipMemsetAsync(P->scount, 0, sizeof(int64_t) * m, s));
  HIPCHK(hipMemsetAsync(P->sinbox, 0, sizeof(int64_t), s));
  HIPCHK(hipMemsetAsync(P->sbad, 0, sizeof(int32_t), s));
  HIPCHK(hipMemsetAsync(P->g, 0, sizeof(double) * m, s));
  // one chunk's hash
  for (int k = 0; k < 2; ++k) {
    GET(P->ckey[k], mc);
    GET(P->cval[k], mc);
  }
  P->crtmp = P->alloc_bytes(rbf::radix_temp_bytes(mc));
  if (!P->crtmp) return fail(RBF_ERR_OOM, "sort workspace allocation failed");
  GET(P->cps, dim * mc);
  GET(P->cpp, mc);
  GET(P->cpcs, P->grid.ncell + 2);
  GET(P->chs, mc);
  return RBF_OK;
}

// Staging slots and the copy stream of host chunks, made at the first one.
int ensure_staging(rbf_plan* P) {
  if (P->copy_stream) return RBF_OK;
  const int64_t mc = P->max_chunk;
  for (int k = 0; k < 2; ++k) {
    GET(P->stage_x[k], P->dim * mc);
    GET(P->stage_h[k], mc);
    HIPCHK(hipEventCreateWithFlags(&P->ev_copied[k], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_used[k], hipEventDisableTiming));
  }
  HIPCHK(hipStreamCreateWithFlags(&P->copy_stream, hipStreamNonBlocking));
  return RBF_OK;
}

// One chunk (device SoA coordinates x [dim][n], values h [n]) into the
// accumulators, on the plan's stream.
int stream_chunk(rbf_plan* P, int64_t n, const double* x, const double* h) {
  hipStream_t s = P->stream;
  HIPCHK(rbf::launch_chunk_check(x, h, n, P->dim, P->sbad, s));
  // the chunk's hash, into the plan's chunk workspace (no synchronisation)
  int rc = hash_core(P, x, n, P->ckey[0], P->ckey[1], P->cval[0], P->cval[1], P->crtmp, P->cps,
                     P->cpp, P->cpcs, true);
  if (rc) return rc;
  HIPCHK(rbf::launch_stream_inbox(P->cpcs + P->grid.ncell, P->sinbox, s));
  HIPCHK(rbf::launch_gather(h, P->cpp, n, P->chs, s));
  rbf::PlanView v = P->view();
  v.n = n;
  v.ps = P->cps;
  v.pcs = P->cpcs;
  v.pperm = P->cpp;
  HIPCHK(rbf::launch_stream_accum(v, P->phi, P->stream_prec == RBF_PREC_FP32_REFINE,
                                  P->stream_grouped, P->chs, P->cptr, P->cup, P->ccol, P->sacc,
                                  P->smark, P->scount, P->g, s));
  return RBF_OK;
}

// The system of the streamed points: active set, pattern, solver layout,
// values, ridge and preconditioner (as build_plan and rbf_assemble form them).
int finish_stream(rbf_plan* P) {
  const int64_t m = P->m;
  hipStream_t s = P->stream;
  GET(P->support, m);
  GET(P->active, m);
  HIPCHK(rbf::launch_stream_active(P->scount, m, P->min_support, P->support, P->active, s));
  int64_t* apos;
  GET(P->amap, m);
  GET(P->srow, m);
  GET(apos, m + 1);
  void* atmp = P->alloc_bytes(rbf::scan_temp_bytes(m + 1));
  if (!atmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(rbf::launch_solver_rows(P->active, m, apos, atmp, P->amap, P->srow, s));
  int64_t* cnt;
  int32_t* maxd;
  GET(cnt, m + 1);
  GET(maxd, 2);
  GET(P->lower_cnt, m);
  GET(P->row_ptr, m + 1);
  HIPCHK(hipMemsetAsync(maxd, 0, 2 * sizeof(int32_t), s));
  // without a ridge, identical columns of A make B singular
  if (P->lambda_rel == 0.0) HIPCHK(rbf::launch_duplicate_centres(P->view(), maxd + 1, s));
  HIPCHK(hipMemsetAsync(cnt + m, 0, sizeof(int64_t), s));
  HIPCHK(rbf::launch_stream_rows(P->cptr, P->cup, P->ccol, P->smark, P->active, m, cnt,
                                 P->lower_cnt, maxd, s));
  void* stmp = P->alloc_bytes(rbf::scan_temp_bytes(m + 1));
  if (!stmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(rbf::exclusive_scan(cnt, P->row_ptr, m + 1, stmp, s));
  int64_t nnz = 0, ms = 0;
  int32_t dm[2] = {0, 0}, bad = 0;
  HIPCHK(hipMemcpyAsync(&nnz, P->row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&ms, apos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(dm, maxd, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&bad, P->sbad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(stmp);
  P->release(maxd);
  P->release(cnt);
  P->release(atmp);
  P->release(apos);
  if (bad) return fail(RBF_ERR_NONFINITE, "non-finite point coordinate or value in a chunk");
  if (nnz >= (int64_t(1) << 31)) return fail(RBF_ERR_INVALID, "pattern exceeds 2^31 entries");
  if (dm[1])
    return fail(RBF_ERR_SINGULAR,
                "two active centres have the same coordinates and radius and lambda_rel is 0: "
                "B is singular");
  P->ms = ms;
  P->nnz_full = nnz;
  P->col16 = dm[0] + rbf::kSortRows <= 32767;
  int64_t* src;
  GET(P->col, nnz);
  GET(src, nnz);
  HIPCHK(rbf::launch_stream_fill(P->cptr, P->cup, P->ccol, P->smark, P->active, m, P->row_ptr,
                                 P->col, src, s));
  int rc = build_layout(P);
  if (rc) return rc;
  const bool fp32 = P->stream_prec == RBF_PREC_FP32_REFINE;
  const int64_t nv = P->nsell + rbf::kSellTail;
  void* val;
  if (fp32) {
    GET(P->val32, nv);
    GET(P->dinv32, m);
    HIPCHK(hipMemsetAsync(P->val32, 0, sizeof(float) * nv, s));
    val = P->val32;
  } else {
    GET(P->val64, nv);
    HIPCHK(hipMemsetAsync(P->val64, 0, sizeof(double) * nv, s));
    val = P->val64;
  }
  HIPCHK(rbf::launch_stream_values(P->row_ptr, P->col, src, P->amap, P->active, P->sacc, P->sptr,
                                   P->lanes, m, fp32, val, P->diag, P->g, s));
  void* dinv = fp32 ? (void*)P->dinv32 : (void*)P->dinv64;
  if (!P->ridge_part) GET(P->ridge_part, rbf::kRidgePartDoubles);
  HIPCHK(rbf::launch_finalize(m, P->active, ms, P->srow, P->sptr, P->lanes, P->lower_cnt, P->diag,
                              P->lambda_rel, P->lam, fp32, val, dinv, P->dinv64,
                              P->ridge_part, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(src);
  P->prec = P->stream_prec;
  return RBF_OK;
}

// The float64 system of a finished chunked plan from its float64 accumulators
// (the float64 fallback of a float32 solve: the points are gone).  The
// accumulators' index of every stored entry is rebuilt by the fill pass that
// finish_stream ran (it rewrites the same columns).
int stream_values64(rbf_plan* P) {
  const int64_t m = P->m, nnz = P->nnz_full;
  hipStream_t s = P->stream;
  const int64_t nv = P->nsell + rbf::kSellTail;
  if (!P->val64) {
    GET(P->val64, nv);
    HIPCHK(hipMemsetAsync(P->val64, 0, sizeof(double) * nv, s));
  }
  int64_t* src;
  GET(src, std::max<int64_t>(nnz, 1));
  HIPCHK(rbf::launch_stream_fill(P->cptr, P->cup, P->ccol, P->smark, P->active, m, P->row_ptr,
                                 P->col, src, s));
  HIPCHK(rbf::launch_stream_values(P->row_ptr, P->col, src, P->amap, P->active, P->sacc, P->sptr,
                                   P->lanes, m, false, P->val64, P->diag, P->g, s));
  if (!P->ridge_part) GET(P->ridge_part, rbf::kRidgePartDoubles);
  HIPCHK(rbf::launch_finalize(m, P->active, P->ms, P->srow, P->sptr, P->lanes, P->lower_cnt,
                              P->diag, P->lambda_rel, P->lam, false, P->val64, P->dinv64,
                              P->dinv64, P->ridge_part, s));
  HIPCHK(hipStreamSynchronize(s));
  P->release(src);
  return RBF_OK;
}

template <typename XT>
rbf::CgArgs<XT> make_args(rbf_plan* P, void** vec, const XT* dinv) {
  rbf::CgArgs<XT> a;
  a.m = P->ms;
  a.st[0] = (rbf::CgState<XT>*)vec[0];
  a.st[1] = (rbf::CgState<XT>*)vec[1];
  a.p = (XT*)vec[2];
  a.xlo = (XT*)vec[3];
  a.dinv = dinv;
  a.xhi = P->xhi;
  a.r64 = P->r64;
  a.sc = P->sc;
  a.snap = nullptr;
  a.flag = &P->host_sc_dev[2].done;
  a.part[0] = P->part_it;
  a.part[1] = P->part_it + rbf::kCgParts * rbf::kCgMaxBlocks;
  a.part_ref = P->part_ref;
  rbf::cg_grid(P->nslices, &a.blocks, &a.threads, &a.xg);
  a.np = P->npoly;
  a.Q = P->npoly ? (sizeof(XT) == 4 ? (const XT*)(const void*)P->q32 : (const XT*)(const void*)P->q64)
                 : nullptr;
  a.psys = P->psys;
  a.pst[0] = P->pst;
  a.pst[1] = P->pst ? P->pst + 1 : nullptr;
  a.xpoly = P->xpoly;
  return a;
}

int ensure_solver(rbf_plan* P, bool fp32) {
  const int64_t m = P->m;
  if (!P->xhi) {
    GET(P->xhi, m);
    GET(P->r64, m);
    GET(P->g_s, m);
    GET(P->sc, 1);
    GET(P->part_it, 2 * rbf::kCgParts * rbf::kCgMaxBlocks);
    GET(P->part_ref, rbf::kCgParts * rbf::kCgMaxBlocks);
  }
  void** vec = fp32 ? P->vec32 : P->vec64;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  const size_t per_row[4] = {4, 4, 1, 1};
  for (int k = 0; k < 4; ++k) {
    if (!vec[k]) {
      vec[k] = P->alloc_bytes(per_row[k] * es * (size_t)m);
      if (!vec[k]) return fail(RBF_ERR_OOM, "solver vector allocation failed");
    }
  }
  if (!P->host_sc) {
    P->host_sc = pinned_acquire();
    if (!P->host_sc) return fail(RBF_ERR_OOM, "pinned host allocation failed");
    HIPCHK(hipHostGetDevicePointer((void**)&P->host_sc_dev, P->host_sc, 0));
  }
  for (hipEvent_t& e : P->snap_ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return RBF_OK;
}

int read_scalars(rbf_plan* P) {
  HIPCHK(hipMemcpyAsync(P->host_sc, P->sc, sizeof(rbf::CgScalars), hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return RBF_OK;
}

// The point tiles of a resident plan and their windows; tile_state 2 when a
// window would exceed the kernels' limit (the rows paths are then used).
int tile_setup(rbf_plan* P) {
  hipStream_t s = P->stream;
  const rbf::PlanView v = P->view();
  const int64_t nc = P->grid.ncell;
  uint32_t *cnt, *off, *wcnt, *woff;
  int32_t* maxw;
  GET(cnt, nc + 1);
  GET(off, nc + 1);
  GET(wcnt, nc + 1);
  GET(woff, nc + 1);
  GET(maxw, 1);
  void* tmp = P->alloc_bytes(rbf::scan_temp_bytes(nc + 1));
  if (!tmp) return fail(RBF_ERR_OOM, "scan workspace allocation failed");
  HIPCHK(hipMemsetAsync(maxw, 0, sizeof(int32_t), s));
  HIPCHK(rbf::launch_tile_count(v, P->cell_size, cnt, wcnt, maxw, s));
  HIPCHK(rbf::exclusive_scan(cnt, off, nc + 1, tmp, s));
  HIPCHK(rbf::exclusive_scan(wcnt, woff, nc + 1, tmp, s));
  uint32_t nt = 0, nwin = 0;
  int32_t mw = 0;
  HIPCHK(hipMemcpyAsync(&nt, off + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&nwin, woff + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&mw, maxw, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->tile_window = mw;
  P->ntiles = nt;
  P->tile_state = 2;
  if (mw <= rbf::tile_window_max(P->dim) && nt > 0) {
    GET(P->tiles, (int64_t)nt);
    GET(P->wids, std::max<int64_t>(nwin, 1));
    HIPCHK(rbf::launch_tile_fill(v, P->cell_size, off, woff, P->tiles, P->wids, s));
    P->tile_state = 1;
  }
  HIPCHK(hipStreamSynchronize(s));
  P->release(tmp);
  P->release(maxw);
  P->release(woff);
  P->release(wcnt);
  P->release(off);
  P->release(cnt);
  return RBF_OK;
}

int assemble_into(rbf_plan* P, int phi, bool fp32) {
  hipStream_t s = P->stream;
  rbf::PlanView v = P->view();
  // padding entries of the sliced-ELL layout are never written: zero them once
  // (and the zeroed tail the CG kernels' batched loads may reach)
  const int64_t nv = P->nsell + rbf::kSellTail;
  if (fp32) {
    if (!P->val32) {
      GET(P->val32, nv);
      HIPCHK(hipMemsetAsync(P->val32, 0, sizeof(float) * nv, s));
    }
    if (!P->dinv32) GET(P->dinv32, P->m);
  } else {
    if (!P->val64) {
      GET(P->val64, nv);
      HIPCHK(hipMemsetAsync(P->val64, 0, sizeof(double) * nv, s));
    }
  }
  void* val = fp32 ? (void*)P->val32 : (void*)P->val64;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (P->prof_on) {
    e0 = P->event();
    e1 = P->event();
    if (!e0 || !e1) return fail(RBF_ERR_HIP, "hipEventCreate failed");
    HIPCHK(hipEventRecord(e0, s));
  }
  // rows wider than one wave on average: the grouped path (see assemble_kernels.hip)
  const double upper_mean =
      (double)(P->nnz_full + P->ms) / (2.0 * (double)std::max<int64_t>(P->ms, 1));
  P->grouped = upper_mean > 64.0;
  if (!P->row_assembly && P->tile_state == 0 && P->pcs) {
    const int rc = tile_setup(P);
    if (rc) return rc;
  }
  P->tiled = !P->row_assembly && P->tile_state == 1;
  if (P->tiled && !P->tacc) {
    GET(P->tacc, std::max<int64_t>(P->nnz_full, 1));
    GET(P->kexp, P->m);
    GET(P->tile_err, 1);
  }
  if (P->tiled) {
    // g by the rows' support stream (the same sums as the rows path gives),
    // with the rows' fixed-point exponents; then B by point tiles
    HIPCHK(hipMemsetAsync(P->tacc, 0, sizeof(unsigned long long) * P->nnz_full, s));
    HIPCHK(hipMemsetAsync(P->tile_err, 0, sizeof(int32_t), s));
    HIPCHK(rbf::launch_rhs(v, phi, fp32, P->grouped, P->hs, P->g, s, P->kexp));
    HIPCHK(rbf::launch_tile_assemble(v, phi, fp32, P->tiles, P->ntiles, P->wids, P->row_ptr,
                                     P->col, P->kexp, P->tacc, P->tile_err, s));
    HIPCHK(rbf::launch_tile_finish(v, fp32, P->row_ptr, P->lower_cnt, P->col, P->kexp, P->tacc,
                                   P->sptr, P->lanes, val, P->diag, s));
  } else {
    HIPCHK(rbf::launch_assemble(v, phi, fp32, P->grouped, P->hs, P->row_ptr, P->lower_cnt,
                                P->col, P->sptr, P->lanes, val, P->g, P->diag, s));
  }
  if (P->prof_on) {
    HIPCHK(hipEventRecord(e1, s));
    P->pending.push_back({2, -1, e0, e1});
  }
  void* dinv = fp32 ? (void*)P->dinv32 : (void*)P->dinv64;
  if (!P->ridge_part) GET(P->ridge_part, rbf::kRidgePartDoubles);
  HIPCHK(rbf::launch_finalize(P->m, P->active, P->ms, P->srow, P->sptr, P->lanes, P->lower_cnt,
                              P->diag, P->lambda_rel, P->lam, fp32, val, dinv, P->dinv64,
                              P->ridge_part, s));
  if (P->npoly) {
    // the polynomial blocks of eq. 10, phi in the same precision as B and g
    const int nb = rbf::poly_gram_blocks(P->n);
    if (!P->psys) {
      GET(P->q64, (int64_t)P->npoly * std::max<int64_t>(P->ms, 1));
      GET(P->gram_part, 14 * 1024);
      GET(P->psys, 1);
      GET(P->pst, 2);
      GET(P->xpoly, rbf::kMaxPoly);
    }
    if (fp32 && !P->q32) GET(P->q32, (int64_t)P->npoly * std::max<int64_t>(P->ms, 1));
    HIPCHK(rbf::launch_poly_system(v, phi, P->pbasis, P->ms, P->hs, P->q64,
                                   fp32 ? P->q32 : nullptr, P->gram_part, nb, P->psys, s));
  }
  if (P->tiled) {
    int32_t te = 0;
    HIPCHK(hipMemcpyAsync(&te, P->tile_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (te)
      return fail(RBF_ERR_HIP, "internal error in the tile assembly (window overflow)");
  }
  return RBF_OK;
}

// Reliable-update Jacobi-PCG (see cg_kernels.hip).  Returns a status; the
// float64 solution is left in P->xhi.
//
// Iterations are launched in chunks of at most check_every (sized by
// rbf::ChunkPlanner); the last launch of a chunk writes the scalars into one
// of two pinned host slots, and an event follows it.  The next chunk is always queued before the host
// waits on the previous one, so the GPU never idles on a convergence check;
// launches after a raised flag return at entry.  The iteration that raises a
// flag also sets a pinned host word, and a chunk being queued when it is seen
// ends with the next launch (which returns at entry and writes the slot), so
// that few launches are queued past a flag.  Launches never exceed the
// iteration budget.
template <typename VT, typename XT>
int run_cg(rbf_plan* P, const VT* val, const XT* dinv, void** vec, const rbf_solve_opts& o,
           int64_t* iters, int64_t* updates, int stall_limit) {
  hipStream_t s = P->stream;
  rbf::CgArgs<XT> a = make_args<XT>(P, vec, dinv);
  const rbf::CgMatrix A = P->matrix(val, (int)sizeof(XT));
  HIPCHK(rbf::cg_setup<XT>(a, P->g_s, o.rtol, o.reliable_delta, s));
  // start: float64 residual of the initial x on state buffer 0, direction reset
  HIPCHK(rbf::cg_refresh<VT, XT>(a, A, P->g_s, 0, 1, 1, s));
  // every refresh moves the state to the other buffer, as every iteration does
  int64_t refreshes = 1;
  const int64_t base_iter = *iters;
  const int64_t budget = std::max<int64_t>(o.max_iter - base_iter, 0);
  int64_t launched = 0;  // iterations launched since the start (>= executed)
  bool fixed = true;     // the next launch takes its scalars from the refresh
  // stall_limit 0: never give up on a stall (the float64 iteration)
  rbf::StallWatch stall(stall_limit);

  rbf::ChunkPlanner plan(o.check_every);
  int64_t slot_len[2] = {0, 0};
  // the flag word the iterations set (no launch of this plan is in flight)
  volatile int32_t* const flag_h = &P->host_sc[2].done;
  *flag_h = 0;
  // queue one chunk and its snapshot into slot `slot` (the other slot's
  // chunk, if queued, is still unobserved); false if none is left
  auto enqueue = [&](int slot, bool* queued) -> int {
    *queued = false;
    const int64_t step = plan.next(slot_len[slot ^ 1]);
    int64_t chunk = std::min<int64_t>(budget - launched, step);
    slot_len[slot] = 0;
    if (chunk <= 0) return RBF_OK;
    for (int64_t it = 0; it < chunk; ++it) {
      // a flag already raised: this launch ends the chunk
      if (it < chunk - 1 && *flag_h != 0) chunk = it + 1;
      const int q = (int)((launched + refreshes) & 1);
      // one launch in kProfPeriod carries start/stop events when timing is on
      const bool timed = P->prof_on && launched % kProfPeriod == kProfPeriod - 1;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        e0 = P->event();
        e1 = P->event();
        if (!e0 || !e1) return fail(RBF_ERR_HIP, "hipEventCreate failed");
      }
      // the chunk's last launch writes the scalars into the host slot
      a.snap = it == chunk - 1 ? P->host_sc_dev + slot : nullptr;
      HIPCHK(rbf::cg_iterate<VT, XT>(a, A, q, fixed ? 1 : 0, e0, e1, s));
      if (timed) P->pending.push_back({0, base_iter + launched, e0, e1});
      fixed = false;
      ++launched;
    }
    a.snap = nullptr;
    slot_len[slot] = chunk;
    HIPCHK(hipEventRecord(P->snap_ev[slot], s));
    *queued = true;
    return RBF_OK;
  };
  auto wait_slot = [&](int slot, rbf::CgScalars* h) -> int {
    HIPCHK(hipEventSynchronize(P->snap_ev[slot]));
    *h = P->host_sc[slot];
    return RBF_OK;
  };

  int cur = 0;
  bool cur_q = false;
  int rc = enqueue(cur, &cur_q);
  if (rc) return rc;
  for (;;) {
    rbf::CgScalars h;
    if (cur_q) {
      bool next_q = false;
      rc = enqueue(cur ^ 1, &next_q);
      if (rc) return rc;
      rc = wait_slot(cur, &h);
      if (rc) return rc;
      slot_len[cur] = 0;
      plan.seen(h.iter, 1, &h.rr, &h.trigger2, nullptr);
      if (h.done == 0 && next_q) {
        *iters = base_iter + h.iter;
        if (P->prof_on) P->resolve(*iters, false);
        cur ^= 1;
        continue;
      }
      // a flag is up (or the budget is spent): the other chunk has run its
      // course too, take the latest state
      if (next_q) {
        rc = wait_slot(cur ^ 1, &h);
        if (rc) return rc;
      }
    } else {
      // nothing was queued: the budget was spent before any launch
      rc = read_scalars(P);
      if (rc) return rc;
      h = *P->host_sc;
    }
    *iters = base_iter + h.iter;
    // every queued launch has run by now
    if (P->prof_on) P->resolve(*iters, true);
    const int q = (int)((h.iter + refreshes) & 1);
    if (h.done == 3) return RBF_OK;
    if (h.done == 2) return fail(RBF_ERR_BREAKDOWN, "CG breakdown after %lld iterations",
                                 (long long)h.iter);
    if (h.done == 1) {
      if (stall.update(h.rr_true) && stall_limit > 0) return RBF_WARN_FALLBACK;
      HIPCHK(rbf::cg_refresh<VT, XT>(a, A, P->g_s, q, q ^ 1, 0, s));
      ++refreshes;
      *updates += 1;
      fixed = true;
      plan.restart();     // the refresh sets a new trigger
      slot_len[0] = slot_len[1] = 0;
      launched = h.iter;  // every queued launch has run; later ones returned at entry
      *flag_h = 0;        // the flag of the iteration that raised it
      cur = 0;
      rc = enqueue(cur, &cur_q);
      if (rc) return rc;
      if (cur_q) continue;
    }
    // iteration budget spent: the float64 residual decides
    HIPCHK(rbf::cg_refresh<VT, XT>(a, A, P->g_s, q, q ^ 1, 1, s));
    rc = read_scalars(P);
    if (rc) return rc;
    return P->host_sc->done == 3 ? RBF_OK : RBF_WARN_MAXITER;
  }
}

// Batched solve of nr right-hand sides (see run_cg; one CG kernel per
// iteration serves all of them).  A trigger of any right-hand side refreshes
// them all; a converged one is frozen by the refresh.  The float64 solutions
// are left in P->bxhi.
template <typename VT, typename XT>
int run_cgn(rbf_plan* P, const VT* val, const XT* dinv, int nr, int prec_idx,
            const rbf_solve_opts& o, int64_t* iters, int64_t* updates) {
  hipStream_t s = P->stream;
  rbf::CgArgsN<XT> a;
  a.m = P->ms;
  a.nr = nr;
  a.st[0] = P->bst[prec_idx][0];
  a.st[1] = P->bst[prec_idx][1];
  a.p = (XT*)P->bvec[prec_idx][0];
  a.xlo = (XT*)P->bvec[prec_idx][1];
  a.dinv = dinv;
  a.xhi = P->bxhi;
  a.r64 = P->br64;
  a.sc = P->bsc;
  a.snap = nullptr;
  a.flag = &P->host_bsc_dev[2].done;
  a.part[0] = P->bpart_it;
  a.part[1] = P->bpart_it + 6 * rbf::kMaxRhs * rbf::kCgMaxBlocks;
  a.part_ref = P->bpart_ref;
  rbf::cg_grid(P->nslices, &a.blocks, &a.threads, &a.xg);
  const int rch = build_halo(P);
  if (rch) return rch;
  const rbf::CgMatrix A = P->matrix(val, (int)sizeof(XT), nr);
  HIPCHK(rbf::cgn_setup<XT>(a, P->bg, o.rtol, o.reliable_delta, s));
  // start: float64 residuals of the initial x on state buffer 0
  HIPCHK(rbf::cgn_refresh<VT, XT>(a, A, P->bg, 0, 1, 1, s));
  int64_t refreshes = 1, launched = 0;
  const int64_t budget = o.max_iter;
  bool fixed = true;
  rbf::ChunkPlanner plan(o.check_every);
  int64_t slot_len[2] = {0, 0};
  // the flag word the iterations set (no launch of this plan is in flight)
  volatile int32_t* const flag_h = &P->host_bsc[2].done;
  *flag_h = 0;
  // queue one chunk and its snapshot into slot `slot` (as run_cg: a flag seen
  // while queueing ends the chunk with the next launch)
  auto enqueue = [&](int slot, bool* queued) -> int {
    *queued = false;
    const int64_t step = plan.next(slot_len[slot ^ 1]);
    int64_t chunk = std::min<int64_t>(budget - launched, step);
    slot_len[slot] = 0;
    if (chunk <= 0) return RBF_OK;
    for (int64_t it = 0; it < chunk; ++it) {
      if (it < chunk - 1 && *flag_h != 0) chunk = it + 1;
      const int q = (int)((launched + refreshes) & 1);
      const bool timed = P->prof_on && launched % kProfPeriod == kProfPeriod - 1;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        e0 = P->event();
        e1 = P->event();
        if (!e0 || !e1) return fail(RBF_ERR_HIP, "hipEventCreate failed");
      }
      // the chunk's last launch writes the scalars into the host slot
      a.snap = it == chunk - 1 ? P->host_bsc_dev + slot : nullptr;
      HIPCHK(rbf::cgn_iterate<VT, XT>(a, A, q, fixed ? 1 : 0, e0, e1, s));
      if (timed) P->pending.push_back({1, launched, e0, e1});
      fixed = false;
      ++launched;
    }
    a.snap = nullptr;
    slot_len[slot] = chunk;
    HIPCHK(hipEventRecord(P->snap_ev[slot], s));
    *queued = true;
    return RBF_OK;
  };
  int cur = 0;
  bool cur_q = false;
  int rc = enqueue(cur, &cur_q);
  if (rc) return rc;
  for (;;) {
    rbf::CgScalarsN h;
    if (cur_q) {
      bool next_q = false;
      rc = enqueue(cur ^ 1, &next_q);
      if (rc) return rc;
      HIPCHK(hipEventSynchronize(P->snap_ev[cur]));
      h = P->host_bsc[cur];
      slot_len[cur] = 0;
      plan.seen(h.iter, nr, h.rr, h.trigger2, h.active);
      if (h.done == 0 && next_q) {
        *iters = h.iter;
        if (P->prof_on) P->resolve(h.iter, false);
        cur ^= 1;
        continue;
      }
      // a flag is up (or the budget is spent): take the latest state
      if (next_q) {
        HIPCHK(hipEventSynchronize(P->snap_ev[cur ^ 1]));
        h = P->host_bsc[cur ^ 1];
      }
    } else {
      HIPCHK(hipMemcpyAsync(P->host_bsc, P->bsc, sizeof(rbf::CgScalarsN), hipMemcpyDeviceToHost,
                            s));
      HIPCHK(hipStreamSynchronize(s));
      h = *P->host_bsc;
    }
    *iters = h.iter;
    if (P->prof_on) P->resolve(h.iter, true);
    const int q = (int)((h.iter + refreshes) & 1);
    if (h.done == 3) return RBF_OK;
    if (h.done == 2) return fail(RBF_ERR_BREAKDOWN, "CG breakdown after %lld iterations",
                                 (long long)h.iter);
    if (h.done == 1) {
      HIPCHK(rbf::cgn_refresh<VT, XT>(a, A, P->bg, q, q ^ 1, 0, s));
      ++refreshes;
      *updates += 1;
      fixed = true;
      plan.restart();
      slot_len[0] = slot_len[1] = 0;
      launched = h.iter;  // every queued launch has run; later ones returned at entry
      *flag_h = 0;        // the flag of the iteration that raised it
      cur = 0;
      rc = enqueue(cur, &cur_q);
      if (rc) return rc;
      if (cur_q) continue;
    }
    // iteration budget spent: the float64 residuals decide
    HIPCHK(rbf::cgn_refresh<VT, XT>(a, A, P->bg, q, q ^ 1, 1, s));
    HIPCHK(hipMemcpyAsync(P->host_bsc, P->bsc, sizeof(rbf::CgScalarsN), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    return P->host_bsc->done == 3 ? RBF_OK : RBF_WARN_MAXITER;
  }
}

// Buffers of the batched solve (sized for kMaxRhs right-hand sides).
int ensure_batch(rbf_plan* P, bool fp32) {
  const int64_t m = std::max<int64_t>(P->ms, 1);
  const int64_t nb = (int64_t)rbf::kMaxRhs * m;
  if (!P->bsc) {
    GET(P->bxhi, nb);
    GET(P->br64, nb);
    GET(P->bg, nb);
    GET(P->bpart_it, 2 * 6 * rbf::kMaxRhs * rbf::kCgMaxBlocks);
    GET(P->bpart_ref, 6 * rbf::kMaxRhs * rbf::kCgMaxBlocks);
    GET(P->bsc, 1);
  }
  const int pi = fp32 ? 1 : 0;
  const size_t rec = fp32 ? sizeof(rbf::CgStateN<float, rbf::kMaxRhs>)
                          : sizeof(rbf::CgStateN<double, rbf::kMaxRhs>);
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  for (int b = 0; b < 2; ++b) {
    if (!P->bst[pi][b]) {
      P->bst[pi][b] = P->alloc_bytes(rec * (size_t)m);
      if (!P->bst[pi][b]) return fail(RBF_ERR_OOM, "batched solver state allocation failed");
    }
    if (!P->bvec[pi][b]) {
      P->bvec[pi][b] = P->alloc_bytes(es * (size_t)nb);
      if (!P->bvec[pi][b]) return fail(RBF_ERR_OOM, "batched solver vector allocation failed");
    }
  }
  if (!P->host_bsc) {
    void* h = nullptr;
    // mapped and coherent: the CG kernel that ends a chunk writes its slot;
    // the third slot's `done` is the word an iteration raising a flag sets
    if (hipHostMalloc(&h, 3 * sizeof(rbf::CgScalarsN),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RBF_ERR_OOM, "pinned host allocation failed");
    }
    P->host_bsc = static_cast<rbf::CgScalarsN*>(h);
    HIPCHK(hipHostGetDevicePointer((void**)&P->host_bsc_dev, P->host_bsc, 0));
  }
  for (hipEvent_t& e : P->snap_ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return RBF_OK;
}

// Partial sums of the squared error of an evaluation (the most blocks
// sq_err_blocks gives), then their total.
constexpr int64_t kEvalParts = 1024;

// The allocation-free evaluation's workspace: one static device array per GPU
// the library runs on, held until the process ends.  Host code never uses the
// array's name as an address: noalloc_scratch() takes the device address of
// this GPU's copy once (with the GPU current) and keeps it per device.
constexpr int64_t kNoAllocScratch = RBF_NOALLOC_MAX_CENTERS + kEvalParts + 1;  // doubles
static __device__ __align__(256) double scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RBF_ERR_INVALID, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RBF_ERR_HIP, "hipGetSymbolAddress returned no address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return RBF_OK;
}

}  // namespace

extern "C" {

const char* rbf_last_error(void) { return g_last_error.c_str(); }

int rbf_build_checked(void) { return RBF_CHECKED_BUILD; }

const char* rbf_status_string(int status) {
  switch (status) {
    case RBF_OK: return "ok";
    case RBF_WARN_MAXITER: return "warning: iteration limit reached";
    case RBF_WARN_FALLBACK: return "warning: mixed precision fell back to float64";
    case RBF_ERR_INVALID: return "invalid argument";
    case RBF_ERR_NONFINITE: return "non-finite input";
    case RBF_ERR_SINGULAR: return "singular system";
    case RBF_ERR_BREAKDOWN: return "conjugate-gradient breakdown";
    case RBF_ERR_HIP: return "HIP runtime error";
    case RBF_ERR_OOM: return "out of device memory";
    default: return "unknown status";
  }
}

static int fit_plan_impl(const rbf_plan_desc* d, const rbf_allocator* allocator, void* stream,
                         rbf_plan** out) {
  if (!out) return fail(RBF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!d) return fail(RBF_ERR_INVALID, "desc is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(RBF_ERR_INVALID, "dim must be 2 or 3");
  if (d->n_points < 1 || d->n_points >= (int64_t(1) << 31))
    return fail(RBF_ERR_INVALID, "n_points must be in [1, 2^31)");
  if (d->n_centers < 1 || d->n_centers >= (int64_t(1) << 31))
    return fail(RBF_ERR_INVALID, "n_centers must be in [1, 2^31)");
  if (!d->points || !d->centers) return fail(RBF_ERR_INVALID, "points/centers is NULL");
  if (!d->rho_per_center && !(d->rho > 0.0 && isfinite(d->rho)))
    return fail(d->rho > 0.0 ? RBF_ERR_NONFINITE : RBF_ERR_INVALID,
                "rho must be finite and > 0");
  if (d->min_support < 1) return fail(RBF_ERR_INVALID, "min_support must be >= 1");
  if (d->polynomial != 0 && d->polynomial != 1)
    return fail(RBF_ERR_INVALID, "polynomial must be 0 (none) or 1 (linear)");
  if (d->flags & ~(RBF_PLAN_NO_STAGING | RBF_PLAN_ROW_ASSEMBLY))
    return fail(RBF_ERR_INVALID, "unknown plan flags");
  if (!(d->lambda_rel >= 0.0 && isfinite(d->lambda_rel)))
    return fail(RBF_ERR_INVALID, "lambda_rel must be finite and >= 0");
  if (allocator && (!allocator->alloc || !allocator->release))
    return fail(RBF_ERR_INVALID, "allocator callbacks are NULL");
  rbf_plan* P = new rbf_plan();
  if (allocator) {
    P->alloc = *allocator;
    P->custom_alloc = true;
  }
  P->stream = (hipStream_t)stream;
  P->dim = d->dim;
  P->n = d->n_points;
  P->m = d->n_centers;
  P->min_support = d->min_support;
  P->lambda_rel = d->lambda_rel;
  P->npoly = d->polynomial ? d->dim + 1 : 0;
  P->staging = (d->flags & RBF_PLAN_NO_STAGING) == 0;
  P->row_assembly = (d->flags & RBF_PLAN_ROW_ASSEMBLY) != 0;
  const int rc = build_plan(P, d);
  if (rc != RBF_OK) {
    delete P;
    return rc;
  }
  *out = P;
  return RBF_OK;
}

int rbf_plan_info(const rbf_plan* P, rbf_plan_stats* o) {
  if (!P || !o) return fail(RBF_ERR_INVALID, "NULL argument");
  if (P->stream_state == 1) return fail(RBF_ERR_INVALID, "rbf_stream_finish must come first");
  memset(o, 0, sizeof *o);
  o->dim = P->dim;
  for (int k = 0; k < 3; ++k) o->grid[k] = P->grid.g[k];
  o->n_points = P->n;
  o->n_centers = P->m;
  o->nnz_full = P->nnz_full;
  o->cell_size = P->cell_size;
  std::vector<int32_t> sup(P->m), low(P->m);
  std::vector<int64_t> rp(P->m + 1);
  std::vector<uint8_t> act(P->m);
  int32_t in_box = 0;
  HIPCHK(hipMemcpyAsync(sup.data(), P->support, sizeof(int32_t) * P->m, hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipMemcpyAsync(rp.data(), P->row_ptr, sizeof(int64_t) * (P->m + 1),
                        hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipMemcpyAsync(act.data(), P->active, P->m, hipMemcpyDeviceToHost, P->stream));
  int64_t in_box64 = 0;
  if (P->pcs)
    HIPCHK(hipMemcpyAsync(&in_box, P->pcs + P->grid.ncell, sizeof(int32_t), hipMemcpyDeviceToHost,
                          P->stream));
  else
    HIPCHK(hipMemcpyAsync(&in_box64, P->sinbox, sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  int64_t na = 0, tot = 0;
  int32_t smax = 0, rmax = 0;
  for (int64_t j = 0; j < P->m; ++j) {
    na += act[j] ? 1 : 0;
    tot += sup[j];
    smax = std::max(smax, sup[j]);
    rmax = std::max<int32_t>(rmax, (int32_t)(rp[j + 1] - rp[j]));
  }
  o->n_active = na;
  o->support_total = tot;
  o->support_max = smax;
  o->row_max = rmax;
  o->nnz_upper = (P->nnz_full + na) / 2;
  o->n_points_in_box = P->pcs ? (int64_t)in_box : in_box64;
  o->density = (double)P->nnz_full / ((double)P->m * (double)P->m);
  o->assembly_tiles = P->tiled ? 1 : 0;
  o->tile_window = P->tile_window;
  o->solver_rows_sorted = P->rows_sorted ? 1 : 0;
  o->pad_ = 0;
  o->solver_entries = P->nsell;
  o->solver_col_bytes = P->col16 ? 2 : 4;
  o->solver_lanes = P->lanes;
  o->n_poly = P->npoly;
  o->solver_staged = P->hslot ? P->halo_max : 0;
  return RBF_OK;
}

int rbf_plan_pattern(const rbf_plan* P, int64_t* row_ptr_h, int32_t* col_h,
                     int32_t* support_count_h) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (P->stream_state == 1) return fail(RBF_ERR_INVALID, "rbf_stream_finish must come first");
  const int64_t m = P->m;
  std::vector<int64_t> rp(m + 1);
  std::vector<int32_t> low(m), colf(P->nnz_full);
  HIPCHK(hipMemcpyAsync(rp.data(), P->row_ptr, sizeof(int64_t) * (m + 1), hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipMemcpyAsync(low.data(), P->lower_cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                        P->stream));
  if (col_h && P->nnz_full)
    HIPCHK(hipMemcpyAsync(colf.data(), P->col, sizeof(int32_t) * P->nnz_full,
                          hipMemcpyDeviceToHost, P->stream));
  if (support_count_h)
    HIPCHK(hipMemcpyAsync(support_count_h, P->support, sizeof(int32_t) * m,
                          hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  int64_t pos = 0;
  if (row_ptr_h) row_ptr_h[0] = 0;
  for (int64_t j = 0; j < m; ++j) {
    const int64_t a = rp[j] + low[j], b = rp[j + 1];
    if (col_h)
      for (int64_t e = a; e < b; ++e) col_h[pos + (e - a)] = colf[e];
    pos += b - a;
    if (row_ptr_h) row_ptr_h[j + 1] = pos;
  }
  return RBF_OK;
}

static int assemble_impl(rbf_plan* P, rbf_phi phi, rbf_precision prec, const double* values) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!P->ps) return fail(RBF_ERR_INVALID, "a stream plan holds no points to assemble from");
  if ((int)phi < 0 || (int)phi > 3) return fail(RBF_ERR_INVALID, "unknown basis function");
  if ((int)prec < 0 || (int)prec > 1) return fail(RBF_ERR_INVALID, "unknown precision");
  if (!values) return fail(RBF_ERR_INVALID, "values is NULL");
  if (!P->hs) GET(P->hs, P->n);
  if (!P->g) {
    GET(P->g, P->m);
    GET(P->diag, P->m);
    GET(P->lam, 1);
    GET(P->dinv64, P->m);
  }
  HIPCHK(rbf::launch_gather(values, P->pperm, P->n, P->hs, P->stream));
  const int rc = assemble_into(P, (int)phi, prec == RBF_PREC_FP32_REFINE);
  if (rc) return rc;
  P->phi = (int)phi;
  P->prec = (int)prec;
  return RBF_OK;
}

int rbf_set_values(rbf_plan* P, const double* values) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!P->ps) return fail(RBF_ERR_INVALID, "a stream plan holds no points");
  if (P->prec < 0) return fail(RBF_ERR_INVALID, "rbf_assemble must precede rbf_set_values");
  if (!values) return fail(RBF_ERR_INVALID, "values is NULL");
  hipStream_t s = P->stream;
  HIPCHK(rbf::launch_gather(values, P->pperm, P->n, P->hs, s));
  HIPCHK(rbf::launch_rhs(P->view(), P->phi, P->prec == RBF_PREC_FP32_REFINE, P->grouped, P->hs,
                         P->g, s));
  if (P->npoly)
    HIPCHK(rbf::launch_poly_gram(P->view(), P->pbasis, P->hs, P->gram_part,
                                 rbf::poly_gram_blocks(P->n), P->psys, s));
  return RBF_OK;
}

int rbf_system_export(const rbf_plan* P, double* val_upper_h, double* g_h, double* lambda_h) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (P->prec < 0) return fail(RBF_ERR_INVALID, "nothing assembled");
  const int64_t m = P->m;
  if (val_upper_h) {
    std::vector<int64_t> rp(m + 1), sp(P->nslices + 1);
    std::vector<int32_t> low(m), amap(m);
    HIPCHK(hipMemcpyAsync(amap.data(), P->amap, sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                          P->stream));
    std::vector<double> v64;
    std::vector<float> v32;
    HIPCHK(hipMemcpyAsync(rp.data(), P->row_ptr, sizeof(int64_t) * (m + 1),
                          hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipMemcpyAsync(sp.data(), P->sptr, sizeof(int64_t) * (P->nslices + 1),
                          hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipMemcpyAsync(low.data(), P->lower_cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                          P->stream));
    if (P->prec == RBF_PREC_FP64) {
      v64.resize(std::max<int64_t>(P->nsell, 1));
      HIPCHK(hipMemcpyAsync(v64.data(), P->val64, sizeof(double) * P->nsell,
                            hipMemcpyDeviceToHost, P->stream));
    } else {
      v32.resize(std::max<int64_t>(P->nsell, 1));
      HIPCHK(hipMemcpyAsync(v32.data(), P->val32, sizeof(float) * P->nsell,
                            hipMemcpyDeviceToHost, P->stream));
    }
    HIPCHK(hipStreamSynchronize(P->stream));
    int64_t pos = 0;
    for (int64_t j = 0; j < m; ++j)
      for (int64_t e = rp[j] + low[j]; e < rp[j + 1]; ++e) {
        const int64_t e4 = rbf::sell_pos(sp.data(), P->lanes, amap[j], e - rp[j]);
        val_upper_h[pos++] = P->prec == RBF_PREC_FP64 ? v64[e4] : (double)v32[e4];
      }
  }
  if (g_h) HIPCHK(hipMemcpyAsync(g_h, P->g, sizeof(double) * m, hipMemcpyDeviceToHost, P->stream));
  if (lambda_h) HIPCHK(hipMemcpyAsync(lambda_h, P->lam, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return RBF_OK;
}

int rbf_poly_export(const rbf_plan* P, double* q_h, double* c_h, double* e_h) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!P->npoly) return fail(RBF_ERR_INVALID, "the plan has no polynomial");
  if (P->prec < 0 || !P->psys) return fail(RBF_ERR_INVALID, "nothing assembled");
  const int np = P->npoly, dim = P->dim;
  const int64_t m = P->m, ms = P->ms;
  rbf::PolySys S;
  std::vector<double> q((size_t)np * std::max<int64_t>(ms, 1));
  std::vector<int32_t> amap(m);
  HIPCHK(hipMemcpyAsync(&S, P->psys, sizeof S, hipMemcpyDeviceToHost, P->stream));
  if (q_h) {
    if (ms > 0)
      HIPCHK(hipMemcpyAsync(q.data(), P->q64, sizeof(double) * np * ms, hipMemcpyDeviceToHost,
                            P->stream));
    HIPCHK(hipMemcpyAsync(amap.data(), P->amap, sizeof(int32_t) * m, hipMemcpyDeviceToHost,
                          P->stream));
  }
  HIPCHK(hipStreamSynchronize(P->stream));
  // the paper's basis (x^T, 1) is the scaled one times T: T[d][d] = s_d,
  // T[dim][d] = o_d, T[dim][dim] = 1; Q T, T^T C T and T^T e
  double T[rbf::kMaxPoly][rbf::kMaxPoly] = {};
  for (int d = 0; d < dim; ++d) {
    T[d][d] = P->pbasis.s[d];
    T[dim][d] = P->pbasis.o[d];
  }
  T[dim][dim] = 1.0;
  if (q_h) {
    for (int64_t j = 0; j < m; ++j) {
      const int32_t k = amap[j];
      for (int t = 0; t < np; ++t) {
        double v = 0.0;
        if (k >= 0)
          for (int u = 0; u < np; ++u) v += q[(size_t)u * ms + k] * T[u][t];
        q_h[j * np + t] = v;
      }
    }
  }
  if (c_h) {
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        double v = 0.0;
        for (int u = 0; u < np; ++u)
          for (int w = 0; w < np; ++w) v += T[u][a] * S.C[u][w] * T[w][b];
        c_h[a * np + b] = v;
      }
  }
  if (e_h) {
    for (int a = 0; a < np; ++a) {
      double v = 0.0;
      for (int u = 0; u < np; ++u) v += T[u][a] * S.e[u];
      e_h[a] = v;
    }
  }
  return RBF_OK;
}

int rbf_solve(rbf_plan* P, const rbf_solve_opts* opts, double* coeffs, rbf_solve_info* info) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!coeffs) return fail(RBF_ERR_INVALID, "coeffs is NULL");
  if (P->prec < 0)
    return fail(RBF_ERR_INVALID, "rbf_assemble (or rbf_stream_finish) must precede rbf_solve");
  rbf_solve_opts o;
  o.rtol = 1e-10;
  o.max_iter = 100000;
  o.warm_start = 0;
  o.check_every = 32;
  o.reliable_delta = 0.1;
  o.stall_limit = 0;
  if (opts) o = *opts;
  if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1 ||
      !(o.reliable_delta > 0.0 && o.reliable_delta < 1.0) || o.stall_limit < 0)
    return fail(RBF_ERR_INVALID, "bad solve options");
  const bool fp32 = P->prec == RBF_PREC_FP32_REFINE;
  int rc = ensure_solver(P, fp32);
  if (rc) return rc;
  hipStream_t s = P->stream;
  if (P->npoly) {
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, &P->psys->bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad)
      return fail(RBF_ERR_SINGULAR,
                  "P^T P of the linear polynomial is singular (points on a line or plane)");
    if (o.warm_start)
      HIPCHK(rbf::launch_poly_coeffs(coeffs + P->m, P->pbasis, P->dim, false, P->xpoly, s));
    else
      HIPCHK(hipMemsetAsync(P->xpoly, 0, sizeof(double) * rbf::kMaxPoly, s));
  }
  if (P->ms == 0) {
    // no centre has a support: every coefficient is 0, the polynomial (if
    // any) fits alone
    HIPCHK(hipMemsetAsync(coeffs, 0, sizeof(double) * P->m, s));
    if (P->npoly) {
      HIPCHK(rbf::launch_poly_only(P->psys, P->xpoly, s));
      HIPCHK(rbf::launch_poly_coeffs(P->xpoly, P->pbasis, P->dim, true, coeffs + P->m, s));
    }
    double lam = 0.0;
    HIPCHK(hipMemcpyAsync(&lam, P->lam, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (info) {
      info->iterations = 0;
      info->reliable_updates = 0;
      info->rel_residual = 0.0;
      info->lambda = lam;
      info->precision = P->prec;
      info->status = RBF_OK;
    }
    return RBF_OK;
  }
  // the solver works on the active centres (rows in order)
  HIPCHK(rbf::launch_gather(P->g, P->srow, P->ms, P->g_s, s));
  if (o.warm_start)
    HIPCHK(rbf::launch_gather(coeffs, P->srow, P->ms, P->xhi, s));
  else
    HIPCHK(hipMemsetAsync(P->xhi, 0, sizeof(double) * P->ms, s));
  int64_t iters = 0, updates = 0;
  int used = P->prec;
  if (fp32) {
    const int limit = o.stall_limit > 0 ? o.stall_limit : rbf::kDefaultStallLimit;
    rc = run_cg<float, float>(P, P->val32, P->dinv32, P->vec32, o, &iters, &updates, limit);
    // decided on the host before any launch (solve_policy.h)
    const rbf::Fallback act = rbf::fallback_action(rc, RBF_WARN_FALLBACK, RBF_ERR_BREAKDOWN, true,
                                                   P->ps != nullptr, o.max_iter - iters);
    if (act == rbf::Fallback::kNone && rc == RBF_WARN_FALLBACK) rc = RBF_WARN_MAXITER;
    if (act != rbf::Fallback::kNone) {
      // the float64 system, then the float64 iteration from the current
      // float64 solution; the plan is a float64 plan from here on
      int rc2 = ensure_solver(P, false);
      if (rc2) return rc2;
      rc2 = act == rbf::Fallback::kReassemble ? assemble_into(P, P->phi, false)
                                              : stream_values64(P);
      if (rc2) return rc2;
      P->prec = RBF_PREC_FP64;
      HIPCHK(rbf::launch_gather(P->g, P->srow, P->ms, P->g_s, s));
      rc2 = build_halo(P);
      if (rc2) return rc2;
      const int rc4 = run_cg<double, double>(P, P->val64, P->dinv64, P->vec64, o, &iters,
                                             &updates, 0);
      rc = rc4 == RBF_OK ? RBF_WARN_FALLBACK : rc4;
      used = RBF_PREC_FP64;
    }
  } else {
    rc = build_halo(P);
    if (rc) return rc;
    rc = run_cg<double, double>(P, P->val64, P->dinv64, P->vec64, o, &iters, &updates, 0);
  }
  if (rc < 0 && rc != RBF_ERR_BREAKDOWN) return rc;
  HIPCHK(rbf::launch_scatter_rows(P->xhi, P->amap, P->m, coeffs, s));
  if (P->npoly)
    HIPCHK(rbf::launch_poly_coeffs(P->xpoly, P->pbasis, P->dim, true, coeffs + P->m, s));
  const int rcr = read_scalars(P);
  if (rcr) return rcr;
  double lam = 0.0;
  HIPCHK(hipMemcpyAsync(&lam, P->lam, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    info->iterations = iters;
    info->reliable_updates = updates;
    const double gg = P->host_sc->gg;
    info->rel_residual = gg > 0 ? sqrt(P->host_sc->rr_true / gg) : 0.0;
    info->lambda = lam;
    info->precision = used;
    info->status = rc;
  }
  return rc;
}

// The LSQR solve's operators on the extended system: rows [A P] (the points,
// sorted order) and, with a ridge, sqrt(lambda) [I 0] (the centres); unknowns
// (c in caller order, k in the scaled basis), nA = m + npoly values.
struct LsqrOps {
  rbf_plan* P;
  double damp;
  int64_t n, m, na;
  // t_n = [A P] x (points), and u_d = damp x_c when out_d is not NULL
  int apply(const double* x, double* tn, double* kp) {
    hipStream_t s = P->stream;
    HIPCHK(rbf::launch_gather(x, P->cperm, m, P->cs_sorted, s));
    if (P->npoly) HIPCHK(rbf::launch_poly_coeffs(x + m, P->pbasis, P->dim, true, kp, s));
    HIPCHK(rbf::launch_eval(P->view(), P->phi, n, P->ps, P->cs_sorted, P->rho2_s, P->irho_s,
                            P->npoly ? kp : nullptr, tn, s));
    return RBF_OK;
  }
  // t = [A P]^T u (+ damp u_d on the c part)
  int adjoint(const double* u, const double* ud, double* t) {
    hipStream_t s = P->stream;
    HIPCHK(rbf::launch_rhs(P->view(), P->phi, false, P->grouped, u, t, s));
    if (P->npoly)
      HIPCHK(rbf::lsqr_poly_adjoint(P->ps, n, P->dim, P->pbasis, u, P->lq_part, t + m, s));
    if (damp > 0.0) HIPCHK(rbf::lsqr_axpby(m, damp, ud, 1.0, t, s));
    return RBF_OK;
  }
  // ||a||^2 (+ ||b||^2) read back to the host
  int norm2(const double* a, int64_t na_, const double* b, int64_t nb_, double* out) {
    hipStream_t s = P->stream;
    HIPCHK(rbf::lsqr_sumsq(a, na_, P->lq_part, P->lq_sc, s));
    if (b) HIPCHK(rbf::lsqr_sumsq(b, nb_, P->lq_part, P->lq_sc + 1, s));
    double h[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(h, P->lq_sc, sizeof(double) * (b ? 2 : 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = h[0] + h[1];
    return RBF_OK;
  }
};

int rbf_solve_batch(rbf_plan* P, int32_t nrhs, const double* values,
                    const rbf_solve_opts* opts, double* coeffs, rbf_solve_info* info) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!P->ps) return fail(RBF_ERR_INVALID, "a stream plan holds no points");
  if (!values || !coeffs) return fail(RBF_ERR_INVALID, "values/coeffs is NULL");
  if (nrhs < 2 || nrhs > rbf::kMaxRhs)
    return fail(RBF_ERR_INVALID, "nrhs must be in [2, %d]", rbf::kMaxRhs);
  if (P->prec < 0) return fail(RBF_ERR_INVALID, "rbf_assemble must precede rbf_solve_batch");
  if (P->npoly)
    return fail(RBF_ERR_INVALID,
                "the batched solve takes no polynomial block (use rbf_set_values and "
                "rbf_solve per component)");
  rbf_solve_opts o;
  o.rtol = 1e-10;
  o.max_iter = 100000;
  o.warm_start = 0;
  o.check_every = 32;
  o.reliable_delta = 0.1;
  o.stall_limit = 0;
  if (opts) o = *opts;
  if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1 ||
      !(o.reliable_delta > 0.0 && o.reliable_delta < 1.0) || o.stall_limit < 0)
    return fail(RBF_ERR_INVALID, "bad solve options");
  const bool fp32 = P->prec == RBF_PREC_FP32_REFINE;
  int rc = ensure_solver(P, fp32);
  if (rc) return rc;
  rc = ensure_batch(P, fp32);
  if (rc) return rc;
  hipStream_t s = P->stream;
  const int64_t m = P->m, ms = P->ms;
  double lam = 0.0;
  int64_t iters = 0, updates = 0;
  if (ms == 0) {
    // no centre has a support: every coefficient is 0
    HIPCHK(hipMemsetAsync(coeffs, 0, sizeof(double) * m * nrhs, s));
  } else {
    // g of every component as rbf_set_values forms it, over the solver rows
    for (int k = 0; k < nrhs; ++k) {
      HIPCHK(rbf::launch_gather(values + (int64_t)k * P->n, P->pperm, P->n, P->hs, s));
      HIPCHK(rbf::launch_rhs(P->view(), P->phi, fp32, P->grouped, P->hs, P->g, s));
      HIPCHK(rbf::launch_gather(P->g, P->srow, ms, P->bg + (int64_t)k * ms, s));
      if (o.warm_start)
        HIPCHK(rbf::launch_gather(coeffs + (int64_t)k * m, P->srow, ms,
                                  P->bxhi + (int64_t)k * ms, s));
    }
    if (!o.warm_start) HIPCHK(hipMemsetAsync(P->bxhi, 0, sizeof(double) * ms * nrhs, s));
    if (fp32)
      rc = run_cgn<float, float>(P, P->val32, P->dinv32, nrhs, 1, o, &iters, &updates);
    else
      rc = run_cgn<double, double>(P, P->val64, P->dinv64, nrhs, 0, o, &iters, &updates);
    if (rc < 0 && rc != RBF_ERR_BREAKDOWN) return rc;
    for (int k = 0; k < nrhs; ++k)
      HIPCHK(rbf::launch_scatter_rows(P->bxhi + (int64_t)k * ms, P->amap, m,
                                      coeffs + (int64_t)k * m, s));
    HIPCHK(hipMemcpyAsync(P->host_bsc, P->bsc, sizeof(rbf::CgScalarsN), hipMemcpyDeviceToHost,
                          s));
  }
  HIPCHK(hipMemcpyAsync(&lam, P->lam, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    for (int k = 0; k < nrhs; ++k) {
      rbf_solve_info& f = info[k];
      f.reliable_updates = updates;
      f.lambda = lam;
      f.precision = P->prec;
      f.status = ms == 0 ? RBF_OK : rc;
      if (ms == 0) {
        f.iterations = 0;
        f.rel_residual = 0.0;
        continue;
      }
      const rbf::CgScalarsN& h = *P->host_bsc;
      f.iterations = h.conv_iter[k] >= 0 ? h.conv_iter[k] : iters;
      f.rel_residual = h.gg[k] > 0 ? sqrt(h.rr_true[k] / h.gg[k]) : 0.0;
    }
  }
  return ms == 0 ? RBF_OK : rc;
}

int rbf_solve_lsqr(rbf_plan* P, const rbf_solve_opts* opts, double* coeffs,
                   rbf_solve_info* info) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (!coeffs) return fail(RBF_ERR_INVALID, "coeffs is NULL");
  if (P->prec < 0 || P->phi < 0)
    return fail(RBF_ERR_INVALID, "rbf_assemble must precede rbf_solve_lsqr");
  if (!P->ps) return fail(RBF_ERR_INVALID, "a plan made from point chunks holds no points");
  rbf_solve_opts o;
  o.rtol = 1e-12;
  o.max_iter = 100000;
  o.warm_start = 0;
  o.check_every = 1;
  o.reliable_delta = 0.1;
  o.stall_limit = 0;
  if (opts) o = *opts;
  if (!(o.rtol > 0.0) || o.max_iter < 1) return fail(RBF_ERR_INVALID, "bad solve options");
  hipStream_t s = P->stream;
  const int64_t n = P->n, m = P->m, na = m + P->npoly;
  if (!P->lq_u) {
    GET(P->lq_u, std::max<int64_t>(n, 1));
    GET(P->lq_tn, std::max<int64_t>(n, 1));
    GET(P->lq_ud, m);
    GET(P->lq_v, m + rbf::kMaxPoly);
    GET(P->lq_w, m + rbf::kMaxPoly);
    GET(P->lq_x, m + rbf::kMaxPoly);
    GET(P->lq_t, m + rbf::kMaxPoly);
    GET(P->lq_part, rbf::kLsqrParts * rbf::kMaxPoly);
    GET(P->lq_sc, 2 + rbf::kMaxPoly);
  }
  if (!P->cs_sorted) GET(P->cs_sorted, m);
  double lam = 0.0;
  HIPCHK(hipMemcpyAsync(&lam, P->lam, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  LsqrOps ops{P, lam > 0.0 ? sqrt(lam) : 0.0, n, m, na};
  double* kp = P->lq_sc + 2;  // polynomial coefficients in the paper's basis
  double *u = P->lq_u, *ud = P->lq_ud, *v = P->lq_v, *w = P->lq_w, *x = P->lq_x;
  double *t = P->lq_t, *tn = P->lq_tn;
  // x0: the caller's guess (inactive centres forced to 0) or 0
  if (o.warm_start) {
    HIPCHK(hipMemcpyAsync(x, coeffs, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    HIPCHK(rbf::lsqr_mask(P->active, m, x, s));
    if (P->npoly)
      HIPCHK(rbf::launch_poly_coeffs(coeffs + m, P->pbasis, P->dim, false, x + m, s));
  } else {
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * na, s));
  }
  // ||[A P]^T h|| for the final relative residual (the damping rows' right-hand
  // side is 0)
  double gnorm2 = 0.0;
  const double damp = ops.damp;
  ops.damp = 0.0;
  int rc = ops.adjoint(P->hs, ud, t);
  ops.damp = damp;
  if (rc) return rc;
  rc = ops.norm2(t, na, nullptr, 0, &gnorm2);
  if (rc) return rc;
  // u = h - [A P] x, u_d = -damp x_c; beta = ||(u, u_d)||
  rc = ops.apply(x, tn, kp);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(u, P->hs, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(rbf::lsqr_axpby(n, -1.0, tn, 1.0, u, s));
  if (ops.damp > 0.0) {
    HIPCHK(hipMemsetAsync(ud, 0, sizeof(double) * m, s));
    HIPCHK(rbf::lsqr_axpby(m, -ops.damp, x, 0.0, ud, s));
  }
  double bb = 0.0;
  rc = ops.norm2(u, n, ops.damp > 0.0 ? ud : nullptr, m, &bb);
  if (rc) return rc;
  double beta = sqrt(bb), alpha = 0.0;
  if (beta > 0.0) {
    HIPCHK(rbf::lsqr_scale(n, 1.0 / beta, u, s));
    if (ops.damp > 0.0) HIPCHK(rbf::lsqr_scale(m, 1.0 / beta, ud, s));
    rc = ops.adjoint(u, ud, v);
    if (rc) return rc;
    double aa = 0.0;
    rc = ops.norm2(v, na, nullptr, 0, &aa);
    if (rc) return rc;
    alpha = sqrt(aa);
  }
  if (alpha > 0.0) HIPCHK(rbf::lsqr_scale(na, 1.0 / alpha, v, s));
  HIPCHK(hipMemcpyAsync(w, v, sizeof(double) * na, hipMemcpyDeviceToDevice, s));
  double phibar = beta, rhobar = alpha, anorm2 = 0.0;
  int64_t it = 0;
  bool done = alpha == 0.0 || beta == 0.0;
  while (!done && it < o.max_iter) {
    ++it;
    // Golub-Kahan bidiagonalisation: beta u = A v - alpha u, alpha v = A^T u - beta v
    rc = ops.apply(v, tn, kp);
    if (rc) return rc;
    HIPCHK(rbf::lsqr_axpby(n, 1.0, tn, -alpha, u, s));
    if (ops.damp > 0.0) HIPCHK(rbf::lsqr_axpby(m, ops.damp, v, -alpha, ud, s));
    rc = ops.norm2(u, n, ops.damp > 0.0 ? ud : nullptr, m, &bb);
    if (rc) return rc;
    beta = sqrt(bb);
    anorm2 += alpha * alpha + beta * beta;
    if (beta > 0.0) {
      HIPCHK(rbf::lsqr_scale(n, 1.0 / beta, u, s));
      if (ops.damp > 0.0) HIPCHK(rbf::lsqr_scale(m, 1.0 / beta, ud, s));
      rc = ops.adjoint(u, ud, t);
      if (rc) return rc;
      HIPCHK(rbf::lsqr_axpby(na, 1.0, t, -beta, v, s));
      double aa = 0.0;
      rc = ops.norm2(v, na, nullptr, 0, &aa);
      if (rc) return rc;
      alpha = sqrt(aa);
      if (alpha > 0.0) HIPCHK(rbf::lsqr_scale(na, 1.0 / alpha, v, s));
    }
    // plane rotation eliminating beta from the lower bidiagonal
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double cs = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -cs * alpha;
    const double phi = cs * phibar;
    phibar = sn * phibar;
    HIPCHK(rbf::lsqr_step(na, phi / rho, -theta / rho, v, w, x, s));
    // ||[A P]^T r|| / (||[A P]|| ||r||) estimated from the recurrences
    const double test2 = anorm2 > 0.0 ? alpha * fabs(cs) / sqrt(anorm2) : 0.0;
    if (!(std::isfinite(rho) && std::isfinite(phibar)))
      return fail(RBF_ERR_BREAKDOWN, "LSQR: non-finite recurrence after %lld iterations",
                  (long long)it);
    if (test2 <= o.rtol || phibar == 0.0 || alpha == 0.0 || beta == 0.0) done = true;
  }
  rc = done ? RBF_OK : RBF_WARN_MAXITER;
  // the normal-equation residual of the result, recomputed: [A P]^T (h - [A P] x) - lambda x_c
  int rr = ops.apply(x, tn, kp);
  if (rr) return rr;
  HIPCHK(hipMemcpyAsync(u, P->hs, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(rbf::lsqr_axpby(n, -1.0, tn, 1.0, u, s));
  ops.damp = 0.0;
  rr = ops.adjoint(u, ud, t);
  ops.damp = damp;
  if (rr) return rr;
  if (lam > 0.0) HIPCHK(rbf::lsqr_axpby(m, -lam, x, 1.0, t, s));
  double res2 = 0.0;
  rr = ops.norm2(t, na, nullptr, 0, &res2);
  if (rr) return rr;
  HIPCHK(hipMemcpyAsync(coeffs, x, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  if (P->npoly)
    HIPCHK(rbf::launch_poly_coeffs(x + m, P->pbasis, P->dim, true, coeffs + m, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    info->iterations = it;
    info->reliable_updates = 0;
    info->rel_residual = gnorm2 > 0.0 ? sqrt(res2 / gnorm2) : 0.0;
    info->lambda = lam;
    info->precision = RBF_PREC_FP64;
    info->status = rc;
  }
  return rc;
}

static int eval_impl(const rbf_plan* Pc, int64_t nq, const double* queries, const double* coeffs,
                     double* out, const double* values, double* rmse_h) {
  rbf_plan* P = const_cast<rbf_plan*>(Pc);
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (nq < 0) return fail(RBF_ERR_INVALID, "n_query < 0");
  if (nq > 0 && (!queries || !coeffs || !out)) return fail(RBF_ERR_INVALID, "NULL pointer");
  if (values && !rmse_h) return fail(RBF_ERR_INVALID, "rmse_h is NULL");
  hipStream_t s = P->stream;
  if (!P->cs_sorted) GET(P->cs_sorted, P->m);
  if (nq > 0) {
    HIPCHK(rbf::launch_gather(coeffs, P->cperm, P->m, P->cs_sorted, s));
    HIPCHK(rbf::launch_eval(P->view(), P->phi < 0 ? 1 : P->phi, nq, queries, P->cs_sorted,
                            P->rho2_s, P->irho_s, P->npoly ? coeffs + P->m : nullptr, out, s));
  }
  if (values) {
    if (nq == 0) {
      *rmse_h = 0.0;
      return RBF_OK;
    }
    if (!P->eval_part) GET(P->eval_part, kEvalParts + 1);
    const int nb = rbf::sq_err_blocks(nq);
    HIPCHK(rbf::launch_sq_err(out, values, nq, P->eval_part, nb, P->eval_part + kEvalParts, s));
    double sum = 0.0;
    HIPCHK(hipMemcpyAsync(&sum, P->eval_part + kEvalParts, sizeof(double), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    *rmse_h = sqrt(sum / (double)nq);
  }
  return RBF_OK;
}

static int eval_noalloc_impl(const rbf_plan* Pc, int64_t nq, const double* queries,
                             const double* coeffs, double* out, const double* values,
                             double* rmse_h) {
  rbf_plan* P = const_cast<rbf_plan*>(Pc);
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (nq < 0) return fail(RBF_ERR_INVALID, "n_query < 0");
  if (nq > 0 && (!queries || !coeffs || !out)) return fail(RBF_ERR_INVALID, "NULL pointer");
  if (values && !rmse_h) return fail(RBF_ERR_INVALID, "rmse_h is NULL");
  if (P->m > RBF_NOALLOC_MAX_CENTERS)
    return fail(RBF_ERR_INVALID,
                "rbf_eval_noalloc takes at most %lld centres (the plan has %lld); use rbf_eval",
                (long long)RBF_NOALLOC_MAX_CENTERS, (long long)P->m);
  double* scr = nullptr;
  const int rc = noalloc_scratch(&scr);
  if (rc) return rc;
  // scratch: the coefficients in centre-hash order [M], then the squared-error
  // partial sums [kEvalParts] and their total
  double* cs_sorted = scr;
  double* part = scr + RBF_NOALLOC_MAX_CENTERS;
  hipStream_t s = P->stream;
  if (nq > 0) {
    HIPCHK(rbf::launch_gather(coeffs, P->cperm, P->m, cs_sorted, s));
    HIPCHK(rbf::launch_eval(P->view(), P->phi < 0 ? 1 : P->phi, nq, queries, cs_sorted,
                            P->rho2_s, P->irho_s, P->npoly ? coeffs + P->m : nullptr, out, s));
  }
  if (values) {
    if (nq == 0) {
      *rmse_h = 0.0;
      return RBF_OK;
    }
    const int nb = rbf::sq_err_blocks(nq);
    HIPCHK(rbf::launch_sq_err(out, values, nq, part, nb, part + kEvalParts, s));
    double sum = 0.0;
    HIPCHK(hipMemcpyAsync(&sum, part + kEvalParts, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *rmse_h = sqrt(sum / (double)nq);
  }
  return RBF_OK;
}

int rbf_stream_begin(const rbf_stream_desc* d, const rbf_allocator* allocator, void* stream,
                     rbf_plan** out) {
  if (!out) return fail(RBF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!d) return fail(RBF_ERR_INVALID, "desc is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(RBF_ERR_INVALID, "dim must be 2 or 3");
  if (d->n_centers < 1 || d->n_centers >= (int64_t(1) << 31))
    return fail(RBF_ERR_INVALID, "n_centers must be in [1, 2^31)");
  if (!d->centers) return fail(RBF_ERR_INVALID, "centers is NULL");
  if (!d->rho_per_center && !(d->rho > 0.0 && isfinite(d->rho)))
    return fail(d->rho > 0.0 ? RBF_ERR_NONFINITE : RBF_ERR_INVALID,
                "rho must be finite and > 0");
  if (d->min_support < 1) return fail(RBF_ERR_INVALID, "min_support must be >= 1");
  if (!(d->lambda_rel >= 0.0 && isfinite(d->lambda_rel)))
    return fail(RBF_ERR_INVALID, "lambda_rel must be finite and >= 0");
  if ((int)d->phi < 0 || (int)d->phi > 3) return fail(RBF_ERR_INVALID, "unknown basis function");
  if ((int)d->precision < 0 || (int)d->precision > 1)
    return fail(RBF_ERR_INVALID, "unknown precision");
  if (d->max_chunk < 1 || d->max_chunk >= (int64_t(1) << 31))
    return fail(RBF_ERR_INVALID, "max_chunk must be in [1, 2^31)");
  if (d->flags & ~(RBF_PLAN_NO_STAGING | RBF_PLAN_ROW_ASSEMBLY))
    return fail(RBF_ERR_INVALID, "unknown plan flags");
  if (allocator && (!allocator->alloc || !allocator->release))
    return fail(RBF_ERR_INVALID, "allocator callbacks are NULL");
  rbf_plan* P = new rbf_plan();
  if (allocator) {
    P->alloc = *allocator;
    P->custom_alloc = true;
  }
  P->stream = (hipStream_t)stream;
  P->dim = d->dim;
  P->n = 0;
  P->m = d->n_centers;
  P->min_support = d->min_support;
  P->lambda_rel = d->lambda_rel;
  P->staging = (d->flags & RBF_PLAN_NO_STAGING) == 0;
  P->row_assembly = (d->flags & RBF_PLAN_ROW_ASSEMBLY) != 0;
  P->max_chunk = d->max_chunk;
  P->phi = (int)d->phi;
  P->stream_prec = (int)d->precision;
  int rc = setup_centres(P, d->centers, d->rho_per_center, d->rho, nullptr);
  if (!rc) rc = build_stream(P);
  if (rc != RBF_OK) {
    delete P;
    return rc;
  }
  P->stream_state = 1;
  *out = P;
  return RBF_OK;
}

int rbf_stream_add(rbf_plan* P, int64_t n, const double* points, const double* values,
                   int32_t on_host) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (P->stream_state != 1)
    return fail(RBF_ERR_INVALID, P->stream_state ? "the stream is finished"
                                                 : "not a stream plan (rbf_stream_begin)");
  if (n < 0 || n > P->max_chunk)
    return fail(RBF_ERR_INVALID, "chunk of %lld points (max_chunk %lld)", (long long)n,
                (long long)P->max_chunk);
  if (n == 0) return RBF_OK;
  if (!points || !values) return fail(RBF_ERR_INVALID, "points/values is NULL");
  const double* x = points;
  const double* h = values;
  int slot = -1;
  if (on_host) {
    int rc = ensure_staging(P);
    if (rc) return rc;
    slot = P->stage_next;
    P->stage_next ^= 1;
    // the slot's previous chunk has been consumed by the plan's stream
    if (P->stage_pending[slot]) HIPCHK(hipStreamWaitEvent(P->copy_stream, P->ev_used[slot], 0));
    const int dim = P->dim;
    for (int d = 0; d < dim; ++d)
      HIPCHK(hipMemcpyAsync(P->stage_x[slot] + d * n, points + d * n, sizeof(double) * n,
                            hipMemcpyHostToDevice, P->copy_stream));
    HIPCHK(hipMemcpyAsync(P->stage_h[slot], values, sizeof(double) * n, hipMemcpyHostToDevice,
                          P->copy_stream));
    HIPCHK(hipEventRecord(P->ev_copied[slot], P->copy_stream));
    HIPCHK(hipStreamWaitEvent(P->stream, P->ev_copied[slot], 0));
    x = P->stage_x[slot];
    h = P->stage_h[slot];
  }
  int rc = stream_chunk(P, n, x, h);
  if (rc) return rc;
  if (on_host) {
    HIPCHK(hipEventRecord(P->ev_used[slot], P->stream));
    P->stage_pending[slot] = true;
    // the previous host chunk has been copied: its memory is the caller's again
    const int prev = slot ^ 1;
    if (P->stage_pending[prev]) HIPCHK(hipEventSynchronize(P->ev_copied[prev]));
  }
  P->n += n;
  return RBF_OK;
}

static int stream_finish_impl(rbf_plan* P) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  if (P->stream_state != 1)
    return fail(RBF_ERR_INVALID, P->stream_state ? "the stream is finished"
                                                 : "not a stream plan (rbf_stream_begin)");
  if (P->copy_stream) HIPCHK(hipStreamSynchronize(P->copy_stream));
  const int rc = finish_stream(P);
  if (rc) return rc;
  P->stream_state = 2;
  return RBF_OK;
}

int rbf_profile(rbf_plan* P, int32_t enable) {
  if (!P) return fail(RBF_ERR_INVALID, "plan is NULL");
  HIPCHK(hipStreamSynchronize(P->stream));
  P->resolve(INT64_MAX, true);
  for (int k = 0; k < 3; ++k) {
    P->prof_launches[k] = 0;
    P->prof_ms[k] = 0.0;
  }
  P->prof_on = enable != 0;
  return RBF_OK;
}

int rbf_profile_read(rbf_plan* P, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!P || kernel < 0 || kernel > 2) return fail(RBF_ERR_INVALID, "bad plan or kernel id");
  HIPCHK(hipStreamSynchronize(P->stream));
  P->resolve(INT64_MAX, true);
  if (launches) *launches = P->prof_launches[kernel];
  if (total_ms) *total_ms = P->prof_ms[kernel];
  return RBF_OK;
}

void rbf_plan_destroy(rbf_plan* P) { delete P; }

}  // extern "C"

// ---------------------------------------------------------------- learned radius
struct rbf_mlp {
  hipStream_t stream = nullptr;
  float* params = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* scale = nullptr;  // input standardisation {mean[16], std[16]}
  int64_t t = 0;  // Adam steps taken
  ~rbf_mlp() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (params) (void)hipFree(params);
    if (m1) (void)hipFree(m1);
    if (m2) (void)hipFree(m2);
    if (scale) (void)hipFree(scale);
  }
};

namespace {

int ensure_cbox(rbf_plan* P) {
  if (!P->cbox_dev) {
    GET(P->cbox_dev, 6);
    HIPCHK(hipMemcpyAsync(P->cbox_dev, P->cbox, sizeof P->cbox, hipMemcpyHostToDevice, P->stream));
  }
  return RBF_OK;
}

int check_blocks(const rbf_plan* P, int32_t bpd, int* nblocks) {
  if (bpd < 1) return fail(RBF_ERR_INVALID, "blocks_per_dim must be >= 1");
  int64_t nb = 1;
  for (int d = 0; d < P->dim; ++d) nb *= bpd;
  if (nb > 65536) return fail(RBF_ERR_INVALID, "too many blocks");
  *nblocks = (int)nb;
  return RBF_OK;
}

template <typename T>
struct DevTmp {
  T* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(int64_t n) { return hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(n, 1)); }
};

}  // namespace

extern "C" {

int rbf_density_features(rbf_plan* P, int32_t n_radii, const double* radii_h,
                         int32_t blocks_per_dim, float* feats) {
  if (!P || !radii_h || !feats) return fail(RBF_ERR_INVALID, "NULL argument");
  if (!P->ps) return fail(RBF_ERR_INVALID, "a stream plan holds no points");
  if (n_radii < 1 || n_radii > rbf::kMaxRadii)
    return fail(RBF_ERR_INVALID, "n_radii must be in [1, %d]", rbf::kMaxRadii);
  double rmax = 0.0;
  for (int s = 0; s < n_radii; ++s) {
    if (!(radii_h[s] > 0.0) || !isfinite(radii_h[s])) return fail(RBF_ERR_INVALID, "bad radius");
    rmax = std::max(rmax, radii_h[s]);
  }
  int nblocks = 0;
  int rc = check_blocks(P, blocks_per_dim, &nblocks);
  if (rc) return rc;
  rc = ensure_cbox(P);
  if (rc) return rc;
  const int reach = (int)ceil(rmax / P->cell_size);
  if (reach > 4) return fail(RBF_ERR_INVALID, "sweep radius exceeds four hash cells");
  hipStream_t s = P->stream;
  DevTmp<double> radii;
  DevTmp<int32_t> counts, blk;
  HIPCHK(radii.alloc(n_radii));
  HIPCHK(counts.alloc(P->m * n_radii));
  HIPCHK(blk.alloc(P->m));
  HIPCHK(hipMemcpyAsync(radii.p, radii_h, sizeof(double) * n_radii, hipMemcpyHostToDevice, s));
  HIPCHK(rbf::launch_density_counts(P->view(), radii.p, n_radii, reach, counts.p, s));
  HIPCHK(rbf::launch_centre_blocks(P->ctr, P->m, P->dim, P->cbox_dev, blocks_per_dim, blk.p, s));
  HIPCHK(rbf::launch_block_features(counts.p, blk.p, P->m, n_radii, nblocks, feats, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBF_OK;
}

int rbf_block_sq_err(rbf_plan* P, int64_t n_query, const double* queries, const double* f,
                     const double* h, int32_t blocks_per_dim, double* sums_h, int64_t* counts_h) {
  if (!P || !sums_h || !counts_h) return fail(RBF_ERR_INVALID, "NULL argument");
  if (n_query < 0 || (n_query > 0 && (!queries || !f || !h)))
    return fail(RBF_ERR_INVALID, "bad queries");
  int nblocks = 0;
  int rc = check_blocks(P, blocks_per_dim, &nblocks);
  if (rc) return rc;
  rc = ensure_cbox(P);
  if (rc) return rc;
  hipStream_t s = P->stream;
  DevTmp<double> sums;
  DevTmp<int64_t> counts;
  HIPCHK(sums.alloc(nblocks));
  HIPCHK(counts.alloc(nblocks));
  HIPCHK(rbf::launch_block_sq_err(queries, n_query, P->dim, f, h, P->cbox_dev, blocks_per_dim,
                                  nblocks, sums.p, counts.p, s));
  HIPCHK(hipMemcpyAsync(sums_h, sums.p, sizeof(double) * nblocks, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(counts_h, counts.p, sizeof(int64_t) * nblocks, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBF_OK;
}

int rbf_radius_broadcast(rbf_plan* P, const float* pred_log, int32_t blocks_per_dim,
                         double spacing, double rho_min, double rho_max, double rho_fallback,
                         double* rho_out) {
  if (!P || !pred_log || !rho_out) return fail(RBF_ERR_INVALID, "NULL argument");
  if (!(spacing > 0.0) || !(rho_min > 0.0) || !(rho_max >= rho_min) || !(rho_fallback > 0.0))
    return fail(RBF_ERR_INVALID, "bad radius bounds");
  int nblocks = 0;
  int rc = check_blocks(P, blocks_per_dim, &nblocks);
  if (rc) return rc;
  rc = ensure_cbox(P);
  if (rc) return rc;
  hipStream_t s = P->stream;
  DevTmp<int32_t> blk;
  HIPCHK(blk.alloc(P->m));
  HIPCHK(rbf::launch_centre_blocks(P->ctr, P->m, P->dim, P->cbox_dev, blocks_per_dim, blk.p, s));
  HIPCHK(rbf::launch_radius_broadcast(pred_log, blk.p, P->m, spacing, rho_min, rho_max,
                                      rho_fallback, rho_out, s));
  HIPCHK(hipStreamSynchronize(s));
  return RBF_OK;
}

int rbf_mlp_create(const float* params_h, void* stream, rbf_mlp** out) {
  if (!out || !params_h) return fail(RBF_ERR_INVALID, "NULL argument");
  *out = nullptr;
  rbf_mlp* M = new rbf_mlp();
  M->stream = (hipStream_t)stream;
  const size_t bytes = sizeof(float) * rbf::kMlpParams;
  if (hipMalloc(&M->params, bytes) != hipSuccess || hipMalloc(&M->m1, bytes) != hipSuccess ||
      hipMalloc(&M->m2, bytes) != hipSuccess ||
      hipMalloc(&M->scale, sizeof(float) * 2 * rbf::kMlpInputs) != hipSuccess) {
    (void)hipGetLastError();
    delete M;
    return fail(RBF_ERR_OOM, "MLP allocation failed");
  }
  float unit[2 * rbf::kMlpInputs];
  for (int i = 0; i < rbf::kMlpInputs; ++i) {
    unit[i] = 0.0f;
    unit[rbf::kMlpInputs + i] = 1.0f;
  }
  hipError_t e = hipMemcpyAsync(M->params, params_h, bytes, hipMemcpyHostToDevice, M->stream);
  if (e == hipSuccess) e = hipMemsetAsync(M->m1, 0, bytes, M->stream);
  if (e == hipSuccess) e = hipMemsetAsync(M->m2, 0, bytes, M->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(M->scale, unit, sizeof(unit), hipMemcpyHostToDevice, M->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
  if (e != hipSuccess) {
    delete M;
    return fail(RBF_ERR_HIP, "MLP set-up failed: %s", hipGetErrorString(e));
  }
  *out = M;
  return RBF_OK;
}

int rbf_mlp_params(const rbf_mlp* M, float* params_h) {
  if (!M || !params_h) return fail(RBF_ERR_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(params_h, M->params, sizeof(float) * rbf::kMlpParams,
                        hipMemcpyDeviceToHost, M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  return RBF_OK;
}

int rbf_mlp_grad(rbf_mlp* M, const float* x, const float* y, int64_t n, float* grad_h,
                 float* loss_h) {
  if (!M || !x || !y || !grad_h || !loss_h) return fail(RBF_ERR_INVALID, "NULL argument");
  if (n < 1) return fail(RBF_ERR_INVALID, "n must be >= 1");
  DevTmp<float> g;
  HIPCHK(g.alloc(rbf::kMlpParams + 1));
  HIPCHK(rbf::launch_mlp_grad(M->params, M->scale, x, y, n, g.p, g.p + rbf::kMlpParams,
                              M->stream));
  HIPCHK(hipMemcpyAsync(grad_h, g.p, sizeof(float) * rbf::kMlpParams, hipMemcpyDeviceToHost,
                        M->stream));
  HIPCHK(hipMemcpyAsync(loss_h, g.p + rbf::kMlpParams, sizeof(float), hipMemcpyDeviceToHost,
                        M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  return RBF_OK;
}

int rbf_mlp_train(rbf_mlp* M, const float* x, const float* y, int64_t n_rows,
                  const int32_t* order, int32_t steps, int32_t batch, float lr, float* losses_h) {
  if (!M || !x || !y || !order) return fail(RBF_ERR_INVALID, "NULL argument");
  if (n_rows < 1 || steps < 0 || batch < 1 || batch > 4096 || !(lr > 0.0f))
    return fail(RBF_ERR_INVALID, "bad training arguments");
  if (steps == 0) return RBF_OK;
  const int64_t total = (int64_t)steps * batch;
  // every row index is read by the kernel: check them on the host first
  std::vector<int32_t> ord(total);
  HIPCHK(hipMemcpyAsync(ord.data(), order, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                        M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  for (int64_t k = 0; k < total; ++k)
    if (ord[k] < 0 || ord[k] >= n_rows) return fail(RBF_ERR_INVALID, "order index out of range");
  DevTmp<float> losses;
  HIPCHK(losses.alloc(steps));
  HIPCHK(rbf::launch_mlp_train(M->params, M->m1, M->m2, M->scale, x, y, order, steps, batch, lr,
                               (int)M->t, losses.p, M->stream));
  M->t += steps;
  if (losses_h)
    HIPCHK(hipMemcpyAsync(losses_h, losses.p, sizeof(float) * steps, hipMemcpyDeviceToHost,
                          M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  return RBF_OK;
}

int rbf_mlp_infer_bf16(const rbf_mlp* M, const float* x, int64_t n, float* out) {
  if (!M || (n > 0 && (!x || !out))) return fail(RBF_ERR_INVALID, "NULL argument");
  if (n < 0) return fail(RBF_ERR_INVALID, "n < 0");
  HIPCHK(rbf::launch_mlp_infer_bf16(M->params, M->scale, x, n, out, M->stream));
  return RBF_OK;
}

int rbf_mlp_set_input_scaling(rbf_mlp* M, const float* mean_h, const float* std_h) {
  if (!M || !mean_h || !std_h) return fail(RBF_ERR_INVALID, "NULL argument");
  float sc[2 * rbf::kMlpInputs];
  for (int i = 0; i < rbf::kMlpInputs; ++i) {
    if (!std::isfinite(mean_h[i]) || !std::isfinite(std_h[i]) || !(std_h[i] > 0.0f))
      return fail(RBF_ERR_INVALID, "input scaling: mean must be finite and std finite and > 0");
    sc[i] = mean_h[i];
    sc[rbf::kMlpInputs + i] = std_h[i];
  }
  HIPCHK(hipMemcpyAsync(M->scale, sc, sizeof(sc), hipMemcpyHostToDevice, M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  return RBF_OK;
}

int rbf_mlp_state(const rbf_mlp* M, float* params_h, float* m1_h, float* m2_h, int64_t* step_h,
                  float* mean_h, float* std_h) {
  if (!M) return fail(RBF_ERR_INVALID, "NULL argument");
  const size_t bytes = sizeof(float) * rbf::kMlpParams;
  const size_t half = sizeof(float) * rbf::kMlpInputs;
  if (params_h)
    HIPCHK(hipMemcpyAsync(params_h, M->params, bytes, hipMemcpyDeviceToHost, M->stream));
  if (m1_h) HIPCHK(hipMemcpyAsync(m1_h, M->m1, bytes, hipMemcpyDeviceToHost, M->stream));
  if (m2_h) HIPCHK(hipMemcpyAsync(m2_h, M->m2, bytes, hipMemcpyDeviceToHost, M->stream));
  if (mean_h) HIPCHK(hipMemcpyAsync(mean_h, M->scale, half, hipMemcpyDeviceToHost, M->stream));
  if (std_h)
    HIPCHK(hipMemcpyAsync(std_h, M->scale + rbf::kMlpInputs, half, hipMemcpyDeviceToHost,
                          M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  if (step_h) *step_h = M->t;
  return RBF_OK;
}

int rbf_mlp_load_state(rbf_mlp* M, const float* params_h, const float* m1_h, const float* m2_h,
                       int64_t step, const float* mean_h, const float* std_h) {
  if (!M || !params_h || !m1_h || !m2_h || !mean_h || !std_h)
    return fail(RBF_ERR_INVALID, "NULL argument");
  if (step < 0 || step > (int64_t)1 << 30) return fail(RBF_ERR_INVALID, "bad Adam step count");
  const int rc = rbf_mlp_set_input_scaling(M, mean_h, std_h);
  if (rc) return rc;
  const size_t bytes = sizeof(float) * rbf::kMlpParams;
  HIPCHK(hipMemcpyAsync(M->params, params_h, bytes, hipMemcpyHostToDevice, M->stream));
  HIPCHK(hipMemcpyAsync(M->m1, m1_h, bytes, hipMemcpyHostToDevice, M->stream));
  HIPCHK(hipMemcpyAsync(M->m2, m2_h, bytes, hipMemcpyHostToDevice, M->stream));
  HIPCHK(hipStreamSynchronize(M->stream));
  M->t = step;
  return RBF_OK;
}

void rbf_mlp_destroy(rbf_mlp* M) { delete M; }


// The exported entry points whose kernels carry the checked build's device
// checks (checks.h): in that build a failed check turns the status into
// RBF_ERR_HIP naming the place; in a normal build they pass the status on.

int rbf_fit_plan(const rbf_plan_desc* d, const rbf_allocator* allocator, void* stream,
                 rbf_plan** out) {
  int rc = fit_plan_impl(d, allocator, stream, out);
  if (rc < 0) return rc;
  rc = device_checks(*out, rc);
  if (rc < 0) {
    delete *out;
    *out = nullptr;
  }
  return rc;
}

int rbf_assemble(rbf_plan* P, rbf_phi phi, rbf_precision prec, const double* values) {
  const int rc = assemble_impl(P, phi, prec, values);
  return rc < 0 ? rc : device_checks(P, rc);
}

int rbf_eval(const rbf_plan* P, int64_t nq, const double* queries, const double* coeffs,
             double* out, const double* values, double* rmse_h) {
  const int rc = eval_impl(P, nq, queries, coeffs, out, values, rmse_h);
  return rc < 0 ? rc : device_checks(P, rc);
}

int rbf_eval_noalloc(const rbf_plan* P, int64_t nq, const double* queries, const double* coeffs,
                     double* out, const double* values, double* rmse_h) {
  const int rc = eval_noalloc_impl(P, nq, queries, coeffs, out, values, rmse_h);
  return rc < 0 ? rc : device_checks(P, rc);
}

int rbf_stream_finish(rbf_plan* P) {
  const int rc = stream_finish_impl(P);
  return rc < 0 ? rc : device_checks(P, rc);
}
}  // extern "C"
