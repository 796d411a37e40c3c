// Neighbourhoods of the solver's slices, for the CG iteration that stages
// them in LDS (see CgMatrix).  For slice s (rows s*S .. s*S + S - 1 of the
// sliced-ELL layout) the set U_s of distinct columns its stored entries
// reference, padding included, is sorted; column c gets the slot
// rank(c) in U_s.  Stored per slice: |U_s| (hcount, -1 when the slice does not
// qualify), the members as int16 offsets from the slice's first row (hrow,
// at hptr[s]), and per stored entry its slot (hslot, at the entry's sliced-ELL
// position).  One wave per slice: a bitmap over the slice's column range in
// LDS, popcounts for the ranks.
#include "plan_kernels.h"
#include "solver.h"

namespace rbf {
namespace {

constexpr int kHaloWords = kHaloSpan / 32;
constexpr int kHaloWaves = 4;

template <typename CT>
__device__ __forceinline__ int32_t entry_col(const CgMatrix& A, int64_t ms, int64_t slice,
                                             int lane, int step, int L) {
  const int64_t rows = kWave / L;
  const int64_t row = slice * rows + lane / L;
  const int32_t rowc = (int32_t)(row < ms ? row : ms - 1);
  const int64_t o = A.sptr[slice] + lane + (int64_t)step * kWave;
  return rowc + (int32_t)static_cast<const CT*>(A.col)[o];
}

// Column range of the slice over all its stored entries (wave-uniform).
template <typename CT>
__device__ __forceinline__ void slice_range(const CgMatrix& A, int64_t ms, int64_t slice, int L,
                                            int32_t* cmin, int32_t* cmax) {
  const int lane = threadIdx.x & (kWave - 1);
  const int steps = A.slen[slice] / L;
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  for (int t = 0; t < steps; ++t) {
    const int32_t c = entry_col<CT>(A, ms, slice, lane, t, L);
    lo = c < lo ? c : lo;
    hi = c > hi ? c : hi;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t a = __shfl_xor(lo, off, kWave), b = __shfl_xor(hi, off, kWave);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  *cmin = lo;
  *cmax = hi;
}

// Marks the slice's columns in the wave's bitmap (cleared first).
template <typename CT>
__device__ __forceinline__ void slice_bitmap(const CgMatrix& A, int64_t ms, int64_t slice, int L,
                                             int32_t cmin, uint32_t* bits) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int w = lane; w < kHaloWords; w += kWave) bits[w] = 0u;
  wave_sync();
  const int steps = A.slen[slice] / L;
  for (int t = 0; t < steps; ++t) {
    const int32_t b = entry_col<CT>(A, ms, slice, lane, t, L) - cmin;
    atomicOr(&bits[b >> 5], 1u << (b & 31));
  }
  wave_sync();
}

// |U_s| of every slice, or -1 when its column range exceeds kHaloSpan bits,
// its offsets do not fit int16, or it has more than `cap` columns.
template <typename CT>
__global__ __launch_bounds__(kWave* kHaloWaves) void k_halo_count(CgMatrix A, int64_t ms, int L,
                                                                  int cap,
                                                                  int32_t* __restrict__ hcount) {
  __shared__ uint32_t bits[kHaloWaves][kHaloWords];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t slice = (int64_t)blockIdx.x * kHaloWaves + wave;
  if (slice >= A.nslices) return;
  int32_t cmin, cmax;
  slice_range<CT>(A, ms, slice, L, &cmin, &cmax);
  const int64_t first = slice * (kWave / L);
  const bool fits = (int64_t)cmax - cmin + 1 <= kHaloSpan && cmin - first >= -32768 &&
                    cmax - first <= 32767;
  if (!fits) {
    if (lane == 0) hcount[slice] = -1;
    return;
  }
  slice_bitmap<CT>(A, ms, slice, L, cmin, bits[wave]);
  int n = 0;
  for (int w = lane; w < kHaloWords; w += kWave) n += __popc(bits[wave][w]);
  n = wave_sum_int(n);
  if (lane == 0) hcount[slice] = n <= cap ? n : -1;
}

// Members (hrow) and entry slots (hslot) of every qualifying slice.
template <typename CT>
__global__ __launch_bounds__(kWave* kHaloWaves) void k_halo_fill(
    CgMatrix A, int64_t ms, int L, const int32_t* __restrict__ hcount,
    const int64_t* __restrict__ hptr, int16_t* __restrict__ hrow, int16_t* __restrict__ hslot) {
  __shared__ uint32_t bits[kHaloWaves][kHaloWords];
  __shared__ int32_t rank[kHaloWaves][kHaloWords];  // set bits below each word
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t slice = (int64_t)blockIdx.x * kHaloWaves + wave;
  if (slice >= A.nslices || hcount[slice] < 0) return;
  int32_t cmin, cmax;
  slice_range<CT>(A, ms, slice, L, &cmin, &cmax);
  slice_bitmap<CT>(A, ms, slice, L, cmin, bits[wave]);
  // exclusive prefix of the words' popcounts: lane-contiguous runs of words
  constexpr int kPer = kHaloWords / kWave;
  int run = 0;
  for (int k = 0; k < kPer; ++k) run += __popc(bits[wave][lane * kPer + k]);
  int incl = run;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int v = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += v;
  }
  int acc = incl - run;
  for (int k = 0; k < kPer; ++k) {
    const int w = lane * kPer + k;
    rank[wave][w] = acc;
    acc += __popc(bits[wave][w]);
  }
  wave_sync();
  const int64_t first = slice * (kWave / L);
  const int64_t base = hptr[slice];
  // members in ascending order
  for (int k = 0; k < kPer; ++k) {
    const int w = lane * kPer + k;
    uint32_t word = bits[wave][w];
    int r = rank[wave][w];
    while (word) {
      const int b = __ffs(word) - 1;
      word &= word - 1;
      hrow[base + r] = (int16_t)((int64_t)cmin + w * 32 + b - first);
      ++r;
    }
  }
  // slot of every stored entry
  const int steps = A.slen[slice] / L;
  for (int t = 0; t < steps; ++t) {
    const int32_t b = entry_col<CT>(A, ms, slice, lane, t, L) - cmin;
    const uint32_t word = bits[wave][b >> 5];
    const int32_t slot = rank[wave][b >> 5] + __popc(word & ((1u << (b & 31)) - 1u));
    hslot[A.sptr[slice] + lane + (int64_t)t * kWave] = (int16_t)slot;
  }
}

}  // namespace

hipError_t launch_halo_count(const CgMatrix& A, int64_t ms, int cap, int32_t* hcount,
                             hipStream_t s) {
  if (A.nslices <= 0) return hipSuccess;
  const dim3 grid((unsigned)((A.nslices + kHaloWaves - 1) / kHaloWaves));
  if (A.col16)
    hipLaunchKernelGGL(k_halo_count<int16_t>, grid, dim3(kWave * kHaloWaves), 0, s, A, ms, A.lanes,
                       cap, hcount);
  else
    hipLaunchKernelGGL(k_halo_count<int32_t>, grid, dim3(kWave * kHaloWaves), 0, s, A, ms, A.lanes,
                       cap, hcount);
  return hipGetLastError();
}

hipError_t launch_halo_fill(const CgMatrix& A, int64_t ms, const int32_t* hcount,
                            const int64_t* hptr, int16_t* hrow, int16_t* hslot, hipStream_t s) {
  if (A.nslices <= 0) return hipSuccess;
  const dim3 grid((unsigned)((A.nslices + kHaloWaves - 1) / kHaloWaves));
  if (A.col16)
    hipLaunchKernelGGL(k_halo_fill<int16_t>, grid, dim3(kWave * kHaloWaves), 0, s, A, ms, A.lanes,
                       hcount, hptr, hrow, hslot);
  else
    hipLaunchKernelGGL(k_halo_fill<int32_t>, grid, dim3(kWave * kHaloWaves), 0, s, A, ms, A.lanes,
                       hcount, hptr, hrow, hslot);
  return hipGetLastError();
}

}  // namespace rbf
