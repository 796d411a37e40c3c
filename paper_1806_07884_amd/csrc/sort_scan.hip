// Prefix sums, stable LSD radix sort and cell-start extraction for the
// uniform-grid hash.  Every result is deterministic: no floating point, and
// the only atomics are integer histogram counts in LDS.
#include "internal.h"

namespace rbf {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // 2048
constexpr int kWavesPerBlock = kThreads / kWave;

template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int off) {
  if constexpr (sizeof(T) == 8) {
    return (T)__shfl_up((long long)v, off, kWave);
  } else {
    return (T)__shfl_up((int)v, off, kWave);
  }
}

// Exclusive scan of one value per thread over a 256-thread block.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wsum, T* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  T incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T t = shfl_up_t(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    T x = wsum[w];
    if (w < wave) pre += x;
    tot += x;
  }
  *total = tot;
  __syncthreads();
  return pre + incl - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_tile_sums(const T* __restrict__ in, int64_t n,
                                                        T* __restrict__ sums) {
  __shared__ T wsum[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T acc = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
    if (idx < n) acc += in[idx];
  }
  T tot;
  block_exclusive_scan(acc, wsum, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of `n` values by one block, tile after tile with a carry.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_single(T* __restrict__ data, int64_t n) {
  __shared__ T wsum[kWavesPerBlock];
  T carry = 0;
  for (int64_t base = 0; base < n; base += kTile) {
    T v[kItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
      v[i] = idx < n ? data[idx] : (T)0;
      s += v[i];
    }
    T tot;
    T run = carry + block_exclusive_scan(s, wsum, &tot);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
      if (idx < n) data[idx] = run;
      run += v[i];
    }
    carry += tot;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const T* in, T* out, int64_t n,
                                                         const T* __restrict__ tile_off) {
  __shared__ T wsum[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T v[kItems];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
    v[i] = idx < n ? in[idx] : (T)0;
    s += v[i];
  }
  T tot;
  T run = tile_off[blockIdx.x] + block_exclusive_scan(s, wsum, &tot);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
}

template <typename T>
hipError_t scan_impl(const T* in, T* out, int64_t n, void* temp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + kTile - 1) / kTile;
  T* sums = static_cast<T*>(temp);
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(kThreads), 0, s, sums, tiles);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out, n,
                     (const T*)sums);
  return hipGetLastError();
}

// ---- radix sort ----------------------------------------------------------
constexpr int kBins = 256;

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         int64_t n, int shift,
                                                         uint32_t* __restrict__ hist,
                                                         int nblocks) {
  __shared__ uint32_t h[kBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kBins - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: within a 64-lane wave, lanes with equal digits are ranked by
// lane order through ballot match masks; waves are ranked in order through
// per-digit counters in LDS; tiles through the scanned histogram.
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t n, int shift, const uint32_t* __restrict__ offs,
    int nblocks) {
  __shared__ uint32_t run[kBins];
  __shared__ uint32_t wc[kWavesPerBlock][kBins];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const uint64_t lt = lanemask_lt();
  for (int i = 0; i < kItems; ++i) {
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t idx = base + (int64_t)i * kThreads + tid;
    const bool valid = idx < n;
    uint32_t key = valid ? kin[idx] : 0u;
    int32_t val = valid ? vin[idx] : 0;
    const uint32_t d = (key >> shift) & (kBins - 1);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & lt);
    const int cnt = __popcll(m);
    if (valid && rank == cnt - 1) wc[wave][d] = (uint32_t)cnt;
    __syncthreads();
    {
      uint32_t o = run[tid];
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) {
        uint32_t c = wc[w][tid];
        wc[w][tid] = o;
        o += c;
      }
      run[tid] = o;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = wc[wave][d] + (uint32_t)rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

__global__ void k_cell_starts(const uint32_t* __restrict__ keys, int64_t n, int32_t ncell,
                              int shift, int32_t* __restrict__ cell_start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  // boundary between sorted position i-1 and i: cells (prev, cur] start at i
  const int64_t prev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> shift);
  const int64_t cur = i == n ? (int64_t)ncell + 1 : (int64_t)(keys[i] >> shift);
  for (int64_t c = prev + 1; c <= cur; ++c) cell_start[c] = (int32_t)i;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
  const int64_t tiles = (n + kTile - 1) / kTile;
  return (size_t)(tiles + 1) * sizeof(int64_t);
}

hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s) {
  return scan_impl<uint32_t>(in, out, n, temp, s);
}
hipError_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, temp, s);
}

size_t radix_temp_bytes(int64_t n) {
  const int64_t nblocks = (n + kTile - 1) / kTile;
  const int64_t hist = nblocks * kBins;
  return (size_t)hist * sizeof(uint32_t) + scan_temp_bytes(hist) + 256;
}

hipError_t radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                            int64_t n, int key_bits, void* temp, hipStream_t s, bool* in_alt) {
  *in_alt = false;
  if (n <= 0) return hipSuccess;
  const int nblocks = (int)((n + kTile - 1) / kTile);
  const int64_t hn = (int64_t)nblocks * kBins;
  uint32_t* hist = static_cast<uint32_t*>(temp);
  char* stemp = static_cast<char*>(temp) + (((size_t)hn * sizeof(uint32_t) + 255) & ~(size_t)255);
  uint32_t* ka = keys;
  int32_t* va = vals;
  uint32_t* kb = keys_alt;
  int32_t* vb = vals_alt;
  const int passes = key_bits <= 0 ? 0 : (key_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kThreads), 0, s, (const uint32_t*)ka, n,
                       shift, hist, nblocks);
    hipError_t e = scan_impl<uint32_t>(hist, hist, hn, stemp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kThreads), 0, s, (const uint32_t*)ka,
                       (const int32_t*)va, kb, vb, n, shift, (const uint32_t*)hist, nblocks);
    uint32_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  *in_alt = (passes & 1) != 0;
  return hipGetLastError();
}

hipError_t cell_starts(const uint32_t* sorted_keys, int64_t n, int32_t ncell, int shift,
                       int32_t* cell_start, hipStream_t s) {
  const int64_t threads = n + 1;
  const int bs = 256;
  hipLaunchKernelGGL(k_cell_starts, dim3((unsigned)((threads + bs - 1) / bs)), dim3(bs), 0, s,
                     sorted_keys, n, ncell, shift, cell_start);
  return hipGetLastError();
}

}  // namespace rbf
