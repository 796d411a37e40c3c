// Device-side building blocks shared by the CS-RBF kernels (gfx950, wave64).
//
//  * the canonical squared distance and the strict support predicate of
//    Algorithm 1 / eq. 18;
//  * the Wendland basis functions of Table 2 (plus phi_{3,2});
//  * the uniform-grid cell geometry used for every neighbour search;
//  * wave64 reductions and stream compaction helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbf {

constexpr int kWave = 64;

// Uniform grid over the box [lo, lo + g * cs) in every dimension.  Cell ids are
// row-major with the first coordinate fastest, so the cells (x0..x1, y, z) form
// one contiguous id range.  Id ``ncell`` is the "outside the box" sentinel.
struct Grid {
  double lo[3];
  double inv_cs;
  int32_t g[3];
  int32_t ncell;
};

// s = (dx*dx + dy*dy) + dz*dz with dx = a - b, every operation rounded on its
// own.  Contraction into fused multiply-adds is switched off so that the value
// (and therefore every support decision) is the same bit pattern the CPU
// computes for the same inputs.
template <int DIM>
__device__ __forceinline__ double sqdist(const double* a, const double* b) {
#pragma clang fp contract(off)
  double d0 = a[0] - b[0];
  double s = d0 * d0;
  double d1 = a[1] - b[1];
  s = s + d1 * d1;
  if constexpr (DIM == 3) {
    double d2 = a[2] - b[2];
    s = s + d2 * d2;
  }
  return s;
}

// Cell coordinate of one value, -1 or g when it falls outside the box.
__device__ __forceinline__ int cell_coord(double x, double lo, double inv_cs, int g) {
  double t = (x - lo) * inv_cs;
  if (!(t >= 0.0)) return -1;            // also catches NaN
  if (t >= (double)g) return g;
  return (int)t;
}

template <int DIM>
__device__ __forceinline__ bool cell_of(const Grid& G, const double* x, int* c) {
  bool in = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    c[d] = cell_coord(x[d], G.lo[d], G.inv_cs, G.g[d]);
    in = in && c[d] >= 0 && c[d] < G.g[d];
  }
  return in;
}

template <int DIM>
__device__ __forceinline__ int cell_id(const Grid& G, const int* c) {
  int id = c[0] + G.g[0] * c[1];
  if constexpr (DIM == 3) id += G.g[0] * G.g[1] * c[2];
  return id;
}

// Wendland CS-RBFs phi_{3,s}(r) for 0 <= r (values for r >= 1 are 0).
//   s=0: (1-r)^2   s=1: (1-r)^4 (4r+1)   s=2: (1-r)^6 (35r^2+18r+3)
//   s=3: (1-r)^8 (32r^3+25r^2+8r+1)
template <int PHI, typename T>
__device__ __forceinline__ T wendland(T r) {
  T t = (T)1 - r;
  t = t > (T)0 ? t : (T)0;
  T t2 = t * t;
  if constexpr (PHI == 0) {
    return t2;
  } else if constexpr (PHI == 1) {
    T t4 = t2 * t2;
    return t4 * ((T)4 * r + (T)1);
  } else if constexpr (PHI == 2) {
    T t6 = t2 * t2 * t2;
    return t6 * (((T)35 * r + (T)18) * r + (T)3);
  } else {
    T t4 = t2 * t2;
    T t8 = t4 * t4;
    return t8 * ((((T)32 * r + (T)25) * r + (T)8) * r + (T)1);
  }
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Compensated (Kahan) accumulation.
struct Kahan32 {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

// Walk over the cells within ``reach`` cells of cell c (clipped to the grid) as
// contiguous id ranges: one range per (y, z) row, (2 reach + 1)^(DIM-1) rows.
template <int DIM>
struct NbrWalk {
  int x0, x1, cy, cz, reach, gx, gy, gz;
  __device__ __forceinline__ NbrWalk(const Grid& G, const int* c, int r) {
    reach = r;
    gx = G.g[0];
    gy = G.g[1];
    gz = DIM == 3 ? G.g[2] : 1;
    x0 = c[0] - r < 0 ? 0 : c[0] - r;
    x1 = c[0] + r >= gx ? gx - 1 : c[0] + r;
    cy = c[1];
    cz = DIM == 3 ? c[2] : 0;
  }
  __device__ __forceinline__ int rows() const {
    return DIM == 2 ? 2 * reach + 1 : (2 * reach + 1) * (2 * reach + 1);
  }
  // id range [lo, hi] (inclusive) of row k; false when the row is off the grid
  __device__ __forceinline__ bool range(int k, int& lo, int& hi) const {
    const int w = 2 * reach + 1;
    int y = cy + (k % w) - reach;
    int z = DIM == 3 ? cz + (k / w) - reach : 0;
    if (y < 0 || y >= gy || z < 0 || z >= gz) return false;
    lo = x0 + gx * (y + gy * z);
    hi = x1 + gx * (y + gy * z);
    return true;
  }
};

}  // namespace rbf
