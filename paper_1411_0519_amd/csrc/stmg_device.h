// Device helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace stmg {
namespace dev {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// element j of lane l is D[row(l/16, j)][l%16].  The row mapping differs between
// the two instructions (measured on gfx950): f64 interleaves, f32 is blocked.
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int g, int j) { return g + 4 * j; }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int g, int j) { return 4 * g + j; }
};

__device__ inline long long slab_index() {
  return (long long)blockIdx.y + (long long)gridDim.y * blockIdx.z;
}

inline dim3 slab_grid(unsigned gx, long long slabs) {
  const long long ymax = 65535;
  unsigned gy = (unsigned)(slabs < ymax ? slabs : ymax);
  unsigned gz = (unsigned)((slabs + ymax - 1) / ymax);
  return dim3(gx, gy, gz);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Map dispatch index b (of B) to a logical index so that every XCD processes
// one contiguous range of logical workgroups: neighbours in memory (halo rows,
// the previous slab, cache lines split between column groups) then meet in the
// same L2.  A bijection on [0, B) for any B.
__device__ inline long long xcd_linear(long long b, long long B) {
  const long long q = B >> 3, rm = B & 7;
  const long long x = b & 7, i = b >> 3;
  return x * q + (x < rm ? x : rm) + i;
}

// q = e / n for 0 <= e < 2^20 via a float reciprocal and one correction step.
__device__ inline int div_small(int e, int n, float inv_n) {
  int q = (int)((float)e * inv_n);
  if (q * n > e) --q;
  else if ((q + 1) * n <= e) ++q;
  return q;
}
}  // namespace dev
}  // namespace stmg
