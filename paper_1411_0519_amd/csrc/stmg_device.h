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
// Mass and stiffness stencils of all N_t time components at interior node
// (x, y, z):  mu[l] = (M_h u_l), ku[l] = (K_h u_l).  Separable: 1-D row sums
// along x, then combined with the y/z weights.
template <typename T, int D, int NT>
__device__ inline void stencil_mk(const T* __restrict__ base, long long nx, int n, int x, int y,
                                  int z, const T* wm, const T* wk, T* mu, T* ku) {
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    mu[l] = T(0);
    ku[l] = T(0);
  }
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= n) continue;
#pragma unroll
    for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= n) continue;
      const long long row = ((long long)zz * n + yy) * n;
      T sm[NT], sk[NT];
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        sm[l] = T(0);
        sk[l] = T(0);
      }
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx;
        if (xx < 0 || xx >= n) continue;
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          const T v = base[l * nx + row + xx];
          sm[l] += wm[dx + 1] * v;
          sk[l] += wk[dx + 1] * v;
        }
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        if (D == 1) {
          mu[l] += sm[l];
          ku[l] += sk[l];
        } else if (D == 2) {
          mu[l] += wm[dy + 1] * sm[l];
          ku[l] += wk[dy + 1] * sm[l] + wm[dy + 1] * sk[l];
        } else {
          const T mzy = wm[dz + 1] * wm[dy + 1];
          mu[l] += mzy * sm[l];
          ku[l] += (wk[dz + 1] * wm[dy + 1] + wm[dz + 1] * wk[dy + 1]) * sm[l] + mzy * sk[l];
        }
      }
    }
  }
}

// The same for a node index below 2^31 with 32-bit arithmetic.
template <int D>
__device__ inline void node_coords32(int j, int n, int& x, int& y, int& z) {
  const unsigned uj = (unsigned)j, un = (unsigned)n;
  if (D == 1) {
    x = j;
    y = z = 0;
    return;
  }
  const unsigned q = uj / un;
  x = (int)(uj - q * un);
  if (D == 2) {
    y = (int)q;
    z = 0;
  } else {
    const unsigned q2 = q / un;
    y = (int)(q - q2 * un);
    z = (int)q2;
  }
}

template <int D>
__device__ inline void node_coords(long long j, int n, int& x, int& y, int& z) {
  x = (int)(j % n);
  y = (D >= 2) ? (int)((j / n) % n) : 0;
  z = (D == 3) ? (int)(j / ((long long)n * n)) : 0;
}

}  // namespace dev
}  // namespace stmg
