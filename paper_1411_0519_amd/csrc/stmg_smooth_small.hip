// Damped block-Jacobi step for small levels: one workgroup per slab keeps the
// slab in LDS and performs u_out = u_in + omega D^{-1} (F - L u_in)
// (eq. chap4_smoother with the exact block inverse, eq. chap4_smootherExact):
// residual with the Q1 stencils and the coupling to the neighbouring slab,
// forward DST-I along every axis, the per-mode N_t x N_t solve, the inverse
// DST-I and the damped update.  u_in and u_out are different buffers (Jacobi:
// every slab reads its neighbour's old values).  The plain (unfolded) DST-I
// matrix is read through the L1 cache; the per-mode blocks are stored in the
// folded spectral order, so plain mode k maps to spectral index s(k).
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

__device__ inline int spectral_of(int k, int n) {
  const int kk = k + 1, h = (n + 1) >> 1;
  return (kk & 1) ? (kk - 1) >> 1 : h + (kk >> 1) - 1;
}

template <typename T, int D>
__device__ inline void coords(int j, int n, int& x, int& y, int& z) {
  x = j % n;
  y = D >= 2 ? (j / n) % n : 0;
  z = D == 3 ? j / (n * n) : 0;
}

// one DST-I pass along `axis` over the NT components: out = S * in along the axis
// (four independent partial sums per output, so that the loads of a row overlap)
template <typename T, int D, int NT>
__device__ inline void dst_axis(const T* __restrict__ S, const T* in, T* out, int n, int nx, int axis) {
  const int stride = axis == 0 ? 1 : (axis == 1 ? n : n * n);
  for (int e = threadIdx.x; e < NT * nx; e += blockDim.x) {
    const int l = e / nx, j = e - (e / nx) * nx;
    const int k = (j / stride) % n;
    const int base = l * nx + j - k * stride;
    const T* srow = S + k * n;
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    int i = 0;
    for (; i + 4 <= n; i += 4) {
      a0 += srow[i] * in[base + i * stride];
      a1 += srow[i + 1] * in[base + (i + 1) * stride];
      a2 += srow[i + 2] * in[base + (i + 2) * stride];
      a3 += srow[i + 3] * in[base + (i + 3) * stride];
    }
    for (; i < n; ++i) a0 += srow[i] * in[base + i * stride];
    out[e] = (a0 + a1) + (a2 + a3);
  }
}

template <typename T, int D, int NT>
__global__ __launch_bounds__(512) void k_smooth_small(const T* __restrict__ u_in, T* __restrict__ u_out,
                                                      const T* __restrict__ F, const T* __restrict__ Sg,
                                                      const T* __restrict__ G, SmallArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const ResidArgs<T>& ra = a.r;
  const int n = ra.n;
  const int nx = (int)ra.nx;
  T* U = reinterpret_cast<T*>(lds_raw);   // NT * nx
  T* W = U + NT * nx;                     // nx   (coupling combination of the neighbour slab)
  T* R = W + nx;                          // NT * nx
  T* Q = R + NT * nx;                     // NT * nx
  T* Sl = Q + NT * nx;                    // n * n (the sine matrix, when a.s_lds)
  const long long slab = slab_index();
  if (slab >= (long long)ra.batch * ra.N) return;
  const int sn = (int)(slab % ra.N);
  const long long slabsz = (long long)NT * nx;
  const bool couple = !a.u_zero && sn + ra.dir >= 0 && sn + ra.dir < ra.N;
  for (int e = threadIdx.x; e < NT * nx; e += blockDim.x) U[e] = a.u_zero ? T(0) : u_in[slab * slabsz + e];
  if (a.s_lds)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Sl[e] = Sg[e];
  const T* S = a.s_lds ? Sl : Sg;
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    T w = T(0);
    if (couple) {
      const T* up = u_in + (slab + ra.dir) * slabsz;
#pragma unroll
      for (int k = 0; k < NT; ++k) w += ra.cb[k] * up[k * nx + j];
    }
    W[j] = w;
  }
  __syncthreads();
  // ---- residual R = F - A u + ca (M_h w)
  const T* Fn = F + slab * slabsz;
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    int x, y, z;
    coords<T, D>(j, n, x, y, z);
    T mu[NT + 1], ku[NT];
#pragma unroll
    for (int c = 0; c <= NT; ++c) mu[c] = T(0);
#pragma unroll
    for (int c = 0; c < NT; ++c) ku[c] = T(0);
    if (!a.u_zero) {
      for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz) {
        const int zz = z + dz;
        if (zz < 0 || zz >= n) continue;
        for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
          const int yy = y + dy;
          if (yy < 0 || yy >= n) continue;
          const int row = (zz * n + yy) * n;
          const T wzy = (D == 3 ? ra.wm[dz + 1] : T(1)) * (D >= 2 ? ra.wm[dy + 1] : T(1));
          T kzy = T(0);   // weight of the x-mass row sum in the stiffness
          if (D == 2) kzy = ra.wk[dy + 1];
          if (D == 3) kzy = ra.wk[dz + 1] * ra.wm[dy + 1] + ra.wm[dz + 1] * ra.wk[dy + 1];
#pragma unroll
          for (int c = 0; c <= NT; ++c) {
            const T* src = c < NT ? U + c * nx : W;
            T sm = T(0), sk = T(0);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const int xx = x + dx;
              if (xx < 0 || xx >= n) continue;
              const T v = src[row + xx];
              sm += ra.wm[dx + 1] * v;
              sk += ra.wk[dx + 1] * v;
            }
            mu[c] += wzy * sm;
            if (c < NT) ku[c] += kzy * sm + wzy * sk;
          }
        }
      }
    }
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T acc = Fn[l * nx + j] + ra.ca[l] * mu[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) acc -= ra.K[l * NT + k] * mu[k] + ra.M[l * NT + k] * ku[k];
      R[l * nx + j] = acc;
    }
  }
  __syncthreads();
  // ---- forward transforms, per-mode solve, inverse transforms
  T* cur = R;
  T* oth = Q;
  for (int axis = 0; axis < D; ++axis) {
    dst_axis<T, D, NT>(S, cur, oth, n, nx, axis);
    __syncthreads();
    T* t = cur;
    cur = oth;
    oth = t;
  }
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    int x, y, z;
    coords<T, D>(j, n, x, y, z);
    int js = spectral_of(x, n);
    if (D >= 2) js += n * spectral_of(y, n);
    if (D == 3) js += n * n * spectral_of(z, n);
    const T* g = G + (long long)js * NT * NT;
    T v[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) v[k] = cur[k * nx + j];
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) acc += (a.transpose ? g[k * NT + l] : g[l * NT + k]) * v[k];
      cur[l * nx + j] = acc;
    }
  }
  __syncthreads();
  for (int axis = D - 1; axis >= 0; --axis) {
    dst_axis<T, D, NT>(S, cur, oth, n, nx, axis);
    __syncthreads();
    T* t = cur;
    cur = oth;
    oth = t;
  }
  T* uo = u_out + slab * slabsz;
  for (int e = threadIdx.x; e < NT * nx; e += blockDim.x) uo[e] = U[e] + a.omega * cur[e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ in, T* __restrict__ out, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = in[i];
}

}  // namespace

size_t smooth_small_lds(int dim, int n, long long nx, int nt, size_t elem) {
  if (dim < 1 || dim > 3 || nt < 1 || nt > NT_MAX) return 0;
  const size_t bytes = (size_t)(3 * nt + 1) * (size_t)nx * elem;
  if (bytes > 64 * 1024) return 0;
  const size_t with_s = bytes + (size_t)n * n * elem;   // the sine matrix too, where it fits
  return with_s <= 64 * 1024 ? with_s : bytes;
}

template <typename T>
hipError_t launch_smooth_small(int dim, int nt, const T* u_in, T* u_out, const T* F, const T* Splain,
                               const T* G, const SmallArgs<T>& a, hipStream_t s) {
  const size_t lds = smooth_small_lds(dim, a.r.n, a.r.nx, nt, sizeof(T));
  if (lds == 0) return hipErrorInvalidValue;
  SmallArgs<T> b = a;
  b.s_lds = lds > (size_t)(3 * nt + 1) * (size_t)a.r.nx * sizeof(T) ? 1 : 0;
  const dim3 grid = slab_grid(1, (long long)a.r.batch * a.r.N);
#define SMALL_CASE(D, NT)                                                                     \
  if (dim == D && nt == NT) {                                                                 \
    hipLaunchKernelGGL((k_smooth_small<T, D, NT>), grid, dim3(512), lds, s, u_in, u_out, F, Splain, G, b); \
    return hipGetLastError();                                                                 \
  }
  SMALL_CASE(1, 1) SMALL_CASE(1, 2) SMALL_CASE(1, 3) SMALL_CASE(1, 4)
  SMALL_CASE(2, 1) SMALL_CASE(2, 2) SMALL_CASE(2, 3) SMALL_CASE(2, 4)
  SMALL_CASE(3, 1) SMALL_CASE(3, 2) SMALL_CASE(3, 3) SMALL_CASE(3, 4)
#undef SMALL_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_copy(const T* in, T* out, long long len, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, in, out, len);
  return hipGetLastError();
}

template hipError_t launch_smooth_small<double>(int, int, const double*, double*, const double*, const double*,
                                                const double*, const SmallArgs<double>&, hipStream_t);
template hipError_t launch_smooth_small<float>(int, int, const float*, float*, const float*, const float*,
                                               const float*, const SmallArgs<float>&, hipStream_t);
template hipError_t launch_copy<double>(const double*, double*, long long, hipStream_t);
template hipError_t launch_copy<float>(const float*, float*, long long, hipStream_t);

}  // namespace stmg
