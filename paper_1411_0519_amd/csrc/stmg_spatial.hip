// Kernels of the inexact block-Jacobi smoother (Remark V-cycleApproxSpace):
// the exact slab inverse D^{-1} is replaced by one geometric multigrid cycle
// in space for every slab matrix A = K (x) M_h + M (x) K_h.  Slabs do not
// interact; each kernel sees the level as b*N independent slabs with the
// usual [slab][time dof l][z][y][x] layout.
//
//   k_spatial          damped block-Jacobi step y = x + omega_x Dinv (f - A x)
//                      or the defect y = f - A x, written as y, scale*y or
//                      base + scale*y (the last step of a cycle writes the
//                      smoothed iterate u += omega_t x directly)
//   k_restrict_space   full weighting in space, time untouched
//   k_prolong_space    (bi/tri)linear interpolation in space, added
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

inline unsigned blocks_for(long long total) { return (unsigned)((total + 255) / 256); }

template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_spatial(const T* __restrict__ x, const T* __restrict__ f,
                                                 const T* base, T* out, SpatialArgs<T> a) {
  const long long slab = slab_index();
  if (slab >= a.slabs) return;
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nx) return;
  const long long nx = a.nx;
  const long long off = slab * NT * nx + j;
  T mu[NT], ku[NT], xv[NT];
  if (a.x_zero) {
#pragma unroll
    for (int l = 0; l < NT; ++l) mu[l] = ku[l] = xv[l] = T(0);
  } else {
    int px, py, pz;
    node_coords<D>(j, a.n, px, py, pz);
    stencil_mk<T, D, NT>(x + slab * NT * nx, nx, a.n, px, py, pz, a.wm, a.wk, mu, ku);
#pragma unroll
    for (int l = 0; l < NT; ++l) xv[l] = x[off + l * nx];
  }
  T r[NT];
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = f[off + l * nx];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
    r[l] = acc;
  }
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T y = r[l];
    if (a.op == SP_JACOBI) {
      T c = T(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) c += a.Dinv[l * NT + k] * r[k];
      y = xv[l] + a.omega * c;
    }
    T o = y;
    if (a.upd == UPD_ADD) o = base[off + l * nx] + a.scale * y;
    else if (a.upd == UPD_SET) o = a.scale * y;
    out[off + l * nx] = o;
  }
}

// 1-D full-weighting factors (1/2, 1, 1/2) around fine node 2c+1.
template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_restrict_space(const T* __restrict__ rf, T* __restrict__ fc, int nf,
                                                        int nc, long long slabs) {
  const long long slab = slab_index();
  if (slab >= slabs) return;
  const long long jc = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nxc = nc, nxf = nf;
  for (int i = 1; i < D; ++i) {
    nxc *= nc;
    nxf *= nf;
  }
  if (jc >= nxc) return;
  int cx, cy, cz;
  node_coords<D>(jc, nc, cx, cy, cz);
  const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = 2 * cz + 1;   // 1 <= f <= nf - 2
  const T* src = rf + slab * NT * nxf;
  T* dst = fc + slab * NT * nxc;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = T(0);
#pragma unroll
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
        const T wzy = (dz == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
        const long long zz = (D == 3) ? fz + dz : 0;
        const long long yy = (D >= 2) ? fy + dy : 0;
        const T* line = src + l * nxf + (zz * nf + yy) * nf;
        acc += wzy * (T(0.5) * line[fx - 1] + line[fx] + T(0.5) * line[fx + 1]);
      }
    dst[l * nxc + jc] = acc;
  }
}

// Coarse neighbours of fine index f along one axis: odd f = 2c+1 takes coarse c
// with weight 1; even f takes c = f/2 - 1 and f/2 with weight 1/2 each (those
// inside 0..nc-1; the Dirichlet boundary contributes zero).
__device__ inline int coarse_taps(int f, int nc, int* c, float* w) {
  if (f & 1) {
    c[0] = (f - 1) >> 1;
    w[0] = 1.f;
    return 1;
  }
  int k = 0;
  const int c0 = (f >> 1) - 1, c1 = f >> 1;
  if (c0 >= 0) {
    c[k] = c0;
    w[k++] = 0.5f;
  }
  if (c1 < nc) {
    c[k] = c1;
    w[k++] = 0.5f;
  }
  return k;
}

template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_prolong_space(const T* __restrict__ ec, T* __restrict__ uf, int nf,
                                                       int nc, long long slabs) {
  const long long slab = slab_index();
  if (slab >= slabs) return;
  const long long jf = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nxc = nc, nxf = nf;
  for (int i = 1; i < D; ++i) {
    nxc *= nc;
    nxf *= nf;
  }
  if (jf >= nxf) return;
  int x, y, z;
  node_coords<D>(jf, nf, x, y, z);
  int cxs[2], cys[2] = {0, 0}, czs[2] = {0, 0};
  float wx[2], wy[2] = {1.f, 1.f}, wz[2] = {1.f, 1.f};
  const int kx = coarse_taps(x, nc, cxs, wx);
  const int ky = (D >= 2) ? coarse_taps(y, nc, cys, wy) : 1;
  const int kz = (D == 3) ? coarse_taps(z, nc, czs, wz) : 1;
  const T* src = ec + slab * NT * nxc;
  T* dst = uf + slab * NT * nxf;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = T(0);
    for (int iz = 0; iz < kz; ++iz)
      for (int iy = 0; iy < ky; ++iy)
        for (int ix = 0; ix < kx; ++ix) {
          const long long jc = ((long long)czs[iz] * nc + cys[iy]) * nc + cxs[ix];
          acc += (T)(wz[iz] * wy[iy] * wx[ix]) * src[l * nxc + jc];
        }
    dst[l * nxf + jf] += acc;
  }
}

}  // namespace

#define SPATIAL_DISPATCH(KERNEL, GX, ...)                                                             \
  const dim3 grid = slab_grid(GX, slabs);                                                           \
  if (dim == 1 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 1, 1>), grid, dim3(256), 0, s, __VA_ARGS__);  \
  else if (dim == 1 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 1, 2>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 1 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 1, 3>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 1 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 1, 4>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 2, 1>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 2, 2>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 2, 3>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 2, 4>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 3, 1>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 3, 2>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 3, 3>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 3, 4>), grid, dim3(256), 0, s, __VA_ARGS__); \
  else return hipErrorInvalidValue;                                                                 \
  return hipGetLastError();

long long ipow(long long b, int e) {
  long long r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

template <typename T>
hipError_t launch_spatial(int dim, int nt, const T* x, const T* f, const T* base, T* out,
                          const SpatialArgs<T>& a, hipStream_t s) {
  const long long slabs = a.slabs;
  SPATIAL_DISPATCH(k_spatial, blocks_for(a.nx), x, f, base, out, a)
}

template <typename T>
hipError_t launch_restrict_space(int dim, int nt, const T* rf, T* fc, int nf, int nc, long long slabs,
                                 hipStream_t s) {
  SPATIAL_DISPATCH(k_restrict_space, blocks_for(ipow(nc, dim)), rf, fc, nf, nc, slabs)
}

template <typename T>
hipError_t launch_prolong_space(int dim, int nt, const T* ec, T* uf, int nf, int nc, long long slabs,
                                hipStream_t s) {
  SPATIAL_DISPATCH(k_prolong_space, blocks_for(ipow(nf, dim)), ec, uf, nf, nc, slabs)
}
#undef SPATIAL_DISPATCH

#define INST(T)                                                                                       \
  template hipError_t launch_spatial<T>(int, int, const T*, const T*, const T*, T*, const SpatialArgs<T>&, \
                                        hipStream_t);                                                 \
  template hipError_t launch_restrict_space<T>(int, int, const T*, T*, int, int, long long, hipStream_t); \
  template hipError_t launch_prolong_space<T>(int, int, const T*, T*, int, int, long long, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
