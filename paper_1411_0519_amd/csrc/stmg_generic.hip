// Kernels for high DG orders (N_t > 4 time dofs per slab): the time dimension
// is a runtime size and the N_t x N_t time matrices live in device tables.
// The block solve of such levels runs the sine-transform passes along every
// spatial axis (they do not depend on N_t) and the per-mode time solve below
// as a separate kernel.
//
//   k_residual_gen     r = F - L u (eq. chap4_generalLinearSystem), fused
//                      per-block partial sums of r^2
//   k_time_solve_gen   x-hat = G_k r-hat per spatial sine mode k
//   k_restrict_gen,    time blocks R1, R2 (eq. chap4_restrictionTime) with
//   k_prolong_gen      optional full weighting / linear interpolation in space
//   k_rhs_gen,         load vector and its transpose (Sec. 1)
//   k_rhs_adjoint_gen
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

inline unsigned blocks_for(long long total) { return (unsigned)((total + 255) / 256); }

__device__ inline double block_sum_gen(double v) {
  __shared__ double red[8];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
  }
  return s;
}

// (M_h v)(node) of one component v.
template <typename T, int D>
__device__ inline T mass1(const T* __restrict__ v, int n, int x, int y, int z, const T* wm) {
  T acc = T(0);
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= n) continue;
    for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= n) continue;
      const long long row = ((long long)zz * n + yy) * n;
      T s = T(0);
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx;
        if (xx < 0 || xx >= n) continue;
        s += wm[dx + 1] * v[row + xx];
      }
      acc += ((D == 3) ? wm[dz + 1] : T(1)) * ((D >= 2) ? wm[dy + 1] : T(1)) * s;
    }
  }
  return acc;
}

template <typename Tin, typename Tout, int D>
__global__ __launch_bounds__(256) void k_residual_gen(const Tin* __restrict__ u, const Tin* __restrict__ F,
                                                      Tout* __restrict__ r, GenArgs<Tin> a,
                                                      double* __restrict__ partial) {
  typedef Tin T;
  const long long slab = slab_index();
  const long long nslab = (long long)a.batch * a.N;
  if (slab >= nslab) return;
  const long long nx = a.nx;
  const int n = a.n, nt = a.nt;
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int sn = (int)(slab % a.N);
  double ss = 0.0;
  if (j < nx) {
    int x, y, z;
    node_coords<D>(j, n, x, y, z);
    const long long slabsz = (long long)nt * nx;
    const T* un = u + slab * slabsz;
    T mu[NT_BIG], ku[NT_BIG];
    for (int l = 0; l < nt; ++l) stencil_mk<T, D, 1>(un + l * nx, nx, n, x, y, z, a.wm, a.wk, &mu[l], &ku[l]);
    T mw = T(0);
    const int sp = sn + a.dir;
    if (sp >= 0 && sp < a.N) {
      const T* up = u + (slab + a.dir) * slabsz;
      for (int l = 0; l < nt; ++l) mw += a.cb[l] * mass1<T, D>(up + l * nx, n, x, y, z, a.wm);
    }
    const T* Fn = F + slab * slabsz;
    Tout* rn = r + slab * slabsz;
    for (int l = 0; l < nt; ++l) {
      T acc = Fn[l * nx + j] + a.ca[l] * mw;
      for (int k = 0; k < nt; ++k) acc -= a.K[l * nt + k] * mu[k] + a.tau * a.M[l * nt + k] * ku[k];
      rn[l * nx + j] = (Tout)acc;
      ss += (double)acc * (double)acc;
    }
  }
  if (partial != nullptr) {
    const double s = block_sum_gen(ss);
    if (threadIdx.x == 0) partial[slab * gridDim.x + blockIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_time_solve_gen(const T* in, T* out, const T* __restrict__ G, long long nx,
                                                        int nt, long long slabs, int transpose, T omega, int mode) {
  const long long slab = slab_index();
  if (slab >= slabs) return;
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nx) return;
  const T* v = in + slab * nt * nx + j;
  const T* g = G + j * nt * nt;
  T y[NT_BIG];
  for (int l = 0; l < nt; ++l) {
    T acc = T(0);
    for (int m = 0; m < nt; ++m) acc += (transpose ? g[m * nt + l] : g[l * nt + m]) * v[m * nx];
    y[l] = acc;
  }
  T* o = out + slab * nt * nx + j;
  for (int l = 0; l < nt; ++l) {
    const T old = mode == MODE_ADD_SCALED ? o[l * nx] : T(0);
    o[l * nx] = mode == MODE_STORE ? y[l] : (mode == MODE_ADD_SCALED ? old + omega * y[l] : omega * y[l]);
  }
}

template <typename T, int D, bool FULL>
__global__ __launch_bounds__(256) void k_restrict_gen(const T* __restrict__ rf, T* __restrict__ Fc,
                                                      GenTransfer<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nxc = a.nxc, nxf = a.nxf;
  const int nt = a.nt;
  if (idx >= nxc * a.Nc * a.batch) return;
  const long long jc = idx % nxc;
  const long long cs = idx / nxc;
  const long long m = cs % a.Nc;
  const long long bi = cs / a.Nc;
  const long long fs0 = bi * (2LL * a.Nc) + 2 * m;
  T v0[NT_BIG], v1[NT_BIG];
  for (int s = 0; s < 2; ++s) {
    T* v = s == 0 ? v0 : v1;
    const T* base = rf + (fs0 + s) * nt * nxf;
    for (int k = 0; k < nt; ++k) {
      if (FULL) {
        int cx, cy, cz;
        node_coords<D>(jc, a.nc, cx, cy, cz);
        const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = 2 * cz + 1, nf = a.nf;
        T acc = T(0);
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
          for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
            const T wzy = (dz == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
            const long long rz = (D == 3) ? (fz + dz) : 0;
            const long long ry = (D >= 2) ? (fy + dy) : 0;
            const T* line = base + k * nxf + (rz * nf + ry) * nf;
            acc += wzy * (T(0.5) * line[fx - 1] + line[fx] + T(0.5) * line[fx + 1]);
          }
        v[k] = acc;
      } else {
        v[k] = base[k * nxf + jc];
      }
    }
  }
  T* out = Fc + cs * nt * nxc + jc;
  for (int l = 0; l < nt; ++l) {
    T acc = T(0);
    for (int k = 0; k < nt; ++k) acc += a.R1T[k * nt + l] * v0[k] + a.R2T[k * nt + l] * v1[k];
    out[l * nxc] = acc;
  }
}

template <typename T, int D, bool FULL>
__global__ __launch_bounds__(256) void k_prolong_gen(const T* __restrict__ ec, T* __restrict__ uf, GenTransfer<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nxc = a.nxc, nxf = a.nxf;
  const int nt = a.nt;
  if (idx >= nxf * a.Nc * a.batch) return;
  const long long jf = idx % nxf;
  const long long cs = idx / nxf;
  const long long m = cs % a.Nc;
  const long long bi = cs / a.Nc;
  const long long fs0 = bi * (2LL * a.Nc) + 2 * m;
  const T* ecs = ec + cs * nt * nxc;
  T e[NT_BIG];
  for (int k = 0; k < nt; ++k) e[k] = T(0);
  if (FULL) {
    int fc[3];
    node_coords<D>(jf, a.nf, fc[0], fc[1], fc[2]);
    const int nc = a.nc;
    int c[3][2], cnt[3];
    T w[3][2];
    for (int ax = 0; ax < 3; ++ax) {
      if (ax >= D) {
        c[ax][0] = 0;
        w[ax][0] = T(1);
        cnt[ax] = 1;
        continue;
      }
      const int f = fc[ax];
      if (f & 1) {
        c[ax][0] = (f - 1) >> 1;
        w[ax][0] = T(1);
        cnt[ax] = 1;
      } else {
        cnt[ax] = 0;
        if ((f >> 1) - 1 >= 0) {
          c[ax][cnt[ax]] = (f >> 1) - 1;
          w[ax][cnt[ax]++] = T(0.5);
        }
        if ((f >> 1) < nc) {
          c[ax][cnt[ax]] = f >> 1;
          w[ax][cnt[ax]++] = T(0.5);
        }
      }
    }
    for (int iz = 0; iz < cnt[2]; ++iz)
      for (int iy = 0; iy < cnt[1]; ++iy)
        for (int ix = 0; ix < cnt[0]; ++ix) {
          const long long jc = ((long long)c[2][iz] * nc + c[1][iy]) * nc + c[0][ix];
          const T ww = w[2][iz] * w[1][iy] * w[0][ix];
          for (int k = 0; k < nt; ++k) e[k] += ww * ecs[k * nxc + jc];
        }
  } else {
    for (int k = 0; k < nt; ++k) e[k] = ecs[k * nxc + jf];
  }
  T* u0 = uf + fs0 * nt * nxf + jf;
  T* u1 = u0 + nt * nxf;
  for (int l = 0; l < nt; ++l) {
    T a0 = T(0), a1 = T(0);
    for (int k = 0; k < nt; ++k) {
      a0 += a.R1T[l * nt + k] * e[k];
      a1 += a.R2T[l * nt + k] * e[k];
    }
    u0[l * nxf] += a0;
    u1[l * nxf] += a1;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_rhs_gen(const T* __restrict__ f, const T* __restrict__ u0,
                                                 T* __restrict__ F, GenArgs<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nx = a.nx;
  if (idx >= nx * a.N * a.batch) return;
  const long long j = idx % nx;
  const long long s = idx / nx;
  const long long sn = s % a.N;
  const long long bi = s / a.N;
  int x, y, z;
  node_coords<D>(j, a.n, x, y, z);
  const T mf = mass1<T, D>(f + s * nx, a.n, x, y, z, a.wm);
  T mu0 = T(0);
  if (sn == 0 && u0 != nullptr) mu0 = mass1<T, D>(u0 + bi * nx, a.n, x, y, z, a.wm);
  T* out = F + s * a.nt * nx + j;
  for (int l = 0; l < a.nt; ++l) out[l * nx] = a.tau * a.ints[l] * mf + a.ca[l] * mu0;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_rhs_adjoint_gen(const T* __restrict__ lam, T* __restrict__ gf,
                                                         T* __restrict__ gu0, GenArgs<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nx = a.nx;
  if (idx >= nx * a.N * a.batch) return;
  const long long j = idx % nx;
  const long long s = idx / nx;
  const long long sn = s % a.N;
  const long long bi = s / a.N;
  int x, y, z;
  node_coords<D>(j, a.n, x, y, z);
  const T* ls = lam + s * a.nt * nx;
  if (gf != nullptr) {
    T acc = T(0);
    for (int l = 0; l < a.nt; ++l) acc += a.tau * a.ints[l] * mass1<T, D>(ls + l * nx, a.n, x, y, z, a.wm);
    gf[s * nx + j] = acc;
  }
  if (gu0 != nullptr && sn == 0) {
    T acc = T(0);
    for (int l = 0; l < a.nt; ++l) acc += a.ca[l] * mass1<T, D>(ls + l * nx, a.n, x, y, z, a.wm);
    gu0[bi * nx + j] = acc;
  }
}

}  // namespace

template <typename Tin, typename Tout>
hipError_t launch_residual_gen(int dim, const Tin* u, const Tin* F, Tout* r, const GenArgs<Tin>& a, double* partial,
                               hipStream_t s) {
  const dim3 grid = slab_grid(blocks_for(a.nx), (long long)a.batch * a.N);
  if (dim == 1) hipLaunchKernelGGL((k_residual_gen<Tin, Tout, 1>), grid, dim3(256), 0, s, u, F, r, a, partial);
  else if (dim == 2) hipLaunchKernelGGL((k_residual_gen<Tin, Tout, 2>), grid, dim3(256), 0, s, u, F, r, a, partial);
  else if (dim == 3) hipLaunchKernelGGL((k_residual_gen<Tin, Tout, 3>), grid, dim3(256), 0, s, u, F, r, a, partial);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

unsigned residual_gen_blocks_per_slab(long long nx) { return blocks_for(nx); }

template <typename T>
hipError_t launch_time_solve_gen(const T* in, T* out, const T* G, long long nx, int nt, long long slabs, int transpose,
                                 T omega, int mode, hipStream_t s) {
  const dim3 grid = slab_grid(blocks_for(nx), slabs);
  hipLaunchKernelGGL((k_time_solve_gen<T>), grid, dim3(256), 0, s, in, out, G, nx, nt, slabs, transpose, omega, mode);
  return hipGetLastError();
}

#define GEN_TRANSFER(KERNEL, TOTAL, ...)                                                         \
  const unsigned grid = blocks_for(TOTAL);                                                       \
  if (full) {                                                                                    \
    if (dim == 1) hipLaunchKernelGGL((KERNEL<T, 1, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 2) hipLaunchKernelGGL((KERNEL<T, 2, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 3) hipLaunchKernelGGL((KERNEL<T, 3, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else return hipErrorInvalidValue;                                                            \
  } else {                                                                                       \
    hipLaunchKernelGGL((KERNEL<T, 1, false>), dim3(grid), dim3(256), 0, s, __VA_ARGS__);         \
  }                                                                                              \
  return hipGetLastError();

template <typename T>
hipError_t launch_restrict_gen(int dim, bool full, const T* rf, T* Fc, const GenTransfer<T>& a, hipStream_t s) {
  GEN_TRANSFER(k_restrict_gen, a.nxc * a.Nc * a.batch, rf, Fc, a)
}

template <typename T>
hipError_t launch_prolong_gen(int dim, bool full, const T* ec, T* uf, const GenTransfer<T>& a, hipStream_t s) {
  GEN_TRANSFER(k_prolong_gen, a.nxf * a.Nc * a.batch, ec, uf, a)
}
#undef GEN_TRANSFER

template <typename T>
hipError_t launch_rhs_gen(int dim, const T* f, const T* u0, T* F, const GenArgs<T>& a, hipStream_t s) {
  const unsigned grid = blocks_for(a.nx * a.N * a.batch);
  if (dim == 1) hipLaunchKernelGGL((k_rhs_gen<T, 1>), dim3(grid), dim3(256), 0, s, f, u0, F, a);
  else if (dim == 2) hipLaunchKernelGGL((k_rhs_gen<T, 2>), dim3(grid), dim3(256), 0, s, f, u0, F, a);
  else if (dim == 3) hipLaunchKernelGGL((k_rhs_gen<T, 3>), dim3(grid), dim3(256), 0, s, f, u0, F, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs_adjoint_gen(int dim, const T* lam, T* gf, T* gu0, const GenArgs<T>& a, hipStream_t s) {
  const unsigned grid = blocks_for(a.nx * a.N * a.batch);
  if (dim == 1) hipLaunchKernelGGL((k_rhs_adjoint_gen<T, 1>), dim3(grid), dim3(256), 0, s, lam, gf, gu0, a);
  else if (dim == 2) hipLaunchKernelGGL((k_rhs_adjoint_gen<T, 2>), dim3(grid), dim3(256), 0, s, lam, gf, gu0, a);
  else if (dim == 3) hipLaunchKernelGGL((k_rhs_adjoint_gen<T, 3>), dim3(grid), dim3(256), 0, s, lam, gf, gu0, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_residual_gen<double, double>(int, const double*, const double*, double*,
                                                        const GenArgs<double>&, double*, hipStream_t);
template hipError_t launch_residual_gen<double, float>(int, const double*, const double*, float*,
                                                       const GenArgs<double>&, double*, hipStream_t);
template hipError_t launch_residual_gen<float, float>(int, const float*, const float*, float*, const GenArgs<float>&,
                                                      double*, hipStream_t);
#define INST(T)                                                                                         \
  template hipError_t launch_time_solve_gen<T>(const T*, T*, const T*, long long, int, long long, int, T, int, \
                                               hipStream_t);                                            \
  template hipError_t launch_restrict_gen<T>(int, bool, const T*, T*, const GenTransfer<T>&, hipStream_t); \
  template hipError_t launch_prolong_gen<T>(int, bool, const T*, T*, const GenTransfer<T>&, hipStream_t);  \
  template hipError_t launch_rhs_gen<T>(int, const T*, const T*, T*, const GenArgs<T>&, hipStream_t);      \
  template hipError_t launch_rhs_adjoint_gen<T>(int, const T*, T*, T*, const GenArgs<T>&, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
