// Kernels of the inexact block-Jacobi smoother (Remark V-cycleApproxSpace):
// the exact slab inverse D^{-1} is replaced by one geometric multigrid cycle
// in space for every slab matrix A = K (x) M_h + M (x) K_h.  Slabs do not
// interact; each kernel sees the level as b*N independent slabs with the
// usual [slab][time dof l][z][y][x] layout.
//
//   k_spatial          damped block-Jacobi step y = x + omega_x Dinv (f - A x)
//                      (k_spatial_tile2d: the 2-D form on an LDS tile)
//                      or the defect y = f - A x, written as y, scale*y or
//                      base + scale*y (the last step of a cycle writes the
//                      smoothed iterate u += omega_t x directly)
//   k_restrict_space   full weighting in space, time untouched
//   k_prolong_space    (bi/tri)linear interpolation in space, added
//   k_spatial_tail     the coarse end of the cycle (from a sub-level whose
//                      vectors fit in LDS down to one node and back), one
//                      workgroup per slab
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

// The same step in 2-D on an LDS tile: one workgroup owns one slab and TY
// rows (all x), stages rows y0-1 .. y0+TY of the N_t components of x (zero
// outside the domain) and applies the separable 9-point stencils from LDS.
// The staged rows, the tile's f and (for UPD_ADD) its base are contiguous
// ranges of the slab, so thread t handles elements t + 256 i, i < SIT, and
// every global load is issued before the first use.  Dynamic LDS:
// NT * (TY + 2) * n elements; requires (TY + 2) n <= 256 SIT.
template <typename T, int NT, int SIT>
__global__ __launch_bounds__(256) void k_spatial_tile2d(const T* __restrict__ x, const T* __restrict__ f,
                                                        const T* base, T* out, SpatialArgs<T> a, int TY) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* U = reinterpret_cast<T*>(lds_raw);
  const long long lg = xcd_linear(blockIdx.x + (long long)gridDim.x * slab_index(),
                                  (long long)gridDim.x * gridDim.y * gridDim.z);
  const long long slab = lg / gridDim.x;
  const int tile = (int)(lg - slab * gridDim.x);
  if (slab >= a.slabs) return;
  const int n = a.n;
  const long long nx = a.nx;
  const int y0 = tile * TY;
  const int plane = (TY + 2) * n;
  const int ylast = y0 + TY < n ? y0 + TY : n;
  const int nout = (ylast - y0) * n;
  const long long sbase = slab * NT * nx;
  const long long s0 = (long long)(y0 - 1) * n;
  const long long o0 = (long long)y0 * n;
  const bool xz = a.x_zero != 0;
  const bool add = a.upd == UPD_ADD;
  T fv[SIT][NT], xv[SIT][NT], bv[SIT][NT];
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    const long long so = s0 + e;
    const bool in = !xz && e < plane && so >= 0 && so < nx;
    const bool o = e < nout;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      xv[i][k] = in ? x[sbase + k * nx + so] : T(0);
      fv[i][k] = o ? f[sbase + k * nx + o0 + e] : T(0);
      bv[i][k] = (o && add) ? base[sbase + k * nx + o0 + e] : T(0);
    }
  }
  if (!xz) {
#pragma unroll
    for (int i = 0; i < SIT; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < plane) {
#pragma unroll
        for (int k = 0; k < NT; ++k) U[k * plane + e] = xv[i][k];
      }
    }
    __syncthreads();
  }
  const float inv_n = 1.0f / (float)n;
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e >= nout) continue;
    T mu[NT], ku[NT], xc[NT];
    if (xz) {
#pragma unroll
      for (int c = 0; c < NT; ++c) mu[c] = ku[c] = xc[c] = T(0);
    } else {
      const int yy = div_small(e, n, inv_n);
      const int px = e - yy * n;
      const bool hl = px > 0, hr = px < n - 1;
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        T m = T(0), kk = T(0);
#pragma unroll
        for (int dr = 0; dr < 3; ++dr) {
          const T* row = U + c * plane + (yy + dr) * n + px;
          const T l = hl ? row[-1] : T(0);
          const T m0 = row[0];
          const T rt = hr ? row[1] : T(0);
          const T sm = a.wm[0] * l + a.wm[1] * m0 + a.wm[2] * rt;
          const T sk = a.wk[0] * l + a.wk[1] * m0 + a.wk[2] * rt;
          m += a.wm[dr] * sm;
          kk += a.wk[dr] * sm + a.wm[dr] * sk;
          if (dr == 1) xc[c] = m0;
        }
        mu[c] = m;
        ku[c] = kk;
      }
    }
    T r[NT];
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T acc = fv[i][l];
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
        y = xc[l] + a.omega * c;
      }
      T o = y;
      if (add) o = bv[i][l] + a.scale * y;
      else if (a.upd == UPD_SET) o = a.scale * y;
      out[sbase + l * nx + o0 + e] = o;
    }
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

// Whole spatial cycle from one sub-level down, one workgroup per slab, all
// vectors in LDS: per sub-level j the iterate pair X_j / Y_j and the right-hand
// side F_j (NT * n_j^d values each), laid out one sub-level after another.
template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_spatial_tail(const T* __restrict__ f, const T* base, T* out,
                                                      TailArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const long long slab = slab_index();
  if (slab >= a.slabs) return;
  T* X[TAIL_MAX];
  T* Y[TAIL_MAX];
  T* F[TAIL_MAX];
  long long nxs[TAIL_MAX];
  {
    long long off = 0;
    for (int j = 0; j < a.levels; ++j) {
      long long nx = a.n[j];
      for (int i = 1; i < D; ++i) nx *= a.n[j];
      nxs[j] = nx;
      X[j] = lds + off;
      Y[j] = lds + off + NT * nx;
      F[j] = lds + off + 2 * NT * nx;
      off += 3 * NT * nx;
    }
  }
  const long long nx0 = nxs[0];
  const T* fs = f + slab * NT * nx0;
  for (long long e = threadIdx.x; e < NT * nx0; e += blockDim.x) F[0][e] = fs[e];
  __syncthreads();
  // y = x + w Dinv (f - A x) on sub-level j (x treated as 0 when xz), or the defect
  auto sweep = [&](int j, const T* x, const T* fj, T* y, bool xz, bool defect, T w) {
    const long long nx = nxs[j];
    const int n = a.n[j];
    for (long long p = threadIdx.x; p < nx; p += blockDim.x) {
      T mu[NT], ku[NT], xv[NT];
      if (xz) {
#pragma unroll
        for (int l = 0; l < NT; ++l) mu[l] = ku[l] = xv[l] = T(0);
      } else {
        int px, py, pz;
        node_coords<D>(p, n, px, py, pz);
        stencil_mk<T, D, NT>(x, nx, n, px, py, pz, a.wm[j], a.wk[j], mu, ku);
#pragma unroll
        for (int l = 0; l < NT; ++l) xv[l] = x[l * nx + p];
      }
      T r[NT];
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = fj[l * nx + p];
#pragma unroll
        for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
        r[l] = acc;
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T v = r[l];
        if (!defect) {
          T c = T(0);
#pragma unroll
          for (int k = 0; k < NT; ++k) c += a.Dinv[j][l * NT + k] * r[k];
          v = xv[l] + w * c;
        }
        y[l * nx + p] = v;
      }
    }
    __syncthreads();
  };
  const int J = a.levels - 1;
  int cur[TAIL_MAX];          // 0: result in X_j, 1: in Y_j
  for (int j = 0; j < J; ++j) {
    T* P[2] = {X[j], Y[j]};
    int c = 0;
    if (a.nu1 == 0) {
      for (long long e = threadIdx.x; e < NT * nxs[j]; e += blockDim.x) X[j][e] = T(0);
      __syncthreads();
    }
    for (int i = 0; i < a.nu1; ++i) {
      if (i == 0) sweep(j, nullptr, F[j], P[0], true, false, a.omega);
      else {
        sweep(j, P[c], F[j], P[1 - c], false, false, a.omega);
        c ^= 1;
      }
    }
    sweep(j, P[c], F[j], P[1 - c], a.nu1 == 0, true, a.omega);      // defect into the free buffer
    // full weighting of the defect into F_{j+1}
    const T* rf = P[1 - c];
    const int nf = a.n[j], nc = a.n[j + 1];
    const long long nxf = nxs[j], nxc = nxs[j + 1];
    for (long long q = threadIdx.x; q < nxc; q += blockDim.x) {
      int cx, cy, cz;
      node_coords<D>(q, nc, cx, cy, cz);
      const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = 2 * cz + 1;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = T(0);
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
          for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
            const T wzy = (dz == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
            const long long zz = (D == 3) ? fz + dz : 0;
            const long long yy = (D >= 2) ? fy + dy : 0;
            const T* line = rf + l * nxf + (zz * nf + yy) * nf;
            acc += wzy * (T(0.5) * line[fx - 1] + line[fx] + T(0.5) * line[fx + 1]);
          }
        F[j + 1][l * nxc + q] = acc;
      }
    }
    __syncthreads();
    cur[j] = c;
  }
  // one node: exact N_t x N_t solve
  sweep(J, nullptr, F[J], X[J], true, false, T(1));
  cur[J] = 0;
  for (int j = J - 1; j >= 0; --j) {
    T* P[2] = {X[j], Y[j]};
    int c = cur[j];
    const T* ec = cur[j + 1] ? Y[j + 1] : X[j + 1];
    const int nf = a.n[j], nc = a.n[j + 1];
    const long long nxf = nxs[j], nxc = nxs[j + 1];
    for (long long p = threadIdx.x; p < nxf; p += blockDim.x) {
      int x, y, z;
      node_coords<D>(p, nf, x, y, z);
      int cxs[2], cys[2] = {0, 0}, czs[2] = {0, 0};
      float wx[2], wy[2] = {1.f, 1.f}, wz[2] = {1.f, 1.f};
      const int kx = coarse_taps(x, nc, cxs, wx);
      const int ky = (D >= 2) ? coarse_taps(y, nc, cys, wy) : 1;
      const int kz = (D == 3) ? coarse_taps(z, nc, czs, wz) : 1;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = T(0);
        for (int iz = 0; iz < kz; ++iz)
          for (int iy = 0; iy < ky; ++iy)
            for (int ix = 0; ix < kx; ++ix)
              acc += (T)(wz[iz] * wy[iy] * wx[ix]) * ec[l * nxc + ((long long)czs[iz] * nc + cys[iy]) * nc + cxs[ix]];
        P[c][l * nxf + p] += acc;
      }
    }
    __syncthreads();
    for (int i = 0; i < a.nu2; ++i) {
      sweep(j, P[c], F[j], P[1 - c], false, false, a.omega);
      c ^= 1;
    }
    cur[j] = c;
  }
  const T* res = cur[0] ? Y[0] : X[0];
  const long long o0 = slab * NT * nx0;
  for (long long e = threadIdx.x; e < NT * nx0; e += blockDim.x) {
    T v = res[e];
    if (a.upd == UPD_ADD) v = base[o0 + e] + a.scale * v;
    else if (a.upd == UPD_SET) v = a.scale * v;
    out[o0 + e] = v;
  }
}

}  // namespace

size_t spatial_tail_lds(int dim, int n, int nt, size_t elem) {
  size_t tot = 0;
  int levels = 0;
  for (int m = n; m >= 1; m = (m - 1) / 2) {
    size_t nx = 1;
    for (int i = 0; i < dim; ++i) nx *= (size_t)m;
    tot += 3 * (size_t)nt * nx * elem;
    ++levels;
    if (m == 1) break;
  }
  if (levels > TAIL_MAX || tot > 65536) return 0;
  return tot;
}

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
  if (dim == 2) {
    const int ty = residual_tile_rows(nt, a.n);
    if (ty == 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)nt * (ty + 2) * a.n * sizeof(T);
    const int sit = ((ty + 2) * a.n + 255) / 256;
    const dim3 grid = slab_grid((unsigned)((a.n + ty - 1) / ty), slabs);
#define SPT_CASE(NT, SIT)                                                                               \
  if (nt == NT && sit == SIT) {                                                                         \
    hipLaunchKernelGGL((k_spatial_tile2d<T, NT, SIT>), grid, dim3(256), lds, s, x, f, base, out, a, ty); \
    return hipGetLastError();                                                                           \
  }
#define SPT_NT(NT) SPT_CASE(NT, 1) SPT_CASE(NT, 2) SPT_CASE(NT, 3) SPT_CASE(NT, 4) SPT_CASE(NT, 5) \
                   SPT_CASE(NT, 6)
    SPT_NT(1) SPT_NT(2) SPT_NT(3) SPT_NT(4)
#undef SPT_NT
#undef SPT_CASE
    return hipErrorInvalidValue;
  }
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
template <typename T>
hipError_t launch_spatial_tail(int dim, int nt, const T* f, const T* base, T* out, const TailArgs<T>& a,
                               hipStream_t s) {
  const size_t lds = spatial_tail_lds(dim, a.n[0], nt, sizeof(T));
  if (lds == 0) return hipErrorInvalidValue;
  const dim3 grid = slab_grid(1, a.slabs);
#define TAIL_CASE(D, NT)                                                                           \
  if (dim == D && nt == NT) {                                                                      \
    hipLaunchKernelGGL((k_spatial_tail<T, D, NT>), grid, dim3(256), lds, s, f, base, out, a);      \
    return hipGetLastError();                                                                      \
  }
  TAIL_CASE(1, 1) TAIL_CASE(1, 2) TAIL_CASE(1, 3) TAIL_CASE(1, 4)
  TAIL_CASE(2, 1) TAIL_CASE(2, 2) TAIL_CASE(2, 3) TAIL_CASE(2, 4)
  TAIL_CASE(3, 1) TAIL_CASE(3, 2) TAIL_CASE(3, 3) TAIL_CASE(3, 4)
#undef TAIL_CASE
  return hipErrorInvalidValue;
}
#undef SPATIAL_DISPATCH

#define INST(T)                                                                                       \
  template hipError_t launch_spatial<T>(int, int, const T*, const T*, const T*, T*, const SpatialArgs<T>&, \
                                        hipStream_t);                                                 \
  template hipError_t launch_restrict_space<T>(int, int, const T*, T*, int, int, long long, hipStream_t); \
  template hipError_t launch_prolong_space<T>(int, int, const T*, T*, int, int, long long, hipStream_t); \
  template hipError_t launch_spatial_tail<T>(int, int, const T*, const T*, T*, const TailArgs<T>&, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
