// HIP kernels of the space-time multigrid V-cycle for gfx950 (MI355X).
//
// Vector layout: [batch][slab][time dof l][z][y][x], x fastest.  One level has
// n interior nodes per dimension (nx = n^d), N slabs and N_t = p_t + 1 time dofs.
//
//   k_residual  r = F - L u: Q1 mass/stiffness stencils (3/9/27 points, applied
//               separably), N_t x N_t time mixing, upwind coupling to the
//               neighbouring slab (eq. chap4_generalLinearSystem).  Fused
//               per-block partial sums of r^2 for the norm.
//   (the slab solves by fast diagonalisation live in stmg_transform.hip)
//   k_restrict  F_c[m] = R1 r[2m] + R2 r[2m+1], optional full weighting in space
//               (eq. chap4_restrictionTime, eq. chap4_spaceRestrictionProlongation).
//   k_prolong   u[2m] += R1^T e_c[m], u[2m+1] += R2^T e_c[m], optional
//               (bi/tri)linear interpolation in space.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

// (M_h w)(node) for w = sum_l coef[l] v_l (v_l the N_t components at `base`).
template <typename T, int D, int NT>
__device__ inline T mass_combo(const T* __restrict__ base, long long nx, int n, int x, int y, int z,
                               const T* wm, const T* coef) {
  T acc = T(0);
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= n) continue;
#pragma unroll
    for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= n) continue;
      const long long row = ((long long)zz * n + yy) * n;
      T s = T(0);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = x + dx;
        if (xx < 0 || xx >= n) continue;
        T w = T(0);
#pragma unroll
        for (int l = 0; l < NT; ++l) w += coef[l] * base[l * nx + row + xx];
        s += wm[dx + 1] * w;
      }
      T wy = (D >= 2) ? wm[dy + 1] : T(1);
      T wz = (D == 3) ? wm[dz + 1] : T(1);
      acc += wz * wy * s;
    }
  }
  return acc;
}

__device__ inline double block_sum(double v) {
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

// ------------------------------------------------------------------ residual
template <typename Tin, typename Tout, int D, int NT>
__global__ __launch_bounds__(256) void k_residual(const Tin* __restrict__ u,
                                                  const Tin* __restrict__ F,
                                                  Tout* __restrict__ r, ResidArgs<Tin> a,
                                                  double* __restrict__ partial) {
  typedef Tin T;
  const long long slab = slab_index();
  const long long nslab = (long long)a.batch * a.N;
  if (slab >= nslab) return;
  const long long nx = a.nx;
  const int n = a.n;
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int sn = (int)(slab % a.N);
  double ss = 0.0;
  if (j < nx) {
    int x, y, z;
    node_coords<D>(j, n, x, y, z);
    const long long slabsz = (long long)NT * nx;
    const T* un = u + slab * slabsz;
    T mu[NT], ku[NT];
    stencil_mk<T, D, NT>(un, nx, n, x, y, z, a.wm, a.wk, mu, ku);
    T mw = T(0);
    const int sp = sn + a.dir;
    if (sp >= 0 && sp < a.N) {
      mw = mass_combo<T, D, NT>(u + (slab + a.dir) * slabsz, nx, n, x, y, z, a.wm, a.cb);
    }
    const T* Fn = F + slab * slabsz;
    Tout* rn = r + slab * slabsz;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T acc = Fn[l * nx + j] + a.ca[l] * mw;
#pragma unroll
      for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
      rn[l * nx + j] = (Tout)acc;
      ss += (double)acc * (double)acc;
    }
  }
  if (partial != nullptr) {
    const double s = block_sum(ss);
    if (threadIdx.x == 0) partial[slab * gridDim.x + blockIdx.x] = s;
  }
}

// 2-D residual on an LDS tile: one workgroup owns one slab and TY rows
// (all x).  It stages the N_t components of u and the coupling combination
// w = sum_k cb[k] u_{n+dir,k} for rows y0-1 .. y0+TY (zero outside the
// domain), then applies the separable 9-point mass/stiffness stencils from
// LDS.  Dynamic LDS: (NT + 1) * (TY + 2) * n elements.  The staged rows and
// the tile's right-hand side are contiguous ranges of the slab, so thread t
// handles elements t + 256 i, i < SIT, and the domain test is a range test
// on the offset; every global load of the workgroup is issued before the
// first use.  Requires (TY + 2) n <= 256 SIT.
template <typename Tin, typename Tout, int NT, int SIT>
__global__ __launch_bounds__(256) void k_residual_tile2d(const Tin* __restrict__ u,
                                                            const Tin* __restrict__ F,
                                                            Tout* __restrict__ r, ResidArgs<Tin> a,
                                                            double* __restrict__ partial, int TY) {
  typedef Tin T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* U = reinterpret_cast<T*>(lds_raw);
  const long long lg = xcd_linear(blockIdx.x + (long long)gridDim.x * slab_index(),
                                  (long long)gridDim.x * gridDim.y * gridDim.z);
  const long long slab = lg / gridDim.x;
  const int tile = (int)(lg - slab * gridDim.x);
  const long long nslab = (long long)a.batch * a.N;
  if (slab >= nslab) return;
  const int n = a.n;
  const long long nx = a.nx;
  const int y0 = tile * TY;
  const int plane = (TY + 2) * n;
  const int ylast = y0 + TY < n ? y0 + TY : n;
  const int nout = (ylast - y0) * n;
  const int sn = (int)(slab % a.N);
  const bool couple = (sn + a.dir >= 0) && (sn + a.dir < a.N);
  const long long slabsz = (long long)NT * nx;
  const T* un = u + slab * slabsz;
  const T* up = u + (slab + a.dir) * slabsz;
  const T* Fn = F + slab * slabsz;
  const long long s0 = (long long)(y0 - 1) * n;   // first staged offset (may be -n)
  const long long o0 = (long long)y0 * n;         // first output offset
  T fv[SIT][NT], uv[SIT][NT], pv[SIT][NT];
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    const long long so = s0 + e;
    const bool in = e < plane && so >= 0 && so < nx;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      uv[i][k] = in ? un[k * nx + so] : T(0);
      pv[i][k] = (in && couple) ? up[k * nx + so] : T(0);
      fv[i][k] = e < nout ? Fn[k * nx + o0 + e] : T(0);
    }
  }
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < plane) {
      T w = T(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        U[k * plane + e] = uv[i][k];
        w += a.cb[k] * pv[i][k];
      }
      U[NT * plane + e] = w;
    }
  }
  __syncthreads();
  double ss = 0.0;
  Tout* rn = r + slab * slabsz;
  const float inv_n = 1.0f / (float)n;
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < nout) {
      const int yy = div_small(e, n, inv_n);
      const int x = e - yy * n;
      const bool hl = x > 0, hr = x < n - 1;
      T mu[NT + 1], ku[NT];
#pragma unroll
      for (int c = 0; c <= NT; ++c) {
        T m = T(0), kk = T(0);
#pragma unroll
        for (int dr = 0; dr < 3; ++dr) {
          const T* row = U + c * plane + (yy + dr) * n + x;
          const T l = hl ? row[-1] : T(0);
          const T m0 = row[0];
          const T rt = hr ? row[1] : T(0);
          const T sm = a.wm[0] * l + a.wm[1] * m0 + a.wm[2] * rt;
          m += a.wm[dr] * sm;
          if (c < NT) {
            const T sk = a.wk[0] * l + a.wk[1] * m0 + a.wk[2] * rt;
            kk += a.wk[dr] * sm + a.wm[dr] * sk;
          }
        }
        mu[c] = m;
        if (c < NT) ku[c] = kk;
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = fv[i][l] + a.ca[l] * mu[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
        rn[l * nx + o0 + e] = (Tout)acc;
        ss += (double)acc * (double)acc;
      }
    }
  }
  if (partial != nullptr) {
    const double s2 = block_sum(ss);
    if (threadIdx.x == 0) partial[slab * gridDim.x + tile] = s2;
  }
}

// 3-D residual, marching in z.  One workgroup owns one slab, TY rows of y
// (all x) and the z-planes z0 .. z1-1.  The separable 27-point stencils split
// into planar parts: per plane p and component c, A_c(p) = (m (x) m) u_c(p) and
// B_c(p) = (k (x) m + m (x) k) u_c(p) (y (x) x), and A_w(p) for the coupling
// combination w = sum_k cb[k] u_{n+dir,k}.  Then
//   (M_h u_c)(z) = sum_dz m[dz] A_c(z+dz),
//   (K_h u_c)(z) = sum_dz k[dz] A_c(z+dz) + m[dz] B_c(z+dz),
// so a thread keeps the planar values of three consecutive planes in
// registers and every plane of u (and of the neighbour slab) is staged in LDS
// once: rows y0-1 .. y0+TY (zero outside the domain), (NT + 1) (TY + 2) n
// elements.  The next plane's loads and the next output plane's right-hand
// side are issued before the current plane's stencils.  Planes -1 and n are
// the Dirichlet boundary (zero).  Thread t of the BS threads owns output
// positions t + BS i, i < OIT (TY n <= BS OIT), and staged positions
// t + BS i, i < SIT ((TY + 2) n <= BS SIT).
template <typename Tin, typename Tout, int NT, int BS, int OIT, int SIT>
__global__ __launch_bounds__(BS) void k_residual_tile3d(const Tin* __restrict__ u,
                                                            const Tin* __restrict__ F,
                                                            Tout* __restrict__ r, ResidArgs<Tin> a,
                                                            double* __restrict__ partial, int TY, int ZC) {
  typedef Tin T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* U = reinterpret_cast<T*>(lds_raw);
  const long long lg = xcd_linear(blockIdx.x + (long long)gridDim.x * slab_index(),
                                  (long long)gridDim.x * gridDim.y * gridDim.z);
  const long long slab = lg / gridDim.x;
  const int tile = (int)(lg - slab * gridDim.x);
  const long long nslab = (long long)a.batch * a.N;
  if (slab >= nslab) return;
  const int n = a.n;
  const long long nx = a.nx;
  const long long nn = (long long)n * n;
  const int nyt = (n + TY - 1) / TY;
  const int yt = tile % nyt;
  const int z0 = (tile / nyt) * ZC;
  const int z1 = z0 + ZC < n ? z0 + ZC : n;
  const int y0 = yt * TY;
  const int ylast = y0 + TY < n ? y0 + TY : n;
  const int plane = (TY + 2) * n;
  const int nout = (ylast - y0) * n;
  const int sn = (int)(slab % a.N);
  const bool couple = (sn + a.dir >= 0) && (sn + a.dir < a.N);
  const long long slabsz = (long long)NT * nx;
  const T* un = u + slab * slabsz;
  const T* up = u + (slab + a.dir) * slabsz;
  const T* Fn = F + slab * slabsz;
  Tout* rn = r + slab * slabsz;
  const long long s0 = (long long)(y0 - 1) * n;   // first staged offset within a plane (may be -n)
  const long long o0 = (long long)y0 * n;         // first output offset within a plane

  // output positions of this thread
  const float inv_n = 1.0f / (float)n;
  int oy[OIT], ox[OIT];
#pragma unroll
  for (int i = 0; i < OIT; ++i) {
    const int e = threadIdx.x + BS * i;
    oy[i] = div_small(e, n, inv_n);
    ox[i] = e - oy[i] * n;
  }
  T uv[SIT][NT], pv[SIT][NT];     // staged values of the next plane
  T fv[OIT][NT], fn[OIT][NT];     // right-hand side of the output plane / the next one
  T A[3][OIT][NT + 1], B[3][OIT][NT];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int i = 0; i < OIT; ++i) {
#pragma unroll
      for (int c = 0; c <= NT; ++c) A[q][i][c] = T(0);
#pragma unroll
      for (int c = 0; c < NT; ++c) B[q][i][c] = T(0);
    }
  auto load_plane = [&](int p) {
    const bool pin = p >= 0 && p < n;
    const long long po = (long long)p * nn;
#pragma unroll
    for (int i = 0; i < SIT; ++i) {
      const int e = threadIdx.x + BS * i;
      const long long so = s0 + e;
      const bool in = pin && e < plane && so >= 0 && so < nn;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        uv[i][k] = in ? un[k * nx + po + so] : T(0);
        pv[i][k] = (in && couple) ? up[k * nx + po + so] : T(0);
      }
    }
  };
  auto load_rhs = [&](int p) {
    const long long po = (long long)p * nn + o0;
#pragma unroll
    for (int i = 0; i < OIT; ++i) {
      const int e = threadIdx.x + BS * i;
#pragma unroll
      for (int k = 0; k < NT; ++k) fn[i][k] = e < nout ? Fn[k * nx + po + e] : T(0);
    }
  };
#pragma unroll
  for (int i = 0; i < OIT; ++i)
#pragma unroll
    for (int k = 0; k < NT; ++k) fn[i][k] = T(0);
  load_plane(z0 - 1);
  double ss = 0.0;
  for (int p = z0 - 1; p <= z1; ++p) {
    __syncthreads();   // the previous plane's stencils are done with the LDS
#pragma unroll
    for (int i = 0; i < SIT; ++i) {
      const int e = threadIdx.x + BS * i;
      if (e < plane) {
        T w = T(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          U[k * plane + e] = uv[i][k];
          w += a.cb[k] * pv[i][k];
        }
        U[NT * plane + e] = w;
      }
    }
    // the right-hand side of this iteration's output plane p - 1 was loaded
    // one iteration ago; load the one of plane p (output next iteration)
#pragma unroll
    for (int i = 0; i < OIT; ++i)
#pragma unroll
      for (int k = 0; k < NT; ++k) fv[i][k] = fn[i][k];
    if (p < z1) load_plane(p + 1);
    if (p >= z0 && p < z1) load_rhs(p);
    __syncthreads();
    // planar stencils of plane p; the window slides by one plane
#pragma unroll
    for (int i = 0; i < OIT; ++i) {
#pragma unroll
      for (int c = 0; c <= NT; ++c) {
        A[0][i][c] = A[1][i][c];
        A[1][i][c] = A[2][i][c];
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        B[0][i][c] = B[1][i][c];
        B[1][i][c] = B[2][i][c];
      }
      const int e = threadIdx.x + BS * i;
      if (e < nout) {
        const int x = ox[i];
        const bool hl = x > 0, hr = x < n - 1;
#pragma unroll
        for (int c = 0; c <= NT; ++c) {
          T m = T(0), kk = T(0);
#pragma unroll
          for (int dr = 0; dr < 3; ++dr) {
            const T* row = U + c * plane + (oy[i] + dr) * n + x;
            const T l = hl ? row[-1] : T(0);
            const T m0 = row[0];
            const T rt = hr ? row[1] : T(0);
            const T sm = a.wm[0] * l + a.wm[1] * m0 + a.wm[2] * rt;
            m += a.wm[dr] * sm;
            if (c < NT) {
              const T sk = a.wk[0] * l + a.wk[1] * m0 + a.wk[2] * rt;
              kk += a.wk[dr] * sm + a.wm[dr] * sk;
            }
          }
          A[2][i][c] = m;
          if (c < NT) B[2][i][c] = kk;
          // one component's nine LDS reads at a time: keeps the register
          // count (and with it the occupancy) of the FP64 kernel in check
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    const int o = p - 1;   // output plane: needs planes o - 1, o, o + 1 = p
    if (o >= z0) {
      const long long po = (long long)o * nn + o0;
#pragma unroll
      for (int i = 0; i < OIT; ++i) {
        const int e = threadIdx.x + BS * i;
        if (e < nout) {
          T mu[NT + 1], ku[NT];
#pragma unroll
          for (int c = 0; c <= NT; ++c)
            mu[c] = a.wm[0] * A[0][i][c] + a.wm[1] * A[1][i][c] + a.wm[2] * A[2][i][c];
#pragma unroll
          for (int c = 0; c < NT; ++c)
            ku[c] = a.wk[0] * A[0][i][c] + a.wk[1] * A[1][i][c] + a.wk[2] * A[2][i][c] +
                    a.wm[0] * B[0][i][c] + a.wm[1] * B[1][i][c] + a.wm[2] * B[2][i][c];
#pragma unroll
          for (int l = 0; l < NT; ++l) {
            T acc = fv[i][l] + a.ca[l] * mu[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
            rn[l * nx + po + e] = (Tout)acc;
            ss += (double)acc * (double)acc;
          }
        }
      }
    }
  }
  if (partial != nullptr) {
    const double s2 = block_sum(ss);
    if (threadIdx.x == 0) partial[slab * gridDim.x + tile] = s2;
  }
}

// ---------------------------------------------------------------- transfers
template <typename T, int D, int NT, bool FULL>
__global__ __launch_bounds__(256) void k_restrict(const T* __restrict__ rf, T* __restrict__ Fc,
                                                  TransferArgs<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nxc = a.nxc, nxf = a.nxf;
  const long long total = nxc * a.Nc * a.batch;
  if (idx >= total) return;
  const long long jc = idx % nxc;
  const long long cs = idx / nxc;             // global coarse slab (batch-major)
  const long long m = cs % a.Nc;
  const long long bi = cs / a.Nc;
  const long long fs0 = bi * (2LL * a.Nc) + 2 * m;
  T v[2][NT];
  if (FULL) {
    int cx, cy, cz;
    node_coords<D>(jc, a.nc, cx, cy, cz);
    const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = 2 * cz + 1;
    const int nf = a.nf;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* base = rf + (fs0 + s) * NT * nxf;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        T acc = T(0);
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
          for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
            const T wzy = (dz == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
            const long long rz = (D == 3) ? (fz + dz) : 0;
            const long long ry = (D >= 2) ? (fy + dy) : 0;
            const T* line = base + k * nxf + (rz * nf + ry) * nf;
            acc += wzy * (T(0.5) * line[fx - 1] + line[fx] + T(0.5) * line[fx + 1]);
          }
        v[s][k] = acc;
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int k = 0; k < NT; ++k) v[s][k] = rf[(fs0 + s) * NT * nxf + k * nxf + jc];
  }
  T* out = Fc + cs * NT * nxc + jc;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) acc += a.R1T[k * NT + l] * v[0][k] + a.R2T[k * NT + l] * v[1][k];
    out[l * nxc] = acc;
  }
}

template <typename T, int D, int NT, bool FULL>
__global__ __launch_bounds__(256) void k_prolong(const T* __restrict__ ec, T* __restrict__ uf,
                                                 TransferArgs<T> a) {
  // grid: x over the fine nodes of a slab, (y, z) over the coarse slabs: the
  // slab decode is per workgroup and the node decode 32-bit
  const long long cs = slab_index();           // coarse slab (batch-major)
  const int jf = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (cs >= (long long)a.Nc * a.batch || jf >= a.nxf) return;
  const long long nxc = a.nxc, nxf = a.nxf;
  const long long m = cs % a.Nc;
  const long long bi = cs / a.Nc;
  const long long fs0 = bi * (2LL * a.Nc) + 2 * m;
  const T* ecs = ec + cs * NT * nxc;
  T e[NT];
  if (FULL) {
    int fx, fy, fz;
    node_coords32<D>(jf, a.nf, fx, fy, fz);
    const int nc = a.nc;
    // per dimension: odd fine index 2c+1 -> coarse c (weight 1); even 2c -> c-1, c (1/2 each)
    int cxs[2], cys[2], czs[2];
    T wx[2], wy[2], wz[2];
    int nxs, nys, nzs;
    auto axis = [nc](int f, int* cs_, T* ws, int& cnt) {
      if (f & 1) {
        cs_[0] = (f - 1) >> 1;
        ws[0] = T(1);
        cnt = 1;
      } else {
        cs_[0] = (f >> 1) - 1;
        ws[0] = T(0.5);
        cs_[1] = f >> 1;
        ws[1] = T(0.5);
        cnt = 2;
      }
      (void)nc;
    };
    axis(fx, cxs, wx, nxs);
    if (D >= 2) axis(fy, cys, wy, nys); else { cys[0] = 0; wy[0] = T(1); nys = 1; }
    if (D == 3) axis(fz, czs, wz, nzs); else { czs[0] = 0; wz[0] = T(1); nzs = 1; }
#pragma unroll
    for (int k = 0; k < NT; ++k) e[k] = T(0);
    for (int iz = 0; iz < nzs; ++iz) {
      if (czs[iz] < 0 || czs[iz] >= (D == 3 ? nc : 1)) continue;
      for (int iy = 0; iy < nys; ++iy) {
        if (cys[iy] < 0 || cys[iy] >= (D >= 2 ? nc : 1)) continue;
        for (int ix = 0; ix < nxs; ++ix) {
          if (cxs[ix] < 0 || cxs[ix] >= nc) continue;
          const long long jc = ((long long)czs[iz] * nc + cys[iy]) * nc + cxs[ix];
          const T w = wz[iz] * wy[iy] * wx[ix];
#pragma unroll
          for (int k = 0; k < NT; ++k) e[k] += w * ecs[k * nxc + jc];
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NT; ++k) e[k] = ecs[k * nxc + jf];
  }
  T* u0 = uf + fs0 * NT * nxf + jf;
  T* u1 = u0 + NT * nxf;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      a0 += a.R1T[l * NT + k] * e[k];
      a1 += a.R2T[l * NT + k] * e[k];
    }
    u0[l * nxf] += a0;
    u1[l * nxf] += a1;
  }
}

// ------------------------------------------------ residual + full restriction
// The pre-restriction defect of a fully coarsened level without storing it:
// F_c[m] = R1 W r[2m] + R2 W r[2m+1] (eq. chap4_generalLinearSystem for r =
// F - L u, eq. chap4_restrictionTime for R1, R2, W the full weighting (1/2, 1,
// 1/2) per axis of eq. chap4_spaceRestrictionProlongation).  k_resid_weigh
// computes, per fine slab s = 2m + j, h_s = R_{j+1} W r[s] on coarse nodes;
// k_pair_sum adds the two slabs of each pair.  A workgroup takes fine slab s,
// coarse rows cy0 .. cy1 - 1 of y (3-D; the whole x line in 2-D) and coarse
// planes cz0 .. cz1 - 1 of the slowest axis (z in 3-D, y in 2-D), and marches
// the fine planes 2 cz0 .. 2 cz1 (n = 2 n_c + 1: coarse node c sits on fine node
// 2c + 1, so a coarse plane takes fine planes 2c .. 2c + 2 and neighbouring
// tiles share one fine row or plane, which both compute).  The stencils use
// the planar split of the 3-D residual (per staged plane A_c = mass and
// B_c = stiffness parts within the plane, x only in 2-D), kept as the open
// sums of the two output planes the last staged plane contributes to; each
// fine output plane's R_{j+1}^T-combined defect goes through LDS for the
// in-plane weighting, which runs after the next barrier beside the next
// plane's staging; sums over fine planes stay in registers.  Thread t owns
// fine positions t + BS i (i < OIT; R rows of n), coarse position t and staged
// positions t + BS i (i < SIT; R + 2 rows in 3-D).
template <typename T, int D, int NT, int BS, int OIT, int SIT>
__global__ __launch_bounds__(BS) void k_resid_weigh(const T* __restrict__ u, const T* __restrict__ F,
                                                    T* __restrict__ Hs, ResidArgs<T> a, TransferArgs<T> t,
                                                    int TYC, int ZCC) {
  constexpr int H = D == 3 ? 1 : 0;        // halo rows of y in a staged plane
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* U = reinterpret_cast<T*>(lds_raw);
  const long long lg = xcd_linear(blockIdx.x + (long long)gridDim.x * slab_index(),
                                  (long long)gridDim.x * gridDim.y * gridDim.z);
  const long long slab = lg / gridDim.x;   // fine slab (batch-major)
  const int tile = (int)(lg - slab * gridDim.x);
  if (slab >= (long long)a.batch * a.N) return;
  const int n = a.n, nc = t.nc;
  const long long nx = a.nx, nxc = t.nxc;
  const int nyt = D == 3 ? (nc + TYC - 1) / TYC : 1;
  const int cy0 = D == 3 ? (tile % nyt) * TYC : 0;
  const int cy1 = D == 3 ? (cy0 + TYC < nc ? cy0 + TYC : nc) : 1;
  const int cz0 = (tile / nyt) * ZCC;
  const int cz1 = cz0 + ZCC < nc ? cz0 + ZCC : nc;
  const int R = D == 3 ? 2 * (cy1 - cy0) + 1 : 1;   // fine rows computed
  const int plane = (R + 2 * H) * n;               // staged elements per component
  const int nout = R * n;
  const int ncout = (cy1 - cy0) * nc;
  const long long pn = D == 3 ? (long long)n * n : n;
  const long long pnc = D == 3 ? (long long)nc * nc : nc;
  const long long s0 = (long long)(2 * cy0 - H) * n;   // first staged offset within a fine plane
  const long long o0 = (long long)(2 * cy0) * n;       // first output offset
  const int sn = (int)(slab % a.N);
  const bool couple = (sn + a.dir >= 0) && (sn + a.dir < a.N);
  const long long slabsz = (long long)NT * nx;
  const T* un = u + slab * slabsz;
  const T* up = u + (slab + a.dir) * slabsz;
  const T* Fn = F + slab * slabsz;
  const T* RT = (sn & 1) ? t.R2T : t.R1T;
  T* out = Hs + slab * NT * nxc + (long long)cy0 * nc;
  T* G = U + (NT + 1) * plane;             // [NT][nout]

  const float inv_n = 1.0f / (float)n;
  int oy[OIT], ox[OIT];
#pragma unroll
  for (int i = 0; i < OIT; ++i) {
    const int e = threadIdx.x + BS * i;
    oy[i] = D == 3 ? div_small(e, n, inv_n) : 0;
    ox[i] = e - oy[i] * n;
  }
  const bool cact = threadIdx.x < ncout;
  const int cyl = D == 3 ? div_small(threadIdx.x, nc, 1.0f / (float)nc) : 0;
  const int cx = threadIdx.x - cyl * nc;

  T uv[SIT][NT], pv[SIT][NT];        // staged loads of the next plane: own slab, upwind neighbour
  T fv[OIT][NT], fn[OIT][NT];        // right-hand side of the output plane / the next one
  // mass (NT + 1) and stiffness (NT) sums of the two output planes still open
  T P0[OIT][2 * NT + 1], P1[OIT][2 * NT + 1], acc[NT];
#pragma unroll
  for (int i = 0; i < OIT; ++i) {
#pragma unroll
    for (int c = 0; c <= 2 * NT; ++c) P0[i][c] = P1[i][c] = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) fn[i][k] = T(0);
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) acc[k] = T(0);
  auto load_plane = [&](int p) {
    const bool pin = p >= 0 && p < n;
    const long long po = (long long)p * pn;
#pragma unroll
    for (int i = 0; i < SIT; ++i) {
      const int e2 = threadIdx.x + BS * i;
      const long long so = s0 + e2;
      const bool in = pin && e2 < plane && so >= 0 && so < pn;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        uv[i][k] = in ? un[k * nx + po + so] : T(0);
        pv[i][k] = (in && couple) ? up[k * nx + po + so] : T(0);
      }
    }
  };
  auto load_rhs = [&](int p) {
    const long long po = (long long)p * pn + o0;
#pragma unroll
    for (int i = 0; i < OIT; ++i) {
      const int e = threadIdx.x + BS * i;
#pragma unroll
      for (int k = 0; k < NT; ++k) fn[i][k] = e < nout ? Fn[k * nx + po + e] : T(0);
    }
  };
  // in-plane full weighting of fine plane o and its share of the coarse planes
  auto weigh = [&](int o) {
    if (!cact) return;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T gc = T(0);
#pragma unroll
      for (int dr = 0; dr < 2 * H + 1; ++dr) {
        const T* row = G + l * nout + (2 * cyl + dr) * n + 2 * cx;
        const T v = T(0.5) * row[0] + row[1] + T(0.5) * row[2];
        gc += (D == 3 && dr != 1) ? T(0.5) * v : v;
      }
      if (o & 1) {
        acc[l] += gc;                       // fine plane 2c + 1: weight 1 on coarse plane c
      } else {
        if (o > 2 * cz0) {                  // fine plane 2c: last part of coarse plane c - 1
          acc[l] += T(0.5) * gc;
          out[l * nxc + (long long)(o / 2 - 1) * pnc + (long long)cyl * nc + cx] = acc[l];
        }
        acc[l] = T(0.5) * gc;               // first part of coarse plane c
      }
    }
  };
  const int f0 = 2 * cz0, f1 = 2 * cz1;   // fine output planes f0 .. f1
  load_plane(f0 - 1);
  for (int p = f0 - 1; p <= f1 + 1; ++p) {
    __syncthreads();   // the previous plane's stencils and contributions are done
    if (p - 2 >= f0) weigh(p - 2);
#pragma unroll
    for (int i = 0; i < SIT; ++i) {
      const int e2 = threadIdx.x + BS * i;
      if (e2 < plane) {
        T w = T(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          U[k * plane + e2] = uv[i][k];
          w += a.cb[k] * pv[i][k];
        }
        U[NT * plane + e2] = w;
      }
    }
#pragma unroll
    for (int i = 0; i < OIT; ++i)
#pragma unroll
      for (int k = 0; k < NT; ++k) fv[i][k] = fn[i][k];
    if (p <= f1) load_plane(p + 1);
    if (p >= f0 && p <= f1) load_rhs(p);
    __syncthreads();
    const int o = p - 1;   // fine output plane: complete once plane p = o + 1 is in
#pragma unroll
    for (int i = 0; i < OIT; ++i) {
      const int e = threadIdx.x + BS * i;
      if (e >= nout) continue;
      const int x = ox[i];
      const bool hl = x > 0, hr = x < n - 1;
      T Ap[NT + 1], Bp[NT];
#pragma unroll
      for (int c = 0; c <= NT; ++c) {
        T mm = T(0), kk = T(0);
#pragma unroll
        for (int dr = 0; dr < 2 * H + 1; ++dr) {
          const T* row = U + c * plane + (oy[i] + dr) * n + x;
          const T l = hl ? row[-1] : T(0);
          const T m0 = row[0];
          const T rt = hr ? row[1] : T(0);
          const T sm = a.wm[0] * l + a.wm[1] * m0 + a.wm[2] * rt;
          if (D == 3) {
            mm += a.wm[dr] * sm;
            if (c < NT) kk += a.wk[dr] * sm + a.wm[dr] * (a.wk[0] * l + a.wk[1] * m0 + a.wk[2] * rt);
          } else {
            mm = sm;
            if (c < NT) kk = a.wk[0] * l + a.wk[1] * m0 + a.wk[2] * rt;
          }
        }
        Ap[c] = mm;
        if (c < NT) Bp[c] = kk;
        __builtin_amdgcn_sched_barrier(0);
      }
      // plane p closes output plane o (weights [2]), adds to plane p (weights
      // [1]) and opens plane p + 1 (weights [0]); P1 holds plane o, P0 plane p
#pragma unroll
      for (int c = 0; c <= NT; ++c) {
        P1[i][c] += a.wm[2] * Ap[c];
        P0[i][c] += a.wm[1] * Ap[c];
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        P1[i][NT + 1 + c] += a.wk[2] * Ap[c] + a.wm[2] * Bp[c];
        P0[i][NT + 1 + c] += a.wk[1] * Ap[c] + a.wm[1] * Bp[c];
      }
      if (o >= f0) {
        T r[NT];
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          T s = fv[i][l] + a.ca[l] * P1[i][NT];
#pragma unroll
          for (int k = 0; k < NT; ++k) s -= a.K[l * NT + k] * P1[i][k] + a.M[l * NT + k] * P1[i][NT + 1 + k];
          r[l] = s;
        }
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          T g = T(0);
#pragma unroll
          for (int k = 0; k < NT; ++k) g += RT[k * NT + l] * r[k];
          G[l * nout + e] = g;
        }
      }
#pragma unroll
      for (int c = 0; c <= NT; ++c) {
        P1[i][c] = P0[i][c];
        P0[i][c] = a.wm[0] * Ap[c];
      }
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        P1[i][NT + 1 + c] = P0[i][NT + 1 + c];
        P0[i][NT + 1 + c] = a.wk[0] * Ap[c] + a.wm[0] * Bp[c];
      }
    }
  }
  __syncthreads();
  weigh(f1);
}

// F_c[m] = h[2m] + h[2m + 1] per coarse slab (len = values of the coarse vector).
template <typename T>
__global__ __launch_bounds__(256) void k_pair_sum(const T* __restrict__ Hs, T* __restrict__ Fc, long long per,
                                                  long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const long long cs = i / per, rem = i - cs * per;
  const T* h = Hs + 2 * cs * per + rem;
  Fc[i] = h[0] + h[per];
}

// --------------------------------------------------------------- load vector
template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_rhs(const T* __restrict__ f, const T* __restrict__ u0,
                                             T* __restrict__ F, RhsArgs<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nx = a.nx;
  const long long total = nx * a.N * a.batch;
  if (idx >= total) return;
  const long long j = idx % nx;
  const long long s = idx / nx;          // global slab
  const long long sn = s % a.N;
  const long long bi = s / a.N;
  int x, y, z;
  node_coords<D>(j, a.n, x, y, z);
  const T one[1] = {T(1)};
  const T mf = mass_combo<T, D, 1>(f + s * nx, nx, a.n, x, y, z, a.wm, one);
  T mu0 = T(0);
  if (sn == 0 && u0 != nullptr) mu0 = mass_combo<T, D, 1>(u0 + bi * nx, nx, a.n, x, y, z, a.wm, one);
  T* out = F + s * NT * nx + j;
#pragma unroll
  for (int l = 0; l < NT; ++l) out[l * nx] = a.ints[l] * mf + a.ca[l] * mu0;
}

template <typename T, int D, int NT>
__global__ __launch_bounds__(256) void k_rhs_adjoint(const T* __restrict__ lam, T* __restrict__ gf,
                                                     T* __restrict__ gu0, RhsArgs<T> a) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nx = a.nx;
  const long long total = nx * a.N * a.batch;
  if (idx >= total) return;
  const long long j = idx % nx;
  const long long s = idx / nx;
  const long long sn = s % a.N;
  const long long bi = s / a.N;
  int x, y, z;
  node_coords<D>(j, a.n, x, y, z);
  const T* ls = lam + s * NT * nx;
  if (gf != nullptr) gf[s * nx + j] = mass_combo<T, D, NT>(ls, nx, a.n, x, y, z, a.wm, a.ints);
  if (gu0 != nullptr && sn == 0) gu0[bi * nx + j] = mass_combo<T, D, NT>(ls, nx, a.n, x, y, z, a.wm, a.ca);
}

// ---------------------------------------------------------------- reductions
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* __restrict__ v, long long len,
                                               double* __restrict__ partial) {
  const long long b = blockIdx.y;
  const T* p = v + b * len;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = (double)p[i];
    s += x * x;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[b * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partial,
                                                    long long per_batch, double* __restrict__ out) {
  const long long b = blockIdx.x;
  double s = 0.0;
  for (long long i = threadIdx.x; i < per_batch; i += blockDim.x) s += partial[b * per_batch + i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[b] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ v, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) v[i] = T(0);
}

// One wave that idles for `ticks` of the constant-rate wall clock (bounded by an
// iteration cap as well), so that work queued behind it starts back to back.
__global__ __launch_bounds__(64) void k_spin(long long ticks) {
  const long long t0 = (long long)wall_clock64();
  for (int it = 0; it < (1 << 22); ++it) {
    if ((long long)wall_clock64() - t0 >= ticks) break;
    __builtin_amdgcn_s_sleep(2);
  }
}

__global__ __launch_bounds__(256) void k_axpy_f32_f64(double* __restrict__ u,
                                                      const float* __restrict__ e, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) u[i] += (double)e[i];
}
__global__ __launch_bounds__(256) void k_cast_f64_f32(const double* __restrict__ in,
                                                      float* __restrict__ out, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = (float)in[i];
}
__global__ __launch_bounds__(256) void k_cast_f32_f64(const float* __restrict__ in,
                                                      double* __restrict__ out, long long len) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = (double)in[i];
}

inline unsigned blocks_for(long long total) { return (unsigned)((total + 255) / 256); }

}  // namespace

// ================================================================ launchers

// Rows per 2-D residual tile: 8/6/4 for N_t <= 2 / 3 / 4, fewer for wide
// grids so that the staged rows fit one set of prefetched loads (at most
// RES_PF_MAX elements; n <= 255 leaves at least 4 rows).
constexpr int RES_PF_SIT = 6;
constexpr int RES_PF_MAX = 256 * RES_PF_SIT;
int residual_tile_rows(int nt, int n) {
  const int ty = nt <= 2 ? 8 : (nt == 3 ? 6 : 4);
  if ((ty + 2) * n <= RES_PF_MAX) return ty;
  const int fit = RES_PF_MAX / n - 2;
  return fit >= 1 ? fit : 0;
}

// 3-D residual tiles: TY rows of y per workgroup (TY n <= 512 output
// positions for N_t <= 2, 256 above) on 256 threads, two positions per thread
// when TY n > 256 (STMG_RES3D_OIT=1: 512 threads with one each instead; on
// 63^3 x 1024 slabs 3.4 ms against 3.0 ms), z-planes in chunks of ZC so that
// a level has about 4096 workgroups or more (chunks of at least 8 planes).
struct Res3dShape {
  int ty, zc, nyt, nzt, bs, oit, sit;
};
Res3dShape residual3d_shape(int nt, int n, long long slabs) {
  static const int oit_env = [] {
    const char* e = std::getenv("STMG_RES3D_OIT");
    return e ? std::atoi(e) : 2;
  }();
  Res3dShape sh{};
  const int cap = nt <= 2 ? 512 : 256;
  sh.ty = cap / n < 1 ? 1 : (cap / n > n ? n : cap / n);
  sh.nyt = (n + sh.ty - 1) / sh.ty;
  long long want = (4096 + (long long)sh.nyt * slabs - 1) / ((long long)sh.nyt * slabs);
  const int maxc = (n + 7) / 8;
  const int nzc = (int)(want < 1 ? 1 : (want > maxc ? maxc : want));
  sh.zc = (n + nzc - 1) / nzc;
  sh.nzt = (n + sh.zc - 1) / sh.zc;
  sh.bs = (sh.ty * n > 256 && oit_env == 1) ? 512 : 256;
  sh.oit = (sh.ty * n + sh.bs - 1) / sh.bs;
  sh.sit = ((sh.ty + 2) * n + sh.bs - 1) / sh.bs;
  return sh;
}

unsigned residual_blocks_per_slab(int dim, int n, long long nx, int nt, long long slabs) {
  if (dim == 2) {
    const int ty = residual_tile_rows(nt, n);
    return ty > 0 ? (unsigned)((n + ty - 1) / ty) : 0u;
  }
  if (dim == 3) {
    const Res3dShape sh = residual3d_shape(nt, n, slabs);
    return (unsigned)(sh.nyt * sh.nzt);
  }
  return (unsigned)((nx + 255) / 256);
}

template <typename Tin, typename Tout>
hipError_t launch_residual(int dim, int nt, const Tin* u, const Tin* F, Tout* r,
                           const ResidArgs<Tin>& a, double* partial, hipStream_t s) {
  const long long slabs = (long long)a.batch * a.N;
  const unsigned gx = residual_blocks_per_slab(dim, a.n, a.nx, nt, slabs);
  const dim3 grid = slab_grid(gx, slabs);
  if (dim == 3) {
    const Res3dShape sh = residual3d_shape(nt, a.n, slabs);
    const size_t lds = (size_t)(nt + 1) * (sh.ty + 2) * a.n * sizeof(Tin);
#define RES3_CASE(NT, BS, OIT, SIT)                                                                    \
  if (nt == NT && sh.bs == BS && sh.oit == OIT && sh.sit == SIT) {                                     \
    hipLaunchKernelGGL((k_residual_tile3d<Tin, Tout, NT, BS, OIT, SIT>), grid, dim3(BS), lds, s, u, F, r, \
                       a, partial, sh.ty, sh.zc);                                                     \
    return hipGetLastError();                                                                          \
  }
#define RES3_NT(NT) RES3_CASE(NT, 256, 1, 1) RES3_CASE(NT, 256, 1, 2) RES3_CASE(NT, 256, 1, 3) \
                    RES3_CASE(NT, 512, 1, 2) RES3_CASE(NT, 256, 2, 2) RES3_CASE(NT, 256, 2, 3) \
                    RES3_CASE(NT, 256, 2, 4)
    RES3_NT(1) RES3_NT(2) RES3_NT(3) RES3_NT(4)
#undef RES3_NT
#undef RES3_CASE
    return hipErrorInvalidValue;
  }
  if (dim == 2) {
    const int ty = residual_tile_rows(nt, a.n);
    if (ty == 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)(nt + 1) * (ty + 2) * a.n * sizeof(Tin);
    const int sit = ((ty + 2) * a.n + 255) / 256;
#define RESPF_CASE(NT, SIT)                                                                     \
  if (nt == NT && sit == SIT) {                                                                 \
    hipLaunchKernelGGL((k_residual_tile2d<Tin, Tout, NT, SIT>), grid, dim3(256), lds, s, u, F, r, \
                       a, partial, ty);                                                         \
    return hipGetLastError();                                                                   \
  }
#define RESPF_NT(NT) RESPF_CASE(NT, 1) RESPF_CASE(NT, 2) RESPF_CASE(NT, 3) RESPF_CASE(NT, 4) \
                     RESPF_CASE(NT, 5) RESPF_CASE(NT, 6)
    RESPF_NT(1) RESPF_NT(2) RESPF_NT(3) RESPF_NT(4)
#undef RESPF_NT
#undef RESPF_CASE
    return hipErrorInvalidValue;
  }
#define RES_CASE(D, NT)                                                                \
  if (dim == D && nt == NT) {                                                          \
    hipLaunchKernelGGL((k_residual<Tin, Tout, D, NT>), grid, dim3(256), 0, s, u, F, r, a, \
                       partial);                                                       \
    return hipGetLastError();                                                          \
  }
  RES_CASE(1, 1) RES_CASE(1, 2) RES_CASE(1, 3) RES_CASE(1, 4)
#undef RES_CASE
  return hipErrorInvalidValue;
}

// Shape of the residual with the restricting epilogue: 3-D workgroups of 256
// threads own TYC coarse rows (R = 2 TYC + 1 fine rows of n, R n <= 512, two
// positions a thread), 2-D workgroups one x line (n <= 512; 128, 256 or 512
// threads); chunks of ZCC coarse planes so that a level has about 8192
// workgroups (at least 4 planes a chunk).
bool resid_restrict_shape(int dim, int nt, int n, int nc, long long slabs, int tbytes, ResRestrictShape& sh) {
  if ((dim != 2 && dim != 3) || nt < 1 || nt > 4 || nc < 1 || n != 2 * nc + 1) return false;
  sh = ResRestrictShape{};
  int R;
  if (dim == 3) {
    sh.bs = 256;
    sh.tyc = (2 * sh.bs / n - 1) / 2;
    if (sh.tyc < 1) return false;
    if (sh.tyc > nc) sh.tyc = nc;
    R = 2 * sh.tyc + 1;
    sh.nyt = (nc + sh.tyc - 1) / sh.tyc;
  } else {
    if (n > 512) return false;
    sh.bs = n <= 128 ? 128 : (n <= 256 ? 256 : 512);
    sh.tyc = 1;
    R = 1;
    sh.nyt = 1;
  }
  const int plane = (R + (dim == 3 ? 2 : 0)) * n;
  sh.oit = (R * n + sh.bs - 1) / sh.bs;
  sh.sit = (plane + sh.bs - 1) / sh.bs;
  if (sh.oit > 2 || sh.sit > 3) return false;
  const long long per = (long long)sh.nyt * slabs;
  const long long want = (8192 + per - 1) / per;
  long long zc = (nc + want - 1) / want;
  const int zmin = nc < 4 ? nc : 4;
  if (zc < zmin) zc = zmin;
  sh.zcc = (int)zc;
  sh.nzt = (nc + sh.zcc - 1) / sh.zcc;
  sh.lds = ((size_t)(nt + 1) * plane + (size_t)nt * R * n) * (size_t)tbytes;
  return sh.lds <= 65536;
}

template <typename T>
hipError_t launch_resid_restrict(int dim, int nt, const T* u, const T* F, T* Fc, T* Hs, const ResidArgs<T>& a,
                                 const TransferArgs<T>& t, hipStream_t s) {
  const long long slabs = (long long)a.batch * a.N;
  ResRestrictShape sh;
  if (!resid_restrict_shape(dim, nt, a.n, t.nc, slabs, (int)sizeof(T), sh) || t.nf != a.n || a.N != 2 * t.Nc ||
      a.batch != t.batch)
    return hipErrorInvalidValue;
  const dim3 grid = slab_grid((unsigned)(sh.nyt * sh.nzt), slabs);
  bool done = false;
#define RR_CASE(D, NT, BS, OIT, SIT)                                                                       \
  if (!done && dim == D && nt == NT && sh.bs == BS && sh.oit == OIT && sh.sit == SIT) {                    \
    hipLaunchKernelGGL((k_resid_weigh<T, D, NT, BS, OIT, SIT>), grid, dim3(BS), sh.lds, s, u, F, Hs, a, t, \
                       sh.tyc, sh.zcc);                                                                     \
    done = true;                                                                                           \
  }
#define RR_NT(NT) RR_CASE(3, NT, 256, 2, 1) RR_CASE(3, NT, 256, 2, 2) RR_CASE(3, NT, 256, 2, 3) \
                  RR_CASE(3, NT, 256, 1, 1) RR_CASE(3, NT, 256, 1, 2) \
                  RR_CASE(2, NT, 128, 1, 1) RR_CASE(2, NT, 256, 1, 1) RR_CASE(2, NT, 512, 1, 1)
  RR_NT(1) RR_NT(2) RR_NT(3) RR_NT(4)
#undef RR_NT
#undef RR_CASE
  if (!done) return hipErrorInvalidValue;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long per = (long long)nt * t.nxc;
  const long long len = per * t.Nc * t.batch;
  hipLaunchKernelGGL((k_pair_sum<T>), dim3(blocks_for(len)), dim3(256), 0, s, Hs, Fc, per, len);
  return hipGetLastError();
}

#define TRANSFER_DISPATCH(KERNEL, TOTAL, ...)                                            \
  const unsigned grid = blocks_for(TOTAL);                                               \
  if (full) {                                                                            \
    if (dim == 1 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 1, 1, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 1 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 1, 2, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 1 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 1, 3, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 1 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 1, 4, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 2 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 2, 1, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 2 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 2, 2, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 2 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 2, 3, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 2 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 2, 4, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 3 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 3, 1, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 3 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 3, 2, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 3 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 3, 3, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (dim == 3 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 3, 4, true>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else return hipErrorInvalidValue;                                                   \
  } else {                                                                               \
    if (nt == 1) hipLaunchKernelGGL((KERNEL<T, 1, 1, false>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (nt == 2) hipLaunchKernelGGL((KERNEL<T, 1, 2, false>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (nt == 3) hipLaunchKernelGGL((KERNEL<T, 1, 3, false>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else if (nt == 4) hipLaunchKernelGGL((KERNEL<T, 1, 4, false>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
    else return hipErrorInvalidValue;                                                   \
  }                                                                                      \
  return hipGetLastError();

template <typename T>
hipError_t launch_restrict(int dim, int nt, bool full, const T* rf, T* Fc, const TransferArgs<T>& a,
                           hipStream_t s) {
  TRANSFER_DISPATCH(k_restrict, a.nxc * a.Nc * a.batch, rf, Fc, a)
}

template <typename T>
hipError_t launch_prolong(int dim, int nt, bool full, const T* ec, T* uf, const TransferArgs<T>& a,
                          hipStream_t s) {
  if (a.nxf > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 pgrid = slab_grid(blocks_for(a.nxf), (long long)a.Nc * a.batch);
#define PR_CASE(D, NT, FULL) \
  if (dim == D && nt == NT && full == FULL) { hipLaunchKernelGGL((k_prolong<T, D, NT, FULL>), pgrid, dim3(256), 0, s, ec, uf, a); return hipGetLastError(); }
#define PR_NT(NT) PR_CASE(1, NT, true) PR_CASE(2, NT, true) PR_CASE(3, NT, true) \
                  PR_CASE(1, NT, false) PR_CASE(2, NT, false) PR_CASE(3, NT, false)
  PR_NT(1) PR_NT(2) PR_NT(3) PR_NT(4)
#undef PR_NT
#undef PR_CASE
  return hipErrorInvalidValue;
}
#undef TRANSFER_DISPATCH

#define RHS_DISPATCH(KERNEL, ...)                                                          \
  const unsigned grid = blocks_for(a.nx * a.N * a.batch);                                  \
  if (dim == 1 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 1, 1>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 1 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 1, 2>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 1 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 1, 3>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 1 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 1, 4>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 2, 1>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 2, 2>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 2, 3>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 2 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 2, 4>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 1) hipLaunchKernelGGL((KERNEL<T, 3, 1>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 2) hipLaunchKernelGGL((KERNEL<T, 3, 2>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 3) hipLaunchKernelGGL((KERNEL<T, 3, 3>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else if (dim == 3 && nt == 4) hipLaunchKernelGGL((KERNEL<T, 3, 4>), dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  else return hipErrorInvalidValue;                                                        \
  return hipGetLastError();

template <typename T>
hipError_t launch_rhs(int dim, int nt, const T* f, const T* u0, T* F, const RhsArgs<T>& a,
                      hipStream_t s) {
  RHS_DISPATCH(k_rhs, f, u0, F, a)
}

template <typename T>
hipError_t launch_rhs_adjoint(int dim, int nt, const T* lam, T* gf, T* gu0, const RhsArgs<T>& a,
                              hipStream_t s) {
  RHS_DISPATCH(k_rhs_adjoint, lam, gf, gu0, a)
}
#undef RHS_DISPATCH

template <typename T>
hipError_t launch_sumsq(const T* v, long long len, int batch, double* partial, unsigned gx,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_sumsq<T>), dim3(gx, batch), dim3(256), 0, s, v, len, partial);
  return hipGetLastError();
}

hipError_t launch_norm_final(const double* partial, long long per_batch, int batch, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_norm_final, dim3(batch), dim3(256), 0, s, partial, per_batch, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* v, long long len, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(len)), dim3(256), 0, s, v, len);
  return hipGetLastError();
}

hipError_t launch_spin(double microseconds, hipStream_t s) {
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  if (khz <= 0) khz = 100000;
  const double us = microseconds < 0 ? 0.0 : (microseconds > 5000.0 ? 5000.0 : microseconds);
  hipLaunchKernelGGL(k_spin, dim3(1), dim3(64), 0, s, (long long)(us * 1e-3 * khz));
  return hipGetLastError();
}

hipError_t launch_axpy_f32_f64(double* u, const float* e, long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_f32_f64, dim3(blocks_for(len)), dim3(256), 0, s, u, e, len);
  return hipGetLastError();
}
hipError_t launch_cast_f64_f32(const double* in, float* out, long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f64_f32, dim3(blocks_for(len)), dim3(256), 0, s, in, out, len);
  return hipGetLastError();
}
hipError_t launch_cast_f32_f64(const float* in, double* out, long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f32_f64, dim3(blocks_for(len)), dim3(256), 0, s, in, out, len);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_residual<double, double>(int, int, const double*, const double*, double*,
                                                    const ResidArgs<double>&, double*, hipStream_t);
template hipError_t launch_residual<double, float>(int, int, const double*, const double*, float*,
                                                   const ResidArgs<double>&, double*, hipStream_t);
template hipError_t launch_residual<float, float>(int, int, const float*, const float*, float*,
                                                  const ResidArgs<float>&, double*, hipStream_t);
#define INST(T)                                                                                     \
  template hipError_t launch_restrict<T>(int, int, bool, const T*, T*, const TransferArgs<T>&,      \
                                         hipStream_t);                                              \
  template hipError_t launch_prolong<T>(int, int, bool, const T*, T*, const TransferArgs<T>&,       \
                                        hipStream_t);                                               \
  template hipError_t launch_resid_restrict<T>(int, int, const T*, const T*, T*, T*, const ResidArgs<T>&, \
                                               const TransferArgs<T>&, hipStream_t);                       \
  template hipError_t launch_rhs<T>(int, int, const T*, const T*, T*, const RhsArgs<T>&, hipStream_t); \
  template hipError_t launch_rhs_adjoint<T>(int, int, const T*, T*, T*, const RhsArgs<T>&,          \
                                            hipStream_t);                                           \
  template hipError_t launch_sumsq<T>(const T*, long long, int, double*, unsigned, hipStream_t); \
  template hipError_t launch_fill<T>(T*, long long, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
