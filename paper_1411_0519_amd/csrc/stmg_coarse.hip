// The coarse end of a space-time cycle in one workgroup (Sec. 2 cycle with the
// exact block-Jacobi smoother, eq. chap4_smoother / chap4_smootherExact):
// from a level whose vectors, and those of every coarser level, fit in LDS,
// the whole cycle -- smoothing steps (residual, sine transforms, per-mode
// N_t x N_t solves, damped update), restriction, gamma coarse cycles,
// prolongation and the exact solve on the single coarsest slab -- runs with
// barriers instead of kernel launches.  On these levels the launches and the
// global-memory round trips between them cost far more than the arithmetic.
//
// LDS: per level q the plain DST matrix S_q (n x n), the per-mode inverse
// blocks G_q (spectral order), the iterate U_q and the right-hand side F_q
// (all b N_q slabs, layout as in global memory), plus two scratch vectors of
// the largest level.  The cycle's recursion is unrolled into a loop over an
// explicit per-level stage (uniform across the workgroup).
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

constexpr int CB = 512;   // threads per workgroup

__device__ inline int spectral_index(int k, int n) {   // plain mode k (0-based) -> folded order
  const int kk = k + 1, h = (n + 1) >> 1;
  return (kk & 1) ? (kk - 1) >> 1 : h + (kk >> 1) - 1;
}

// q = e / d for 0 <= e < 2^20 from a float reciprocal and one correction
// (the indices here stay below the 64 KB LDS budget, far inside that range).
__device__ inline int fdiv(int e, int d, float r) {
  int q = (int)((float)e * r);
  if (q * d > e) --q;
  else if ((q + 1) * d <= e) ++q;
  return q;
}

template <int D>
__device__ inline void coords3(int j, int n, float rn, int& x, int& y, int& z) {
  const int t = fdiv(j, n, rn);
  x = j - t * n;
  if (D >= 2) {
    z = D == 3 ? fdiv(t, n, rn) : 0;
    y = t - z * n;
  } else {
    y = 0;
    z = 0;
  }
}

template <typename T, int D, int NT>
struct Ctx {
  const CoarseArgs<T>& a;
  T* lds;
  int b;
  __device__ T* S(int q) const { return lds + a.lv[q].offS; }
  __device__ T* G(int q) const { return lds + a.lv[q].offG; }
  __device__ T* U(int q) const { return lds + a.lv[q].offU; }
  __device__ T* F(int q) const { return lds + a.lv[q].offF; }
  __device__ T* R() const { return lds + a.offR; }
  __device__ T* Q() const { return lds + a.offQ; }
  __device__ int slabs(int q) const { return b * a.lv[q].N; }
  __device__ int dof(int q) const { return slabs(q) * NT * a.lv[q].nx; }

  // R = F - L U on level q (U treated as zero: R = F)
  __device__ void residual(int q, bool zero) const {
    const CoarseLevel<T>& L = a.lv[q];
    const int n = L.n, nx = L.nx, N = L.N, ns = slabs(q);
    const T* u = U(q);
    const T* f = F(q);
    T* r = R();
    for (int e = threadIdx.x; e < ns * nx; e += blockDim.x) {
      const int sl = fdiv(e, nx, L.rnx), j = e - sl * nx, s = sl - fdiv(sl, N, L.rN) * N;
      T mu[NT + 1], ku[NT];
#pragma unroll
      for (int c = 0; c <= NT; ++c) mu[c] = T(0);
#pragma unroll
      for (int c = 0; c < NT; ++c) ku[c] = T(0);
      if (!zero) {
        const bool couple = s + a.dir >= 0 && s + a.dir < N;
        int x, y, z;
        coords3<D>(j, n, L.rn, x, y, z);
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz) {
          const int zz = z + dz;
          if (zz < 0 || zz >= n) continue;
          for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= n) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              const int xx = x + dx;
              if (xx < 0 || xx >= n) continue;
              const int idx = (zz * n + yy) * n + xx;
              const T mx = L.wm[dx + 1], my = D >= 2 ? L.wm[dy + 1] : T(1), mz = D == 3 ? L.wm[dz + 1] : T(1);
              T wmass = mx * my * mz;
              T wstiff = L.wk[dx + 1] * my * mz;
              if (D >= 2) wstiff += mx * L.wk[dy + 1] * mz;
              if (D == 3) wstiff += mx * my * L.wk[dz + 1];
#pragma unroll
              for (int c = 0; c < NT; ++c) {
                const T v = u[(sl * NT + c) * nx + idx];
                mu[c] += wmass * v;
                ku[c] += wstiff * v;
              }
              if (couple) {
                T w = T(0);
#pragma unroll
                for (int k = 0; k < NT; ++k) w += L.cb[k] * u[((sl + a.dir) * NT + k) * nx + idx];
                mu[NT] += wmass * w;
              }
            }
          }
        }
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = f[(sl * NT + l) * nx + j] + L.ca[l] * mu[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) acc -= L.K[l * NT + k] * mu[k] + L.M[l * NT + k] * ku[k];
        r[(sl * NT + l) * nx + j] = acc;
      }
    }
    __syncthreads();
  }

  // out = S along one axis (the plain DST-I is symmetric, its own inverse)
  __device__ void dst_axis(int q, int axis, const T* in, T* out) const {
    const CoarseLevel<T>& L = a.lv[q];
    const int n = L.n, nx = L.nx;
    const int stride = axis == 0 ? 1 : (axis == 1 ? n : n * n);
    const T* s = S(q);
    const int total = slabs(q) * NT * nx;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int v = fdiv(e, nx, L.rnx), j = e - v * nx;
      int x0, y0, z0;
      coords3<D>(j, n, L.rn, x0, y0, z0);
      const int k = axis == 0 ? x0 : (axis == 1 ? y0 : z0);
      const int base = v * nx + j - k * stride;
      T acc = T(0);
      for (int i = 0; i < n; ++i) acc += s[k * n + i] * in[base + i * stride];
      out[e] = acc;
    }
    __syncthreads();
  }

  // The last forward pass (along the slowest axis) for all N_t components of a
  // node at once, followed by that sine mode's N_t x N_t solve (G or G^T).
  __device__ void dst_last_and_solve(int q, const T* in, T* out) const {
    const CoarseLevel<T>& L = a.lv[q];
    const int n = L.n, nx = L.nx;
    const int axis = D - 1, stride = axis == 0 ? 1 : (axis == 1 ? n : n * n);
    const T* s = S(q);
    const T* g0 = G(q);
    for (int e = threadIdx.x; e < slabs(q) * nx; e += blockDim.x) {
      const int sl = fdiv(e, nx, L.rnx), j = e - sl * nx;
      int x0, y0, z0;
      coords3<D>(j, n, L.rn, x0, y0, z0);
      const int k = axis == 0 ? x0 : (axis == 1 ? y0 : z0);
      const int base = j - k * stride;
      T v[NT];
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const T* src = in + (sl * NT + c) * nx + base;
        T acc = T(0);
        for (int i = 0; i < n; ++i) acc += s[k * n + i] * src[i * stride];
        v[c] = acc;
      }
      int js = spectral_index(x0, n);
      if (D >= 2) js += n * spectral_index(y0, n);
      if (D == 3) js += n * n * spectral_index(z0, n);
      const T* g = g0 + js * NT * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < NT; ++c) acc += (a.transpose ? g[c * NT + l] : g[l * NT + c]) * v[c];
        out[(sl * NT + l) * nx + j] = acc;
      }
    }
    __syncthreads();
  }

  // The last inverse pass (along x) written into U: U = scale y (set) or
  // U += scale y.
  __device__ void dst_first_into(int q, const T* in, bool set, T scale) const {
    const CoarseLevel<T>& L = a.lv[q];
    const int n = L.n, nx = L.nx;
    const T* s = S(q);
    T* u = U(q);
    for (int e = threadIdx.x; e < dof(q); e += blockDim.x) {
      const int v = fdiv(e, nx, L.rnx), j = e - v * nx;
      const int k = j - fdiv(j, n, L.rn) * n;
      const T* src = in + v * nx + j - k;
      T acc = T(0);
      for (int i = 0; i < n; ++i) acc += s[k * n + i] * src[i];
      u[e] = set ? scale * acc : u[e] + scale * acc;
    }
    __syncthreads();
  }

  // U = scale D^{-1} src (set) or U += scale D^{-1} src; src is R or F(q)
  __device__ void block_solve_into(int q, const T* src, bool set, T scale) const {
    const T* cur = src;
    T* bufs[2] = {Q(), R()};
    int w = 0;
    if (src == Q()) w = 1;
    for (int ax = 0; ax < D - 1; ++ax) {   // leading forward passes
      dst_axis(q, ax, cur, bufs[w]);
      cur = bufs[w];
      w ^= 1;
    }
    dst_last_and_solve(q, cur, bufs[w]);
    cur = bufs[w];
    w ^= 1;
    for (int ax = D - 1; ax >= 1; --ax) {   // inverse passes down to y
      dst_axis(q, ax, cur, bufs[w]);
      cur = bufs[w];
      w ^= 1;
    }
    dst_first_into(q, cur, set, scale);
  }

  // U = omega D^{-1} F (zero) or U += omega D^{-1} (F - L U)
  __device__ void smooth(int q, bool zero) const {
    if (zero) {
      block_solve_into(q, F(q), true, a.omega);
      return;
    }
    residual(q, false);
    block_solve_into(q, R(), false, a.omega);
  }

  // F_{q+1} = R_transfer (R): time blocks and, for full coarsening, full weighting
  __device__ void restrict_to(int q, const T* rf) const {
    const CoarseLevel<T>& Lf = a.lv[q];
    const CoarseLevel<T>& Lc = a.lv[q + 1];
    const int nf = Lf.n, nc = Lc.n, nxf = Lf.nx, nxc = Lc.nx, Nc = Lc.N;
    T* fc = F(q + 1);
    for (int e = threadIdx.x; e < slabs(q + 1) * nxc; e += blockDim.x) {
      const int cs = fdiv(e, nxc, Lc.rnx), jc = e - cs * nxc;
      const int bi = fdiv(cs, Nc, Lc.rN), m = cs - bi * Nc;
      const int fs0 = bi * 2 * Nc + 2 * m;
      T v[2][NT];
      if (Lf.full) {
        int cx, cy, cz;
        coords3<D>(jc, nc, Lc.rn, cx, cy, cz);
        const int fx = 2 * cx + 1, fy = 2 * cy + 1, fz = 2 * cz + 1;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            const T* base = rf + ((fs0 + s) * NT + k) * nxf;
            T acc = T(0);
            for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
              for (int dy = (D >= 2 ? -1 : 0); dy <= (D >= 2 ? 1 : 0); ++dy) {
                const T wzy = (dz == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
                const int rz = D == 3 ? fz + dz : 0, ry = D >= 2 ? fy + dy : 0;
                const T* line = base + (rz * nf + ry) * nf;
                acc += wzy * (T(0.5) * line[fx - 1] + line[fx] + T(0.5) * line[fx + 1]);
              }
            v[s][k] = acc;
          }
      } else {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int k = 0; k < NT; ++k) v[s][k] = rf[((fs0 + s) * NT + k) * nxf + jc];
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) acc += a.R1T[k * NT + l] * v[0][k] + a.R2T[k * NT + l] * v[1][k];
        fc[(cs * NT + l) * nxc + jc] = acc;
      }
    }
    __syncthreads();
  }

  // U_q += P U_{q+1}
  __device__ void prolong_from(int q) const {
    const CoarseLevel<T>& Lf = a.lv[q];
    const CoarseLevel<T>& Lc = a.lv[q + 1];
    const int nf = Lf.n, nc = Lc.n, nxf = Lf.nx, nxc = Lc.nx, Nc = Lc.N, Nf = Lf.N;
    const T* ec = U(q + 1);
    T* uf = U(q);
    for (int e = threadIdx.x; e < slabs(q) * nxf; e += blockDim.x) {
      const int fsl = fdiv(e, nxf, Lf.rnx), jf = e - fsl * nxf;
      const int bi = fdiv(fsl, Nf, Lf.rN), fs = fsl - bi * Nf, m = fs >> 1;
      const T* blk = (fs & 1) ? a.R2T : a.R1T;
      const T* src = ec + (bi * Nc + m) * NT * nxc;
      T ev[NT];
      if (Lf.full) {
        int fx, fy, fz;
        coords3<D>(jf, nf, Lf.rn, fx, fy, fz);
        int cc[3][2];
        T ww[3][2];
        int cnt[3];
        const int f3[3] = {fx, fy, fz};
        for (int ax = 0; ax < 3; ++ax) {
          if (ax >= D) {
            cc[ax][0] = 0;
            ww[ax][0] = T(1);
            cnt[ax] = 1;
            continue;
          }
          const int f = f3[ax];
          if (f & 1) {
            cc[ax][0] = (f - 1) >> 1;
            ww[ax][0] = T(1);
            cnt[ax] = 1;
          } else {
            cc[ax][0] = (f >> 1) - 1;
            ww[ax][0] = T(0.5);
            cc[ax][1] = f >> 1;
            ww[ax][1] = T(0.5);
            cnt[ax] = 2;
          }
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) ev[k] = T(0);
        for (int iz = 0; iz < cnt[2]; ++iz) {
          const int cz = cc[2][iz];
          if (cz < 0 || cz >= (D == 3 ? nc : 1)) continue;
          for (int iy = 0; iy < cnt[1]; ++iy) {
            const int cy = cc[1][iy];
            if (cy < 0 || cy >= (D >= 2 ? nc : 1)) continue;
            for (int ix = 0; ix < cnt[0]; ++ix) {
              const int cx = cc[0][ix];
              if (cx < 0 || cx >= nc) continue;
              const T w = ww[0][ix] * ww[1][iy] * ww[2][iz];
              const int jc = (cz * nc + cy) * nc + cx;
#pragma unroll
              for (int k = 0; k < NT; ++k) ev[k] += w * src[k * nxc + jc];
            }
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < NT; ++k) ev[k] = src[k * nxc + jf];
      }
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) acc += blk[l * NT + k] * ev[k];
        uf[(fsl * NT + l) * nxf + jf] += acc;
      }
    }
    __syncthreads();
  }

  // exact solve on the coarsest level (one slab per right-hand side): U = D^{-1} F
  __device__ void exact(int q) const { block_solve_into(q, F(q), true, T(1)); }
};

template <typename T, int D, int NT>
__global__ __launch_bounds__(CB) void k_coarse_cycle(const CoarseArgs<T>* __restrict__ ap, const T* __restrict__ Ftop,
                                                     T* __restrict__ utop, int batch, int u_zero) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const CoarseArgs<T>& a = *ap;
  Ctx<T, D, NT> c{a, reinterpret_cast<T*>(lds_raw), batch};
  const int last = a.levels - 1;
  // stage the tables of every level and the top level's F (and U)
  for (int q = 0; q <= last; ++q) {
    const int n = a.lv[q].n, nx = a.lv[q].nx;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) c.S(q)[e] = a.lv[q].gS[e];
    for (int e = threadIdx.x; e < nx * NT * NT; e += blockDim.x) c.G(q)[e] = a.lv[q].gG[e];
  }
  for (int e = threadIdx.x; e < c.dof(0); e += blockDim.x) {
    c.F(0)[e] = Ftop[e];
    c.U(0)[e] = u_zero ? T(0) : utop[e];
  }
  __syncthreads();
  int stage[CT_MAX], done[CT_MAX], zero[CT_MAX];
  int q = 0;
  stage[0] = 0;
  zero[0] = u_zero;
  while (q >= 0) {
    if (q == last) {
      c.exact(q);
      --q;
      continue;
    }
    if (stage[q] == 0) {
      const bool z = zero[q] != 0;
      for (int i = 0; i < a.nu1; ++i) c.smooth(q, z && i == 0);
      if (a.nu1 == 0 && z) {   // nothing smoothed yet: the iterate is zero, the defect is F
        for (int e = threadIdx.x; e < c.dof(q); e += blockDim.x) c.U(q)[e] = T(0);
        __syncthreads();
      }
      if (a.nu1 == 0 && z) c.restrict_to(q, c.F(q));   // the defect of a zero iterate is F
      else {
        c.residual(q, false);
        c.restrict_to(q, c.R());
      }
      done[q] = 0;
      stage[q] = 1;
      zero[q + 1] = 1;
      stage[q + 1] = 0;
      ++q;
      continue;
    }
    if (++done[q] < a.gamma) {   // another coarse cycle, from the previous coarse result
      zero[q + 1] = 0;
      stage[q + 1] = 0;
      ++q;
      continue;
    }
    c.prolong_from(q);
    for (int i = 0; i < a.nu2; ++i) c.smooth(q, false);
    --q;
  }
  for (int e = threadIdx.x; e < c.dof(0); e += blockDim.x) utop[e] = c.U(0)[e];
}

}  // namespace

template <typename T>
hipError_t launch_coarse_cycle(int dim, int nt, const CoarseArgs<T>* args, size_t lds, const T* F, T* u, int batch,
                               int u_zero, hipStream_t s) {
  if (lds > 65536) return hipErrorInvalidValue;
#define CC(D, NT)                                                                                        \
  if (dim == D && nt == NT) {                                                                            \
    hipLaunchKernelGGL((k_coarse_cycle<T, D, NT>), dim3(1), dim3(CB), lds, s, args, F, u, batch, u_zero); \
    return hipGetLastError();                                                                            \
  }
  CC(1, 1) CC(1, 2) CC(1, 3) CC(1, 4)
  CC(2, 1) CC(2, 2) CC(2, 3) CC(2, 4)
  CC(3, 1) CC(3, 2) CC(3, 3) CC(3, 4)
#undef CC
  return hipErrorInvalidValue;
}

template hipError_t launch_coarse_cycle<double>(int, int, const CoarseArgs<double>*, size_t, const double*, double*,
                                                int, int, hipStream_t);
template hipError_t launch_coarse_cycle<float>(int, int, const CoarseArgs<float>*, size_t, const float*, float*, int,
                                               int, hipStream_t);

}  // namespace stmg
