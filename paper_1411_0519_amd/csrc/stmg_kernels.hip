// HIP kernels of the space-time multigrid V-cycle for gfx950 (MI355X).
//
// Vector layout: [batch][slab][time dof l][z][y][x], x fastest.  One level has
// n interior nodes per dimension (nx = n^d), N slabs and N_t = p_t + 1 time dofs.
//
//   k_residual  r = F - L u: Q1 mass/stiffness stencils (3/9/27 points, applied
//               separably), N_t x N_t time mixing, upwind coupling to the
//               neighbouring slab (eq. chap4_generalLinearSystem).  Fused
//               per-block partial sums of r^2 for the norm.
//   k_dst       one sine-transform pass along one axis as a tall GEMM on the
//               matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32):
//               out[o][k][c] = sum_i S[k][i] in[o][i][c], S the orthonormal
//               DST-I (S = S^T = S^{-1}); epilogue store / u += omega out.
//   k_tsolve    per sine mode k the N_t x N_t solve G_k = (mu_k K + nu_k M)^{-1}
//               (fast diagonalisation of the slab block A = K (x) M_h + M (x) K_h).
//   k_restrict  F_c[m] = R1 r[2m] + R2 r[2m+1], optional full weighting in space
//               (eq. chap4_restrictionTime, eq. chap4_spaceRestrictionProlongation).
//   k_prolong   u[2m] += R1^T e_c[m], u[2m+1] += R2^T e_c[m], optional
//               (bi/tri)linear interpolation in space.
#include <hip/hip_runtime.h>

#include "stmg_internal.h"

namespace stmg {

namespace {

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

template <int D>
__device__ inline void node_coords(long long j, int n, int& x, int& y, int& z) {
  x = (int)(j % n);
  y = (D >= 2) ? (int)((j / n) % n) : 0;
  z = (D == 3) ? (int)(j / ((long long)n * n)) : 0;
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

// ------------------------------------------------------------- DST contraction
// One workgroup (4 waves) owns TILE_COLS = 64 columns and all n rows of the
// contracted axis.  The data tile is staged in LDS (row stride 65 to spread
// banks); the transform matrix is read from global memory in MFMA fragment
// order (Sfrag[(kb*(NP/4) + ib)*64 + lane] = S[16 kb + lane%16][4 ib + lane/16]),
// which makes every fragment load one coalesced 64-lane access.
template <typename T, int NB, bool XAXIS>
__global__ __launch_bounds__(256) void k_dst(const T* __restrict__ in, T* __restrict__ out,
                                             const T* __restrict__ Sfrag, int n, long long inner,
                                             long long ncols, T omega, int mode) {
  constexpr int NP = 16 * NB;
  constexpr int LD = TILE_COLS + 1;
  constexpr int KPW = (NB >= 4) ? NB / 4 : NB;   // k-blocks per wave
  constexpr int CPW = (NB >= 4) ? 4 : 1;         // 16-column blocks per wave
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T tile[NP * LD];

  const int tid = threadIdx.x;
  const long long col0 = (long long)blockIdx.x * TILE_COLS;
  const long long ncol_here = (ncols - col0) < TILE_COLS ? (ncols - col0) : TILE_COLS;

  // ---- stage the input tile: tile[i][c] = X[i][col0 + c]
  if (XAXIS) {
    const long long base = col0 * n;
    const int total = TILE_COLS * n;
    const long long maxe = ncol_here * n;
    for (int e = tid; e < total; e += 256) {
      const int c = e / n;
      const int i = e - c * n;
      tile[i * LD + c] = (e < maxe) ? in[base + e] : T(0);
    }
  } else {
    const int c = tid & (TILE_COLS - 1);
    const long long col = col0 + c;
    const bool valid = c < ncol_here;
    const long long o = valid ? col / inner : 0;
    const long long cc = valid ? col - o * inner : 0;
    const T* src = in + o * (long long)n * inner + cc;
    for (int i = tid >> 6; i < n; i += 4) tile[i * LD + c] = valid ? src[(long long)i * inner] : T(0);
  }
  for (int e = tid; e < (NP - n) * TILE_COLS; e += 256) {
    const int i = n + e / TILE_COLS;
    tile[i * LD + (e % TILE_COLS)] = T(0);
  }
  __syncthreads();

  // ---- contraction on the matrix cores
  const int lane = tid & 63;
  const int wave = tid >> 6;
  acc_t acc[KPW][CPW];
#pragma unroll
  for (int q = 0; q < KPW; ++q)
#pragma unroll
    for (int p = 0; p < CPW; ++p) acc[q][p] = acc_t{0, 0, 0, 0};
  const int ibmax = (n + 3) >> 2;
  const int brow = lane >> 4, bcol = lane & 15;
  for (int ib = 0; ib < ibmax; ++ib) {
    T bf[CPW];
#pragma unroll
    for (int p = 0; p < CPW; ++p) {
      const int cb = (NB >= 4) ? p : wave;
      bf[p] = tile[(ib * 4 + brow) * LD + cb * 16 + bcol];
    }
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
      const int kb = (NB >= 4) ? wave + 4 * q : q;
      const T af = Sfrag[((long long)kb * (NP / 4) + ib) * 64 + lane];
#pragma unroll
      for (int p = 0; p < CPW; ++p) acc[q][p] = Mfma<T>::op(af, bf[p], acc[q][p]);
    }
  }
  __syncthreads();
  // ---- accumulators back to LDS
#pragma unroll
  for (int q = 0; q < KPW; ++q) {
    const int kb = (NB >= 4) ? wave + 4 * q : q;
#pragma unroll
    for (int p = 0; p < CPW; ++p) {
      const int cb = (NB >= 4) ? p : wave;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int k = kb * 16 + Mfma<T>::row(brow, jj);
        tile[k * LD + cb * 16 + bcol] = acc[q][p][jj];
      }
    }
  }
  __syncthreads();

  // ---- store with epilogue
  if (XAXIS) {
    const long long base = col0 * n;
    const long long maxe = ncol_here * n;
    const int total = TILE_COLS * n;
    for (int e = tid; e < total && e < maxe; e += 256) {
      const int c = e / n;
      const int i = e - c * n;
      const T v = tile[i * LD + c];
      T* dst = out + base + e;
      if (mode == MODE_STORE) *dst = v;
      else if (mode == MODE_ADD_SCALED) *dst += omega * v;
      else *dst = omega * v;
    }
  } else {
    const int c = tid & (TILE_COLS - 1);
    if (c < ncol_here) {
      const long long col = col0 + c;
      const long long o = col / inner;
      const long long cc = col - o * inner;
      T* dstb = out + o * (long long)n * inner + cc;
      for (int i = tid >> 6; i < n; i += 4) {
        const T v = tile[i * LD + c];
        T* dst = dstb + (long long)i * inner;
        if (mode == MODE_STORE) *dst = v;
        else if (mode == MODE_ADD_SCALED) *dst += omega * v;
        else *dst = omega * v;
      }
    }
  }
}

// ------------------------------------------------------------- per-mode solve
template <typename T, int NT>
__global__ __launch_bounds__(256) void k_tsolve(T* __restrict__ buf, const T* __restrict__ G,
                                                long long nx, long long nslab, int transpose) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nx * nslab) return;
  const long long s = idx / nx;
  const long long j = idx - s * nx;
  T* p = buf + s * NT * nx + j;
  T v[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) v[k] = p[k * nx];
  const T* g = G + j * NT * NT;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) acc += (transpose ? g[k * NT + l] : g[l * NT + k]) * v[k];
    p[l * nx] = acc;
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
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nxc = a.nxc, nxf = a.nxf;
  const long long total = nxf * a.Nc * a.batch;
  if (idx >= total) return;
  const long long jf = idx % nxf;
  const long long cs = idx / nxf;
  const long long m = cs % a.Nc;
  const long long bi = cs / a.Nc;
  const long long fs0 = bi * (2LL * a.Nc) + 2 * m;
  const T* ecs = ec + cs * NT * nxc;
  T e[NT];
  if (FULL) {
    int fx, fy, fz;
    node_coords<D>(jf, a.nf, fx, fy, fz);
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

unsigned residual_blocks_per_slab(long long nx) { return (unsigned)((nx + 255) / 256); }

template <typename Tin, typename Tout>
hipError_t launch_residual(int dim, int nt, const Tin* u, const Tin* F, Tout* r,
                           const ResidArgs<Tin>& a, double* partial, hipStream_t s) {
  const unsigned gx = residual_blocks_per_slab(a.nx);
  const dim3 grid = slab_grid(gx, (long long)a.batch * a.N);
#define RES_CASE(D, NT)                                                                \
  if (dim == D && nt == NT) {                                                          \
    hipLaunchKernelGGL((k_residual<Tin, Tout, D, NT>), grid, dim3(256), 0, s, u, F, r, a, \
                       partial);                                                       \
    return hipGetLastError();                                                          \
  }
  RES_CASE(1, 1) RES_CASE(1, 2) RES_CASE(1, 3) RES_CASE(1, 4)
  RES_CASE(2, 1) RES_CASE(2, 2) RES_CASE(2, 3) RES_CASE(2, 4)
  RES_CASE(3, 1) RES_CASE(3, 2) RES_CASE(3, 3) RES_CASE(3, 4)
#undef RES_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dst(int np, bool xaxis, const T* in, T* out, const T* Sfrag, int n,
                      long long inner, long long ncols, T omega, int mode, hipStream_t s) {
  const unsigned grid = (unsigned)((ncols + TILE_COLS - 1) / TILE_COLS);
#define DST_CASE(NB)                                                                       \
  if (np == 16 * NB) {                                                                     \
    if (xaxis)                                                                             \
      hipLaunchKernelGGL((k_dst<T, NB, true>), dim3(grid), dim3(256), 0, s, in, out, Sfrag, \
                         n, inner, ncols, omega, mode);                                    \
    else                                                                                   \
      hipLaunchKernelGGL((k_dst<T, NB, false>), dim3(grid), dim3(256), 0, s, in, out,       \
                         Sfrag, n, inner, ncols, omega, mode);                             \
    return hipGetLastError();                                                              \
  }
  DST_CASE(1) DST_CASE(2) DST_CASE(4) DST_CASE(8) DST_CASE(16)
#undef DST_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_tsolve(int nt, T* buf, const T* G, long long nx, long long nslab, int transpose,
                         hipStream_t s) {
  const unsigned grid = blocks_for(nx * nslab);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_tsolve<T, 1>), dim3(grid), dim3(256), 0, s, buf, G, nx, nslab, transpose); break;
    case 2: hipLaunchKernelGGL((k_tsolve<T, 2>), dim3(grid), dim3(256), 0, s, buf, G, nx, nslab, transpose); break;
    case 3: hipLaunchKernelGGL((k_tsolve<T, 3>), dim3(grid), dim3(256), 0, s, buf, G, nx, nslab, transpose); break;
    case 4: hipLaunchKernelGGL((k_tsolve<T, 4>), dim3(grid), dim3(256), 0, s, buf, G, nx, nslab, transpose); break;
    default: return hipErrorInvalidValue;
  }
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
  TRANSFER_DISPATCH(k_prolong, a.nxf * a.Nc * a.batch, ec, uf, a)
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
  template hipError_t launch_dst<T>(int, bool, const T*, T*, const T*, int, long long, long long, T, \
                                    int, hipStream_t);                                              \
  template hipError_t launch_tsolve<T>(int, T*, const T*, long long, long long, int, hipStream_t);  \
  template hipError_t launch_restrict<T>(int, int, bool, const T*, T*, const TransferArgs<T>&,      \
                                         hipStream_t);                                              \
  template hipError_t launch_prolong<T>(int, int, bool, const T*, T*, const TransferArgs<T>&,       \
                                        hipStream_t);                                               \
  template hipError_t launch_rhs<T>(int, int, const T*, const T*, T*, const RhsArgs<T>&, hipStream_t); \
  template hipError_t launch_rhs_adjoint<T>(int, int, const T*, T*, T*, const RhsArgs<T>&,          \
                                            hipStream_t);                                           \
  template hipError_t launch_sumsq<T>(const T*, long long, int, double*, unsigned, hipStream_t); \
  template hipError_t launch_fill<T>(T*, long long, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
