// Kernels of the P1 mesh path (the setting of the numerical examples, Sec. 4).
// Space is an unstructured P1 discretisation: M_h and K_h of the interior
// nodes in CSR with one shared pattern (the same matrices for every slab), so
// every operator is a gather over a node's row.  Vectors keep the slab layout
// [batch][slab][time dof l][interior node]; each thread owns one node of one
// slab and all N_t time components of it.
//
//   k_mesh_residual        r = F - L u (or L^T), squared norms per workgroup
//   k_mesh_smooth          node-block Jacobi step or defect of the slab matrix
//                          A = K (x) M_h + M (x) K_h (spatial cycle of the
//                          inexact smoother, Remark V-cycleApproxSpace)
//   k_mesh_restrict_space  P^T in space per slab;  k_mesh_prolong_space  + P
//   k_mesh_dense           exact slab solve by a dense inverse (coarse mesh,
//                          coarsest level)
//   k_mesh_restrict / k_mesh_prolong  space-time transfers (R = P^T)
//   k_mesh_rhs / k_mesh_rhs_adjoint   load vector and its transpose
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

constexpr int MB = MESH_TILE;   // one thread per row of a tile (the host builds the tile halos)

// Blocks run over (slab, node tile) with the tiles of a slab adjacent and the
// dispatch order remapped so that each XCD works through a contiguous range of
// slabs: the gathers of a row then hit the slab vectors its own L2 holds.
__device__ inline void slab_tile(long long tiles, long long& slab, long long& tile) {
  const long long b = xcd_linear(blockIdx.x, gridDim.x);
  slab = b / tiles;
  tile = b - slab * tiles;
}

__device__ inline double block_sum(double v) {
  __shared__ double red[MB / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < MB / 64; ++w) s += red[w];
  return s;
}

// (M_h x_k)_i and (K_h x_k)_i for the N_t components of one slab, over the
// ELL copy (consecutive lanes read consecutive matrix entries).
template <typename T, int NT>
__device__ inline void row_mk(const MeshOp<T>& op, const T* __restrict__ x, long long nx, long long i, T* mu,
                              T* ku) {
#pragma unroll
  for (int k = 0; k < NT; ++k) mu[k] = ku[k] = T(0);
  for (int e = 0; e < op.ew; ++e) {
    const long long q = (long long)e * nx + i;
    const long long c = op.ecol[q];
    const T m = op.emk[2 * q], kk = op.emk[2 * q + 1];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const T v = x[k * nx + c];
      mu[k] += m * v;
      ku[k] += kk * v;
    }
  }
}

template <typename Tin, typename Tout, int NT>
__global__ __launch_bounds__(MB) void k_mesh_residual(const Tin* __restrict__ u, const Tin* __restrict__ F,
                                                      Tout* __restrict__ r, MeshResidArgs<Tin> a,
                                                      double* __restrict__ partial) {
  const long long nx = a.op.nx;
  long long slab, tile;
  slab_tile((nx + MB - 1) / MB, slab, tile);
  const long long i = tile * MB + threadIdx.x;
  const int s = (int)(slab % a.N);
  double ss = 0.0;
  if (i < nx && slab < (long long)a.batch * a.N) {
    const long long off = slab * NT * nx;
    const Tin* us = u + off;
    Tin mu[NT], ku[NT];
    Tin mw = Tin(0);   // coupling to the neighbouring slab: ca (M_h w), w = sum cb_k u_k
    if (s + a.dir >= 0 && s + a.dir < a.N) {
      const Tin* un = u + (slab + a.dir) * NT * nx;
#pragma unroll
      for (int k = 0; k < NT; ++k) mu[k] = ku[k] = Tin(0);
      for (int e = 0; e < a.op.ew; ++e) {
        const long long q = (long long)e * nx + i;
        const long long c = a.op.ecol[q];
        const Tin m = a.op.emk[2 * q], kk = a.op.emk[2 * q + 1];
        Tin w = Tin(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          const Tin v = us[k * nx + c];
          mu[k] += m * v;
          ku[k] += kk * v;
          w += a.cb[k] * un[k * nx + c];
        }
        mw += m * w;
      }
    } else {
      row_mk<Tin, NT>(a.op, us, nx, i, mu, ku);
    }
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      Tin acc = F[off + l * nx + i] + a.ca[l] * mw;
#pragma unroll
      for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
      r[off + l * nx + i] = (Tout)acc;
      ss += (double)acc * (double)acc;
    }
  }
  if (partial != nullptr) {
    const double t = block_sum(ss);
    if (threadIdx.x == 0 && slab < (long long)a.batch * a.N) partial[slab * ((nx + MB - 1) / MB) + tile] = t;
  }
}

// Halo-staged variants: the workgroup first copies the values its rows touch
// (the tile's halo, mostly contiguous thanks to the Z-order numbering) into
// LDS, once per time component, together with the neighbouring slab's
// coupling combination w = sum_k cb_k u_k; the rows are then formed from LDS.
template <typename T, int NT>
__device__ inline void stage_halo(const MeshOp<T>& op, long long tile, const T* __restrict__ xs,
                                  const T* __restrict__ xn, const T* cb, T* lx, T* lw) {
  const long long nx = op.nx;
  const int h0 = op.hoff[tile], hn = op.hoff[tile + 1] - h0;
  for (int j = threadIdx.x; j < hn; j += MB) {
    const long long c = op.hcol[h0 + j];
#pragma unroll
    for (int k = 0; k < NT; ++k) lx[k * op.hmax + j] = xs[k * nx + c];
    if (xn != nullptr) {
      T w = T(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) w += cb[k] * xn[k * nx + c];
      lw[j] = w;
    }
  }
  __syncthreads();
}

template <typename T, int NT>
__device__ inline void row_mk_lds(const MeshOp<T>& op, const T* lx, const T* lw, long long i, T* mu, T* ku,
                                  T& mw) {
  const long long nx = op.nx;
#pragma unroll
  for (int k = 0; k < NT; ++k) mu[k] = ku[k] = T(0);
  mw = T(0);
  for (int e = 0; e < op.ew; ++e) {
    const long long q = (long long)e * nx + i;
    const int lc = op.lcol[q];
    const T m = op.emk[2 * q], kk = op.emk[2 * q + 1];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const T v = lx[k * op.hmax + lc];
      mu[k] += m * v;
      ku[k] += kk * v;
    }
    if (lw != nullptr) mw += m * lw[lc];
  }
}

template <typename Tin, typename Tout, int NT>
__global__ __launch_bounds__(MB) void k_mesh_residual_lds(const Tin* __restrict__ u, const Tin* __restrict__ F,
                                                          Tout* __restrict__ r, MeshResidArgs<Tin> a,
                                                          double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Tin* lx = reinterpret_cast<Tin*>(lds_raw);
  Tin* lw = lx + NT * a.op.hmax;
  const long long nx = a.op.nx;
  const long long tiles = (nx + MB - 1) / MB;
  long long slab, tile;
  slab_tile(tiles, slab, tile);
  const long long i = tile * MB + threadIdx.x;
  const int s = (int)(slab % a.N);
  const bool couple = s + a.dir >= 0 && s + a.dir < a.N;
  const long long off = slab * NT * nx;
  stage_halo<Tin, NT>(a.op, tile, u + off, couple ? u + (slab + a.dir) * NT * nx : nullptr, a.cb, lx, lw);
  double ss = 0.0;
  if (i < nx) {
    Tin mu[NT], ku[NT], mw;
    row_mk_lds<Tin, NT>(a.op, lx, couple ? lw : nullptr, i, mu, ku, mw);
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      Tin acc = F[off + l * nx + i] + a.ca[l] * mw;
#pragma unroll
      for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
      r[off + l * nx + i] = (Tout)acc;
      ss += (double)acc * (double)acc;
    }
  }
  if (partial != nullptr) {
    const double t = block_sum(ss);
    if (threadIdx.x == 0) partial[slab * tiles + tile] = t;
  }
}

// Runs of consecutive slabs: a workgroup takes one node tile of up to SR
// slabs of one right-hand side in the order of the time coupling (increasing
// for the forward operator, decreasing for the adjoint).  Staging a slab's
// halo also forms the coupling combination w = sum_k cb_k u_k that the next
// slab of the run needs (two alternating buffers), so only the first slab of
// a run reads its neighbour from memory (u is read 1 + 1/SR times).  Partial
// sums of r^2 per (slab, tile) as in the one-slab kernels.  Dynamic LDS:
// (N_t + 2) hmax elements.
template <typename Tin, typename Tout, int NT>
__global__ __launch_bounds__(MB) void k_mesh_residual_run(const Tin* __restrict__ u, const Tin* __restrict__ F,
                                                          Tout* __restrict__ r, MeshResidArgs<Tin> a,
                                                          double* __restrict__ partial, int SR) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int hmax = a.op.hmax;
  Tin* lx = reinterpret_cast<Tin*>(lds_raw);
  Tin* lwb = lx + NT * hmax;   // [2][hmax]: coupling combinations, alternating
  const long long nx = a.op.nx;
  const long long tiles = (nx + MB - 1) / MB;
  const long long runs = (a.N + SR - 1) / SR;   // runs per right-hand side
  long long run, tile;
  slab_tile(tiles, run, tile);
  const long long bi = run / runs;
  const int sa = (int)(run - bi * runs) * SR;
  const int sb = sa + SR < a.N ? sa + SR : a.N;
  const long long i = tile * MB + threadIdx.x;
  const int h0 = a.op.hoff[tile], hn = a.op.hoff[tile + 1] - h0;
  for (int q = 0; q < sb - sa; ++q) {
    const int sn = a.dir < 0 ? sa + q : sb - 1 - q;
    const long long slab = bi * a.N + sn;
    const bool couple = sn + a.dir >= 0 && sn + a.dir < a.N;
    const Tin* xs = u + slab * NT * nx;
    const Tin* xn = u + (slab + a.dir) * NT * nx;
    Tin* lw = lwb + (q & 1) * hmax;          // this slab's coupling (formed one slab earlier)
    Tin* lw_next = lwb + (1 - (q & 1)) * hmax;
    for (int j = threadIdx.x; j < hn; j += MB) {
      const long long c = a.op.hcol[h0 + j];
      Tin w = Tin(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const Tin v = xs[k * nx + c];
        lx[k * hmax + j] = v;
        w += a.cb[k] * v;
      }
      lw_next[j] = w;
      if (q == 0 && couple) {
        Tin wn = Tin(0);
#pragma unroll
        for (int k = 0; k < NT; ++k) wn += a.cb[k] * xn[k * nx + c];
        lw[j] = wn;
      }
    }
    __syncthreads();
    double ss = 0.0;
    if (i < nx) {
      const long long off = slab * NT * nx;
      Tin mu[NT], ku[NT], mw;
      row_mk_lds<Tin, NT>(a.op, lx, couple ? lw : nullptr, i, mu, ku, mw);
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        Tin acc = F[off + l * nx + i] + a.ca[l] * mw;
#pragma unroll
        for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
        r[off + l * nx + i] = (Tout)acc;
        ss += (double)acc * (double)acc;
      }
    }
    if (partial != nullptr) {
      const double t = block_sum(ss);
      if (threadIdx.x == 0) partial[slab * tiles + tile] = t;
    }
    __syncthreads();   // every row is done with lx and lw before the next slab is staged
  }
}

// Solve D y = r for the node block D = m K + k M (N_t x N_t) by elimination
// without pivoting: the symmetric part of D is positive definite (that of K is
// semidefinite for the DG basis, M and the diagonals are positive), so every
// pivot is nonzero.
template <typename T, int NT>
__device__ inline void node_solve(const T* K, const T* M, T m, T k, T* r) {
  T D[NT][NT];
#pragma unroll
  for (int l = 0; l < NT; ++l)
#pragma unroll
    for (int c = 0; c < NT; ++c) D[l][c] = m * K[l * NT + c] + k * M[l * NT + c];
#pragma unroll
  for (int p = 0; p < NT; ++p) {
    const T inv = T(1) / D[p][p];
#pragma unroll
    for (int l = p + 1; l < NT; ++l) {
      const T f = D[l][p] * inv;
#pragma unroll
      for (int c = p + 1; c < NT; ++c) D[l][c] -= f * D[p][c];
      r[l] -= f * r[p];
    }
  }
#pragma unroll
  for (int p = NT - 1; p >= 0; --p) {
    T acc = r[p];
#pragma unroll
    for (int c = p + 1; c < NT; ++c) acc -= D[p][c] * r[c];
    r[p] = acc / D[p][p];
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_smooth(const T* __restrict__ x, const T* __restrict__ f,
                                                    const T* base, T* out, MeshSmoothArgs<T> a) {
  const long long nx = a.op.nx;
  long long slab, tile;
  slab_tile((nx + MB - 1) / MB, slab, tile);
  const long long i = tile * MB + threadIdx.x;
  if (slab >= a.slabs || i >= nx) return;
  const long long off = slab * NT * nx + i;
  T r[NT], xv[NT];
  if (a.x_zero) {
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      r[l] = f[off + l * nx];
      xv[l] = T(0);
    }
  } else {
    T mu[NT], ku[NT];
    row_mk<T, NT>(a.op, x + slab * NT * nx, nx, i, mu, ku);
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T acc = f[off + l * nx];
#pragma unroll
      for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
      r[l] = acc;
      xv[l] = x[off + l * nx];
    }
  }
  if (a.op_kind == SP_JACOBI) {
    node_solve<T, NT>(a.K, a.M, a.op.diag[2 * i], a.op.diag[2 * i + 1], r);
#pragma unroll
    for (int l = 0; l < NT; ++l) r[l] = xv[l] + a.omega * r[l];
  }
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T o = r[l];
    if (a.upd == UPD_ADD) o = base[off + l * nx] + a.scale * o;
    else if (a.upd == UPD_SET) o = a.scale * o;
    out[off + l * nx] = o;
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_smooth_lds(const T* __restrict__ x, const T* __restrict__ f,
                                                        const T* base, T* out, MeshSmoothArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lx = reinterpret_cast<T*>(lds_raw);
  const long long nx = a.op.nx;
  long long slab, tile;
  slab_tile((nx + MB - 1) / MB, slab, tile);
  const long long i = tile * MB + threadIdx.x;
  stage_halo<T, NT>(a.op, tile, x + slab * NT * nx, nullptr, nullptr, lx, nullptr);
  if (i >= nx) return;
  const long long off = slab * NT * nx + i;
  T mu[NT], ku[NT], mw, r[NT], xv[NT];
  row_mk_lds<T, NT>(a.op, lx, nullptr, i, mu, ku, mw);
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = f[off + l * nx];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc -= a.K[l * NT + k] * mu[k] + a.M[l * NT + k] * ku[k];
    r[l] = acc;
    xv[l] = lx[l * a.op.hmax + a.op.ldiag[i]];
  }
  if (a.op_kind == SP_JACOBI) {
    node_solve<T, NT>(a.K, a.M, a.op.diag[2 * i], a.op.diag[2 * i + 1], r);
#pragma unroll
    for (int l = 0; l < NT; ++l) r[l] = xv[l] + a.omega * r[l];
  }
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T o = r[l];
    if (a.upd == UPD_ADD) o = base[off + l * nx] + a.scale * o;
    else if (a.upd == UPD_SET) o = a.scale * o;
    out[off + l * nx] = o;
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_restrict_space(const T* __restrict__ rf, T* __restrict__ fc,
                                                            MeshXfer x, const T* __restrict__ w, long long slabs) {
  long long slab, tile;
  slab_tile((x.nxc + MB - 1) / MB, slab, tile);
  const long long I = tile * MB + threadIdx.x;
  if (slab >= slabs || I >= x.nxc) return;
  const T* src = rf + slab * NT * x.nxf;
  T acc[NT];
#pragma unroll
  for (int l = 0; l < NT; ++l) acc[l] = T(0);
  for (int e = 0; e < x.rw; ++e) {
    const long long c = x.rell[(long long)e * x.nxc + I];
    if (c < 0) break;
    const T wc = w[c];
#pragma unroll
    for (int l = 0; l < NT; ++l) acc[l] += wc * src[l * x.nxf + c];
  }
  T* dst = fc + slab * NT * x.nxc;
#pragma unroll
  for (int l = 0; l < NT; ++l) dst[l * x.nxc + I] = acc[l];
}

// (P^T v)_I for the coarse rows of this workgroup's tile from the tile's halo
// of v staged in LDS (one component at a time, the interpolation weight of the
// fine node folded in).  All threads of the workgroup must call it.
template <typename T>
__device__ inline T restrict_row_lds(const MeshXfer& x, const T* __restrict__ w, long long tile, long long I,
                                     const T* __restrict__ v, T* lx) {
  const int h0 = x.rhoff[tile], hn = x.rhoff[tile + 1] - h0;
  for (int j = threadIdx.x; j < hn; j += MB) {
    const long long c = x.rhcol[h0 + j];
    lx[j] = w[c] * v[c];
  }
  __syncthreads();
  T acc = T(0);
  if (I < x.nxc)
    for (int e = 0; e < x.rw; ++e) {
      const long long q = (long long)e * x.nxc + I;
      if (x.rell[q] < 0) break;
      acc += lx[x.rloc[q]];
    }
  __syncthreads();
  return acc;
}

template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_restrict_space_lds(const T* __restrict__ rf, T* __restrict__ fc,
                                                                MeshXfer x, const T* __restrict__ w,
                                                                long long slabs) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lx = reinterpret_cast<T*>(lds_raw);
  long long slab, tile;
  slab_tile((x.nxc + MB - 1) / MB, slab, tile);
  const long long I = tile * MB + threadIdx.x;
  const T* src = rf + slab * NT * x.nxf;
  T acc[NT];
#pragma unroll
  for (int l = 0; l < NT; ++l) acc[l] = restrict_row_lds<T>(x, w, tile, I, src + l * x.nxf, lx);
  if (I >= x.nxc) return;
  T* dst = fc + slab * NT * x.nxc;
#pragma unroll
  for (int l = 0; l < NT; ++l) dst[l * x.nxc + I] = acc[l];
}

template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_prolong_space(const T* __restrict__ ec, T* __restrict__ uf,
                                                           MeshXfer x, const T* __restrict__ w, long long slabs) {
  long long slab, tile;
  slab_tile((x.nxf + MB - 1) / MB, slab, tile);
  const long long i = tile * MB + threadIdx.x;
  if (slab >= slabs || i >= x.nxf) return;
  const int p0 = x.p[2 * i], p1 = x.p[2 * i + 1];
  const T wi = w[i];
  const T* src = ec + slab * NT * x.nxc;
  T* dst = uf + slab * NT * x.nxf + i;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T v = T(0);
    if (p0 >= 0) v += src[l * x.nxc + p0];
    if (p1 >= 0) v += src[l * x.nxc + p1];
    dst[l * x.nxf] += wi * v;
  }
}

// One workgroup per slab: the slab's right-hand side is staged in LDS, each
// thread forms rows of the dense product.
template <typename T>
__global__ __launch_bounds__(MB) void k_mesh_dense(const T* __restrict__ Ainv, int m, int trans,
                                                   const T* __restrict__ f, const T* base, T* out, int upd, T scale,
                                                   long long slabs) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* fs = reinterpret_cast<T*>(lds_raw);
  const long long slab = slab_index();
  if (slab >= slabs) return;
  const long long off = slab * m;
  for (int c = threadIdx.x; c < m; c += blockDim.x) fs[c] = f[off + c];
  __syncthreads();
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    T acc = T(0);
    if (trans)
      for (int c = 0; c < m; ++c) acc += Ainv[(long long)c * m + r] * fs[c];
    else
      for (int c = 0; c < m; ++c) acc += Ainv[(long long)r * m + c] * fs[c];
    T o = acc;
    if (upd == UPD_ADD) o = base[off + r] + scale * acc;
    else if (upd == UPD_SET) o = scale * acc;
    out[off + r] = o;
  }
}

// Fc[b][m][k][I] = sum_{s=0,1} sum_l R_s^T[l][k] (P_x^T rf[b][2m+s][l])_I
template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_restrict(const T* __restrict__ rf, T* __restrict__ Fc,
                                                      MeshTransferArgs<T> a) {
  const long long nxc = a.x.nxc, nxf = a.x.nxf;
  long long cs, tile;   // cs = b * Nc + m
  slab_tile((nxc + MB - 1) / MB, cs, tile);
  const long long I = tile * MB + threadIdx.x;
  if (cs >= (long long)a.batch * a.Nc || I >= nxc) return;
  const long long b = cs / a.Nc, m = cs % a.Nc;
  T out[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) out[k] = T(0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T* src = rf + ((b * 2 * a.Nc) + 2 * m + s) * NT * nxf;
    const T* blk = s ? a.R2T : a.R1T;
    T g[NT];
    if (a.full) {
#pragma unroll
      for (int l = 0; l < NT; ++l) g[l] = T(0);
      for (int e = 0; e < a.x.rw; ++e) {
        const long long c = a.x.rell[(long long)e * nxc + I];
        if (c < 0) break;
        const T wc = a.w[c];
#pragma unroll
        for (int l = 0; l < NT; ++l) g[l] += wc * src[l * nxf + c];
      }
    } else {
#pragma unroll
      for (int l = 0; l < NT; ++l) g[l] = src[l * nxf + I];
    }
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int l = 0; l < NT; ++l) out[k] += blk[l * NT + k] * g[l];
  }
  T* dst = Fc + cs * NT * nxc + I;
#pragma unroll
  for (int k = 0; k < NT; ++k) dst[k * nxc] = out[k];
}

// the same with full coarsening, the space part from LDS-staged halos
template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_restrict_lds(const T* __restrict__ rf, T* __restrict__ Fc,
                                                          MeshTransferArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lx = reinterpret_cast<T*>(lds_raw);
  const long long nxc = a.x.nxc, nxf = a.x.nxf;
  long long cs, tile;   // cs = b * Nc + m
  slab_tile((nxc + MB - 1) / MB, cs, tile);
  const long long I = tile * MB + threadIdx.x;
  const long long b = cs / a.Nc, m = cs % a.Nc;
  T out[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) out[k] = T(0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T* src = rf + ((b * 2 * a.Nc) + 2 * m + s) * NT * nxf;
    const T* blk = s ? a.R2T : a.R1T;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      const T g = restrict_row_lds<T>(a.x, a.w, tile, I, src + l * nxf, lx);
#pragma unroll
      for (int k = 0; k < NT; ++k) out[k] += blk[l * NT + k] * g;
    }
  }
  if (I >= nxc) return;
  T* dst = Fc + cs * NT * nxc + I;
#pragma unroll
  for (int k = 0; k < NT; ++k) dst[k * nxc] = out[k];
}

// uf[b][fs][l][i] += sum_k R_s^T[l][k] (P_x ec[b][m][k])_i,  fs = 2m + s
template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_prolong(const T* __restrict__ ec, T* __restrict__ uf,
                                                     MeshTransferArgs<T> a) {
  const long long nxc = a.x.nxc, nxf = a.x.nxf;
  long long fsl, tile;   // fsl = b * 2Nc + fs
  slab_tile((nxf + MB - 1) / MB, fsl, tile);
  const long long i = tile * MB + threadIdx.x;
  const long long Nf = 2LL * a.Nc;
  if (fsl >= (long long)a.batch * Nf || i >= nxf) return;
  const long long b = fsl / Nf, fs = fsl % Nf, m = fs >> 1;
  const T* blk = (fs & 1) ? a.R2T : a.R1T;
  const T* src = ec + (b * a.Nc + m) * NT * nxc;
  T e[NT];
  if (a.full) {
    const int p0 = a.x.p[2 * i], p1 = a.x.p[2 * i + 1];
    const T wi = a.w[i];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      T v = T(0);
      if (p0 >= 0) v += src[k * nxc + p0];
      if (p1 >= 0) v += src[k * nxc + p1];
      e[k] = wi * v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NT; ++k) e[k] = src[k * nxc + i];
  }
  T* dst = uf + fsl * NT * nxf + i;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) acc += blk[l * NT + k] * e[k];
    dst[l * nxf] += acc;
  }
}

// F[b][s][l] = ints_l M_h f[b][s] (+ ca_l M_h u0[b] on the first slab)
template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_rhs(const T* __restrict__ f, const T* __restrict__ u0,
                                                 T* __restrict__ F, MeshRhsArgs<T> a) {
  const long long sl = slab_index();   // b * N + s
  const long long i = (long long)blockIdx.x * MB + threadIdx.x;
  const long long nx = a.op.nx;
  if (sl >= (long long)a.batch * a.N || i >= nx) return;
  const long long b = sl / a.N, s = sl % a.N;
  const bool first = s == 0 && u0 != nullptr;
  const T* fs = f + sl * nx;
  const T* us = first ? u0 + b * nx : nullptr;
  T mf = T(0), mu = T(0);
  const int e1 = a.op.rowptr[i + 1];
  for (int e = a.op.rowptr[i]; e < e1; ++e) {
    const long long c = a.op.col[e];
    const T m = a.op.mv[e];
    mf += m * fs[c];
    if (first) mu += m * us[c];
  }
  T* dst = F + sl * NT * nx + i;
#pragma unroll
  for (int l = 0; l < NT; ++l) dst[l * nx] = a.ints[l] * mf + (first ? a.ca[l] * mu : T(0));
}

// grad_f[b][s] = M_h sum_l ints_l lam[b][s][l];  grad_u0[b] = M_h sum_l ca_l lam[b][0][l]
template <typename T, int NT>
__global__ __launch_bounds__(MB) void k_mesh_rhs_adjoint(const T* __restrict__ lam, T* gf, T* gu0,
                                                         MeshRhsArgs<T> a) {
  const long long sl = slab_index();
  const long long i = (long long)blockIdx.x * MB + threadIdx.x;
  const long long nx = a.op.nx;
  if (sl >= (long long)a.batch * a.N || i >= nx) return;
  const long long b = sl / a.N, s = sl % a.N;
  const T* ls = lam + sl * NT * nx;
  const bool first = s == 0 && gu0 != nullptr;
  T acc_f = T(0), acc_u = T(0);
  const int e1 = a.op.rowptr[i + 1];
  for (int e = a.op.rowptr[i]; e < e1; ++e) {
    const long long c = a.op.col[e];
    T vf = T(0), vu = T(0);
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      const T v = ls[l * nx + c];
      vf += a.ints[l] * v;
      vu += a.ca[l] * v;
    }
    acc_f += a.op.mv[e] * vf;
    if (first) acc_u += a.op.mv[e] * vu;
  }
  if (gf) gf[sl * nx + i] = acc_f;
  if (first) gu0[b * nx + i] = acc_u;
}

unsigned blocks_for(long long n) { return (unsigned)((n + MB - 1) / MB); }

}  // namespace

unsigned mesh_blocks_per_slab(long long nx) { return blocks_for(nx); }

#define NT_SWITCH(KERNEL_LAUNCH) \
  switch (nt) {                  \
    case 1: KERNEL_LAUNCH(1); break; \
    case 2: KERNEL_LAUNCH(2); break; \
    case 3: KERNEL_LAUNCH(3); break; \
    case 4: KERNEL_LAUNCH(4); break; \
    default: return hipErrorInvalidValue; \
  }

template <typename Tin, typename Tout>
hipError_t launch_mesh_residual(int nt, const Tin* u, const Tin* F, Tout* r, const MeshResidArgs<Tin>& a,
                                double* partial, hipStream_t s) {
  const long long blocks = (long long)blocks_for(a.op.nx) * a.batch * a.N;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  // runs of SR slabs per workgroup (fewer where the grid would drop below 2048 workgroups)
  const long long tiles = blocks_for(a.op.nx);
  int SR = 8;
  while (SR > 1 && tiles * a.batch * ((a.N + SR - 1) / SR) < 2048) SR /= 2;
  const size_t lds_run = (size_t)(nt + 2) * a.op.hmax * sizeof(Tin);
  if (SR > 1 && lds_run <= 65536) {
    const dim3 rgrid((unsigned)(tiles * a.batch * ((a.N + SR - 1) / SR)));
#define L_(NT) hipLaunchKernelGGL((k_mesh_residual_run<Tin, Tout, NT>), rgrid, dim3(MB), lds_run, s, u, F, r, a, \
                                  partial, SR)
    NT_SWITCH(L_)
#undef L_
    return hipGetLastError();
  }
  const size_t lds = (size_t)(nt + 1) * a.op.hmax * sizeof(Tin);
  if (lds <= 65536) {
#define L_(NT) hipLaunchKernelGGL((k_mesh_residual_lds<Tin, Tout, NT>), grid, dim3(MB), lds, s, u, F, r, a, partial)
    NT_SWITCH(L_)
#undef L_
    return hipGetLastError();
  }
#define L_(NT) hipLaunchKernelGGL((k_mesh_residual<Tin, Tout, NT>), grid, dim3(MB), 0, s, u, F, r, a, partial)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_smooth(int nt, const T* x, const T* f, const T* base, T* out, const MeshSmoothArgs<T>& a,
                              hipStream_t s) {
  const long long blocks = (long long)blocks_for(a.op.nx) * a.slabs;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const size_t lds = (size_t)nt * a.op.hmax * sizeof(T);
  if (!a.x_zero && lds <= 65536) {
#define L_(NT) hipLaunchKernelGGL((k_mesh_smooth_lds<T, NT>), grid, dim3(MB), lds, s, x, f, base, out, a)
    NT_SWITCH(L_)
#undef L_
    return hipGetLastError();
  }
#define L_(NT) hipLaunchKernelGGL((k_mesh_smooth<T, NT>), grid, dim3(MB), 0, s, x, f, base, out, a)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_restrict_space(int nt, const T* rf, T* fc, const MeshXfer& x, const T* w, long long slabs,
                                      hipStream_t s) {
  const long long blocks = (long long)blocks_for(x.nxc) * slabs;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const size_t lds = (size_t)x.rhmax * sizeof(T);
  if (x.rhoff != nullptr && lds <= 65536) {
#define L_(NT) hipLaunchKernelGGL((k_mesh_restrict_space_lds<T, NT>), grid, dim3(MB), lds, s, rf, fc, x, w, slabs)
    NT_SWITCH(L_)
#undef L_
    return hipGetLastError();
  }
#define L_(NT) hipLaunchKernelGGL((k_mesh_restrict_space<T, NT>), grid, dim3(MB), 0, s, rf, fc, x, w, slabs)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_prolong_space(int nt, const T* ec, T* uf, const MeshXfer& x, const T* w, long long slabs,
                                     hipStream_t s) {
  const long long blocks = (long long)blocks_for(x.nxf) * slabs;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
#define L_(NT) hipLaunchKernelGGL((k_mesh_prolong_space<T, NT>), grid, dim3(MB), 0, s, ec, uf, x, w, slabs)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_dense(const T* Ainv, int m, int trans, const T* f, const T* base, T* out, int upd, T scale,
                             long long slabs, hipStream_t s) {
  if (m < 1 || m > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_mesh_dense<T>), slab_grid(1, slabs), dim3(MB), (size_t)m * sizeof(T), s, Ainv, m, trans, f,
                     base, out, upd, scale, slabs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_restrict(int nt, const T* rf, T* Fc, const MeshTransferArgs<T>& a, hipStream_t s) {
  const long long blocks = (long long)blocks_for(a.x.nxc) * a.batch * a.Nc;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const size_t lds = (size_t)a.x.rhmax * sizeof(T);
  if (a.full && a.x.rhoff != nullptr && lds <= 65536) {
#define L_(NT) hipLaunchKernelGGL((k_mesh_restrict_lds<T, NT>), grid, dim3(MB), lds, s, rf, Fc, a)
    NT_SWITCH(L_)
#undef L_
    return hipGetLastError();
  }
#define L_(NT) hipLaunchKernelGGL((k_mesh_restrict<T, NT>), grid, dim3(MB), 0, s, rf, Fc, a)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_prolong(int nt, const T* ec, T* uf, const MeshTransferArgs<T>& a, hipStream_t s) {
  const long long blocks = (long long)blocks_for(a.x.nxf) * a.batch * 2 * a.Nc;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
#define L_(NT) hipLaunchKernelGGL((k_mesh_prolong<T, NT>), grid, dim3(MB), 0, s, ec, uf, a)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_rhs(int nt, const T* f, const T* u0, T* F, const MeshRhsArgs<T>& a, hipStream_t s) {
  const dim3 grid = slab_grid(blocks_for(a.op.nx), (long long)a.batch * a.N);
#define L_(NT) hipLaunchKernelGGL((k_mesh_rhs<T, NT>), grid, dim3(MB), 0, s, f, u0, F, a)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mesh_rhs_adjoint(int nt, const T* lam, T* gf, T* gu0, const MeshRhsArgs<T>& a, hipStream_t s) {
  const dim3 grid = slab_grid(blocks_for(a.op.nx), (long long)a.batch * a.N);
#define L_(NT) hipLaunchKernelGGL((k_mesh_rhs_adjoint<T, NT>), grid, dim3(MB), 0, s, lam, gf, gu0, a)
  NT_SWITCH(L_)
#undef L_
  return hipGetLastError();
}

#undef NT_SWITCH

template hipError_t launch_mesh_residual<double, double>(int, const double*, const double*, double*,
                                                         const MeshResidArgs<double>&, double*, hipStream_t);
template hipError_t launch_mesh_residual<float, float>(int, const float*, const float*, float*,
                                                       const MeshResidArgs<float>&, double*, hipStream_t);
template hipError_t launch_mesh_residual<double, float>(int, const double*, const double*, float*,
                                                        const MeshResidArgs<double>&, double*, hipStream_t);
#define INST(T)                                                                                                    \
  template hipError_t launch_mesh_smooth<T>(int, const T*, const T*, const T*, T*, const MeshSmoothArgs<T>&,      \
                                            hipStream_t);                                                          \
  template hipError_t launch_mesh_restrict_space<T>(int, const T*, T*, const MeshXfer&, const T*, long long,       \
                                                    hipStream_t);                                                  \
  template hipError_t launch_mesh_prolong_space<T>(int, const T*, T*, const MeshXfer&, const T*, long long,        \
                                                   hipStream_t);                                                   \
  template hipError_t launch_mesh_dense<T>(const T*, int, int, const T*, const T*, T*, int, T, long long,          \
                                           hipStream_t);                                                           \
  template hipError_t launch_mesh_restrict<T>(int, const T*, T*, const MeshTransferArgs<T>&, hipStream_t);         \
  template hipError_t launch_mesh_prolong<T>(int, const T*, T*, const MeshTransferArgs<T>&, hipStream_t);          \
  template hipError_t launch_mesh_rhs<T>(int, const T*, const T*, T*, const MeshRhsArgs<T>&, hipStream_t);         \
  template hipError_t launch_mesh_rhs_adjoint<T>(int, const T*, T*, T*, const MeshRhsArgs<T>&, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
