// Exact slab solves by fast diagonalisation on the matrix cores (gfx950).
//
// The slab block A = K_tau (x) M_h + M_tau (x) K_h (eq. chap4_generalLinearSystem)
// is diagonalised in space by the orthonormal DST-I, S[k][j] = c sin(pi k j/(n+1))
// (1-based, c = sqrt(2/(n+1)), S = S^T = S^{-1}), applied along every axis; per
// sine mode the N_t x N_t block G = (mu K_tau + nu M_tau)^{-1} remains
// (eq. chap4_smootherExact is D^{-1} applied exactly).
//
// Folding.  With m = n + 1 and h = m/2, S[k][m-j] = (-1)^(k+1) S[k][j], so a
// length-n transform splits into two half-size products:
//   odd  k = 2s+1 (s < h):   xhat = sum_{j<=h}   S[k][j] a_j,  a_j = x_j + x_{m-j}, a_h = x_h
//   even k = 2s+2 (s < h-1): xhat = sum_{j<h}    S[k][j] d_j,  d_j = x_j - x_{m-j}
// and the inverse y = S xhat is  P = S_odd^T xhat_odd, Q = S_even^T xhat_even,
// y_j = P_j + Q_j, y_{m-j} = P_j - Q_j, y_h = P_h.  This halves the matrix-core
// work.  Transformed data are kept in "spectral order" along every axis: the h
// odd modes first, then the h-1 even modes; the per-mode blocks G use the same
// order.
//
// Kernels (one workgroup = 4 waves = 64 columns of the contracted axis):
//   k_dst_pass   one forward or inverse folded transform along one axis
//                (x: rows contiguous; y/z: strided), epilogue store / u += omega y
//   k_dst_fused  forward transform along the slowest axis, the per-mode time
//                solve, inverse transform, in one pass over HBM: the tile holds
//                all N_t time components of 64 / N_t columns.
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

constexpr int LDT = TILE_COLS + 1;   // LDS row stride (spreads banks)

// Fragment table offset of (direction, half): [dir][half][kb][ib][lane].
template <int HB>
__device__ inline int frag_block(int dir, int half) {
  constexpr int HP = 16 * HB;
  return ((dir * 2 + half) * HB) * (HP / 4) * 64;
}

// Block-diagonal folded product on the tile (rows = contracted axis, 64
// columns).  INV = false: the tile holds a (rows < h) and d (row n-1-i holds
// d_{i+1}); INV = true: the tile holds spectral rows (odd s at row s, even s at
// row h + s).  Results: odd outputs -> acc of odd k-blocks, even -> even.
template <typename T, int HB, bool INV>
struct FoldMma {
  static constexpr int NB = 2 * HB;
  static constexpr int HP = 16 * HB;
  static constexpr int KPW = (NB >= 4) ? NB / 4 : NB;
  static constexpr int CPW = (NB >= 4) ? 4 : 1;
  typedef typename Mfma<T>::acc_t acc_t;

  static __device__ inline int kbt_of(int wave, int q) { return (NB >= 4) ? wave + 4 * q : q; }
  static __device__ inline int cb_of(int wave, int p) { return (NB >= 4) ? p : wave; }

  static __device__ inline void run(const T* tile, const T* __restrict__ Sfrag, int n, int h,
                                    acc_t (&acc)[KPW][CPW]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int brow = lane >> 4, bcol = lane & 15;
#pragma unroll
    for (int q = 0; q < KPW; ++q)
#pragma unroll
      for (int p = 0; p < CPW; ++p) acc[q][p] = acc_t{0, 0, 0, 0};
    const T* sf[KPW];
    bool even[KPW];
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
      const int kbt = kbt_of(wave, q);
      const int half = kbt / HB, kb = kbt % HB;
      even[q] = half == 1;
      sf[q] = Sfrag + frag_block<HB>(INV ? 1 : 0, half) + kb * (HP / 4) * 64 + lane;
    }
    const int ibmax = (h + 3) >> 2;
    T an[KPW];
#pragma unroll
    for (int q = 0; q < KPW; ++q) an[q] = sf[q][0];
    for (int ib = 0; ib < ibmax; ++ib) {
      T af[KPW];
#pragma unroll
      for (int q = 0; q < KPW; ++q) af[q] = an[q];
      if (ib + 1 < ibmax) {
#pragma unroll
        for (int q = 0; q < KPW; ++q) an[q] = sf[q][(ib + 1) * 64];
      }
      const int i = ib * 4 + brow;
      const int rowo = i;                          // odd operand row (valid if i < h)
      const int rowe = INV ? h + i : n - 1 - i;    // even operand row (valid if i < h - 1)
      T bo[CPW], be[CPW];
#pragma unroll
      for (int p = 0; p < CPW; ++p) {
        const int col = cb_of(wave, p) * 16 + bcol;
        bo[p] = (i < h) ? tile[rowo * LDT + col] : T(0);
        be[p] = (i < h - 1) ? tile[rowe * LDT + col] : T(0);
      }
#pragma unroll
      for (int q = 0; q < KPW; ++q)
#pragma unroll
        for (int p = 0; p < CPW; ++p) acc[q][p] = Mfma<T>::op(af[q], even[q] ? be[p] : bo[p], acc[q][p]);
    }
  }

  // acc -> tile: odd output r (< h) at row r, even output r (< h-1) at row h + r.
  static __device__ inline void to_tile(T* tile, int h, const acc_t (&acc)[KPW][CPW]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int brow = lane >> 4, bcol = lane & 15;
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
      const int kbt = kbt_of(wave, q);
      const int half = kbt / HB, kb = kbt % HB;
#pragma unroll
      for (int p = 0; p < CPW; ++p) {
        const int col = cb_of(wave, p) * 16 + bcol;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int r = kb * 16 + Mfma<T>::row(brow, jj);
          if (half == 0) {
            if (r < h) tile[r * LDT + col] = acc[q][p][jj];
          } else {
            if (r < h - 1) tile[(h + r) * LDT + col] = acc[q][p][jj];
          }
        }
      }
    }
  }
};

// In-place butterfly of physical rows: row i <- x_i + x_{n-1-i}, row n-1-i <- x_i - x_{n-1-i}.
template <typename T>
__device__ inline void butterfly(T* tile, int n, int h) {
  for (int e = threadIdx.x; e < (h - 1) * TILE_COLS; e += 256) {
    const int i = e >> 6, c = e & (TILE_COLS - 1);
    const T a = tile[i * LDT + c], b = tile[(n - 1 - i) * LDT + c];
    tile[i * LDT + c] = a + b;
    tile[(n - 1 - i) * LDT + c] = a - b;
  }
}

// Physical value of row p after an inverse product (P at rows < h, Q at h + i).
template <typename T>
__device__ inline T unfold(const T* tile, int n, int h, int p, int c) {
  if (p < h - 1) return tile[p * LDT + c] + tile[(h + p) * LDT + c];
  if (p == h - 1) return tile[p * LDT + c];
  const int i = n - 1 - p;
  return tile[i * LDT + c] - tile[(h + i) * LDT + c];
}

template <typename T>
__device__ inline T epilogue(int mode, T old, T v, T omega) {
  return mode == MODE_STORE ? v : (mode == MODE_ADD_SCALED ? old + omega * v : omega * v);
}

// ------------------------------------------------------------ single pass
template <typename T, int HB, bool XAXIS, bool INV>
__global__ __launch_bounds__(256) void k_dst_pass(const T* __restrict__ in, T* __restrict__ out,
                                                  const T* __restrict__ Sfrag, int n, long long inner,
                                                  long long ncols, T omega, int mode) {
  typedef FoldMma<T, HB, INV> MM;
  constexpr int NP = 32 * HB;                  // >= n rows
  constexpr int EPT = NP * TILE_COLS / 256;
  __shared__ T tile[NP * LDT];
  const int tid = threadIdx.x;
  const long long col0 = xcd_linear(blockIdx.x, gridDim.x) * TILE_COLS;
  const int ncol_here = (int)((ncols - col0) < TILE_COLS ? (ncols - col0) : TILE_COLS);
  const float inv_n = 1.0f / (float)n;
  const int h = (n + 1) >> 1;

  // ---- stage: tile[i][c] = X[i][col0 + c]
  if (XAXIS) {
    const T* src = in + col0 * n;
    const int total = ncol_here * n;
    T v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + 256 * j;
      v[j] = (e < total) ? src[e] : T(0);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + 256 * j;
      if (e < TILE_COLS * n) {
        const int c = div_small(e, n, inv_n);
        tile[(e - c * n) * LDT + c] = v[j];
      }
    }
  } else {
    const int c = tid & (TILE_COLS - 1);
    const bool valid = c < ncol_here;
    const long long col = col0 + c;
    const long long o = valid ? col / inner : 0;
    const long long cc = valid ? col - o * inner : 0;
    const T* src = in + o * (long long)n * inner + cc;
    const int i0 = tid >> 6;
    T v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = i0 + 4 * j;
      v[j] = (valid && i < n) ? src[(long long)i * inner] : T(0);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = i0 + 4 * j;
      if (i < n) tile[i * LDT + c] = v[j];
    }
  }
  __syncthreads();
  if (!INV) {
    butterfly(tile, n, h);
    __syncthreads();
  }
  typename MM::acc_t acc[MM::KPW][MM::CPW];
  MM::run(tile, Sfrag, n, h, acc);
  __syncthreads();
  MM::to_tile(tile, h, acc);
  __syncthreads();

  // ---- store (forward: spectral rows as they are; inverse: unfold)
  if (XAXIS) {
    T* dst = out + col0 * n;
    const int total = ncol_here * n;
    T o[EPT];
    if (mode == MODE_ADD_SCALED) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = tid + 256 * j;
        o[j] = (e < total) ? dst[e] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + 256 * j;
      if (e < total) {
        const int c = div_small(e, n, inv_n);
        const int p = e - c * n;
        const T v = INV ? unfold(tile, n, h, p, c) : tile[p * LDT + c];
        dst[e] = epilogue(mode, o[j], v, omega);
      }
    }
  } else {
    const int c = tid & (TILE_COLS - 1);
    if (c < ncol_here) {
      const long long col = col0 + c;
      const long long o = col / inner;
      const long long cc = col - o * inner;
      T* dstb = out + o * (long long)n * inner + cc;
      const int i0 = tid >> 6;
      T ov[EPT];
      if (mode == MODE_ADD_SCALED) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int i = i0 + 4 * j;
          ov[j] = (i < n) ? dstb[(long long)i * inner] : T(0);
        }
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int p = i0 + 4 * j;
        if (p < n) {
          const T v = INV ? unfold(tile, n, h, p, c) : tile[p * LDT + c];
          dstb[(long long)p * inner] = epilogue(mode, ov[j], v, omega);
        }
      }
    }
  }
}

// ------------------------------------------------ fused last-axis solve
// Column c of the tile is (time component l = c / CT, position cc = c % CT) of
// the linear index lin = blockIdx.x * CT + cc over (slab o, other axes pos):
// element i sits at o*NT*n*inner + l*n*inner + i*inner + pos.  The sine mode
// of spectral row s at position pos is j = pos + inner * s.
template <typename T, int HB, int NT>
__global__ __launch_bounds__(256) void k_dst_fused(const T* in, T* out,
                                                   const T* __restrict__ Sfrag,
                                                   const T* __restrict__ G, int n, long long inner,
                                                   long long outer, int transpose, T omega,
                                                   int mode) {
  typedef FoldMma<T, HB, false> MF;
  typedef FoldMma<T, HB, true> MI;
  constexpr int NP = 32 * HB;
  constexpr int CT = TILE_COLS / NT;
  constexpr int EPT = NP * TILE_COLS / 256;
  __shared__ T tile[NP * LDT];
  __shared__ long long pos_s[TILE_COLS];
  __shared__ long long base_s[TILE_COLS];
  const int tid = threadIdx.x;
  const long long total = outer * inner;
  const long long lin0 = xcd_linear(blockIdx.x, gridDim.x) * CT;
  const int h = (n + 1) >> 1;
  if (tid < TILE_COLS) {
    const int l = tid / CT, cc = tid - (tid / CT) * CT;
    const long long lin = lin0 + cc;
    if (l < NT && lin < total) {
      const long long o = lin / inner;
      const long long pos = lin - o * inner;
      pos_s[tid] = pos;
      base_s[tid] = o * NT * (long long)n * inner + (long long)l * n * inner + pos;
    } else {
      pos_s[tid] = -1;
      base_s[tid] = -1;
    }
  }
  __syncthreads();
  const int c = tid & (TILE_COLS - 1);
  const long long base = base_s[c];
  const int i0 = tid >> 6;
  {
    T v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = i0 + 4 * j;
      v[j] = (base >= 0 && i < n) ? in[base + (long long)i * inner] : T(0);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int i = i0 + 4 * j;
      if (i < n) tile[i * LDT + c] = v[j];
    }
  }
  __syncthreads();
  butterfly(tile, n, h);
  __syncthreads();
  {
    typename MF::acc_t acc[MF::KPW][MF::CPW];
    MF::run(tile, Sfrag, n, h, acc);
    __syncthreads();
    MF::to_tile(tile, h, acc);
  }
  __syncthreads();
  // ---- per-mode N_t x N_t solve on the spectral tile
  for (int e = tid; e < n * CT; e += 256) {
    const int s = e / CT, cc = e - (e / CT) * CT;
    const long long pos = pos_s[cc];
    if (pos < 0) continue;
    const T* g = G + (pos + inner * s) * (NT * NT);
    T v[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) v[k] = tile[s * LDT + k * CT + cc];
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T a = T(0);
#pragma unroll
      for (int k = 0; k < NT; ++k) a += (transpose ? g[k * NT + l] : g[l * NT + k]) * v[k];
      tile[s * LDT + l * CT + cc] = a;
    }
  }
  __syncthreads();
  {
    typename MI::acc_t acc[MI::KPW][MI::CPW];
    MI::run(tile, Sfrag, n, h, acc);
    __syncthreads();
    MI::to_tile(tile, h, acc);
  }
  __syncthreads();
  if (base >= 0) {
    T ov[EPT];
    if (mode == MODE_ADD_SCALED) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int i = i0 + 4 * j;
        ov[j] = (i < n) ? out[base + (long long)i * inner] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int p = i0 + 4 * j;
      if (p < n) out[base + (long long)p * inner] = epilogue(mode, ov[j], unfold(tile, n, h, p, c), omega);
    }
  }
}

// ------------------------------------------------ register-resident kernels
// Each wave owns 16 columns (lin = 16 * global_wave + lane % 16) and all rows of
// the contracted axis; lane (g = lane / 16, r = lane % 16) holds the B-operand
// rows g, g+4, ... and the accumulator rows Mfma<T>::row(g, j) of every
// 16-row block.  For FP64 the accumulator layout (row g + 4j) equals the
// B-operand layout of the next product (row 4 ib + g with ib = 4 kb + j), so a
// forward product, the per-mode solve and the inverse product chain in
// registers; FP32 (row 4g + j) re-lays out each block through LDS.  Element i
// of column lin sits at o*n*inner*NT + l*n*inner + i*inner + pos with
// (o, pos) = divmod(lin, inner).

// Forward operands of one column: a (odd half) and d (even half) per 4-row chunk.
template <typename T, int HB>
__device__ inline void load_folded(const T* __restrict__ src, bool valid, long long inner, int n, int h,
                                   int g, T (&a)[4 * HB], T (&d)[4 * HB]) {
#pragma unroll
  for (int ib = 0; ib < 4 * HB; ++ib) {
    const int i = 4 * ib + g;
    const T x1 = (valid && i < h) ? src[(long long)i * inner] : T(0);
    const T x2 = (valid && i < h - 1) ? src[(long long)(n - 1 - i) * inner] : T(0);
    a[ib] = x1 + x2;
    d[ib] = x1 - x2;
  }
}

// acc[kbt] += S_half(dir) * operand over ib < ceil(h/4); kbt < HB odd, >= HB even.
// The S fragments of chunk ib+1 are loaded while chunk ib multiplies; a
// scheduling barrier per chunk stops the compiler from hoisting every fragment
// load of the unrolled loop (which would exhaust the register file).
template <typename T, int HB, int DIR, typename OpFn>
__device__ inline void folded_mma_core(const T* __restrict__ Sfrag, int h, int lane, OpFn op,
                                       typename Mfma<T>::acc_t (&acc)[2 * HB]) {
#pragma unroll
  for (int k = 0; k < 2 * HB; ++k) acc[k] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  const int ibmax = (h + 3) >> 2;
  const T* s0 = Sfrag + frag_block<HB>(DIR, 0) + lane;
  const T* s1 = Sfrag + frag_block<HB>(DIR, 1) + lane;
  T no[HB], ne[HB];
#pragma unroll
  for (int kb = 0; kb < HB; ++kb) {
    no[kb] = s0[(kb * 4 * HB) * 64];
    ne[kb] = s1[(kb * 4 * HB) * 64];
  }
#pragma unroll
  for (int ib = 0; ib < 4 * HB; ++ib) {
    if (ib < ibmax) {
      T ao[HB], ae[HB];
#pragma unroll
      for (int kb = 0; kb < HB; ++kb) {
        ao[kb] = no[kb];
        ae[kb] = ne[kb];
      }
      if (ib + 1 < ibmax) {
#pragma unroll
        for (int kb = 0; kb < HB; ++kb) {
          no[kb] = s0[(kb * 4 * HB + ib + 1) * 64];
          ne[kb] = s1[(kb * 4 * HB + ib + 1) * 64];
        }
      }
      const T bo = op(0, ib), be = op(1, ib);
#pragma unroll
      for (int kb = 0; kb < HB; ++kb) {
        acc[kb] = Mfma<T>::op(ao[kb], bo, acc[kb]);
        acc[HB + kb] = Mfma<T>::op(ae[kb], be, acc[HB + kb]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <typename T, int HB, int DIR>
__device__ inline void folded_mma(const T* __restrict__ Sfrag, int h, int lane, const T (&bo)[4 * HB],
                                  const T (&be)[4 * HB], typename Mfma<T>::acc_t (&acc)[2 * HB]) {
  folded_mma_core<T, HB, DIR>(Sfrag, h, lane, [&](int half, int ib) { return half ? be[ib] : bo[ib]; }, acc);
}

// Inverse product whose B operands are held in B-operand order: chunk
// ib = 4 kb + j of the odd (even) half is element j of src[kb] (src[HB + kb]).
template <typename T, int HB>
__device__ inline void folded_mma_chain(const T* __restrict__ Sfrag, int h, int lane,
                                        const typename Mfma<T>::acc_t (&src)[2 * HB],
                                        typename Mfma<T>::acc_t (&acc)[2 * HB]) {
  folded_mma_core<T, HB, 1>(Sfrag, h, lane,
                            [&](int half, int ib) { return src[half * HB + (ib >> 2)][ib & 3]; }, acc);
}

// Physical outputs of an inverse product: row i gets P_i + Q_i, row n-1-i gets
// P_i - Q_i (i < h-1), row h-1 gets P_{h-1}; apply the epilogue in place.
template <typename T, int HB>
__device__ inline void store_unfolded(T* __restrict__ dst, bool valid, long long inner, int n, int h, int g,
                                      const typename Mfma<T>::acc_t (&acc)[2 * HB], int mode, T omega) {
  if (!valid) return;
#pragma unroll
  for (int kb = 0; kb < HB; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = kb * 16 + Mfma<T>::row(g, j);
      const T P = acc[kb][j], Q = acc[HB + kb][j];
      if (i < h - 1) {
        T* p0 = dst + (long long)i * inner;
        T* p1 = dst + (long long)(n - 1 - i) * inner;
        const T o0 = (mode == MODE_ADD_SCALED) ? *p0 : T(0);
        const T o1 = (mode == MODE_ADD_SCALED) ? *p1 : T(0);
        *p0 = epilogue(mode, o0, P + Q, omega);
        *p1 = epilogue(mode, o1, P - Q, omega);
      } else if (i == h - 1) {
        T* p0 = dst + (long long)i * inner;
        const T o0 = (mode == MODE_ADD_SCALED) ? *p0 : T(0);
        *p0 = epilogue(mode, o0, P, omega);
      }
    }
}

// GPW column groups per wave (loads of every group issued before the first
// product; scheduling barriers keep the groups' phases apart).  Launched with
// GPW = 1: with two groups the compiler's register demand drops occupancy to
// one wave per SIMD.  UNIT: unit stride along the contracted axis (x passes),
// which lets the loads use immediate offsets from one base address.
template <typename T, int HB, bool INV, int GPW, bool UNIT>
__global__ __launch_bounds__(256) void k_pass_reg(const T* __restrict__ in, T* __restrict__ out,
                                                  const T* __restrict__ Sfrag, int n, long long inner_rt,
                                                  long long ncols, T omega, int mode) {
  typedef typename Mfma<T>::acc_t acc_t;
  const long long inner = UNIT ? 1 : inner_rt;     // UNIT: contiguous columns (x axis)
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const long long wv = xcd_linear(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int h = (n + 1) >> 1;
  bool valid[GPW];
  long long base[GPW];
  T bo[GPW][4 * HB], be[GPW][4 * HB];
#pragma unroll
  for (int q = 0; q < GPW; ++q) {
    const long long lin = (wv * GPW + q) * 16 + r;
    valid[q] = lin < ncols;
    const long long o = valid[q] ? lin / inner : 0;
    const long long pos = valid[q] ? lin - o * inner : 0;
    base[q] = o * (long long)n * inner + pos;
#pragma unroll
    for (int ib = 0; ib < 4 * HB; ++ib) {
      const int i = 4 * ib + g;
      if (!INV) {          // raw pair loads; folded right before the product
        bo[q][ib] = (valid[q] && i < h) ? in[base[q] + (long long)i * inner] : T(0);
        be[q][ib] = (valid[q] && i < h - 1) ? in[base[q] + (long long)(n - 1 - i) * inner] : T(0);
      } else {
        bo[q][ib] = (valid[q] && i < h) ? in[base[q] + (long long)i * inner] : T(0);
        be[q][ib] = (valid[q] && i < h - 1) ? in[base[q] + (long long)(h + i) * inner] : T(0);
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < GPW; ++q) {
    if (!INV) {
#pragma unroll
      for (int ib = 0; ib < 4 * HB; ++ib) {
        const T x1 = bo[q][ib], x2 = be[q][ib];
        bo[q][ib] = x1 + x2;
        be[q][ib] = x1 - x2;
      }
    }
    acc_t acc[2 * HB];
    const T* Sf = Sfrag;
    asm volatile("" : "+s"(Sf));     // no reuse of one group's fragment loads by the next
    folded_mma<T, HB, INV ? 1 : 0>(Sf, h, lane, bo[q], be[q], acc);
    if (!INV) {
      if (valid[q]) {
#pragma unroll
        for (int kb = 0; kb < HB; ++kb)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int i = kb * 16 + Mfma<T>::row(g, j);
            if (i < h) out[base[q] + (long long)i * inner] = acc[kb][j];
            if (i < h - 1) out[base[q] + (long long)(h + i) * inner] = acc[HB + kb][j];
          }
      }
    } else {
      store_unfolded<T, HB>(out + base[q], valid[q], inner, n, h, g, acc, mode, omega);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Fused slowest-axis solve, all N_t time components in one lane (FP64 only:
// relies on the chained layout).
template <int HB, int NT>
__global__ __launch_bounds__(256) void k_fused_reg(const double* in, double* out,
                                                   const double* __restrict__ Sfrag,
                                                   const double* __restrict__ G, int n, long long inner,
                                                   long long outer, int transpose, double omega, int mode) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const long long lin = (xcd_linear(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)) * 16 + r;
  const bool valid = lin < outer * inner;
  const long long o = valid ? lin / inner : 0;
  const long long pos = valid ? lin - o * inner : 0;
  const long long cstride = (long long)n * inner;           // between time components
  const long long base = o * NT * cstride + pos;
  const int h = (n + 1) >> 1;
  v4d spec[NT][2 * HB];
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    double a[4 * HB], d[4 * HB];
    load_folded<double, HB>(in + base + l * cstride, valid, inner, n, h, g, a, d);
    folded_mma<double, HB, 0>(Sfrag, h, lane, a, d, spec[l]);
  }
  if (valid) {
#pragma unroll
    for (int k = 0; k < 2 * HB; ++k) {
      const int half = k / HB, kb = k % HB;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = kb * 16 + g + 4 * j;
        const bool ok = half == 0 ? rr < h : rr < h - 1;
        if (!ok) continue;
        const long long sidx = half == 0 ? rr : h + rr;
        const double* gm = G + (pos + inner * sidx) * (NT * NT);
        double v[NT], w[NT];
#pragma unroll
        for (int l = 0; l < NT; ++l) v[l] = spec[l][k][j];
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < NT; ++m) t += (transpose ? gm[m * NT + l] : gm[l * NT + m]) * v[m];
          w[l] = t;
        }
#pragma unroll
        for (int l = 0; l < NT; ++l) spec[l][k][j] = w[l];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    v4d acc[2 * HB];
    folded_mma_chain<double, HB>(Sfrag, h, lane, spec[l], acc);
    store_unfolded<double, HB>(out + base + l * cstride, valid, inner, n, h, g, acc, mode, omega);
  }
}

// Fused slowest-axis solve with the N_t time components of one 16-column
// group spread over N_t waves of the workgroup (wave w: column group w / NT,
// component w % NT).  Each wave keeps only its own component's spectral
// values; for the per-mode time solve all waves write their blocks to LDS,
// meet at one barrier and read the other components' values.  FP32 additionally re-lays out each solved block
// from accumulator order (row 4g + j) into B-operand order (row 4j + g) through
// a per-wave LDS slot before the inverse product.
template <typename T, int HB, int NT>
__global__ __launch_bounds__(256) void k_fused_pair(const T* in, T* out, const T* __restrict__ Sfrag,
                                                    const T* __restrict__ G, int n, long long inner,
                                                    long long outer, int transpose, T omega, int mode) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr bool CHAIN = sizeof(T) == 8;     // accumulator order == B-operand order
  constexpr int CG = NT >= 3 ? 1 : 4 / NT;   // column groups per workgroup
  __shared__ T xch[2 * HB][CG * NT * 64 * 4];
  __shared__ T rel[CHAIN ? 1 : CG * NT * 256];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int cg = wave / NT, l = wave - (wave / NT) * NT;
  const long long lin = (xcd_linear(blockIdx.x, gridDim.x) * CG + cg) * 16 + r;
  const bool valid = lin < outer * inner;
  const long long o = valid ? lin / inner : 0;
  const long long pos = valid ? lin - o * inner : 0;
  const long long cstride = (long long)n * inner;
  const long long base = o * NT * cstride + (long long)l * cstride + pos;
  const int h = (n + 1) >> 1;
  acc_t spec[2 * HB];
  {
    T a[4 * HB], d[4 * HB];
    load_folded<T, HB>(in + base, valid, inner, n, h, g, a, d);
    folded_mma<T, HB, 0>(Sfrag, h, lane, a, d, spec);
  }
  // every 16-row block of every component to LDS, one barrier, then the
  // per-mode solves read the other components' values without further waits
#pragma unroll
  for (int k = 0; k < 2 * HB; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) xch[k][((cg * NT + l) * 64 + lane) * 4 + j] = spec[k][j];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2 * HB; ++k) {
    const T* slot = xch[k];
    const int half = k / HB, kb = k % HB;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = kb * 16 + Mfma<T>::row(g, j);
      const bool ok = valid && (half == 0 ? rr < h : rr < h - 1);
      T acc = T(0);
      if (ok) {
        const long long sidx = half == 0 ? rr : h + rr;
        const T* gm = G + (pos + inner * sidx) * (NT * NT);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const T v = slot[((cg * NT + m) * 64 + lane) * 4 + j];
          acc += (transpose ? gm[m * NT + l] : gm[l * NT + m]) * v;
        }
      }
      spec[k][j] = acc;
    }
    if (!CHAIN) {
      // accumulator row 4g + j of column r -> B-operand element (chunk 4k + j', row g' = g)
      T* rs = rel + (cg * NT + l) * 256;
#pragma unroll
      for (int j = 0; j < 4; ++j) rs[(4 * g + j) * 16 + r] = spec[k][j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) spec[k][j] = rs[(4 * j + g) * 16 + r];
      __syncthreads();
    }
  }
  acc_t acc[2 * HB];
  folded_mma_chain<T, HB>(Sfrag, h, lane, spec, acc);
  store_unfolded<T, HB>(out + base, valid, inner, n, h, g, acc, mode, omega);
}

}  // namespace

// Register-resident kernels: FP64 up to 4 half blocks (n <= 127), FP32 up to 8
// (n <= 255); the LDS-staged kernels cover the rest and the TRANSFORM_LDS choice.
template <typename T>
bool reg_path(int impl, int hb) {
  if (impl == TRANSFORM_LDS) return false;
  return sizeof(T) == 8 ? hb <= 4 : hb <= 8;
}

template <typename T>
hipError_t launch_pass_reg(int hb, bool inverse, const T* in, T* out, const T* Sfrag, int n,
                           long long inner, long long ncols, T omega, int mode, hipStream_t s) {
  const int gpw = (sizeof(T) == 8 && hb == 4 && inner == 1) ? 2 : 1;
  const unsigned grid = (unsigned)((ncols + 64 * gpw - 1) / (64 * gpw));
#define REG_PASS_GU(HB, G, U)                                                                     \
  if (hb == HB && gpw == G && (inner == 1) == U) {                                                \
    if (inverse)                                                                                  \
      hipLaunchKernelGGL((k_pass_reg<T, HB, true, G, U>), dim3(grid), dim3(256), 0, s, in, out, Sfrag, n, inner, \
                         ncols, omega, mode);                                                     \
    else                                                                                          \
      hipLaunchKernelGGL((k_pass_reg<T, HB, false, G, U>), dim3(grid), dim3(256), 0, s, in, out, Sfrag, n, inner, \
                         ncols, omega, mode);                                                     \
    return hipGetLastError();                                                                     \
  }
#define REG_PASS_G(HB, G) REG_PASS_GU(HB, G, true) REG_PASS_GU(HB, G, false)
#define REG_PASS(HB) REG_PASS_G(HB, 1)
  if (sizeof(T) == 8) {
    REG_PASS_GU(4, 2, true)
  }

  REG_PASS(1) REG_PASS(2) REG_PASS(4)
  if (sizeof(T) == 4) {
    REG_PASS(8)
  }
#undef REG_PASS
#undef REG_PASS_G
#undef REG_PASS_GU
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_fused_pair(int hb, int nt, const T* in, T* out, const T* Sfrag, const T* G, int n,
                             long long inner, long long outer, int transpose, T omega, int mode, hipStream_t s) {
  const int cg = nt >= 3 ? 1 : 4 / nt;
  const unsigned grid = (unsigned)((outer * inner + 16 * cg - 1) / (16 * cg));
  const dim3 block(64 * nt * cg);
#define PAIR(HB, NT)                                                                                 \
  if (hb == HB && nt == NT) {                                                                        \
    hipLaunchKernelGGL((k_fused_pair<T, HB, NT>), dim3(grid), block, 0, s, in, out, Sfrag, G, n, inner, outer, \
                       transpose, omega, mode);                                                      \
    return hipGetLastError();                                                                        \
  }
  PAIR(1, 1) PAIR(1, 2) PAIR(1, 3) PAIR(1, 4)
  PAIR(2, 1) PAIR(2, 2) PAIR(2, 3) PAIR(2, 4)
  PAIR(4, 1) PAIR(4, 2) PAIR(4, 3) PAIR(4, 4)
  if (sizeof(T) == 4) {
    PAIR(8, 1) PAIR(8, 2) PAIR(8, 3) PAIR(8, 4)
  }
#undef PAIR
  return hipErrorInvalidValue;
}

// Fused solve: TRANSFORM_REG keeps all N_t components in one lane when that
// state is small (FP64, hb * N_t <= 8); otherwise the wave-per-component kernel.
template <typename T>
hipError_t launch_fused_any(int impl, int hb, int nt, const T* in, T* out, const T* Sfrag, const T* G, int n,
                            long long inner, long long outer, int transpose, T omega, int mode, hipStream_t s) {
  if (sizeof(T) == 8 && impl == TRANSFORM_REG && hb * nt <= 8) {
    const unsigned grid = (unsigned)((outer * inner + 63) / 64);
    const double* ind = (const double*)in;
    double* outd = (double*)out;
    const double* Sd = (const double*)Sfrag;
    const double* Gd = (const double*)G;
    const double om = (double)omega;
#define REG_FUSED(HB, NT)                                                                          \
    if (hb == HB && nt == NT) {                                                                    \
      hipLaunchKernelGGL((k_fused_reg<HB, NT>), dim3(grid), dim3(256), 0, s, ind, outd, Sd, Gd, n, inner, \
                         outer, transpose, om, mode);                                              \
      return hipGetLastError();                                                                    \
    }
    REG_FUSED(1, 1) REG_FUSED(1, 2) REG_FUSED(1, 3) REG_FUSED(1, 4)
    REG_FUSED(2, 1) REG_FUSED(2, 2) REG_FUSED(2, 3) REG_FUSED(2, 4)
    REG_FUSED(4, 1) REG_FUSED(4, 2)
#undef REG_FUSED
  }
  return launch_fused_pair<T>(hb, nt, in, out, Sfrag, G, n, inner, outer, transpose, omega, mode, s);
}

int transform_half_blocks(int n) {
  const int h = (n + 1) / 2;
  int hb = 1;
  while (16 * hb < h) hb *= 2;
  return hb;
}

template <typename T>
hipError_t launch_dst_pass(int impl, int hb, bool xaxis, bool inverse, const T* in, T* out, const T* Sfrag,
                           int n, long long inner, long long ncols, T omega, int mode,
                           hipStream_t s) {
  if (reg_path<T>(impl, hb)) return launch_pass_reg<T>(hb, inverse, in, out, Sfrag, n, inner, ncols, omega, mode, s);
  const unsigned grid = (unsigned)((ncols + TILE_COLS - 1) / TILE_COLS);
#define PASS_CASE(HB)                                                                          \
  if (hb == HB) {                                                                              \
    if (xaxis && !inverse)                                                                     \
      hipLaunchKernelGGL((k_dst_pass<T, HB, true, false>), dim3(grid), dim3(256), 0, s, in, out, \
                         Sfrag, n, inner, ncols, omega, mode);                                 \
    else if (xaxis && inverse)                                                                 \
      hipLaunchKernelGGL((k_dst_pass<T, HB, true, true>), dim3(grid), dim3(256), 0, s, in, out,  \
                         Sfrag, n, inner, ncols, omega, mode);                                 \
    else if (!inverse)                                                                         \
      hipLaunchKernelGGL((k_dst_pass<T, HB, false, false>), dim3(grid), dim3(256), 0, s, in,     \
                         out, Sfrag, n, inner, ncols, omega, mode);                            \
    else                                                                                       \
      hipLaunchKernelGGL((k_dst_pass<T, HB, false, true>), dim3(grid), dim3(256), 0, s, in, out, \
                         Sfrag, n, inner, ncols, omega, mode);                                 \
    return hipGetLastError();                                                                  \
  }
  PASS_CASE(1) PASS_CASE(2) PASS_CASE(4) PASS_CASE(8)
#undef PASS_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dst_fused(int impl, int hb, int nt, const T* in, T* out, const T* Sfrag, const T* G, int n,
                            long long inner, long long outer, int transpose, T omega, int mode,
                            hipStream_t s) {
  if (reg_path<T>(impl, hb)) return launch_fused_any<T>(impl, hb, nt, in, out, Sfrag, G, n, inner, outer, transpose, omega, mode, s);
  const long long ct = TILE_COLS / nt;
  const unsigned grid = (unsigned)((outer * inner + ct - 1) / ct);
#define FUSED_CASE(HB, NT)                                                                      \
  if (hb == HB && nt == NT) {                                                                   \
    hipLaunchKernelGGL((k_dst_fused<T, HB, NT>), dim3(grid), dim3(256), 0, s, in, out, Sfrag, G, \
                       n, inner, outer, transpose, omega, mode);                                \
    return hipGetLastError();                                                                   \
  }
  FUSED_CASE(1, 1) FUSED_CASE(1, 2) FUSED_CASE(1, 3) FUSED_CASE(1, 4)
  FUSED_CASE(2, 1) FUSED_CASE(2, 2) FUSED_CASE(2, 3) FUSED_CASE(2, 4)
  FUSED_CASE(4, 1) FUSED_CASE(4, 2) FUSED_CASE(4, 3) FUSED_CASE(4, 4)
  FUSED_CASE(8, 1) FUSED_CASE(8, 2) FUSED_CASE(8, 3) FUSED_CASE(8, 4)
#undef FUSED_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_dst_pass<double>(int, int, bool, bool, const double*, double*, const double*,
                                            int, long long, long long, double, int, hipStream_t);
template hipError_t launch_dst_pass<float>(int, int, bool, bool, const float*, float*, const float*, int,
                                           long long, long long, float, int, hipStream_t);
template hipError_t launch_dst_fused<double>(int, int, int, const double*, double*, const double*,
                                             const double*, int, long long, long long, int, double,
                                             int, hipStream_t);
template hipError_t launch_dst_fused<float>(int, int, int, const float*, float*, const float*, const float*,
                                            int, long long, long long, int, float, int, hipStream_t);

}  // namespace stmg
