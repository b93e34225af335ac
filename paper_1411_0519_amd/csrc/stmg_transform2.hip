// Twice-folded sine transforms on the matrix cores: FP64 for n = 63, 127, FP32
// for n = 63, 127, 255, and FP32 data with bf16 operands (BF = true:
// v_mfma_f32_16x16x16_bf16, FP32 accumulation) for the same n.
//
// The first fold pairs x_i with x_{n-1-i} (odd modes see a_i = x_i + x_{n-1-i},
// even modes d_i = x_i - x_{n-1-i}).  Each half has a second mirror symmetry:
// with h = (n+1)/2, the odd-mode rows s and h-1-s of O[s][i] = sin(pi (2s+1)(i+1)
// / (n+1)) agree on even i and differ in sign on odd i; the even-mode rows s and
// h-2-s of E[s][i] = sin(pi (2s+2)(i+1)/(n+1)) likewise (the middle row
// s* = h/2 - 1 vanishes on odd i).  So every half is two (h/2) x (h/2) products
// on the even- and odd-indexed inputs, P and Q, and the outputs are P + Q (row s)
// and P - Q (the mirrored row); the inverse transforms first form the sums and
// differences of mirrored spectral rows.  This halves the matrix-core work of
// the once-folded kernels.  Spectral order in memory is unchanged (odd mode s at
// row s, even mode s at row h + s), so the per-mode blocks G are shared.
//
// Fragment table [dir][mat][kb][ib][lane], mat = 0: O on even i, 1: O on odd i,
// 2: E on even i, 3: E on odd i; dir 0 holds A[s][p] (forward), dir 1 A[p][s]
// (inverse), blocks of 16 rows and chunks of 4 along the contraction.
//
// Register order: chunk ib of a product's contraction holds index 4 ib + g in
// lane group g, and accumulator element j of row block kb holds output row
// 16 kb + g + 4 j.  That is the f64 instruction's own accumulator layout; the
// f32 instruction holds row 4 g + j of its A operand there, so the FP32 table
// stores A row g + 4 j at operand row 4 g + j.  Either way accumulator element
// j of block kb is, in every lane, the operand of chunk 4 kb + j of the next
// product (forward product, per-mode solve and inverse product chain in
// registers), and the four lane groups of a line touch neighbouring elements.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

// contraction index of lane group g in chunk ib; output row of element j of block kb
__device__ inline int cidx(int ib, int g) { return 4 * ib + g; }
__device__ inline int orow(int kb, int g, int j) { return 16 * kb + g + 4 * j; }

// acc[mat][kb] = sum over chunks ib of A(dir, mat, kb, ib) * B(mat, ib); HB2 = h/32
// row blocks per product, 2 HB2 * 4 = h/2 contraction indices.  B(mat, ib) is
// the lane's operand for (mat, chunk ib).
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// BF16 products: chunk c of 16 contraction indices holds values 4c + q (q < 4)
// of a lane, packed; the table is [dir][mat][kb][c][lane] of four bf16.
template <int HB2, int DIR, typename OpFn>
__device__ inline void mma4_bf16(const v4s* __restrict__ F, int lane, OpFn op, v4f (&acc)[4][HB2]) {
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb) acc[m][kb] = v4f{0.f, 0.f, 0.f, 0.f};
  const v4s* f = F + (size_t)DIR * 4 * HB2 * HB2 * 64 + lane;
#pragma unroll
  for (int c = 0; c < HB2; ++c) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v4s b;
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = bf16_bits(op(m, 4 * c + q));
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
        acc[m][kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f[((m * HB2 + kb) * HB2 + c) * 64], b, acc[m][kb], 0,
                                                               0, 0);
    }
  }
}

template <typename T, int HB2, int DIR, bool BF = false, typename OpFn>
__device__ inline void mma4(const T* __restrict__ Sfrag, int lane, OpFn op,
                            typename Mfma<T>::acc_t (&acc)[4][HB2]) {
  if constexpr (BF) {
    mma4_bf16<HB2, DIR>(reinterpret_cast<const v4s*>(Sfrag), lane, op, acc);
    return;
  }
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NC = 4 * HB2;   // chunks of 4 along the contraction (h/2 / 4)
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb) acc[m][kb] = acc_t{0, 0, 0, 0};
  const T* s = Sfrag + (size_t)DIR * 4 * HB2 * NC * 64 + lane;
  T nf[4][HB2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb) nf[m][kb] = s[((m * HB2 + kb) * NC) * 64];
#pragma unroll
  for (int ib = 0; ib < NC; ++ib) {
    T af[4][HB2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb) af[m][kb] = nf[m][kb];
    if (ib + 1 < NC) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int kb = 0; kb < HB2; ++kb) nf[m][kb] = s[((m * HB2 + kb) * NC + ib + 1) * 64];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const T b = op(m, ib);
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb) acc[m][kb] = Mfma<T>::op(af[m][kb], b, acc[m][kb]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// acc[kb] = sum over chunks ib of A(dir, mat, kb, ib) * B(ib): one of the four
// products of mma4.
template <typename T, int HB2, int DIR, typename OpFn>
__device__ inline void mma1(const T* __restrict__ Sfrag, int lane, int mat, OpFn op,
                            typename Mfma<T>::acc_t (&acc)[HB2]) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NC = 4 * HB2;
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb) acc[kb] = acc_t{0, 0, 0, 0};
  const T* s = Sfrag + (size_t)DIR * 4 * HB2 * NC * 64 + (size_t)mat * HB2 * NC * 64 + lane;
#pragma unroll
  for (int ib = 0; ib < NC; ++ib) {
    const T b = op(ib);
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb) acc[kb] = Mfma<T>::op(s[(kb * NC + ib) * 64], b, acc[kb]);
  }
}

// Forward operands of chunk ib for contraction index p = cidx(ib, g): the
// physical values x_{2p}, x_{2p+1} and their partners x_{n-1-2p}, x_{n-2-2p}.
// Returns a_{2p}, a_{2p+1}, d_{2p}, d_{2p+1} (d_{h-1} = 0, a_{h-1} = x_{h-1}).
template <typename T, int HB2, typename I = long long>
__device__ inline void load_twice_folded(const T* __restrict__ src, bool valid, I inner, int n, int g,
                                         T (&op)[4][4 * HB2]) {
  const int h = (n + 1) >> 1;
#pragma unroll
  for (int ib = 0; ib < 4 * HB2; ++ib) {
    const int p = cidx(ib, g);
    const int i0 = 2 * p, i1 = 2 * p + 1;
    T x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    if (valid) {
      x0 = src[(I)i0 * inner];
      y0 = src[(I)(n - 1 - i0) * inner];
      x1 = src[(I)i1 * inner];
      if (i1 < h - 1) y1 = src[(I)(n - 1 - i1) * inner];
    }
    op[0][ib] = x0 + y0;
    op[1][ib] = x1 + y1;
    op[2][ib] = x0 - y0;
    op[3][ib] = (i1 < h - 1) ? x1 - y1 : T(0);
  }
}

template <typename T>
__device__ inline T epi(int mode, T old, T v, T omega) {
  if (mode == MODE_ADD_SCALED) return old + omega * v;
  if (mode == MODE_SET_SCALED) return omega * v;
  return v;
}

// Physical outputs of an inverse product: row p of the four accumulators holds
// P_{2p}, P_{2p+1} (odd modes) and Q_{2p}, Q_{2p+1} (even modes); x_i = P_i + Q_i
// and x_{n-1-i} = P_i - Q_i (i < h-1), x_{h-1} = P_{h-1}.  The four positions of
// element j of block kb are put_pos(); with MODE_ADD_SCALED the old values are
// loaded by load_old() before the products (PRE), so that those loads overlap
// them, or at the store.
__device__ inline void put_pos(int n, int kb, int g, int j, int (&pos)[4], bool& tail) {
  const int h = (n + 1) >> 1;
  const int p = orow(kb, g, j);
  const int i0 = 2 * p, i1 = 2 * p + 1;
  tail = i1 >= h - 1;
  pos[0] = i0;
  pos[1] = n - 1 - i0;
  pos[2] = i1;
  pos[3] = n - 1 - i1;
}

template <typename T, int HB2>
__device__ inline void load_old(const T* __restrict__ dst, bool valid, long long inner, int n, int g,
                                T (&old)[HB2][4][4]) {
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int pos[4];
      bool tail;
      put_pos(n, kb, g, j, pos, tail);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        old[kb][j][c] = (valid && (c < 3 || !tail)) ? dst[(long long)pos[c] * inner] : T(0);
    }
}

template <typename T, int HB2>
__device__ inline void zero_old(T (&old)[HB2][4][4]) {
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) old[kb][j][c] = T(0);
}

template <typename T, int HB2, bool PRE, typename I = long long>
__device__ inline void store_twice_unfolded(T* __restrict__ dst, bool valid, I inner, int n, int g,
                                            const typename Mfma<T>::acc_t (&acc)[4][HB2], int mode, T omega,
                                            const T (&old)[HB2][4][4]) {
  if (!valid) return;
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int pos[4];
      bool tail;
      put_pos(n, kb, g, j, pos, tail);
      const T P0 = acc[0][kb][j], P1 = acc[1][kb][j], Q0 = acc[2][kb][j], Q1 = acc[3][kb][j];
      T v[4] = {P0 + Q0, P0 - Q0, tail ? P1 : P1 + Q1, P1 - Q1};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c == 3 && tail) continue;
        T* q = dst + (I)pos[c] * inner;
        const T o = PRE ? old[kb][j][c] : (mode == MODE_ADD_SCALED ? *q : T(0));
        *q = epi<T>(mode, o, v[c], omega);
      }
    }
}

// Inverse operands from the four spectral values of row s: u = y_o[s] +
// y_o[h-1-s], v = y_o[s] - y_o[h-1-s], ue = y_e[s] + y_e[h-2-s] (y_e[s*] on the
// middle row), ve = y_e[s] - y_e[h-2-s] (0 on the middle row).
template <typename T>
__device__ inline void inverse_operands(T o, T om, T e, T em, bool middle, T& u, T& v, T& ue, T& ve) {
  u = o + om;
  v = o - om;
  ue = middle ? e : e + em;
  ve = middle ? T(0) : e - em;
}

// Row l of the per-mode time block G (of G^T with transpose) from the
// eigenvalues: mode s along the pass axis, (P, Q) = (prod m, sum kappa prod m)
// over the other axes of the lane's position; G = D^{-1} with
// D = mu K_tau + nu M_tau, mu = P m_s, nu = Q m_s + P kappa_s.  N_t = 1, 2 in
// closed form; N_t = 3, 4 by elimination without pivoting on D^T g = e_l
// (D g = e_l for a row of G^T): D's symmetric part is positive definite
// (mu, nu > 0), so every pivot is positive.
template <typename T>
__device__ inline T recip(T d) {
  if constexpr (sizeof(T) == 8) {
    // hardware reciprocal refined by two Newton steps r <- r + r (1 - d r): about one ulp, far
    // cheaper than the IEEE division sequence
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    return r;
  } else {
    // hardware reciprocal (1 ulp) refined by one Newton step
    float r = __builtin_amdgcn_rcpf(d);
    r = __builtin_fmaf(r, __builtin_fmaf(-d, r, 1.0f), r);
    return r;
  }
}

template <typename T, int NT>
__device__ inline void mode_row(const ModeEig<T>& me, const T* eig, int n, T P, T Q, int s, int l, int transpose,
                                T (&g)[NT]) {
  const T ms = eig[s], ks = eig[n + s];
  const T mu = P * ms, nu = Q * ms + P * ks;
  if constexpr (NT == 1) {
    g[0] = T(1) / (mu * me.K[0] + nu * me.M[0]);
  } else if constexpr (NT == 2) {
    const T d00 = mu * me.K[0] + nu * me.M[0], d01 = mu * me.K[1] + nu * me.M[1];
    const T d10 = mu * me.K[2] + nu * me.M[2], d11 = mu * me.K[3] + nu * me.M[3];
    const T inv = recip<T>(d00 * d11 - d01 * d10);   // det > 0: the block is positive definite
    // G = inv [[d11, -d01], [-d10, d00]]
    const T g00 = d11 * inv, g01 = -d01 * inv, g10 = -d10 * inv, g11 = d00 * inv;
    if (l == 0) {
      g[0] = g00;
      g[1] = transpose ? g10 : g01;
    } else {
      g[0] = transpose ? g01 : g10;
      g[1] = g11;
    }
  } else {
    T A[NT][NT], b[NT], piv[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int ij = transpose ? i * NT + j : j * NT + i;
        A[i][j] = mu * me.K[ij] + nu * me.M[ij];
      }
      b[i] = i == l ? T(1) : T(0);
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      piv[k] = recip<T>(A[k][k]);
#pragma unroll
      for (int i = k + 1; i < NT; ++i) {
        const T f = A[i][k] * piv[k];
#pragma unroll
        for (int j = k + 1; j < NT; ++j) A[i][j] -= f * A[k][j];
        b[i] -= f * b[k];
      }
    }
#pragma unroll
    for (int k = NT - 1; k >= 0; --k) {
      T x = b[k];
#pragma unroll
      for (int j = k + 1; j < NT; ++j) x -= A[k][j] * g[j];
      g[k] = x * piv[k];
    }
  }
}

// The whole block of mode s for N_t <= 2 (the rows mode_row gives one at a
// time): G[l][m] = (D^{-1})[l][m], or (D^{-T})[l][m] when transposed.
template <typename T, int NT>
__device__ inline void mode_block(const ModeEig<T>& me, const T* eig, int n, T P, T Q, int s, int transpose,
                                  T (&G)[NT][NT]) {
  static_assert(NT <= 2, "closed form for N_t <= 2");
  const T ms = eig[s], ks = eig[n + s];
  const T mu = P * ms, nu = Q * ms + P * ks;
  if constexpr (NT == 1) {
    G[0][0] = T(1) / (mu * me.K[0] + nu * me.M[0]);
  } else {
    const T d00 = mu * me.K[0] + nu * me.M[0], d01 = mu * me.K[1] + nu * me.M[1];
    const T d10 = mu * me.K[2] + nu * me.M[2], d11 = mu * me.K[3] + nu * me.M[3];
    const T inv = recip<T>(d00 * d11 - d01 * d10);
    G[0][0] = d11 * inv;
    G[1][1] = d00 * inv;
    G[0][1] = (transpose ? -d10 : -d01) * inv;
    G[1][0] = (transpose ? -d01 : -d10) * inv;
  }
}

// (P, Q) of a position `pos` of the axes before the pass axis (spectral order).
template <typename T>
__device__ inline void mode_pq(const ModeEig<T>& me, int n, long long inner, long long pos, T& P, T& Q) {
  if (inner == 1) {
    P = T(1);
    Q = T(0);
  } else if (inner == n) {
    P = me.eig[pos];
    Q = me.eig[n + pos];
  } else {
    const int xs = (int)(pos % n), ys = (int)(pos / n);
    const T mx = me.eig[xs], kx = me.eig[n + xs], my = me.eig[ys], ky = me.eig[n + ys];
    P = mx * my;
    Q = kx * my + mx * ky;
  }
}

// One pass along an axis: a wave transforms the group of 16 lines gi.
template <typename T, int HB2, bool INV, bool UNIT, bool BF>
__device__ __forceinline__ void pass2_group(const T* __restrict__ in, T* __restrict__ out,
                                            const T* __restrict__ Sf, int n, long long inner, long long ncols,
                                            T omega, int mode, long long gi) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int h = (n + 1) >> 1;
  const long long lin = gi * 16 + r;
  const bool valid = lin < ncols;
  const long long o = valid ? lin / inner : 0;
  const long long pos = valid ? lin - o * inner : 0;
  const long long base = o * (long long)n * inner + pos;
  T op[4][4 * HB2];
  if (!INV) {
    load_twice_folded<T, HB2>(in + base, valid, inner, n, g, op);
  } else {
    // spectral rows s = cidx(ib, g) (< h/2) and their mirrors
#pragma unroll
    for (int ib = 0; ib < 4 * HB2; ++ib) {
      const int s = cidx(ib, g);
      const bool middle = s == h / 2 - 1;
      T yo = 0, yom = 0, ye = 0, yem = 0;
      if (valid) {
        yo = in[base + (long long)s * inner];
        yom = in[base + (long long)(h - 1 - s) * inner];
        ye = in[base + (long long)(h + s) * inner];
        if (!middle) yem = in[base + (long long)(h + h - 2 - s) * inner];
      }
      inverse_operands<T>(yo, yom, ye, yem, middle, op[0][ib], op[1][ib], op[2][ib], op[3][ib]);
    }
  }
  T old[HB2][4][4];
  if (INV && mode == MODE_ADD_SCALED) load_old<T, HB2>(out + base, valid, inner, n, g, old);
  else zero_old<T, HB2>(old);
  acc_t acc[4][HB2];
  mma4<T, HB2, INV ? 1 : 0, BF>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
  if (!INV) {
    if (valid) {
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = orow(kb, g, j);
          const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
          out[base + (long long)s * inner] = P + Q;
          out[base + (long long)(h - 1 - s) * inner] = P - Q;
          out[base + (long long)(h + s) * inner] = Pe + Qe;
          if (s != h / 2 - 1) out[base + (long long)(h + h - 2 - s) * inner] = Pe - Qe;
        }
    }
  } else {
    store_twice_unfolded<T, HB2, true>(out + base, valid, inner, n, g, acc, mode, omega, old);
  }
}

// Orders one wave's LDS writes before its later reads by other lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Offset in the x-mode-major layout [slab][s][line in slab] of spectral
// value s of the group's line r, given the slab and in-slab index of the
// group's first line and lps lines per slab.
__device__ inline long long xmode_offset(long long slab0, long long ll0, int r, int s, int n, long long lps) {
  long long ll = ll0 + r, sl = slab0;
  if (ll >= lps) {
    ll -= lps;
    ++sl;
  }
  return (sl * n + s) * lps + ll;
}

// Unit-stride pass (along x) through LDS: the 16 lines of group gi are one
// contiguous run of 16 n values, loaded with consecutive lanes on consecutive
// values (eight loads in flight per lane), transformed from the wave's LDS
// buffer, written back there and stored the same way; the update reads the
// old iterate at the store.  Same arithmetic as the strided path.  buf: 16 n
// values of this wave.  lps > 0: the spectral side (output of the forward
// pass, input of the inverse) is in the x-mode-major layout
// [slab][s][line in slab] with lps lines per slab, moved with the 16 lines
// of one s on 16 consecutive lanes.
template <typename T, int HB2, bool INV, bool BF>
__device__ __forceinline__ void pass2_group_staged(const T* __restrict__ in, T* __restrict__ out,
                                                   const T* __restrict__ Sf, int n, long long ncols, T omega,
                                                   int mode, long long gi, T* buf, long long lps) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int h = (n + 1) >> 1;
  const long long first = gi * 16;
  if (first >= ncols) return;
  const int lines = ncols - first < 16 ? (int)(ncols - first) : 16;
  const int cnt = lines * n;
  const long long off = first * (long long)n;
  long long slab0 = 0, ll0 = 0;
  if (lps > 0) {
    slab0 = first / lps;
    ll0 = first - slab0 * lps;
  }
  if (INV && lps > 0) {
#pragma unroll 1
    for (int e0 = 0; e0 < cnt; e0 += 64 * 8) {
      T v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 64 * i + lane;
        const int s = e / lines, rr = e - s * lines;
        v[i] = e < cnt ? in[xmode_offset(slab0, ll0, rr, s, n, lps)] : T(0);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 64 * i + lane;
        const int s = e / lines, rr = e - s * lines;
        if (e < cnt) buf[rr * n + s] = v[i];
      }
    }
  } else {
#pragma unroll 1
    for (int e0 = 0; e0 < cnt; e0 += 64 * 8) {
      T v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 64 * i + lane;
        v[i] = e < cnt ? in[off + e] : T(0);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 64 * i + lane;
        if (e < cnt) buf[e] = v[i];
      }
    }
  }
  wave_lds_sync();
  const bool valid = r < lines;
  T* lp = buf + (valid ? r : 0) * n;
  T op[4][4 * HB2];
  if (!INV) {
    load_twice_folded<T, HB2, int>(lp, valid, 1, n, g, op);
  } else {
#pragma unroll
    for (int ib = 0; ib < 4 * HB2; ++ib) {
      const int s = cidx(ib, g);
      const bool middle = s == h / 2 - 1;
      T yo = 0, yom = 0, ye = 0, yem = 0;
      if (valid) {
        yo = lp[s];
        yom = lp[h - 1 - s];
        ye = lp[h + s];
        if (!middle) yem = lp[h + h - 2 - s];
      }
      inverse_operands<T>(yo, yom, ye, yem, middle, op[0][ib], op[1][ib], op[2][ib], op[3][ib]);
    }
  }
  acc_t acc[4][HB2];
  mma4<T, HB2, INV ? 1 : 0, BF>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
  wave_lds_sync();
  if (!INV) {
    if (valid) {
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = orow(kb, g, j);
          const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
          lp[s] = P + Q;
          lp[h - 1 - s] = P - Q;
          lp[h + s] = Pe + Qe;
          if (s != h / 2 - 1) lp[h + h - 2 - s] = Pe - Qe;
        }
    }
  } else {
    T none[HB2][4][4];
    zero_old<T, HB2>(none);
    store_twice_unfolded<T, HB2, false, int>(lp, valid, 1, n, g, acc, MODE_STORE, T(1), none);
  }
  wave_lds_sync();
  if (!INV && lps > 0) {
#pragma unroll 1
    for (int e0 = 0; e0 < cnt; e0 += 64 * 8) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + 64 * i + lane;
        const int s = e / lines, rr = e - s * lines;
        if (e < cnt) out[xmode_offset(slab0, ll0, rr, s, n, lps)] = buf[rr * n + s];
      }
    }
    return;
  }
#pragma unroll 1
  for (int e0 = 0; e0 < cnt; e0 += 64 * 8) {
    T o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + 64 * i + lane;
      o[i] = (e < cnt && mode == MODE_ADD_SCALED) ? out[off + e] : T(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + 64 * i + lane;
      if (e < cnt) out[off + e] = epi<T>(mode, o[i], buf[e], omega);
    }
  }
}

// A pass along an axis, a wave per group of 16 lines, workgroups of
// blockDim.x / 64 waves.  PERSIST: the grid is smaller than the group count
// (persistent workgroups); each wave takes a contiguous range of groups and
// the waves of one XCD cover neighbouring ranges.
template <typename T, int HB2, bool INV, bool UNIT, bool BF, bool PERSIST>
__global__ __launch_bounds__(256) void k_pass_reg2(const T* __restrict__ in, T* __restrict__ out,
                                                   const T* __restrict__ Sfrag, int n_arg, long long inner_rt,
                                                   long long ncols, T omega, int mode, long long lps) {
  constexpr int n = 64 * HB2 - 1;   // fixed by the twice folding (the host checks n_arg)
  (void)n_arg;
  const long long inner = UNIT ? 1 : inner_rt;
  const int wpb = blockDim.x >> 6;
  const long long wv = xcd_linear(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* buf = reinterpret_cast<T*>(lds_raw) + (threadIdx.x >> 6) * 16 * n;   // unit stride: 16 n values per wave
  if constexpr (!PERSIST) {
    if constexpr (UNIT) pass2_group_staged<T, HB2, INV, BF>(in, out, Sfrag, n, ncols, omega, mode, wv, buf, lps);
    else pass2_group<T, HB2, INV, UNIT, BF>(in, out, Sfrag, n, inner, ncols, omega, mode, wv);
  } else {
    const long long nwaves = (long long)gridDim.x * wpb;
    const long long ngroups = (ncols + 15) >> 4;
    const long long per = (ngroups + nwaves - 1) / nwaves;
    const long long gbeg = wv * per;
    const long long gend = gbeg + per < ngroups ? gbeg + per : ngroups;
#pragma unroll 1
    for (long long gi = gbeg; gi < gend; ++gi) {
      // an opaque copy of the table pointer: its loads stay inside the loop
      const T* Sf = Sfrag;
      asm volatile("" : "+s"(Sf));
      if constexpr (UNIT) pass2_group_staged<T, HB2, INV, BF>(in, out, Sf, n, ncols, omega, mode, gi, buf, lps);
      else pass2_group<T, HB2, INV, UNIT, BF>(in, out, Sf, n, inner, ncols, omega, mode, gi);
    }
  }
}

// Slowest axis: forward transform, per-mode N_t x N_t solve, inverse transform,
// one wave per time component (as the once-folded k_fused_pair), the
// components exchanged through LDS for the solve.  A workgroup of NT * CG
// waves takes CG groups of 16 columns per tile; with a grid smaller than the
// tile count (persistent workgroups) each workgroup takes a contiguous range
// of tiles.
template <typename T, int HB2, int NT, int CG, bool BF>
__device__ __forceinline__ void fused2_tile(const T* in, T* out, const T* __restrict__ Sf, const T* __restrict__ G,
                                            int n, long long inner, long long ncol, int transpose, T omega,
                                            int mode, const ModeEig<T>& me, const T* eig,
                                            T (&xch)[4 * HB2][CG * NT * 64 * 4], long long t) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int cg = wave / NT, l = wave - (wave / NT) * NT;
  const long long cstride = (long long)n * inner;
  const int h = (n + 1) >> 1;
  const long long lin = (t * CG + cg) * 16 + r;
  const bool valid = lin < ncol;
  const long long o = valid ? lin / inner : 0;
  const long long pos = valid ? lin - o * inner : 0;
  const long long base = o * NT * cstride + (long long)l * cstride + pos;
  acc_t acc[4][HB2];
  {
    T op[4][4 * HB2];
    load_twice_folded<T, HB2>(in + base, valid, inner, n, g, op);
    mma4<T, HB2, 0, BF>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
  }
  // spectral values (o, om, e, em) of every row to LDS, one barrier
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
      const int slot = ((cg * NT + l) * 64 + lane) * 4 + j;
      xch[0 * HB2 + kb][slot] = P + Q;
      xch[1 * HB2 + kb][slot] = P - Q;
      xch[2 * HB2 + kb][slot] = Pe + Qe;
      xch[3 * HB2 + kb][slot] = Pe - Qe;
    }
  __syncthreads();
  T P0 = T(0), Q0 = T(0);
  if (me.eig != nullptr && valid) mode_pq<T>(me, n, inner, pos, P0, Q0);
  // per-mode solve of this wave's component, then the inverse operands
  T op[4][4 * HB2];
#pragma unroll
  for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = orow(kb, g, j);
      const bool middle = s == h / 2 - 1;
      const int mode_idx[4] = {s, h - 1 - s, h + s, h + (middle ? s : h - 2 - s)};
      T y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T a = T(0);
        if (valid) {
          bool done = false;
          if (me.eig != nullptr) {
            T gr[NT];
            mode_row<T, NT>(me, eig, n, P0, Q0, mode_idx[q], l, transpose, gr);
#pragma unroll
            for (int m = 0; m < NT; ++m) a += gr[m] * xch[q * HB2 + kb][((cg * NT + m) * 64 + lane) * 4 + j];
            done = true;
          }
          if (!done) {
            const T* gm = G + (pos + inner * (long long)mode_idx[q]) * (NT * NT);
#pragma unroll
            for (int m = 0; m < NT; ++m) {
              const T v = xch[q * HB2 + kb][((cg * NT + m) * 64 + lane) * 4 + j];
              a += (transpose ? gm[m * NT + l] : gm[l * NT + m]) * v;
            }
          }
        }
        y[q] = a;
      }
      // chunk 4 kb + j, contraction row g: the accumulator layout is the operand layout
      const int ib = 4 * kb + j;
      inverse_operands<T>(y[0], y[1], y[2], y[3], middle, op[0][ib], op[1][ib], op[2][ib], op[3][ib]);
    }
  acc_t out_acc[4][HB2];
  mma4<T, HB2, 1, BF>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, out_acc);
  T none[HB2][4][4];
  zero_old<T, HB2>(none);
  store_twice_unfolded<T, HB2, false>(out + base, valid, inner, n, g, out_acc, mode, omega, none);
}

template <typename T, int HB2, int NT, int CG, bool BF, bool PERSIST>
__global__ __launch_bounds__(256) void k_fused_pair2(const T* in, T* out, const T* __restrict__ Sfrag,
                                                     const T* __restrict__ G, int n_arg, long long inner,
                                                     long long outer, int transpose, T omega, int mode,
                                                     ModeEig<T> me) {
  constexpr int n = 64 * HB2 - 1;   // fixed by the twice folding (the host checks n_arg)
  (void)n_arg;
  __shared__ T xch[4 * HB2][CG * NT * 64 * 4];
  // the 1-D eigenvalues of the per-mode blocks, read by every mode: staged in
  // LDS before the first barrier (n < 2h = 64 HB2)
  __shared__ T eig[128 * HB2];
  if (me.eig != nullptr)
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) eig[i] = me.eig[i];
  const long long ncol = outer * inner;
  if constexpr (!PERSIST) {
    fused2_tile<T, HB2, NT, CG, BF>(in, out, Sfrag, G, n, inner, ncol, transpose, omega, mode, me, eig, xch,
                                    xcd_linear(blockIdx.x, gridDim.x));
  } else {
    const long long tiles = (ncol + 16 * CG - 1) / (16 * CG);
    const long long per = (tiles + gridDim.x - 1) / gridDim.x;
    const long long tbeg = xcd_linear(blockIdx.x, gridDim.x) * per;
    const long long tend = tbeg + per < tiles ? tbeg + per : tiles;
#pragma unroll 1
    for (long long t = tbeg; t < tend; ++t) {
      const T* Sf = Sfrag;
      asm volatile("" : "+s"(Sf));
      fused2_tile<T, HB2, NT, CG, BF>(in, out, Sf, G, n, inner, ncol, transpose, omega, mode, me, eig, xch, t);
      __syncthreads();   // the next tile rewrites the exchange buffer
    }
  }
}

// 2-D slab-resident block solve: one workgroup of WG threads (512) per slab holds
// the slab's N_t x n x n values in LDS and runs the forward x pass, the fused
// y pass with the per-mode solve, and the inverse x pass there, each wave
// taking groups of 16 lines (x passes) or 16 columns with all N_t components
// (y pass), so no component exchange is needed; barriers separate the
// passes.  The slab is read once and written once:
// dst = epi(mode, dst, D^{-1} src).  src and dst may alias (a workgroup reads
// its whole slab before it writes).  Dynamic LDS: N_t n^2 elements.
//
// X3: the same solve on the 2-D blocks of a 3-D level after the forward x
// pass, in the x-mode-major layout [slab][kx][l][z][y] (kx = spectral x index):
// block b = (slab, kx) is one N_t x n x n problem in (z, y) whose per-mode
// blocks also carry kx's eigenvalues (formed from the 1-D eigenvalues in
// `me`; the 2-D form reads the table G).  `slabs` counts blocks.
template <typename T, int HB2, int NT, bool X3, int WG = 512>
__global__ __launch_bounds__(WG) void k_slab_solve2(const T* src, T* dst, const T* __restrict__ Sfrag,
                                                     const T* __restrict__ G, int n_arg, long long slabs,
                                                     int transpose, T omega, int mode, ModeEig<T> me) {
  typedef typename Mfma<T>::acc_t acc_t;
  // the twice-folded transform fixes n = 64 HB2 - 1 (the host checks n_arg): with n a
  // compile-time constant every LDS address of the passes is a base plus an immediate offset
  constexpr int n = 64 * HB2 - 1;
  (void)n_arg;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* R = reinterpret_cast<T*>(lds_raw);
  const long long slab = X3 ? xcd_linear(slab_index(), (long long)gridDim.y * gridDim.z) : slab_index();
  if (slab >= slabs) return;
  // X3: the 1-D eigenvalues (2n) after the plane, read by every mode of the z pass,
  // then the twice-folded fragment tables of both directions (2048 HB2^2 values),
  // read by every product of the four passes
  T* E = R + NT * n * n;
  T* Sl = E + 2 * n;
  constexpr int NFRAG = 2048 * HB2 * HB2;
  if constexpr (X3) {
    for (int i = threadIdx.x; i < 2 * n; i += WG) E[i] = me.eig[i];
    for (int i = threadIdx.x; i < NFRAG; i += WG) Sl[i] = Sfrag[i];
  }
  // the fragment table of the passes: LDS (X3), else global memory through an
  // opaque copy of the pointer (its loads are not hoisted out of the loops and kept live)
  auto frag = [&]() -> const T* {
    if constexpr (X3) {
      return Sl;
    } else {
      const T* Sf = Sfrag;
      asm volatile("" : "+s"(Sf));
      return Sf;
    }
  };
  // x-mode of a 3-D block: its (m, kappa)
  T mxk = T(0), kxk = T(0);
  if constexpr (X3) {
    const int kx = (int)(slab % n);
    mxk = me.eig[kx];
    kxk = me.eig[n + kx];
  }
  const int nn = n * n;
  const int total = NT * nn;
  constexpr int NW = WG / 64;   // waves per workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int h = (n + 1) >> 1;
  const T* sp = src + slab * (long long)total;
  T* dp = dst + slab * (long long)total;
  // ---- slab to LDS: LF loads in flight per thread (the whole 63^2 x 2 plane of a 3-D block at once: nothing
  // else is live yet, so the registers are free)
  constexpr int LF = X3 ? 32 : 8;
#pragma unroll 1
  for (int e0 = threadIdx.x; e0 < total; e0 += WG * LF) {
    T v[LF];
#pragma unroll
    for (int i = 0; i < LF; ++i) {
      const int e = e0 + WG * i;
      v[i] = e < total ? sp[e] : T(0);
    }
#pragma unroll
    for (int i = 0; i < LF; ++i) {
      const int e = e0 + WG * i;
      if (e < total) R[e] = v[i];
    }
  }
  __syncthreads();
  // ---- forward x pass: line = component * n + y, in place in spectral order
  const int xgroups = (NT * n + 15) >> 4;
#pragma unroll 1
  for (int gi = wave; gi < xgroups; gi += NW) {
    // an opaque copy of the table pointer: its loads are not hoisted out of the loop and kept live
    const T* Sf = frag();
    const int line = gi * 16 + r;
    const bool valid = line < NT * n;
    T* lp = R + (valid ? line : 0) * n;
    T op[4][4 * HB2];
    load_twice_folded<T, HB2, int>(lp, valid, 1, n, g, op);
    acc_t acc[4][HB2];
    mma4<T, HB2, 0>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
    if (valid) {
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = orow(kb, g, j);
          const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
          lp[s] = P + Q;
          lp[h - 1 - s] = P - Q;
          lp[h + s] = Pe + Qe;
          if (s != h / 2 - 1) lp[h + h - 2 - s] = Pe - Qe;
        }
    }
  }
  __syncthreads();
  const int ygroups = (n + 15) >> 4;
  if constexpr (X3) {
    // ---- y pass, one wave per (column group, component), where there are
    // fewer column groups than waves (n = 63 on eight waves): forward pass of
    // the component with the spectral column written back in place; barrier;
    // every wave reads all components of its columns' modes and forms its
    // component's solved values; barrier; inverse pass and store.  The
    // all-components-per-wave form below would leave waves idle there.
    const int tasks = ygroups < NW ? ygroups * NT : 0;
    const int iters = (tasks + NW - 1) / NW;
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
      const T* Sf = frag();
      const int t = it * NW + wave;
      const bool active = t < tasks;
      const int gi = active ? t / NT : 0, l = active ? t - (t / NT) * NT : 0;
      const int col = gi * 16 + r;
      const bool valid = active && col < n;
      const int cc = valid ? col : 0;
      T* cp = R + l * nn + cc;
      {
        T op[4][4 * HB2];
        load_twice_folded<T, HB2, int>(cp, valid, n, n, g, op);
        acc_t acc[4][HB2];
        mma4<T, HB2, 0>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
        if (valid) {
#pragma unroll
          for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int s = orow(kb, g, j);
              const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
              cp[s * n] = P + Q;
              cp[(h - 1 - s) * n] = P - Q;
              cp[(h + s) * n] = Pe + Qe;
              if (s != h / 2 - 1) cp[(h + h - 2 - s) * n] = Pe - Qe;
            }
        }
      }
      __syncthreads();
      const T P3 = mxk * E[cc];
      const T Q3 = kxk * E[cc] + mxk * E[n + cc];
      T op[4][4 * HB2];
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = orow(kb, g, j);
          const bool middle = s == h / 2 - 1;
          const int mode_idx[4] = {s, h - 1 - s, h + s, h + (middle ? s : h - 2 - s)};
          T y[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            T a = T(0);
            if (valid) {
              T gr[NT];
              mode_row<T, NT>(me, E, n, P3, Q3, mode_idx[q], l, transpose, gr);
#pragma unroll
              for (int m = 0; m < NT; ++m) a += gr[m] * R[m * nn + mode_idx[q] * n + cc];
            }
            y[q] = a;
          }
          const int ib = 4 * kb + j;
          inverse_operands<T>(y[0], y[1], y[2], y[3], middle, op[0][ib], op[1][ib], op[2][ib], op[3][ib]);
        }
      __syncthreads();   // every component's modes are read before any column is overwritten
      acc_t out_acc[4][HB2];
      mma4<T, HB2, 1>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, out_acc);
      T none[HB2][4][4];
      zero_old<T, HB2>(none);
      store_twice_unfolded<T, HB2, false, int>(cp, valid, n, n, g, out_acc, MODE_STORE, T(1), none);
    }
  }
  // ---- y pass: column c (spectral x index) of every component, forward,
  // per-mode N_t x N_t solve, inverse, in place (3-D blocks: where there are
  // at least as many column groups as waves, n = 63 on four waves)
  if (!X3 || ygroups >= NW) {
#pragma unroll 1
  for (int gi = wave; gi < ygroups; gi += NW) {
    const T* Sf = frag();
    const int col = gi * 16 + r;
    const bool valid = col < n;
    const int cc = valid ? col : 0;
    // (P, Q) of the modes of this column: x-mode and y-mode (3-D blocks)
    const T P3 = X3 ? mxk * E[cc] : T(0);
    const T Q3 = X3 ? kxk * E[cc] + mxk * E[n + cc] : T(0);
    acc_t acc[NT][4][HB2];
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      T op[4][4 * HB2];
      load_twice_folded<T, HB2, int>(R + l * nn + cc, valid, n, n, g, op);
      mma4<T, HB2, 0>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc[l]);
      __builtin_amdgcn_sched_barrier(0);   // one component's operands live at a time
    }
    // per (kb, j): the four modes s, h-1-s, h+s, h+(h-2-s) of every component
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = orow(kb, g, j);
        const bool middle = s == h / 2 - 1;
        const int mode_idx[4] = {s, h - 1 - s, h + s, h + (middle ? s : h - 2 - s)};
        T v[NT][4];
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          const T P = acc[l][0][kb][j], Q = acc[l][1][kb][j], Pe = acc[l][2][kb][j], Qe = acc[l][3][kb][j];
          v[l][0] = P + Q;
          v[l][1] = P - Q;
          v[l][2] = Pe + Qe;
          v[l][3] = Pe - Qe;
        }
        T y[NT][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int l = 0; l < NT; ++l) y[l][q] = T(0);
          if (valid) {
            if constexpr (X3) {
              T gb[NT][NT];   // one block per mode for every component
              mode_block<T, NT>(me, E, n, P3, Q3, mode_idx[q], transpose, gb);
#pragma unroll
              for (int l = 0; l < NT; ++l)
#pragma unroll
                for (int m = 0; m < NT; ++m) y[l][q] += gb[l][m] * v[m][q];
            } else {
              const T* gm = G + (cc + n * mode_idx[q]) * (NT * NT);
#pragma unroll
              for (int l = 0; l < NT; ++l)
#pragma unroll
                for (int m = 0; m < NT; ++m) y[l][q] += (transpose ? gm[m * NT + l] : gm[l * NT + m]) * v[m][q];
            }
          }
        }
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          T u0, u1, u2, u3;
          inverse_operands<T>(y[l][0], y[l][1], y[l][2], y[l][3], middle, u0, u1, u2, u3);
          acc[l][0][kb][j] = u0;   // the operand of chunk 4 kb + j, kept in place
          acc[l][1][kb][j] = u1;
          acc[l][2][kb][j] = u2;
          acc[l][3][kb][j] = u3;
        }
        // keeps the compiler from hoisting every row's block loads (register spills)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      acc_t out_acc[4][HB2];
      mma4<T, HB2, 1>(Sf, lane, [&](int m, int ib) { return (T)acc[l][m][ib >> 2][ib & 3]; }, out_acc);
      T none[HB2][4][4];
      zero_old<T, HB2>(none);
      store_twice_unfolded<T, HB2, false, int>(R + l * nn + cc, valid, n, n, g, out_acc, MODE_STORE, T(1), none);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  }
  __syncthreads();
  // ---- inverse x pass, in place in physical order
#pragma unroll 1
  for (int gi = wave; gi < xgroups; gi += NW) {
    const T* Sf = frag();
    const int line = gi * 16 + r;
    const bool valid = line < NT * n;
    T* lp = R + (valid ? line : 0) * n;
    T op[4][4 * HB2];
#pragma unroll
    for (int ib = 0; ib < 4 * HB2; ++ib) {
      const int s = cidx(ib, g);
      const bool middle = s == h / 2 - 1;
      T yo = 0, yom = 0, ye = 0, yem = 0;
      if (valid) {
        yo = lp[s];
        yom = lp[h - 1 - s];
        ye = lp[h + s];
        if (!middle) yem = lp[h + h - 2 - s];
      }
      inverse_operands<T>(yo, yom, ye, yem, middle, op[0][ib], op[1][ib], op[2][ib], op[3][ib]);
    }
    acc_t acc[4][HB2];
    mma4<T, HB2, 1>(Sf, lane, [&](int m, int ib) { return op[m][ib]; }, acc);
    T none[HB2][4][4];
    zero_old<T, HB2>(none);
    store_twice_unfolded<T, HB2, false, int>(lp, valid, 1, n, g, acc, MODE_STORE, T(1), none);
  }
  __syncthreads();
  // ---- result to dst
#pragma unroll 1
  for (int e0 = threadIdx.x; e0 < total; e0 += WG * 8) {
    T old[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + WG * i;
      old[i] = (e < total && mode == MODE_ADD_SCALED) ? dp[e] : T(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + WG * i;
      if (e < total) dp[e] = epi<T>(mode, old[i], R[e], omega);
    }
  }
}

// 2-D residual fused with the forward x pass (N_t = 2): a workgroup owns one
// slab and 8 rows, stages rows y0-1 .. y0+8 of u and of the coupling
// combination of the neighbouring slab in LDS (every global load issued
// first), forms r = F - L u in registers, puts its 16 lines (2 components x 8
// rows) back into LDS, and the four waves each run one of the four twice-
// folded products (O and E on even and odd inputs) on those 16 lines; the
// sums and differences of their results are the spectral x lines, stored to
// xhat in the layout of r.  The residual itself never reaches HBM; with
// `partial` the workgroup's sum of r^2 is written as the residual kernel does.
// Dynamic LDS: max(3 (TY + 2) n, 2 TY n + 4 * 16 * 16 HB2) elements.
template <typename T, int HB2, int SIT>
__global__ __launch_bounds__(256) void k_resid_xfwd(const T* __restrict__ u, const T* __restrict__ F,
                                                    T* __restrict__ xhat, ResidArgs<T> a,
                                                    const T* __restrict__ Sfrag, double* __restrict__ partial) {
  constexpr int NT = 2, TY = 8;
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
  const int h = (n + 1) >> 1;
  const int y0 = tile * TY;
  const int plane = (TY + 2) * n;
  const int rows = (y0 + TY < n ? y0 + TY : n) - y0;
  const int nout = rows * n;
  const int sn = (int)(slab % a.N);
  const bool couple = (sn + a.dir >= 0) && (sn + a.dir < a.N);
  const long long slabsz = (long long)NT * nx;
  const T* un = u + slab * slabsz;
  const T* up = u + (slab + a.dir) * slabsz;
  const T* Fn = F + slab * slabsz;
  const long long s0 = (long long)(y0 - 1) * n;
  const long long o0 = (long long)y0 * n;
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
  const float inv_n = 1.0f / (float)n;
  T rv[SIT][NT];
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
#pragma unroll
    for (int l = 0; l < NT; ++l) rv[i][l] = T(0);
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
        rv[i][l] = acc;
      }
    }
  }
  if (partial != nullptr) {
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < SIT; ++i)
#pragma unroll
      for (int l = 0; l < NT; ++l) ss += (double)rv[i][l] * (double)rv[i][l];
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) partial[slab * gridDim.x + tile] = red[0] + red[1] + red[2] + red[3];
  }
  __syncthreads();   // every stencil read of U is done
  // r lines into LDS: line l * TY + yy, element x
  T* Rl = U;
#pragma unroll
  for (int i = 0; i < SIT; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < nout) {
#pragma unroll
      for (int l = 0; l < NT; ++l) Rl[l * TY * n + e] = rv[i][l];
    }
  }
  __syncthreads();
  // wave m: product m of the 16 lines; results to Pb[m][line][row]
  constexpr int PR = 16 * HB2;   // rows of one product (h / 2)
  T* Pb = U + NT * TY * n;
  {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int yy = r & (TY - 1);
    const bool valid = yy < rows;
    const T* lp = Rl + r * n;   // line r = component r / TY, row r % TY
    T op[4 * HB2];
#pragma unroll
    for (int ib = 0; ib < 4 * HB2; ++ib) {
      const int p = cidx(ib, g);
      const int i0 = 2 * p, i1 = 2 * p + 1;
      T v = T(0);
      if (valid) {
        if (wave == 0) v = lp[i0] + lp[n - 1 - i0];
        else if (wave == 1) v = i1 < h - 1 ? lp[i1] + lp[n - 1 - i1] : lp[i1];
        else if (wave == 2) v = lp[i0] - lp[n - 1 - i0];
        else v = i1 < h - 1 ? lp[i1] - lp[n - 1 - i1] : T(0);
      }
      op[ib] = v;
    }
    typename Mfma<T>::acc_t acc[HB2];
    mma1<T, HB2, 0>(Sfrag, lane, wave, [&](int ib) { return op[ib]; }, acc);
#pragma unroll
    for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j) Pb[(wave * 16 + r) * PR + orow(kb, g, j)] = acc[kb][j];
  }
  __syncthreads();
  // spectral lines: row s of line L gives positions s, h-1-s, h+s, h+h-2-s
  T* xo = xhat + slab * slabsz;
  for (int it = threadIdx.x; it < 16 * PR; it += 256) {
    const int line = it / PR, sr = it - line * PR;
    const int l = line / TY, yy = line - l * TY;
    if (yy >= rows) continue;
    const T P = Pb[(0 * 16 + line) * PR + sr], Q = Pb[(1 * 16 + line) * PR + sr];
    const T Pe = Pb[(2 * 16 + line) * PR + sr], Qe = Pb[(3 * 16 + line) * PR + sr];
    T* dst = xo + l * nx + (long long)(y0 + yy) * n;
    dst[sr] = P + Q;
    dst[h - 1 - sr] = P - Q;
    dst[h + sr] = Pe + Qe;
    if (sr != h / 2 - 1) dst[h + h - 2 - sr] = Pe - Qe;
  }
}

// 3-D residual fused with the forward x pass into the x-mode-major layout
// [slab][kx][l][z][y] of the slab-resident solves: the z-marching residual
// (TY rows of y per workgroup, zero halo rows and planes at the Dirichlet
// boundary, planar stencil sums kept as the open sums of the two output
// planes the last staged plane contributes to) leaves each output plane's
// N_t TY lines of r (GP groups of 16 for the twice-folded transform) in one
// of PB LDS slots instead of HBM.  After every PB-th plane (and at the end of
// the chunk) each wave runs the forward transform on one group of the slots,
// right after the next staging barrier, and stores the spectral values to
// xhat (TY consecutive y per (kx, l, z)).  With `partial` the workgroup's sum
// of r^2 is written as the residual kernel does.  Dynamic LDS:
// ((N_t + 1)(TY + 2) n + (BS / 64) 16 n) elements.  The register budget is
// capped at 256 (two 256-thread or one 512-thread workgroup per CU; the
// accumulators then stay out of the matrix registers).
template <typename T, int HB2, int NT, int OIT, int SIT, int BS>
__global__ __launch_bounds__(BS, 512 / BS) void k_resid_xfwd3(const T* __restrict__ u, const T* __restrict__ F,
                                                            T* __restrict__ xhat, ResidArgs<T> a,
                                                            const T* __restrict__ Sfrag, double* __restrict__ partial,
                                                            int TY_arg, int ZC) {
  // n = 64 HB2 - 1 and TY = min(16 / N_t, 512 / n) x BS / 256 are fixed by the template (the host
  // checks them); a plane's N_t TY lines are GP groups of 16, and PB planes fill the BS / 64 waves
  constexpr int n = 64 * HB2 - 1;
  constexpr int TY = (16 / NT < 512 / n ? 16 / NT : 512 / n) * (BS / 256);
  constexpr int GP = (NT * TY + 15) / 16;
  constexpr int PB = BS / 64 / GP;
  (void)TY_arg;
  typedef typename Mfma<T>::acc_t acc_t;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* U = reinterpret_cast<T*>(lds_raw);
  const long long lg = xcd_linear(blockIdx.x + (long long)gridDim.x * slab_index(),
                                  (long long)gridDim.x * gridDim.y * gridDim.z);
  const long long slab = lg / gridDim.x;
  const int tile = (int)(lg - slab * gridDim.x);
  if (slab >= (long long)a.batch * a.N) return;
  const long long nx = a.nx;
  constexpr long long nn = (long long)n * n;
  constexpr int h = (n + 1) >> 1;
  constexpr int nyt = (n + TY - 1) / TY;
  const int yt = tile % nyt;
  const int z0 = (tile / nyt) * ZC;
  const int z1 = z0 + ZC < n ? z0 + ZC : n;
  const int y0 = yt * TY;
  const int rows = (y0 + TY < n ? y0 + TY : n) - y0;
  constexpr int plane = (TY + 2) * n;
  const int nout = rows * n;
  const int sn = (int)(slab % a.N);
  const bool couple = (sn + a.dir >= 0) && (sn + a.dir < a.N);
  const long long slabsz = (long long)NT * nx;
  const T* un = u + slab * slabsz;
  const T* up = u + (slab + a.dir) * slabsz;
  const T* Fn = F + slab * slabsz;
  const long long s0 = (long long)(y0 - 1) * n;
  const long long o0 = (long long)y0 * n;
  T* Rb = U + (NT + 1) * plane;   // slots [PB][GP 16 lines][n], line l * TY + row
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;

  int oy[OIT], ox[OIT];
#pragma unroll
  for (int i = 0; i < OIT; ++i) {
    const int e = threadIdx.x + BS * i;
    oy[i] = e / n;
    ox[i] = e - oy[i] * n;
  }
  T uv[SIT][NT], pv[SIT][NT];
  T fv[OIT][NT], fn[OIT][NT];
  T P0[OIT][2 * NT + 1], P1[OIT][2 * NT + 1];
#pragma unroll
  for (int i = 0; i < OIT; ++i) {
#pragma unroll
    for (int c = 0; c <= 2 * NT; ++c) P0[i][c] = P1[i][c] = T(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) fn[i][k] = T(0);
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
  // forward x transform of the nb planes ob .. ob + nb - 1 in the slots: wave w takes plane ob + w
  const long long lps = (long long)NT * nn;
  auto xform = [&](int ob, int nb) {
    const int pw = wave / GP, gp = wave - (wave / GP) * GP;   // plane of the batch, group of the plane
    if (pw >= nb) return;
    const T* Sf = Sfrag;
    asm volatile("" : "+s"(Sf));
    const int zb = ob + pw;
    const int line = gp * 16 + r;
    const int l = line / TY, yl = line - (line / TY) * TY;
    const bool valid = l < NT && yl < rows;
    const T* lp = Rb + ((long long)pw * GP * 16 + (valid ? line : 0)) * n;
    // the four folded products one at a time, each operand formed from LDS
    // (the operands of one product live at a time)
    acc_t acc[4][HB2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      T op[4 * HB2];
#pragma unroll
      for (int ib = 0; ib < 4 * HB2; ++ib) {
        const int pp = cidx(ib, g);
        const int i = 2 * pp + (m & 1);
        const bool pair = (m & 1) == 0 || i < h - 1;   // the odd row h - 1 has no mirror
        T v = T(0);
        if (valid && (pair || m == 1)) {
          const T x = lp[i];
          const T y = pair ? lp[n - 1 - i] : T(0);
          v = m < 2 ? x + y : x - y;
        }
        op[ib] = v;
      }
      mma1<T, HB2, 0>(Sf, lane, m, [&](int ib) { return op[ib]; }, acc[m]);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (valid) {
      T* xo = xhat + slab * n * lps + ((long long)l * n + zb) * n + y0 + yl;
#pragma unroll
      for (int kb = 0; kb < HB2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = orow(kb, g, j);
          const T P = acc[0][kb][j], Q = acc[1][kb][j], Pe = acc[2][kb][j], Qe = acc[3][kb][j];
          xo[(long long)s * lps] = P + Q;
          xo[(long long)(h - 1 - s) * lps] = P - Q;
          xo[(long long)(h + s) * lps] = Pe + Qe;
          if (s != h / 2 - 1) xo[(long long)(h + h - 2 - s) * lps] = Pe - Qe;
        }
    }
  };
  double ss = 0.0;
  int pend_ob = -1, pend_nb = 0;   // a batch of planes in the slots waiting for its transform
  load_plane(z0 - 1);
  for (int p = z0 - 1; p <= z1; ++p) {
    __syncthreads();   // the previous plane's stencils and slot writes are done
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
#pragma unroll
    for (int i = 0; i < OIT; ++i)
#pragma unroll
      for (int k = 0; k < NT; ++k) fv[i][k] = fn[i][k];
    if (pend_nb > 0) {
      // the transform runs between the staging and the next plane's loads, so
      // that its operands and accumulators never share registers with those loads
      __builtin_amdgcn_sched_barrier(0);
      xform(pend_ob, pend_nb);
      __builtin_amdgcn_sched_barrier(0);
      pend_nb = 0;
    }
    if (p < z1) load_plane(p + 1);
    if (p >= z0 && p < z1) load_rhs(p);
    __syncthreads();
    const int o = p - 1;   // output plane: complete once plane p = o + 1 is in
    const int slot = (o - z0) % PB;
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
        for (int dr = 0; dr < 3; ++dr) {
          const T* row = U + c * plane + (oy[i] + dr) * n + x;
          const T lft = hl ? row[-1] : T(0);
          const T m0 = row[0];
          const T rt = hr ? row[1] : T(0);
          const T sm = a.wm[0] * lft + a.wm[1] * m0 + a.wm[2] * rt;
          mm += a.wm[dr] * sm;
          if (c < NT) kk += a.wk[dr] * sm + a.wm[dr] * (a.wk[0] * lft + a.wk[1] * m0 + a.wk[2] * rt);
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
      if (o >= z0) {
        T* sp = Rb + (long long)slot * GP * 16 * n + oy[i] * n + x;
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          T s = fv[i][l] + a.ca[l] * P1[i][NT];
#pragma unroll
          for (int k = 0; k < NT; ++k) s -= a.K[l * NT + k] * P1[i][k] + a.M[l * NT + k] * P1[i][NT + 1 + k];
          sp[l * TY * n] = s;
          ss += (double)s * (double)s;
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
    if (o >= z0 && (slot == PB - 1 || o == z1 - 1)) {
      pend_ob = o - slot;
      pend_nb = slot + 1;
    }
  }
  __syncthreads();
  if (pend_nb > 0) xform(pend_ob, pend_nb);
  if (partial != nullptr) {
    __shared__ double red[BS / 64];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < BS / 64; ++w) t += red[w];
      partial[slab * gridDim.x + tile] = t;
    }
  }
}

}  // namespace

bool twice_folded_ok(int n, int elem_bytes) {
  if (n == 63 || n == 127) return true;
  return elem_bytes == 4 && n == 255;    // FP64 at h/2 = 64 would not fit in registers
}

// Launch shape of the twice-folded passes: waves per workgroup of the x (and y)
// passes (1, 2 or 4; 0 = 4), a cap on their grid in workgroups per compute
// unit (0 = one wave per group of 16 lines), column groups per workgroup of
// the fused pass (0 = 4 / N_t for N_t <= 2, else 1) and its grid cap.
static unsigned capped_grid(long long need, int per_cu, int cus) {
  if (per_cu <= 0 || cus <= 0) return (unsigned)need;
  const long long cap = (long long)per_cu * cus;
  return (unsigned)(need < cap ? need : cap);
}

template <typename T>
hipError_t launch_pass_reg2(int n, bool inverse, const T* in, T* out, const T* Sfrag2, long long inner,
                            long long ncols, T omega, int mode, hipStream_t s, bool bf16, const PassShape& sh,
                            long long lps) {
  if (lps > 0 && inner != 1) return hipErrorInvalidValue;   // the x-mode-major side exists for x passes only
  const int wpg = sh.wpg == 1 || sh.wpg == 2 ? sh.wpg : 4;
  const long long need = (ncols + 16 * wpg - 1) / (16 * wpg);
  const unsigned grid = capped_grid(need, sh.pass_per_cu, sh.cus);
  const bool persist = (long long)grid < need;
  const dim3 block(64 * wpg);
#define P2P(HB2, U, B, P)                                                                                      \
  {                                                                                                            \
    const size_t lds = U ? (size_t)wpg * 16 * n * sizeof(T) : 0;                                               \
    if (inverse)                                                                                               \
      hipLaunchKernelGGL((k_pass_reg2<T, HB2, true, U, B, P>), dim3(grid), block, lds, s, in, out, Sfrag2, n,   \
                         inner, ncols, omega, mode, lps);                                                      \
    else                                                                                                       \
      hipLaunchKernelGGL((k_pass_reg2<T, HB2, false, U, B, P>), dim3(grid), block, lds, s, in, out, Sfrag2, n,  \
                         inner, ncols, omega, mode, lps);                                                      \
    return hipGetLastError();                                                                                  \
  }
#define P2B(HB2, U, B)            \
  if (persist) { P2P(HB2, U, B, true) } \
  P2P(HB2, U, B, false)
#define P2(HB2, U)                      \
  if constexpr (sizeof(T) == 4) {       \
    if (bf16) { P2B(HB2, U, true) }     \
  }                                     \
  P2B(HB2, U, false)
  if (!twice_folded_ok(n, (int)sizeof(T)) || (bf16 && sizeof(T) != 4)) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    if (n == 255) {
      if (inner == 1) { P2(4, true) }
      P2(4, false)
    }
  }
  if (n == 127) {
    if (inner == 1) { P2(2, true) }
    P2(2, false)
  }
  if (n == 63) {
    if (inner == 1) { P2(1, true) }
    P2(1, false)
  }
#undef P2
#undef P2B
#undef P2P
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_fused_pair2(int n, int nt, const T* in, T* out, const T* Sfrag2, const T* G, long long inner,
                              long long outer, int transpose, T omega, int mode, hipStream_t s, bool bf16,
                              const ModeEig<T>* me, const PassShape& sh) {
  ModeEig<T> mev{};
  if (me != nullptr && nt <= NT_MAX) mev = *me;
  const int cgmax = nt >= 3 ? 1 : 4 / nt;
  const int cg = (sh.fused_cg >= 1 && sh.fused_cg <= cgmax && (sh.fused_cg & (sh.fused_cg - 1)) == 0)
                     ? sh.fused_cg : cgmax;
  const long long need = (outer * inner + 16 * cg - 1) / (16 * cg);
  const unsigned grid = capped_grid(need, sh.fused_per_cu, sh.cus);
  const bool persist = (long long)grid < need;
  const dim3 block(64 * nt * cg);
#define F2B(HB2, NT, CG, B)                                                                                      \
  if (nt == NT && cg == CG) {                                                                                    \
    if (persist)                                                                                                 \
      hipLaunchKernelGGL((k_fused_pair2<T, HB2, NT, CG, B, true>), dim3(grid), block, 0, s, in, out, Sfrag2, G,  \
                         n, inner, outer, transpose, omega, mode, mev);                                          \
    else                                                                                                         \
      hipLaunchKernelGGL((k_fused_pair2<T, HB2, NT, CG, B, false>), dim3(grid), block, 0, s, in, out, Sfrag2, G, \
                         n, inner, outer, transpose, omega, mode, mev);                                          \
    return hipGetLastError();                                                                                    \
  }
#define F2C(HB2, B) F2B(HB2, 1, 1, B) F2B(HB2, 1, 2, B) F2B(HB2, 1, 4, B) F2B(HB2, 2, 1, B) F2B(HB2, 2, 2, B) \
                    F2B(HB2, 3, 1, B) F2B(HB2, 4, 1, B)
#define F2(HB2)                                      \
  if constexpr (sizeof(T) == 4) {                    \
    if (bf16) { F2C(HB2, true) }                     \
  }                                                  \
  F2C(HB2, false)
  if (!twice_folded_ok(n, (int)sizeof(T)) || (bf16 && sizeof(T) != 4)) return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    if (n == 255) { F2(4) }
  }
  if (n == 127) { F2(2) }
  if (n == 63) { F2(1) }
#undef F2
#undef F2C
#undef F2B
  return hipErrorInvalidValue;
}

size_t slab_solve2_lds(int dim, int n, int nt, int elem_bytes) {
  if (dim < 2 || dim > 3 || nt < 1 || nt > 2 || !twice_folded_ok(n, elem_bytes) || n > 127) return 0;
  const int hb2 = (n + 1) / 64;   // twice-folded fragment tables in LDS for the 3-D form
  const size_t bytes = ((size_t)nt * n * n + (dim == 3 ? 2 * n + 2048 * hb2 * hb2 : 0)) * elem_bytes;
  return bytes <= 160 * 1024 ? bytes : 0;
}

template <typename T>
hipError_t launch_slab_solve2(int n, int nt, const T* src, T* dst, const T* Sfrag2, const T* G, long long slabs,
                              int transpose, T omega, int mode, hipStream_t s, const ModeEig<T>* me3) {
  const bool x3 = me3 != nullptr;
  const size_t lds = slab_solve2_lds(x3 ? 3 : 2, n, nt, (int)sizeof(T));
  if (lds == 0) return hipErrorInvalidValue;
  ModeEig<T> mev{};
  if (x3) mev = *me3;
  const long long blocks = x3 ? slabs * n : slabs;
  const dim3 grid = slab_grid(1, blocks);
  // 3-D planes: 256 threads (two workgroups per CU, limited by LDS, overlap one's memory phases with the other's
  // matrix phases; 4.37 ms against 4.52 ms with 512 on 63^3 x 1024); STMG_XSLAB_WG=512 selects the wider form
  static const int wg_env = [] {
    const char* e = std::getenv("STMG_XSLAB_WG");
    return e ? std::atoi(e) : 256;
  }();
#define SL2X(HB2, NT, X, W)                                                                                    \
  {                                                                                                            \
    const void* fn = reinterpret_cast<const void*>(&k_slab_solve2<T, HB2, NT, X, W>);                          \
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);              \
    if (e != hipSuccess) return e;                                                                             \
    hipLaunchKernelGGL((k_slab_solve2<T, HB2, NT, X, W>), grid, dim3(W), lds, s, src, dst, Sfrag2, G, n,         \
                       blocks, transpose, omega, mode, mev);                                                   \
    return hipGetLastError();                                                                                  \
  }
#define SL2(HB2, NT)                                    \
  if (nt == NT) {                                       \
    if (x3 && wg_env == 512) SL2X(HB2, NT, true, 512)   \
    if (x3) SL2X(HB2, NT, true, 256)                    \
    SL2X(HB2, NT, false, 512)                           \
  }
  if (n == 63) { SL2(1, 1) SL2(1, 2) }
  if constexpr (sizeof(T) == 4) {
    if (n == 127) { SL2(2, 1) SL2(2, 2) }
  }
#undef SL2
#undef SL2X
  return hipErrorInvalidValue;
}

template hipError_t launch_slab_solve2<double>(int, int, const double*, double*, const double*, const double*,
                                               long long, int, double, int, hipStream_t, const ModeEig<double>*);
template hipError_t launch_slab_solve2<float>(int, int, const float*, float*, const float*, const float*, long long,
                                              int, float, int, hipStream_t, const ModeEig<float>*);
bool resid_xfwd_ok(int dim, int n, int nt, int elem_bytes) {
  return dim == 2 && nt == 2 && (n == 63 || n == 127) && twice_folded_ok(n, elem_bytes);
}

unsigned resid_xfwd_blocks_per_slab(int n) { return (unsigned)((n + 7) / 8); }

template <typename T>
hipError_t launch_resid_xfwd(int n, const T* u, const T* F, T* xhat, const ResidArgs<T>& a, const T* Sfrag2,
                             double* partial, hipStream_t s) {
  if (!resid_xfwd_ok(2, n, 2, (int)sizeof(T)) || a.n != n) return hipErrorInvalidValue;
  const int HB2 = n == 127 ? 2 : 1;
  const size_t elems = std::max<size_t>((size_t)3 * 10 * n, (size_t)2 * 8 * n + (size_t)4 * 16 * 16 * HB2);
  const size_t lds = elems * sizeof(T);
  const dim3 grid = slab_grid(resid_xfwd_blocks_per_slab(n), (long long)a.batch * a.N);
  if (n == 127)
    hipLaunchKernelGGL((k_resid_xfwd<T, 2, 5>), grid, dim3(256), lds, s, u, F, xhat, a, Sfrag2, partial);
  else
    hipLaunchKernelGGL((k_resid_xfwd<T, 1, 3>), grid, dim3(256), lds, s, u, F, xhat, a, Sfrag2, partial);
  return hipGetLastError();
}

// 3-D form: TY rows of y per workgroup of BS threads with N_t TY <= 16 BS /
// 256 lines a plane and TY n <= 2 BS positions (two a thread), z chunks of at
// least 8 planes so that a level has about 4096 workgroups.
bool resid_xfwd3_ok(int n, int nt, int elem_bytes) {
  return (n == 63 || n == 127) && nt >= 1 && nt <= 2 && twice_folded_ok(n, elem_bytes);
}

struct Rx3Shape {
  int ty, zc, nyt, nzt, oit, sit, bs;
  size_t lds;
};
static Rx3Shape rx3_shape(int n, int nt, long long slabs, int elem_bytes) {
  // n = 63: 512-thread workgroups of 16 rows (runs of 16 y in the output: 4.5 instead of 5.9 GB
  // written per launch on 63^3 x 1024, 3.94 against 4.19 ms); tuning knob STMG_RX3_BS=256 takes 8 rows
  static const int bs = [] {
    const char* e = std::getenv("STMG_RX3_BS");
    return e && std::atoi(e) == 256 ? 256 : 512;
  }();
  Rx3Shape sh{};
  sh.bs = n == 63 ? bs : 256;
  sh.ty = std::min(16 / nt, 512 / n) * (sh.bs / 256);
  sh.nyt = (n + sh.ty - 1) / sh.ty;
  const long long want = (4096 + (long long)sh.nyt * slabs - 1) / ((long long)sh.nyt * slabs);
  const int maxc = (n + 7) / 8;
  const int nzc = (int)(want < 1 ? 1 : (want > maxc ? maxc : want));
  sh.zc = (n + nzc - 1) / nzc;
  sh.nzt = (n + sh.zc - 1) / sh.zc;
  sh.oit = (sh.ty * n + sh.bs - 1) / sh.bs;
  sh.sit = ((sh.ty + 2) * n + sh.bs - 1) / sh.bs;
  sh.lds = ((size_t)(nt + 1) * (sh.ty + 2) * n + (size_t)(sh.bs / 64) * 16 * n) * elem_bytes;
  return sh;
}

unsigned resid_xfwd3_blocks_per_slab(int n, int nt, long long slabs, int elem_bytes) {
  if (!resid_xfwd3_ok(n, nt, elem_bytes)) return 0;
  const Rx3Shape sh = rx3_shape(n, nt, slabs, elem_bytes);
  return (unsigned)(sh.nyt * sh.nzt);
}

template <typename T>
hipError_t launch_resid_xfwd3(int n, int nt, const T* u, const T* F, T* xhat, const ResidArgs<T>& a,
                              const T* Sfrag2, double* partial, hipStream_t s) {
  if (!resid_xfwd3_ok(n, nt, (int)sizeof(T)) || a.n != n) return hipErrorInvalidValue;
  const long long slabs = (long long)a.batch * a.N;
  const Rx3Shape sh = rx3_shape(n, nt, slabs, (int)sizeof(T));
  const dim3 grid = slab_grid((unsigned)(sh.nyt * sh.nzt), slabs);
#define RX3(HB2, NT, OIT, SIT, BS)                                                                              \
  if (n == 32 * HB2 * 2 - 1 && nt == NT && sh.oit == OIT && sh.sit == SIT && sh.bs == BS) {                     \
    const void* fn = reinterpret_cast<const void*>(&k_resid_xfwd3<T, HB2, NT, OIT, SIT, BS>);                  \
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);         \
    if (e != hipSuccess) return e;                                                                             \
    hipLaunchKernelGGL((k_resid_xfwd3<T, HB2, NT, OIT, SIT, BS>), grid, dim3(BS), sh.lds, s, u, F, xhat, a,     \
                       Sfrag2, partial, sh.ty, sh.zc);                                                          \
    return hipGetLastError();                                                                                  \
  }
  RX3(1, 1, 2, 3, 256) RX3(1, 2, 2, 3, 256) RX3(2, 1, 2, 3, 256) RX3(2, 2, 2, 3, 256)
  RX3(1, 1, 2, 3, 512) RX3(1, 2, 2, 3, 512)
#undef RX3
  return hipErrorInvalidValue;
}

template hipError_t launch_resid_xfwd3<double>(int, int, const double*, const double*, double*,
                                               const ResidArgs<double>&, const double*, double*, hipStream_t);
template hipError_t launch_resid_xfwd3<float>(int, int, const float*, const float*, float*, const ResidArgs<float>&,
                                              const float*, double*, hipStream_t);
template hipError_t launch_resid_xfwd<double>(int, const double*, const double*, double*, const ResidArgs<double>&,
                                              const double*, double*, hipStream_t);
template hipError_t launch_resid_xfwd<float>(int, const float*, const float*, float*, const ResidArgs<float>&,
                                             const float*, double*, hipStream_t);
template hipError_t launch_pass_reg2<double>(int, bool, const double*, double*, const double*, long long, long long,
                                             double, int, hipStream_t, bool, const PassShape&, long long);
template hipError_t launch_pass_reg2<float>(int, bool, const float*, float*, const float*, long long, long long,
                                            float, int, hipStream_t, bool, const PassShape&, long long);
template hipError_t launch_fused_pair2<double>(int, int, const double*, double*, const double*, const double*,
                                               long long, long long, int, double, int, hipStream_t, bool,
                                               const ModeEig<double>*, const PassShape&);
template hipError_t launch_fused_pair2<float>(int, int, const float*, float*, const float*, const float*, long long,
                                              long long, int, float, int, hipStream_t, bool, const ModeEig<float>*,
                                              const PassShape&);

}  // namespace stmg
