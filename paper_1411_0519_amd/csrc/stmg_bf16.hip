// BF16 matrix-core sine transforms for the FP32 inner V-cycle of the mixed
// solver (ST_MIXED_BF16): vectors stay FP32 in HBM, the folded DST products
// round their operands to bfloat16 and accumulate in FP32
// (v_mfma_f32_16x16x16_bf16), the per-mode time solve is FP32.  The outer
// iterative refinement in FP64 absorbs the ~2^-8 relative error of the inner
// block solves.
//
// Operand layout (measured on gfx950): lane l supplies A[l%16][4(l/16)+q] and
// B[4(l/16)+q][l%16] (q = 0..3, packed bf16) and holds D[4(l/16)+j][l%16].  A
// 16-row chunk c of a column is therefore rows 16c + 4g + q of lane (g, r), and
// an output block kb is rows 16kb + 4g + j: the same rows, so a forward product,
// the per-mode solve and the inverse product chain in registers.
#include <hip/hip_runtime.h>

#include "stmg_device.h"
#include "stmg_internal.h"

namespace stmg {

namespace {

using namespace dev;

typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ inline v4s pack4(float a, float b, float c, float d) {
  v4s v;
  v[0] = bf16_bits(a);
  v[1] = bf16_bits(b);
  v[2] = bf16_bits(c);
  v[3] = bf16_bits(d);
  return v;
}

// Fragment table [dir][half][kb][c][lane] of packed bf16 quadruples.
template <int HB>
__device__ inline const v4s* frag_at(const v4s* F, int dir, int half, int kb, int c, int lane) {
  return F + ((((dir * 2 + half) * HB + kb) * HB + c) * 64 + lane);
}

// acc[kbt] = S_half(dir) * operand over the 16-row chunks c < ceil(h/16).
template <int HB, int DIR, typename OpFn>
__device__ inline void bf16_mma(const v4s* __restrict__ F, int h, int lane, OpFn op, v4f (&acc)[2 * HB]) {
#pragma unroll
  for (int k = 0; k < 2 * HB; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
  const int cmax = (h + 15) >> 4;
#pragma unroll
  for (int c = 0; c < HB; ++c) {
    if (c < cmax) {
      const v4s bo = op(0, c), be = op(1, c);
#pragma unroll
      for (int kb = 0; kb < HB; ++kb) {
        acc[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(*frag_at<HB>(F, DIR, 0, kb, c, lane), bo, acc[kb], 0, 0, 0);
        acc[HB + kb] =
            __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(*frag_at<HB>(F, DIR, 1, kb, c, lane), be, acc[HB + kb], 0, 0, 0);
      }
    }
  }
}

__device__ inline float epi(int mode, float old, float v, float omega) {
  return mode == MODE_STORE ? v : (mode == MODE_ADD_SCALED ? old + omega * v : omega * v);
}

// Physical rows of an inverse product: i gets P + Q, n-1-i gets P - Q (i < h-1),
// h-1 gets P; the epilogue is applied in place.
template <int HB>
__device__ inline void unfold_store(float* __restrict__ dst, bool valid, long long inner, int n, int h, int g,
                                    const v4f (&acc)[2 * HB], int mode, float omega) {
  if (!valid) return;
#pragma unroll
  for (int kb = 0; kb < HB; ++kb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = kb * 16 + 4 * g + j;
      const float P = acc[kb][j], Q = acc[HB + kb][j];
      if (i < h - 1) {
        float* p0 = dst + (long long)i * inner;
        float* p1 = dst + (long long)(n - 1 - i) * inner;
        const float o0 = mode == MODE_ADD_SCALED ? *p0 : 0.f;
        const float o1 = mode == MODE_ADD_SCALED ? *p1 : 0.f;
        *p0 = epi(mode, o0, P + Q, omega);
        *p1 = epi(mode, o1, P - Q, omega);
      } else if (i == h - 1) {
        float* p0 = dst + (long long)i * inner;
        const float o0 = mode == MODE_ADD_SCALED ? *p0 : 0.f;
        *p0 = epi(mode, o0, P, omega);
      }
    }
}

// Folded operands of one column: chunk c holds rows 16c + 4g + q.
template <int HB>
__device__ inline void load_fold_bf16(const float* __restrict__ src, bool valid, long long inner, int n, int h, int g,
                                      v4s (&bo)[HB], v4s (&be)[HB]) {
#pragma unroll
  for (int c = 0; c < HB; ++c) {
    float a[4], d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * c + 4 * g + q;
      const float x1 = (valid && i < h) ? src[(long long)i * inner] : 0.f;
      const float x2 = (valid && i < h - 1) ? src[(long long)(n - 1 - i) * inner] : 0.f;
      a[q] = x1 + x2;
      d[q] = x1 - x2;
    }
    bo[c] = pack4(a[0], a[1], a[2], a[3]);
    be[c] = pack4(d[0], d[1], d[2], d[3]);
  }
}

// One pass along an axis (x: inner = 1), a wave per 16 columns.
template <int HB, bool INV>
__global__ __launch_bounds__(256) void k_pass_bf16(const float* __restrict__ in, float* __restrict__ out,
                                                   const v4s* __restrict__ F, int n, long long inner,
                                                   long long ncols, float omega, int mode) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const long long lin = (xcd_linear(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)) * 16 + r;
  const bool valid = lin < ncols;
  const long long o = valid ? lin / inner : 0;
  const long long pos = valid ? lin - o * inner : 0;
  const long long base = o * (long long)n * inner + pos;
  const int h = (n + 1) >> 1;
  v4s bo[HB], be[HB];
  v4f acc[2 * HB];
  if (!INV) {
    load_fold_bf16<HB>(in + base, valid, inner, n, h, g, bo, be);
    bf16_mma<HB, 0>(F, h, lane, [&](int half, int c) { return half ? be[c] : bo[c]; }, acc);
    if (!valid) return;
#pragma unroll
    for (int kb = 0; kb < HB; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = kb * 16 + 4 * g + j;
        if (i < h) out[base + (long long)i * inner] = acc[kb][j];
        if (i < h - 1) out[base + (long long)(h + i) * inner] = acc[HB + kb][j];
      }
  } else {
#pragma unroll
    for (int c = 0; c < HB; ++c) {
      float a[4], d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * c + 4 * g + q;
        a[q] = (valid && i < h) ? in[base + (long long)i * inner] : 0.f;
        d[q] = (valid && i < h - 1) ? in[base + (long long)(h + i) * inner] : 0.f;
      }
      bo[c] = pack4(a[0], a[1], a[2], a[3]);
      be[c] = pack4(d[0], d[1], d[2], d[3]);
    }
    bf16_mma<HB, 1>(F, h, lane, [&](int half, int c) { return half ? be[c] : bo[c]; }, acc);
    unfold_store<HB>(out + base, valid, inner, n, h, g, acc, mode, omega);
  }
}

// Slowest axis: forward transform, per-mode N_t x N_t solve, inverse transform.
// One wave per time component (wave w: column group w / NT, component w % NT);
// the time solve exchanges one 16-row block at a time through LDS.
template <int HB, int NT>
__global__ __launch_bounds__(256) void k_fused_bf16(const float* in, float* out, const v4s* __restrict__ F,
                                                    const float* __restrict__ G, int n, long long inner,
                                                    long long outer, int transpose, float omega, int mode) {
  constexpr int CG = NT >= 3 ? 1 : 4 / NT;
  __shared__ float xch[2][CG * NT * 64 * 4];
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
  v4f spec[2 * HB];
  {
    v4s bo[HB], be[HB];
    load_fold_bf16<HB>(in + base, valid, inner, n, h, g, bo, be);
    bf16_mma<HB, 0>(F, h, lane, [&](int half, int c) { return half ? be[c] : bo[c]; }, spec);
  }
#pragma unroll
  for (int k = 0; k < 2 * HB; ++k) {
    float* slot = xch[k & 1];
#pragma unroll
    for (int j = 0; j < 4; ++j) slot[((cg * NT + l) * 64 + lane) * 4 + j] = spec[k][j];
    __syncthreads();
    const int half = k / HB, kb = k % HB;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = kb * 16 + 4 * g + j;
      const bool ok = valid && (half == 0 ? rr < h : rr < h - 1);
      float acc = 0.f;
      if (ok) {
        const long long sidx = half == 0 ? rr : h + rr;
        const float* gm = G + (pos + inner * sidx) * (NT * NT);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const float v = slot[((cg * NT + m) * 64 + lane) * 4 + j];
          acc += (transpose ? gm[m * NT + l] : gm[l * NT + m]) * v;
        }
      }
      spec[k][j] = acc;
    }
  }
  v4f acc[2 * HB];
  bf16_mma<HB, 1>(F, h, lane, [&](int half, int c) {
    const v4f& s = spec[half * HB + c];
    return pack4(s[0], s[1], s[2], s[3]);
  }, acc);
  unfold_store<HB>(out + base, valid, inner, n, h, g, acc, mode, omega);
}

}  // namespace

hipError_t launch_pass_bf16(int hb, bool inverse, const float* in, float* out, const void* F, int n, long long inner,
                            long long ncols, float omega, int mode, hipStream_t s) {
  const unsigned grid = (unsigned)((ncols + 63) / 64);
  const v4s* Fv = (const v4s*)F;
#define BF_PASS(HB)                                                                                     \
  if (hb == HB) {                                                                                       \
    if (inverse)                                                                                        \
      hipLaunchKernelGGL((k_pass_bf16<HB, true>), dim3(grid), dim3(256), 0, s, in, out, Fv, n, inner, ncols, \
                         omega, mode);                                                                  \
    else                                                                                                \
      hipLaunchKernelGGL((k_pass_bf16<HB, false>), dim3(grid), dim3(256), 0, s, in, out, Fv, n, inner, ncols, \
                         omega, mode);                                                                  \
    return hipGetLastError();                                                                           \
  }
  BF_PASS(1) BF_PASS(2) BF_PASS(4) BF_PASS(8)
#undef BF_PASS
  return hipErrorInvalidValue;
}

hipError_t launch_fused_bf16(int hb, int nt, const float* in, float* out, const void* F, const float* G, int n,
                             long long inner, long long outer, int transpose, float omega, int mode, hipStream_t s) {
  const int cg = nt >= 3 ? 1 : 4 / nt;
  const unsigned grid = (unsigned)((outer * inner + 16 * cg - 1) / (16 * cg));
  const dim3 block(64 * nt * cg);
  const v4s* Fv = (const v4s*)F;
#define BF_FUSED(HB, NT)                                                                                \
  if (hb == HB && nt == NT) {                                                                           \
    hipLaunchKernelGGL((k_fused_bf16<HB, NT>), dim3(grid), block, 0, s, in, out, Fv, G, n, inner, outer, \
                       transpose, omega, mode);                                                         \
    return hipGetLastError();                                                                           \
  }
  BF_FUSED(1, 1) BF_FUSED(1, 2) BF_FUSED(1, 3) BF_FUSED(1, 4)
  BF_FUSED(2, 1) BF_FUSED(2, 2) BF_FUSED(2, 3) BF_FUSED(2, 4)
  BF_FUSED(4, 1) BF_FUSED(4, 2) BF_FUSED(4, 3) BF_FUSED(4, 4)
  BF_FUSED(8, 1) BF_FUSED(8, 2) BF_FUSED(8, 3) BF_FUSED(8, 4)
#undef BF_FUSED
  return hipErrorInvalidValue;
}

}  // namespace stmg
