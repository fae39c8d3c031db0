// fft_split.h - line FFT whose radix-8 stages run as DFT matmuls on MFMA with
// split-precision operands.
//
// Same Stockham schedule as fft_core.h (same stage radices, spans, output
// positions and twiddles), but every radix-8 stage computes its 8-point DFTs
// as D = W * X on the matrix cores: X holds 16 butterflies as columns, each
// column the 8 complex inputs interleaved (re, im), and W is the 16 x 16 real
// form of the 8-point DFT.  Operands are split so that float32 accuracy
// survives 16-bit inputs: each column is scaled by a power of two so
// |x| < 1, then
//   fp16: x = hi + lo, W = Wh + Wl, D = Wl*Xh + Wh*Xl + Wh*Xh (the lo*lo
//         term, ~2^-22, is dropped);
//   bf16: x = hi + mid + lo (three 8-bit mantissas), same for W, and the six
//         products whose order is <= 2^-16 are kept.
// All products accumulate in float32 and the power of two is undone exactly.
// Radix 2/3/4 stages stay on the vector ALUs in float32.  Twiddles are
// applied in float32 before the split.
//
// Data moves through the wavefront's LDS lines between every stage; a
// radix-8 stage reads its inputs in the matrix-core operand layout (lane
// 16g + n holds legs 2g and 2g+1 of butterflies n, 16 + n, ...), the others
// in the strided layout of fft_core.h.
#pragma once

#include "fft_core.h"

namespace psn {

enum { MODE_FP32 = 0, MODE_SPLIT_FP16 = 1, MODE_SPLIT_BF16 = 2 };

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// exp(-2 pi i k / 8) for k = 0..7 (exact trigonometric values)
__device__ __forceinline__ float2 w8(int k) {
  constexpr float r = 0.70710678118654752440f;
  const float c[8] = {1.f, r, 0.f, -r, -1.f, -r, 0.f, r};
  const float s[8] = {0.f, -r, -1.f, -r, 0.f, r, 1.f, r};
  return make_float2(c[k & 7], s[k & 7]);
}

// entry (row, col) of the 16 x 16 real form of the 8-point DFT, rows and
// columns interleaved (re, im) per leg; the inverse uses exp(+2 pi i pq / 8)
__device__ __forceinline__ float dft8_real(int row, int col, bool inv) {
  const float2 w = w8((row >> 1) * (col >> 1));
  const float c = w.x, s = inv ? -w.y : w.y;
  const bool ro = row & 1, co = col & 1;
  if (!ro && !co) return c;
  if (!ro && co) return -s;
  if (ro && !co) return s;
  return c;
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

// The DFT matrix operand of one lane, split into 2 (fp16) or 3 (bf16) parts.
template <int MODE> struct DftOperand;
template <> struct DftOperand<MODE_SPLIT_FP16> {
  half4_t hi, lo;
  __device__ void init(int lane, bool inv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float a = dft8_real(lane % 16, 4 * (lane / 16) + e, inv);
      const _Float16 h = (_Float16)a;
      hi[e] = h;
      lo[e] = (_Float16)(a - (float)h);
    }
  }
};
template <> struct DftOperand<MODE_SPLIT_BF16> {
  bf4_t hi, mid, lo;
  __device__ void init(int lane, bool inv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float a = dft8_real(lane % 16, 4 * (lane / 16) + e, inv);
      const unsigned short h = bf16_rne(a);
      const float r1 = a - bf16_to_f32(h);
      const unsigned short m = bf16_rne(r1);
      const float r2 = r1 - bf16_to_f32(m);
      hi[e] = (short)h;
      mid[e] = (short)m;
      lo[e] = (short)bf16_rne(r2);
    }
  }
};

// D = W * X for one block of 16 butterflies; x holds this lane's 4 entries
// of X (already scaled to |x| < 1).
template <int MODE>
__device__ __forceinline__ f4_t dft8_mfma(const DftOperand<MODE> &W, const float (&x)[4]) {
  f4_t acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (MODE == MODE_SPLIT_FP16) {
    half4_t xh, xl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const _Float16 h = (_Float16)x[e];
      xh[e] = h;
      xl[e] = (_Float16)(x[e] - (float)h);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(W.lo, xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(W.hi, xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(W.hi, xh, acc, 0, 0, 0);
  } else {
    bf4_t xh, xm, xl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned short h = bf16_rne(x[e]);
      const float r1 = x[e] - bf16_to_f32(h);
      const unsigned short m = bf16_rne(r1);
      const float r2 = r1 - bf16_to_f32(m);
      xh[e] = (short)h;
      xm[e] = (short)m;
      xl[e] = (short)bf16_rne(r2);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.mid, xm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.lo, xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.hi, xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.mid, xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.hi, xm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.hi, xh, acc, 0, 0, 0);
  }
  return acc;
}

// Maximum of a non-negative value over lanes l, l ^ 16, l ^ 32, l ^ 48 (one
// matrix column).  Non-negative floats order like their bit patterns, so an
// integer max needs no NaN canonicalization, and the two lane exchanges are
// the CDNA4 row swaps (VALU, no LDS crossbar): permlane32_swap pairs lane l
// with l ^ 32, permlane16_swap lane l with l ^ 16.
__device__ __forceinline__ float column_max(float v) {
  unsigned u = __float_as_uint(v);
  const auto s32 = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  u = max(s32[0], s32[1]);
  const auto s16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __uint_as_float(max(s16[0], s16[1]));
}

// Twiddle product with one fixed rounding order (one product rounded, the
// other fused).  In a matrix-core stage a line's butterflies land in a block
// chosen by the line's place in the wavefront, and every block is separate
// unrolled code; if the compiler picked the fused form per block, a line's
// result would depend on that place (a batched solve and a lone one would
// differ in the last bit).
template <bool INV> __device__ __forceinline__ float2 cmul_tw_fixed(float2 a, float2 w) {
#pragma clang fp contract(off)
  if constexpr (!INV)
    return make_float2(__builtin_fmaf(a.x, w.x, -(a.y * w.y)), __builtin_fmaf(a.x, w.y, a.y * w.x));
  else
    return make_float2(__builtin_fmaf(a.x, w.x, a.y * w.y), __builtin_fmaf(a.y, w.x, -(a.x * w.y)));
}

// Twiddles of the split transform, read from the table exp(-2 pi i n / L)
// (cached) when a stage needs them: the matrix-core path is short of
// registers, so they are not held across lines.
template <int L> struct SplitTwiddles {
  const float2 *__restrict__ tab;
  __device__ __forceinline__ void load(const float2 *__restrict__ t, int) { tab = t; }
  __device__ __forceinline__ float2 operator()(int n) const { return tab[n]; }
};

template <int MODE> struct SplitOps {
  DftOperand<MODE> fwd, inv;
  __device__ void init(int lane) {
    fwd.init(lane, false);
    inv.init(lane, true);
  }
};

// One stage, LDS to LDS.  `wl` is the wavefront's first line region; line l
// of the wavefront lives at wl + l * line_lds_slots<L>().
// ZHI: the line's upper half is zero on entry (a zero-padded line); CROP:
// only the first half of the outputs is kept.  A radix-8 stage runs on the
// matrix cores except where it touches half the data: the first stage of a
// zero-padded transform (four of eight legs are zero) and the last stage of
// a cropped one.  Those stay on the vector ALUs in float32, where they cost
// less than the split and scaling around a matrix product.
template <int L, int S, bool INV, int MODE, bool ZHI = false, bool CROP = false>
__device__ __forceinline__ void split_stage(float2 *__restrict__ wl, const SplitTwiddles<L> &tw,
                                            const SplitOps<MODE> &ops, int lane) {
  constexpr int E = Shape<L>::E, R = Shape<L>::R[S], NS = span<L>(S), T = kT<L>;
  constexpr int SLOTS = line_lds_slots<L>(), NB = L / R, STEP = L / (NS * R);
  constexpr bool HALF = (S == 0 && ZHI) || (S + 1 == Shape<L>::NR && CROP);
  if constexpr (R == 8 && !HALF) {
    const int gq = lane / 16, n = lane % 16;
    float x[E / 2][4];
    int line[E / 2], jj[E / 2];
    float cmax[E / 2];
#pragma unroll
    for (int b = 0; b < E / 2; ++b) {
      const int beta = 16 * b + n;
      line[b] = beta / NB;
      jj[b] = beta % NB;
      const float2 *src = wl + line[b] * SLOTS;
      cmax[b] = 0.f;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float2 a = src[lds_pad(jj[b] + (2 * gq + u) * NB)];
        if constexpr (S > 0) a = cmul_tw_fixed<INV>(a, tw((jj[b] % NS) * (2 * gq + u) * STEP));
        x[b][2 * u] = a.x;
        x[b][2 * u + 1] = a.y;
        // |x| as bits: non-negative floats order like unsigned integers
        const unsigned ax = __float_as_uint(a.x) & 0x7fffffffu, ay = __float_as_uint(a.y) & 0x7fffffffu;
        cmax[b] = __uint_as_float(max(__float_as_uint(cmax[b]), max(ax, ay)));
      }
    }
    wave_lds_fence();  // all inputs read before outputs overwrite them
#pragma unroll
    for (int b = 0; b < E / 2; ++b) {
      // one power of two per butterfly (matrix column): its 16 entries sit
      // in lanes n, n + 16, n + 32, n + 48; left products by W commute with
      // column scaling, so the scale is undone exactly on the output column
      const float m = column_max(cmax[b]);
      int e2;
      (void)frexpf(m, &e2);  // |x| * 2^-e2 < 1
      // keep both factors finite: columns below 2^-100 (denormal tails of a
      // density) are scaled only by 2^100 and stay far below fp16 resolution
      e2 = max(e2, -100);
      const float down = ldexpf(1.f, -e2), up = ldexpf(1.f, e2);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[b][e] *= down;
      const f4_t d = dft8_mfma<MODE>(INV ? ops.inv : ops.fwd, x[b]);
      float2 *dst = wl + line[b] * SLOTS;
      const int j = jj[b];
      const int base = (j / NS) * NS * 8 + (j % NS);
#pragma unroll
      for (int u = 0; u < 2; ++u)
        dst[lds_pad(base + (2 * gq + u) * NS)] = make_float2(d[2 * u] * up, d[2 * u + 1] * up);
    }
  } else {
    constexpr int B = E / R;
    const int g = lane / T, t = lane % T;
    float2 *ln = wl + g * SLOTS;
    float2 v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = ln[lds_pad(t + T * i)];
    wave_lds_fence();
#pragma unroll
    for (int b = 0; b < B; ++b) {
      float2 a[R];
#pragma unroll
      for (int m = 0; m < R; ++m) a[m] = v[b + m * B];
      const int j = t + T * b;
      if constexpr (S > 0) {
#pragma unroll
        for (int m = 1; m < R; ++m) a[m] = cmul_tw<INV>(a[m], tw((j % NS) * m * STEP));
      }
      dft<R, INV, ZHI && S == 0>(a);
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int m = 0; m < R; ++m) ln[lds_pad(base + m * NS)] = a[m];
    }
  }
  wave_lds_fence();
  if constexpr (S + 1 < Shape<L>::NR) split_stage<L, S + 1, INV, MODE, ZHI, CROP>(wl, tw, ops, lane);
}

// Transform of the wavefront's LPW lines.  v holds lane t's strided elements
// of its line (as in fft_line); `wl` is the wavefront's LDS line block.
template <int L, bool INV, int MODE, bool ZHI = false, bool CROP = false>
__device__ __forceinline__ void fft_line_split(float2 (&v)[Shape<L>::E], const SplitTwiddles<L> &tw,
                                               const SplitOps<MODE> &ops, float2 *__restrict__ wl,
                                               int lane) {
  constexpr int E = Shape<L>::E, T = kT<L>, SLOTS = line_lds_slots<L>();
  float2 *ln = wl + (lane / T) * SLOTS;
  const int t = lane % T;
#pragma unroll
  for (int i = 0; i < E; ++i) ln[lds_pad(t + T * i)] = v[i];
  wave_lds_fence();
  split_stage<L, 0, INV, MODE, ZHI, CROP>(wl, tw, ops, lane);
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = ln[lds_pad(t + T * i)];
  wave_lds_fence();
}

}  // namespace psn
