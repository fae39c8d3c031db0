// fft_core.h - register/LDS Stockham FFT of one line held by T lanes.
//
// The 1D transforms of the customized 3D FFT (paper, Section 3) are batched
// FFTs along one axis.  Here a line of length L is held by T = L/E lanes of
// one wavefront, lane t owning the E elements x[t + T*i], i = 0..E-1.  Each
// radix-R stage does E/R butterflies per lane entirely in registers (the
// "strided" element set of a lane is exactly the input set of its
// butterflies), then the lanes exchange results through the line's LDS
// region.  The last stage needs no exchange: its outputs land in natural
// order, lane t holding X[t + T*i].  All exchanges stay inside one wavefront,
// so no workgroup barrier is needed between stages.
//
// Zero padding (Section 3: the second half of a free axis is zero before its
// transform) is known at compile time: elements i >= E/2 are never loaded,
// and the first stage uses butterflies without their zero legs (ZHI).
// Likewise, outputs a caller never stores (the crop after an inverse
// transform) are dead code.
#pragma once

#include <hip/hip_runtime.h>

namespace psn {

// ------------------------------------------------------------------ shapes
// Per FFT length L: E elements per lane and the radix of each stage.  Every
// radix divides E, and T = L / E is a power of two <= 64 (a line group never
// spans two wavefronts).
template <int L> struct Shape;
#define PSN_SHAPE(LL, EE, NRR, ...)                                          \
  template <> struct Shape<LL> {                                             \
    static constexpr int E = EE, NR = NRR;                                   \
    static constexpr int R[6] = {__VA_ARGS__};                               \
  };
PSN_SHAPE(4, 4, 1, 4)
PSN_SHAPE(6, 6, 2, 3, 2)
PSN_SHAPE(8, 8, 1, 8)
PSN_SHAPE(12, 12, 2, 4, 3)
PSN_SHAPE(16, 8, 2, 8, 2)
PSN_SHAPE(24, 24, 2, 8, 3)
PSN_SHAPE(32, 8, 2, 8, 4)
PSN_SHAPE(48, 24, 3, 8, 3, 2)
PSN_SHAPE(64, 8, 2, 8, 8)
PSN_SHAPE(96, 24, 3, 8, 4, 3)
PSN_SHAPE(128, 8, 3, 8, 8, 2)
PSN_SHAPE(192, 24, 3, 8, 8, 3)
PSN_SHAPE(256, 8, 3, 8, 8, 4)
PSN_SHAPE(384, 24, 4, 8, 8, 3, 2)
PSN_SHAPE(512, 8, 3, 8, 8, 8)
PSN_SHAPE(768, 24, 4, 8, 8, 4, 3)
PSN_SHAPE(1024, 16, 4, 8, 8, 4, 4)
#undef PSN_SHAPE

template <int L> constexpr int kT = L / Shape<L>::E;
// span NS of stage s: product of the radices before it
template <int L> constexpr int span(int s) {
  int p = 1;
  for (int u = 0; u < s; ++u) p *= Shape<L>::R[u];
  return p;
}
constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
// Lane t's butterfly b of stage s has twiddle index k = (t + T b) mod NS.
// Butterflies b and b + P, P = NS / gcd(T, NS), differ by a multiple of
// lcm(T, NS) and so share their twiddles: a lane holds only the first
// min(B, P) butterflies' sets.
template <int L> constexpr int tw_period(int s) {
  const int ns = span<L>(s);
  return ns / cgcd(kT<L>, ns);
}
template <int L> constexpr int tw_sets(int s) {
  const int b = Shape<L>::E / Shape<L>::R[s], p = tw_period<L>(s);
  return b < p ? b : p;
}
// register offset of stage s's twiddles (stage 0 has none)
template <int L> constexpr int tw_offset(int s) {
  int o = 0;
  for (int u = 1; u < s; ++u) o += tw_sets<L>(u) * (Shape<L>::R[u] - 1);
  return o;
}
template <int L> constexpr int tw_count() { return tw_offset<L>(Shape<L>::NR) > 0 ? tw_offset<L>(Shape<L>::NR) : 1; }

// LDS exchange region of one line: float2 slots with one pad slot per 16
// (breaks the power-of-two strides of the Stockham scatter across banks)
__host__ __device__ constexpr int lds_pad(int o) { return o + (o >> 4); }
template <int L> constexpr int line_lds_slots() { return lds_pad(L - 1) + 1; }

// --------------------------------------------------------------- complex ops
// Rounding is fixed in the source: the compiler contracts nothing in this
// file (fp contract off), and the products that should fuse are written as
// fmaf.  A line's result then does not depend on which kernel inlines its
// transform or where (the plane kernel and the separate passes, a batched
// launch and a lone one, every tile schedule give identical bits).
#pragma clang fp contract(off)
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * w (forward) or a * conj(w) (inverse): one product rounded, one fused
template <bool INV> __device__ __forceinline__ float2 cmul_tw(float2 a, float2 w) {
  if constexpr (!INV)
    return make_float2(__builtin_fmaf(a.x, w.x, -(a.y * w.y)), __builtin_fmaf(a.x, w.y, a.y * w.x));
  else
    return make_float2(__builtin_fmaf(a.x, w.x, a.y * w.y), __builtin_fmaf(a.y, w.x, -(a.x * w.y)));
}
// multiply by -i (forward) or +i (inverse)
template <bool INV> __device__ __forceinline__ float2 mul_mi(float2 a) {
  if constexpr (!INV) return make_float2(a.y, -a.x);
  else return make_float2(-a.y, a.x);
}

// ------------------------------------------------------------ small DFTs
// Forward kernels use exp(-2 pi i jk / R), inverse exp(+2 pi i jk / R).
// ZHI: the upper half of the inputs (a[R/2..R-1]) is known to be zero, as in
// the first stage of a transform of a zero-padded line.  Adding a literal
// zero does not fold away in IEEE arithmetic (-0 + 0 = +0), so the first
// radix-2 split is written out as copies instead.
template <bool INV, bool ZHI = false> __device__ __forceinline__ void dft2(float2 *a) {
  if constexpr (ZHI) {
    a[1] = a[0];
  } else {
    float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
}

template <bool INV> __device__ __forceinline__ void dft3(float2 *a) {
  constexpr float c = 0.86602540378443864676f;  // sqrt(3)/2
  float2 s = cadd(a[1], a[2]);
  float2 d = csub(a[1], a[2]);
  float2 m = make_float2(__builtin_fmaf(-0.5f, s.x, a[0].x), __builtin_fmaf(-0.5f, s.y, a[0].y));
  // forward: X1 = m - i c d, X2 = m + i c d (i c d = (-c d.y, c d.x))
  const float2 p = make_float2(__builtin_fmaf(c, d.y, m.x), __builtin_fmaf(-c, d.x, m.y));  // m - i c d
  const float2 q = make_float2(__builtin_fmaf(-c, d.y, m.x), __builtin_fmaf(c, d.x, m.y));  // m + i c d
  a[0] = cadd(a[0], s);
  if constexpr (!INV) { a[1] = p; a[2] = q; }
  else { a[1] = q; a[2] = p; }
}

template <bool INV, bool ZHI = false> __device__ __forceinline__ void dft4(float2 *a) {
  float2 d0, d1, d2, d3;
  if constexpr (ZHI) {
    d0 = d2 = a[0];
    d1 = a[1];
    d3 = mul_mi<INV>(a[1]);
  } else {
    d0 = cadd(a[0], a[2]);
    d2 = csub(a[0], a[2]);
    d1 = cadd(a[1], a[3]);
    d3 = mul_mi<INV>(csub(a[1], a[3]));
  }
  a[0] = cadd(d0, d1);
  a[2] = csub(d0, d1);
  a[1] = cadd(d2, d3);
  a[3] = csub(d2, d3);
}

template <bool INV, bool ZHI = false> __device__ __forceinline__ void dft8(float2 *a) {
  constexpr float r = 0.70710678118654752440f;
  // radix-2 split between a[m] and a[m+4]
  float2 b0, b1, b2, b3, b4, b5, b6, b7;
  if constexpr (ZHI) {
    b0 = b4 = a[0];
    b1 = b5 = a[1];
    b2 = b6 = a[2];
    b3 = b7 = a[3];
  } else {
    b0 = cadd(a[0], a[4]); b4 = csub(a[0], a[4]);
    b1 = cadd(a[1], a[5]); b5 = csub(a[1], a[5]);
    b2 = cadd(a[2], a[6]); b6 = csub(a[2], a[6]);
    b3 = cadd(a[3], a[7]); b7 = csub(a[3], a[7]);
  }
  // odd half times w8^m (forward w8 = (1-i)/sqrt2)
  if constexpr (!INV) {
    b5 = make_float2(r * (b5.x + b5.y), r * (b5.y - b5.x));
    b6 = make_float2(b6.y, -b6.x);
    b7 = make_float2(r * (b7.y - b7.x), -r * (b7.x + b7.y));
  } else {
    b5 = make_float2(r * (b5.x - b5.y), r * (b5.x + b5.y));
    b6 = make_float2(-b6.y, b6.x);
    b7 = make_float2(-r * (b7.x + b7.y), r * (b7.x - b7.y));
  }
  float2 e[4] = {b0, b1, b2, b3};
  float2 o[4] = {b4, b5, b6, b7};
  dft4<INV>(e);
  dft4<INV>(o);
  a[0] = e[0]; a[2] = e[1]; a[4] = e[2]; a[6] = e[3];
  a[1] = o[0]; a[3] = o[1]; a[5] = o[2]; a[7] = o[3];
}

// ZHI is used by the even radices; an odd radix ignores it (its zero inputs
// do not fall in one half of the butterfly).
template <int R, bool INV, bool ZHI = false> __device__ __forceinline__ void dft(float2 *a) {
  if constexpr (R == 2) dft2<INV, ZHI>(a);
  else if constexpr (R == 3) dft3<INV>(a);
  else if constexpr (R == 4) dft4<INV, ZHI>(a);
  else if constexpr (R == 8) dft8<INV, ZHI>(a);
  else static_assert(R == 2, "unsupported radix");
}

// Make LDS writes of this wavefront visible to its other lanes.  LDS
// operations of one wavefront execute in order; the fence keeps the compiler
// from moving accesses across the exchange point.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// -------------------------------------------------------------- twiddles
// Lane t's twiddles for every twiddled stage, loaded once from the table
// tab[n] = exp(-2 pi i n / L) (float64-computed, rounded once).
template <int L> struct Twiddles {
  float2 w[tw_count<L>()];

  __device__ __forceinline__ void load(const float2 *__restrict__ tab, int t) {
    load_stage<1>(tab, t);
  }
  template <int S> __device__ __forceinline__ void load_stage(const float2 *__restrict__ tab, int t) {
    if constexpr (S < Shape<L>::NR) {
      constexpr int R = Shape<L>::R[S], NS = span<L>(S);
      constexpr int T = kT<L>, STEP = L / (NS * R), OFF = tw_offset<L>(S), D = tw_sets<L>(S);
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const int k = (t + T * b) % NS;
#pragma unroll
        for (int m = 1; m < R; ++m) w[OFF + b * (R - 1) + (m - 1)] = tab[k * m * STEP];
      }
      load_stage<S + 1>(tab, t);
    }
  }
};

// ----------------------------------------------------------- the line FFT
// ZHI: elements i >= E/2 of every lane are zero on entry (a zero-padded line).
// In the first stage butterfly b reads v[b + m B], m = 0..R-1, with E = R B,
// so its zero legs are exactly m >= R/2.
template <int L, int S, bool INV, bool ZHI = false>
__device__ __forceinline__ void fft_stage(float2 (&v)[Shape<L>::E], const Twiddles<L> &tw,
                                          float2 *__restrict__ lds, int t) {
  constexpr int E = Shape<L>::E, R = Shape<L>::R[S], B = E / R, NS = span<L>(S), T = kT<L>;
  constexpr int OFF = tw_offset<L>(S), P = tw_period<L>(S);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    float2 a[R];
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = v[b + m * B];
    if constexpr (S > 0) {
#pragma unroll
      for (int m = 1; m < R; ++m) a[m] = cmul_tw<INV>(a[m], tw.w[OFF + (b % P) * (R - 1) + (m - 1)]);
    }
    dft<R, INV, ZHI && S == 0>(a);
#pragma unroll
    for (int m = 0; m < R; ++m) v[b + m * B] = a[m];
  }
  if constexpr (S + 1 < Shape<L>::NR) {
    // Stockham scatter: butterfly j = t + T b, leg m goes to
    // (j / NS) * NS * R + j % NS + m * NS
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + T * b;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int m = 0; m < R; ++m) lds[lds_pad(base + m * NS)] = v[b + m * B];
    }
    wave_lds_fence();
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = lds[lds_pad(t + T * i)];
    wave_lds_fence();
    fft_stage<L, S + 1, INV>(v, tw, lds, t);
  }
}

// Full forward (INV = false) or unnormalized inverse transform of the line
// held by lanes t = 0..T-1 of this line group; lds is the group's region of
// line_lds_slots<L>() float2.
template <int L, bool INV, bool ZHI = false>
__device__ __forceinline__ void fft_line(float2 (&v)[Shape<L>::E], const Twiddles<L> &tw,
                                         float2 *__restrict__ lds, int t) {
  fft_stage<L, 0, INV, ZHI>(v, tw, lds, t);
}

}  // namespace psn
