// fft_mfma.h - split-precision line FFT as two dense DFT products on the
// matrix cores (gfx950 v_mfma_f32_16x16x32_{f16,bf16}).
//
// A line of length L = 16 B is the 16 x B array x[n0 + 16 n1] and its DFT is
// taken in two factors (Cooley-Tukey, four-step form):
//   F0: DFT_B over n1 for every n0          Y[n0][k1]
//       twiddle w_L^(n0 k1)
//   F1: DFT_16 over n0 for every k1         X[k1 + B k0]
// Each factor is a real matrix product on the matrix cores.  The data of a
// factor sits in the operand that puts its contraction index in the K
// dimension: F0 takes the data as the A operand (columns n0 in the lanes),
// F1 as the B operand.  A matrix core writes D[i][j] to lane j + 16 (i/4),
// register i%4, which is exactly where the B operand of the next product
// wants row i: so F0's output is F1's input as it stands, and no lane
// exchange happens between the two factors.  The inverse mirrors this
// (I0: DFT_16 with the data as A, I1: DFT_B with the data as B), and the
// forward output is the inverse input, so the fused forward x K^F x inverse
// of the convolution pass keeps everything in registers.
//
// Operand layouts of the 16x16x32 products (checked with an in-bounds probe
// on gfx950): A[i][k] at lane i + 16 (k/8), element k%8; B[k][j] at lane
// j + 16 (k/8), element k%8; D[i][j] at lane j + 16 (i/4), element i%4.
// K = 32 reals = 16 complex legs (re, im interleaved).  Lengths with B < 16
// pack 16/BS lines per product with a block-diagonal DFT_B (BS = B rounded
// up to a power of two; slots B..BS-1 of a block are unused); B = 24 and 32
// use two K blocks.  So every L = 16 B with B in {2, 3, 4, 6, 8, 12, 16, 24,
// 32} (32 ... 512) runs here.
//
// Complex products with real matrices: the real part of W x takes the
// matrix with entries (Re w, -Im w) against (Re x, Im x); the imaginary part
// is the real part of W (-i x), so one operand serves both and -i x is a
// swap and a sign of the split halves.  The inverse uses the forward matrix
// through conj(W conj(x)).
//
// Precision: each product is split so that float32 accuracy survives 16-bit
// operands, with float32 accumulation.
//   fp16: every line is scaled by one power of two so its largest value
//         lies in [2^9, 2^10) (no factor then leaves the fp16 range), and
//         x = hi + lo, W = Wh + Wl, D = Wh hi + Wh lo + Wl hi.  Keeping the
//         values near 2^10 keeps lo in the normal range for everything
//         within 12 binades of the line maximum; below that the error is
//         under 2^-35 of the maximum.
//   bf16: x = hi + mid + lo (three 8-bit mantissas), the same for W, and
//         the six products of order >= 2^-16 are kept; bf16 has the float32
//         exponent range, so no scaling is needed.
// Twiddles and the K^F product stay float32 on the vector ALUs.
#pragma once

#include "fft_core.h"
#include "fft_split.h"

namespace psn {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

// Lengths the matrix-core engine covers.
template <int L> constexpr bool mfma_length() {
  return L >= 32 && L <= 512 && L % 16 == 0 &&
         (L / 16 == 2 || L / 16 == 3 || L / 16 == 4 || L / 16 == 6 || L / 16 == 8 ||
          L / 16 == 12 || L / 16 == 16 || L / 16 == 24 || L / 16 == 32);
}

template <int L> struct MfmaGeo {
  static constexpr int B = L / 16;
  static constexpr int BS = pow2_ceil(B);              // slot stride of one line
  static constexpr int P = BS <= 16 ? 16 / BS : 1;     // lines per product block
  static constexpr int KB = BS > 16 ? BS / 16 : 1;     // K blocks (and column blocks)
  static constexpr int LPW = 64 / kT<L>;               // lines per wavefront
  static constexpr int NB = LPW / P;                   // product blocks per wavefront
  static constexpr int SLOTS = line_lds_slots<L>();
  static_assert(NB * P == LPW, "lines per wavefront must fill whole blocks");
};

// ------------------------------------------------------ split operands
// fp16 parts are held as packed pairs (one 32-bit register per complex leg:
// re in the low half, im in the high half).
typedef unsigned u4_t __attribute__((ext_vector_type(4)));
template <int MODE> struct MOp;
template <> struct MOp<MODE_SPLIT_FP16> {
  u4_t hi, lo;
};
template <> struct MOp<MODE_SPLIT_BF16> {
  u4_t hi, mid, lo;
};

// One complex leg times the power of two sc, split into packed fp16 parts:
// hi = RNE(x sc), lo = RNE(x sc - hi), both products and the difference
// exact inside the mixed-precision FMA.  CONJ negates the imaginary part.
template <bool CONJ> __device__ __forceinline__ void split_leg(float re, float im, float sc, unsigned &hi, unsigned &lo) {
  if constexpr (!CONJ)
    asm("v_fma_mixlo_f16 %0, %2, %4, 0\n\t"
        "v_fma_mixhi_f16 %0, %3, %4, 0\n\t"
        "v_fma_mixlo_f16 %1, %2, %4, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, %3, %4, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(hi), "=&v"(lo)
        : "v"(re), "v"(im), "v"(sc));
  else
    asm("v_fma_mixlo_f16 %0, %2, %4, 0\n\t"
        "v_fma_mixhi_f16 %0, -%3, %4, 0\n\t"
        "v_fma_mixlo_f16 %1, %2, %4, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, -%3, %4, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(hi), "=&v"(lo)
        : "v"(re), "v"(im), "v"(sc));
}
// The same split with no scale (sc = 1): hi by one packed conversion.
template <bool CONJ> __device__ __forceinline__ void split_leg1(float re, float im, unsigned &hi, unsigned &lo) {
  if constexpr (!CONJ)
    asm("v_cvt_pk_f16_f32 %0, %2, %3\n\t"
        "v_fma_mixlo_f16 %1, 1.0, %2, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, 1.0, %3, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(hi), "=&v"(lo)
        : "v"(re), "v"(im));
  else
    asm("v_cvt_pk_f16_f32 %0, %2, -%3\n\t"
        "v_fma_mixlo_f16 %1, 1.0, %2, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, 1.0, -%3, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(hi), "=&v"(lo)
        : "v"(re), "v"(im));
}
// -i times a packed leg: (re, im) -> (im, -re), exact
__device__ __forceinline__ unsigned rot_leg(unsigned v) {
  unsigned r;
  asm("v_pk_add_f16 %0, %1, 0 op_sel:[1,0] op_sel_hi:[0,0] neg_hi:[1,0]" : "=v"(r) : "v"(v));
  return r;
}

// One complex leg split into packed bf16 parts x = hi + mid + lo (each
// part the round-to-nearest-even bf16 of what the earlier parts leave,
// exact float32 differences), together with the parts of -i x, made from
// (im, -re) by the same conversions.  CONJ negates the imaginary part.
template <bool CONJ>
__device__ __forceinline__ void split_leg_bf16(float re, float im, unsigned &h, unsigned &m, unsigned &l,
                                               unsigned &rh, unsigned &rm, unsigned &rl) {
  unsigned r1a, r1b, r2a, r2b;
  if constexpr (CONJ) im = -im;
  asm("v_cvt_pk_bf16_f32 %0, %10, %11\n\t"
      "v_cvt_pk_bf16_f32 %3, %11, -%10\n\t"
      "v_lshlrev_b32 %6, 16, %0\n\t"
      "v_and_b32 %7, 0xffff0000, %0\n\t"
      "v_sub_f32 %6, %10, %6\n\t"
      "v_sub_f32 %7, %11, %7\n\t"
      "v_cvt_pk_bf16_f32 %1, %6, %7\n\t"
      "v_cvt_pk_bf16_f32 %4, %7, -%6\n\t"
      "v_lshlrev_b32 %8, 16, %1\n\t"
      "v_and_b32 %9, 0xffff0000, %1\n\t"
      "v_sub_f32 %8, %6, %8\n\t"
      "v_sub_f32 %9, %7, %9\n\t"
      "v_cvt_pk_bf16_f32 %2, %8, %9\n\t"
      "v_cvt_pk_bf16_f32 %5, %9, -%8"
      : "=&v"(h), "=&v"(m), "=&v"(l), "=&v"(rh), "=&v"(rm), "=&v"(rl), "=&v"(r1a), "=&v"(r1b),
        "=&v"(r2a), "=&v"(r2b)
      : "v"(re), "v"(im));
}

// The matrix cores read their A and B operands a few cycles after issue,
// and a vector-ALU write shortly before can be missed.  The compiler inserts
// the wait states for its own instructions but cannot see which registers
// the inline assembly above writes, so every finished operand passes
// through this fence: a wait whose in/out operands are the operand
// registers, so every matrix product that reads them comes after it (by
// data dependence: the fence is not volatile and does not hold back other
// instructions).
// (Without it, schedules under high register pressure read stale operand
// halves: the length-384 inverse passes went wrong by up to 1e-2.)
template <int MODE> __device__ __forceinline__ void operand_fence(MOp<MODE> &o) {
  if constexpr (MODE == MODE_SPLIT_FP16)
    asm("s_nop 2" : "+v"(o.hi), "+v"(o.lo));
  else
    asm("s_nop 2" : "+v"(o.hi), "+v"(o.mid), "+v"(o.lo));
}

// Operand of 4 complex legs (times sc, conjugated for the inverse trick) and
// the operand of -i times the same legs.
template <int MODE, bool CONJ, bool UNSCALED = false>
__device__ __forceinline__ void make_operands(const float2 (&c)[4], const float (&sc)[4], MOp<MODE> &o,
                                              MOp<MODE> &r) {
  if constexpr (MODE == MODE_SPLIT_FP16) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      unsigned h, lo;
      if constexpr (UNSCALED) split_leg1<CONJ>(c[l].x, c[l].y, h, lo);
      else split_leg<CONJ>(c[l].x, c[l].y, sc[l], h, lo);
      o.hi[l] = h;
      o.lo[l] = lo;
    }
    // the products of o may start while the rotation is formed
    operand_fence<MODE>(o);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      r.hi[l] = rot_leg(o.hi[l]);
      r.lo[l] = rot_leg(o.lo[l]);
    }
    operand_fence<MODE>(r);
  } else {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      unsigned h, m, lo, rh, rm, rl;
      split_leg_bf16<CONJ>(c[l].x, c[l].y, h, m, lo, rh, rm, rl);
      o.hi[l] = h;
      o.mid[l] = m;
      o.lo[l] = lo;
      r.hi[l] = rh;
      r.mid[l] = rm;
      r.lo[l] = rl;
    }
    operand_fence<MODE>(o);
    operand_fence<MODE>(r);
  }
}
template <int MODE, bool CONJ>
__device__ __forceinline__ MOp<MODE> make_operand(const float2 (&c)[4]) {
  MOp<MODE> o, r;
  const float one[4] = {1.f, 1.f, 1.f, 1.f};
  make_operands<MODE, CONJ, true>(c, one, o, r);
  return o;
}

// acc += (data as A) x (W as B), or (W as A) x (data as B): the split
// products, small terms first.
template <int MODE, bool DATA_A>
__device__ __forceinline__ f4_t mprod(const MOp<MODE> &d, const MOp<MODE> &w, f4_t acc) {
  if constexpr (MODE == MODE_SPLIT_FP16) {
    const h8_t dh = __builtin_bit_cast(h8_t, d.hi), dl = __builtin_bit_cast(h8_t, d.lo);
    const h8_t wh = __builtin_bit_cast(h8_t, w.hi), wl = __builtin_bit_cast(h8_t, w.lo);
    if constexpr (DATA_A) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(dl, wh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(dh, wl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(dh, wh, acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, dl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wl, dh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, dh, acc, 0, 0, 0);
    }
  } else {
    const bf8_t dh = __builtin_bit_cast(bf8_t, d.hi), dm = __builtin_bit_cast(bf8_t, d.mid),
                dl = __builtin_bit_cast(bf8_t, d.lo);
    const bf8_t wh = __builtin_bit_cast(bf8_t, w.hi), wm = __builtin_bit_cast(bf8_t, w.mid),
                wl = __builtin_bit_cast(bf8_t, w.lo);
    if constexpr (DATA_A) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dl, wh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dm, wm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, wl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dm, wh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, wm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dh, wh, acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, dl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, dm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, dh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, dm, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, dh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, dh, acc, 0, 0, 0);
    }
  }
  return acc;
}

// ------------------------------------------------------------ scaling
// fp16 scaling is per line: a line's exponent comes from its own largest
// |value|, so its result does not depend on the lines that share its
// product block (a batched solve equals a lone one bit for bit).  The
// reductions follow each layout's line map; non-negative floats order like
// their bit patterns, so they run on integers.
template <int CTRL> __device__ __forceinline__ unsigned dpp_max(unsigned u) {
  return max(u, (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xf, 0xf, false));
}
// max within aligned segments of N lanes of every row of 16
template <int N> __device__ __forceinline__ unsigned seg_max(unsigned u) {
  if constexpr (N >= 2) u = dpp_max<0xB1>(u);   // quad_perm [1,0,3,2]
  if constexpr (N >= 4) u = dpp_max<0x4E>(u);   // quad_perm [2,3,0,1]
  if constexpr (N >= 8) u = dpp_max<0x141>(u);  // row_half_mirror
  if constexpr (N >= 16) u = dpp_max<0x140>(u); // row_mirror
  return u;
}
// max over row pairs (0,1), (2,3) and over all four rows (CDNA4 row swaps)
__device__ __forceinline__ unsigned rowpair_max(unsigned u) {
  const auto s16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return max(s16[0], s16[1]);
}
__device__ __forceinline__ unsigned allrows_max(unsigned u) {
  const auto s32 = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return rowpair_max(max(s32[0], s32[1]));
}
// exponent s that brings max |x| (as bits) into [2^9, 2^10); 0 for zero
__device__ __forceinline__ int scale_of(unsigned u) {
  const int s = 136 - int(u >> 23);  // biased exponent E: 9 - (E - 127)
  return u == 0 ? 0 : (s < 127 ? s : 127);
}
// 2^s as a float, -126 <= s <= 127
__device__ __forceinline__ float pow2f(int s) { return __uint_as_float(unsigned(127 + s) << 23); }
__device__ __forceinline__ unsigned absmax2(float2 v) {
  return __float_as_uint(fmaxf(fabsf(v.x), fabsf(v.y)));
}
__device__ __forceinline__ int lane_value(int v, int src_lane) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

template <int L, int MODE> struct MfmaLine {
  using G = MfmaGeo<L>;
  static constexpr int B = G::B, BS = G::BS, P = G::P, KB = G::KB, NB = G::NB;
  static constexpr int SLOTS = G::SLOTS, T = kT<L>, E = Shape<L>::E;
  static constexpr bool SCALED = MODE == MODE_SPLIT_FP16;

  MOp<MODE> wb[KB][KB];  // block (a, b) of the block-diagonal DFT_B
  MOp<MODE> w16;         // DFT_16
  const float2 *__restrict__ tab;

  // lane (g, jl) holds W[jl + 16 a][4 g + lam + 16 b], lam = 0..3, as
  // (Re w, -Im w) of the forward matrix, split
  __device__ void init(const float2 *t, int lane) {
    tab = t;
    const int g = lane >> 4, jl = lane & 15;
#pragma unroll
    for (int a = 0; a < KB; ++a)
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        float2 c[4];
#pragma unroll
        for (int lam = 0; lam < 4; ++lam) {
          const int row = jl + 16 * a, col = 4 * g + lam + 16 * b;
          const int rl = row / BS, k = row % BS, cl = col / BS, m = col % BS;
          float2 w = make_float2(0.f, 0.f);
          if (rl == cl && k < B && m < B) w = t[(16 * k * m) % L];
          c[lam] = w;
        }
        wb[a][b] = make_operand<MODE, true>(c);  // (Re w, -Im w)
      }
    float2 c[4];
#pragma unroll
    for (int lam = 0; lam < 4; ++lam) c[lam] = t[(B * jl * (4 * g + lam)) % L];
    w16 = make_operand<MODE, true>(c);
  }

  // ---------------------------------------------------- line scales
  // Exponents per register, for fp16 (0 in bf16).  The forward input (and
  // the inverse output) has element (k, l) of lane (g, jl) in line
  // (4 g + l + 16 k) / BS; the spectrum has it in line (jl + 16 k) / BS.
  template <int NK> __device__ __forceinline__ static void in_scales(const float2 (&x)[KB][4], int (&s)[KB][4]) {
    if constexpr (!SCALED) {
      fill(s, 0);
    } else if constexpr (BS == 2) {  // lines 2g (legs 0, 1) and 2g + 1 (legs 2, 3)
      const int s0 = scale_of(seg_max<16>(max(absmax2(x[0][0]), absmax2(x[0][1]))));
      const int s1 = scale_of(seg_max<16>(max(absmax2(x[0][2]), absmax2(x[0][3]))));
      s[0][0] = s[0][1] = s0;
      s[0][2] = s[0][3] = s1;
    } else {
      unsigned m = 0;
#pragma unroll
      for (int k = 0; k < NK; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) m = max(m, absmax2(x[k][l]));
      m = seg_max<16>(m);                      // line g / (BS/4) spans BS/4 rows
      if constexpr (BS == 8) m = rowpair_max(m);
      // one line per block: the exponent is wavefront-uniform (scalar)
      if constexpr (BS >= 16) m = __builtin_amdgcn_readfirstlane(allrows_max(m));
      fill(s, scale_of(m));
    }
  }
  __device__ __forceinline__ static void spec_scales(const float2 (&x)[KB][4], int (&s)[KB][4]) {
    if constexpr (!SCALED) {
      fill(s, 0);
    } else {
      unsigned m = 0;
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) m = max(m, absmax2(x[k][l]));
      m = allrows_max(seg_max<(BS < 16 ? BS : 16)>(m));
      if constexpr (P == 1) m = __builtin_amdgcn_readfirstlane(m);
      fill(s, scale_of(m));
    }
  }
  // the forward input exponents moved to the spectrum layout: lane (g, jl)
  // needs line jl / BS, whose exponent rows BS (jl / BS) / 4 .. hold
  __device__ __forceinline__ static void in_to_spec(const int (&si)[KB][4], int (&ss)[KB][4], int lane) {
    if constexpr (!SCALED || P == 1) {
      fill(ss, si[0][0]);
    } else {
      const int ls = (lane & 15) / BS, src = 16 * ((ls * BS) / 4);
      int v;
      if constexpr (BS == 2) {
        const int a = lane_value(si[0][0], src), b = lane_value(si[0][2], src);
        v = (ls & 1) ? b : a;
      } else {
        v = lane_value(si[0][0], src);
      }
      fill(ss, v);
    }
  }
  // the spectrum exponents moved to the inverse output layout: element
  // (k, e) of lane (g, jl) is in line (4 g + e) / BS, whose exponent lane
  // BS * line holds
  __device__ __forceinline__ static void spec_to_out(const int (&ss)[KB][4], int (&so)[KB][4], int lane) {
    if constexpr (!SCALED || P == 1) {
      fill(so, ss[0][0]);
    } else if constexpr (BS == 2) {
      const int g = lane >> 4;
      const int a = lane_value(ss[0][0], 4 * g), b = lane_value(ss[0][0], 4 * g + 2);
      so[0][0] = so[0][1] = a;
      so[0][2] = so[0][3] = b;
    } else {
      const int ls = (4 * (lane >> 4)) / BS;
      fill(so, lane_value(ss[0][0], ls * BS));
    }
  }
  __device__ __forceinline__ static void fill(int (&s)[KB][4], int v) {
#pragma unroll
    for (int k = 0; k < KB; ++k)
#pragma unroll
      for (int l = 0; l < 4; ++l) s[k][l] = v;
  }
  __device__ __forceinline__ static void factors(const int (&s)[KB][4], int k, float (&f)[4]) {
#pragma unroll
    for (int l = 0; l < 4; ++l) f[l] = SCALED ? pow2f(s[k][l]) : 1.f;
  }
  // x times 2^-s per register
  __device__ __forceinline__ static void unscale(float2 (&c)[KB][4], const int (&s)[KB][4]) {
    if constexpr (SCALED) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int l = 0; l < 4; ++l)
          c[kb][l] = make_float2(ldexpf(c[kb][l].x, -s[kb][l]), ldexpf(c[kb][l].y, -s[kb][l]));
    }
  }

  // ---------------------------------------------------------- forward
  // in: x[kb][lam] = element jl + 16 n1 of line lam_full / BS, lam_full =
  // 4 g + lam + 16 kb, n1 = lam_full % BS.  out: X[cb][e] = element
  // k1 + B (4 g + e) of line slot / BS, slot = jl + 16 cb, k1 = slot % BS,
  // times 2^s (s returned; 0 in bf16).
  template <bool ZHI>
  __device__ __forceinline__ void forward(float2 (&x)[KB][4], int (&sx)[KB][4], int lane) const {
    const int g = lane >> 4, jl = lane & 15;
    constexpr int KZ = (ZHI && KB > 1) ? KB / 2 : KB;  // K blocks holding data
    int si[KB][4];
    in_scales<KZ>(x, si);
    MOp<MODE> d[KZ], dr[KZ];
#pragma unroll
    for (int kb = 0; kb < KZ; ++kb) {
      float sc[4];
      factors(si, kb, sc);
      make_operands<MODE, false>(x[kb], sc, d[kb], dr[kb]);
    }
    // F0: data as A, output column block cb
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      f4_t re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KZ; ++kb) {
        re = mprod<MODE, true>(d[kb], wb[cb][kb], re);
        im = mprod<MODE, true>(dr[kb], wb[cb][kb], im);
      }
      // twiddle w_L^(n0 k1), n0 = 4 g + e, k1 = slot % BS
      const int k1 = (jl + 16 * cb) % BS;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float2 w = tab[((4 * g + e) * k1) % L];
        x[cb][e] = cmul_tw<false>(make_float2(re[e], im[e]), w);
      }
    }
    // F1: data as B (K = n0 = the four values just made), W16 as A
    const float one[4] = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      MOp<MODE> y, yr;
      make_operands<MODE, false, true>(x[cb], one, y, yr);
      f4_t re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
      re = mprod<MODE, false>(y, w16, re);
      im = mprod<MODE, false>(yr, w16, im);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[cb][e] = make_float2(re[e], im[e]);
    }
    in_to_spec(si, sx, lane);
  }

  // ---------------------------------------------------------- inverse
  // in: the forward's out layout.  out: y[rho][e] = element jl + 16 nb of
  // line M / BS, M = 4 g + e + 16 rho, nb = M % BS (unnormalized inverse),
  // times 2^so (so: exponent of each register's line).  CROP: only nb < B/2 is used (row blocks past
  // the first half skipped).
  template <bool CROP>
  __device__ __forceinline__ void inverse(float2 (&x)[KB][4], int (&so)[KB][4], int lane) const {
    const int jl = lane & 15, g = lane >> 4;
    constexpr int RZ = (CROP && KB > 1) ? KB / 2 : KB;  // output row blocks kept
    int ss[KB][4];
    spec_scales(x, ss);
    // I0: data as A (M = slot, K = k0), W16 as B; conj(W conj x)
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      float sc[4];
      factors(ss, cb, sc);
      MOp<MODE> d, dr;
      make_operands<MODE, true>(x[cb], sc, d, dr);
      f4_t re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
      re = mprod<MODE, true>(d, w16, re);
      im = mprod<MODE, true>(dr, w16, im);
      // twiddle conj(w_L^(n_a k1)), n_a = jl, k1 = (4 g + e + 16 cb) % BS
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k1 = (4 * g + e + 16 * cb) % BS;
        const float2 w = tab[(jl * k1) % L];
        x[cb][e] = cmul_tw<true>(make_float2(re[e], -im[e]), w);
      }
    }
    // I1: W_B as A (rows M = (line, nb)), data as B (K = slot); conj trick
    MOp<MODE> d[KB], dr[KB];
    const float one[4] = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) make_operands<MODE, true, true>(x[kb], one, d[kb], dr[kb]);
#pragma unroll
    for (int rho = 0; rho < RZ; ++rho) {
      f4_t re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        re = mprod<MODE, false>(d[kb], wb[rho][kb], re);
        im = mprod<MODE, false>(dr[kb], wb[rho][kb], im);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) x[rho][e] = make_float2(re[e], -im[e]);
    }
    spec_to_out(ss, so, lane);
  }

  // ------------------------------------------------------ index maps
  // forward input: element of K block kb, leg lam
  __device__ __forceinline__ static int in_line(int lane, int kb, int lam) {
    return (4 * (lane >> 4) + lam + 16 * kb) / BS;
  }
  template <bool ZHI> __device__ __forceinline__ static int in_index(int lane, int kb, int lam) {
    const int n1 = (4 * (lane >> 4) + lam + 16 * kb) % BS;
    return (n1 < B && (!ZHI || 2 * n1 < B)) ? (lane & 15) + 16 * n1 : -1;
  }
  // forward output = inverse input
  __device__ __forceinline__ static int spec_line(int lane, int cb) { return ((lane & 15) + 16 * cb) / BS; }
  __device__ __forceinline__ static int spec_index(int lane, int cb, int e) {
    const int k1 = ((lane & 15) + 16 * cb) % BS;
    return k1 < B ? k1 + B * (4 * (lane >> 4) + e) : -1;
  }
  // inverse output
  __device__ __forceinline__ static int out_line(int lane, int rho, int e) {
    return (4 * (lane >> 4) + e + 16 * rho) / BS;
  }
  template <bool CROP> __device__ __forceinline__ static int out_index(int lane, int rho, int e) {
    const int nb = (4 * (lane >> 4) + e + 16 * rho) % BS;
    return (nb < B && (!CROP || 2 * nb < B)) ? (lane & 15) + 16 * nb : -1;
  }

  // ------------------------------------------------ layouts in LDS lines
  // wl: the block's first line region (lines at stride SLOTS)
  template <bool ZHI> __device__ __forceinline__ static void load_fwd(float2 (&x)[KB][4], const float2 *wl, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int lam = 0; lam < 4; ++lam) {
        const int n = in_index<ZHI>(lane, kb, lam);
        x[kb][lam] = n >= 0 ? wl[in_line(lane, kb, lam) * SLOTS + lds_pad(n)] : make_float2(0.f, 0.f);
      }
  }
  __device__ __forceinline__ static void store_spec(const float2 (&x)[KB][4], float2 *wl, int lane) {
#pragma unroll
    for (int cb = 0; cb < KB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = spec_index(lane, cb, e);
        if (k >= 0) wl[spec_line(lane, cb) * SLOTS + lds_pad(k)] = x[cb][e];
      }
  }
  __device__ __forceinline__ static void load_spec(float2 (&x)[KB][4], const float2 *wl, int lane) {
#pragma unroll
    for (int cb = 0; cb < KB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = spec_index(lane, cb, e);
        x[cb][e] = k >= 0 ? wl[spec_line(lane, cb) * SLOTS + lds_pad(k)] : make_float2(0.f, 0.f);
      }
  }
  template <bool CROP> __device__ __forceinline__ static void store_inv(const float2 (&x)[KB][4], float2 *wl, int lane) {
    constexpr int RZ = (CROP && KB > 1) ? KB / 2 : KB;
#pragma unroll
    for (int rho = 0; rho < RZ; ++rho)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = out_index<CROP>(lane, rho, e);
        if (n >= 0) wl[out_line(lane, rho, e) * SLOTS + lds_pad(n)] = x[rho][e];
      }
  }

  // Transform of the wavefront's LPW lines; v holds lane t's strided
  // elements t + T i of its line (as fft_line), in and out.
  template <bool INV, bool ZHI = false, bool CROP = false>
  __device__ __forceinline__ void run(float2 (&v)[E], float2 *wave_lines, int lane) const {
    float2 *ln = wave_lines + (lane / T) * SLOTS;
    const int t = lane % T;
#pragma unroll
    for (int i = 0; i < E; ++i) ln[lds_pad(t + T * i)] = v[i];
    wave_lds_fence();
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      float2 *wl = wave_lines + blk * P * SLOTS;
      float2 x[KB][4];
      if constexpr (!INV) {
        load_fwd<ZHI>(x, wl, lane);
        wave_lds_fence();
        int s[KB][4];
        forward<ZHI>(x, s, lane);
        unscale(x, s);
        store_spec(x, wl, lane);
      } else {
        load_spec(x, wl, lane);
        wave_lds_fence();
        int s[KB][4];
        inverse<CROP>(x, s, lane);
        unscale(x, s);
        store_inv<CROP>(x, wl, lane);
      }
      wave_lds_fence();
    }
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = ln[lds_pad(t + T * i)];
    wave_lds_fence();
  }

  // Forward, times K^F, inverse, with everything in registers: x in the
  // forward input layout (zero-padded half absent when PC), kf the real
  // kernel values in the spectrum layout; on return x holds the inverse
  // output (cropped when PC).
  template <bool PC> __device__ __forceinline__ void conv(float2 (&x)[KB][4], const float (&kf)[KB][4], int lane) const {
    int s1[KB][4];
    forward<PC>(x, s1, lane);
#pragma unroll
    for (int cb = 0; cb < KB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float k = SCALED ? ldexpf(kf[cb][e], -s1[cb][e]) : kf[cb][e];
        x[cb][e] = make_float2(x[cb][e].x * k, x[cb][e].y * k);
      }
    int s2[KB][4];
    inverse<PC>(x, s2, lane);
    unscale(x, s2);
  }
};

}  // namespace psn
