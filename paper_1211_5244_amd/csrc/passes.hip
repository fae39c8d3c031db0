// passes.hip - the five passes of one solve (paper, Section 3).
//
//   P1 r2c   real-to-complex along p of the density, zero-padded half skipped
//            (spread_X + 1DFFT_X of the paper's step list)
//   P2 c2c   forward along q (transpose/spread_Y + 1DFFT_Y)
//   P3 conv  forward along r, times K^F, inverse along r, crop
//            (spread_Z + 1DFFT_Z + kernel multiplication + inverse_1DFFT_Z +
//            compactification_Z, with the kernel stored in pass order so no
//            final transpose is needed)
//   P4 c2c   inverse along q, crop (compactification_Y + transpose)
//   P5 c2r   complex-to-real along p, crop (inverse_1DFFT_X +
//            compactification_X)
//
// The paper's separate transpose, spread and compaction kernels do not exist
// here: zero padding happens in registers at load time, crops at store time,
// and the transposes are the LDS staging of tiled sides (plan.cpp picks
// layouts so each side of a pass is either one contiguous line per line
// group or rows of W consecutive lines).  Each HBM array is read and written
// once per pass.
//
// Workgroups are persistent over tiles and prefetch the next tile's input
// into registers while the current tile is transformed, so the HBM reads of
// one tile overlap the FFT arithmetic of the previous one.
//
// The real passes transform two real lines per complex FFT: P1 packs lines
// a and b as a + i b and separates X_a[k] = (Z[k] + conj Z[L-k]) / 2,
// X_b[k] = (Z[k] - conj Z[L-k]) / (2i); P5 forms Z = X_a + i X_b from the two
// Hermitian halves, so the real part of its inverse is line a and the
// imaginary part line b.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_core.h"
#include "fft_mfma.h"
#include "fft_split.h"
#include "kernels.h"

namespace psn {

template <int L, int MODE>
hipError_t launch_for_mode(const Pass &P, const PassIO &io, const float2 *tw, const float *kf,
                           int S_q, hipStream_t s);

template <int A, int B> constexpr int cmax() { return A > B ? A : B; }

// Tile schedules of the tiled passes: schedule TS stages tiles of about
// tile_lines(TS) complex lines (16, 8, 4 or 32) per workgroup.  The lines of
// a tile are the W consecutive lines whose elements form the contiguous row
// segments on the tiled side, so TS trades row-segment length (bytes per HBM
// request) against workgroup size and LDS.  Every schedule computes each
// line's transform with the same arithmetic: results do not depend on it.
constexpr int tile_lines(int ts) { return ts == 1 ? 8 : ts == 2 ? 4 : ts == 3 ? 32 : 16; }

// Workgroup geometry for length L: NW waves of LPW line groups of T lanes.
template <int L, int TS = 0> struct Geo {
  static constexpr int E = Shape<L>::E, T = L / E, LPW = 64 / T;
  static constexpr int NW_WANT = tile_lines(TS) / LPW;
  static constexpr int NW = NW_WANT < 1 ? 1 : NW_WANT > 16 ? 16 : NW_WANT;
  static constexpr int NT = NW * 64;
  static constexpr int G = NW * LPW;  // complex lines in flight per workgroup
  static constexpr int SLOTS = line_lds_slots<L>();
  static constexpr int XCH_F2 = G * SLOTS;
};

// LDS (float2 slots) of each tiled kernel; a schedule is compiled only where
// it fits the 160 KiB of a CDNA4 compute unit.
constexpr int kLdsLimitF2 = 160 * 1024 / 8;
template <int L, int TS> constexpr int c2c_lds_f2() {
  using C = Geo<L, TS>;
  return C::XCH_F2 > (L + 1) * (C::G + 1) ? C::XCH_F2 : (L + 1) * (C::G + 1);
}
template <int L, int TS, bool PAD> constexpr int r2c_lds_f2() {
  using C = Geo<L, TS>;
  constexpr int W = 2 * C::G, LDR = W + 2, LDC = W + 1;
  constexpr int ROWS_IN = PAD ? L / 2 : L, ROWS_OUT = L / 2 + 1;
  return cmax<cmax<C::XCH_F2, ROWS_OUT * LDC>(), (ROWS_IN * LDR + 1) / 2>();
}
template <int L, int TS, bool CROP> constexpr int c2r_lds_f2() {
  using C = Geo<L, TS>;
  constexpr int W = 2 * C::G, LDR = W + 2, LDC = W + 1;
  constexpr int ROWS_IN = L / 2 + 1, ROWS_OUT = CROP ? L / 2 : L;
  return cmax<cmax<C::XCH_F2, ROWS_IN * LDC>(), (ROWS_OUT * LDR + 1) / 2>();
}

// A schedule is compiled only if its tile width differs from every lower
// schedule's (a clamped schedule would duplicate one).
template <int L, int TS> constexpr bool tile_distinct() {
  if constexpr (TS == 0) return true;
  else if constexpr (TS == 1) return Geo<L, 1>::G != Geo<L, 0>::G;
  else if constexpr (TS == 2)
    return Geo<L, 2>::G != Geo<L, 0>::G && Geo<L, 2>::G != Geo<L, 1>::G;
  else
    return Geo<L, 3>::G != Geo<L, 0>::G && Geo<L, 3>::G != Geo<L, 1>::G &&
           Geo<L, 3>::G != Geo<L, 2>::G;
}

// Complex lines per tile that schedule ts gives pass P at length L (0 if the
// schedule does not fit).
template <int L> int tile_lines_of(const Pass &P, int ts) {
  auto pick = [&](auto tsc) -> int {
    constexpr int T = decltype(tsc)::value;
    bool fits = true;
    switch (P.kind) {
      case KIND_FWD:
      case KIND_INV: fits = c2c_lds_f2<L, T>() <= kLdsLimitF2; break;
      case KIND_R2C: fits = P.pad ? r2c_lds_f2<L, T, true>() <= kLdsLimitF2
                                  : r2c_lds_f2<L, T, false>() <= kLdsLimitF2; break;
      case KIND_C2R: fits = P.crop ? c2r_lds_f2<L, T, true>() <= kLdsLimitF2
                                   : c2r_lds_f2<L, T, false>() <= kLdsLimitF2; break;
      default: return 0;
    }
    return fits && tile_distinct<L, T>() ? Geo<L, T>::G : 0;
  };
  switch (ts) {
    case 0: return pick(std::integral_constant<int, 0>{});
    case 1: return pick(std::integral_constant<int, 1>{});
    case 2: return pick(std::integral_constant<int, 2>{});
    case 3: return pick(std::integral_constant<int, 3>{});
  }
  return 0;
}

#if !defined(PSN_DISPATCH_ONLY)

// One launch covers `nsolve` solves of identical geometry; the tile index
// runs over solves first-major.  Per-solve array bases are kernel arguments
// (graph-capturable, no device-side pointer tables).
struct PassParams {
  const void *in[kMaxBatch];
  void *out[kMaxBatch];
  const float2 *tw;
  int in_sl, in_st, in_sb;  // element strides (line, tile, batch); arrays < 2^31 elements
  int out_sl, out_st, out_sb;
  int ext_tile;
  int tiles_per_batch;
  int tiles_per_solve;
  int ntiles;
  int xcd;  // 1: XCD-blocked tile order (block_order)
};


// The line transform of a kernel: float32 radix stages on the vector ALUs
// (MODE_FP32), or radix-8 stages as split-precision DFT matmuls on the
// matrix cores (MODE_SPLIT_*).  `line` is this line group's LDS region,
// `wave_lines` the first region of its wavefront.
// Engine kinds: 0 float32 radix stages, 1 radix-8 matrix stages with LDS
// exchanges (fft_split.h), 2 the two-factor matrix-core engine.
template <int L, int MODE> constexpr int engine_kind() {
  return MODE == MODE_FP32 ? 0 : mfma_length<L>() ? 2 : 1;
}
template <int L, int MODE, int KIND = engine_kind<L, MODE>()> struct LineEngine {
  SplitTwiddles<L> tw;
  SplitOps<MODE> ops;
  __device__ __forceinline__ void init(const float2 *tab, int lane) {
    tw.load(tab, lane);
    ops.init(lane);
  }
  // ZHI: upper half of the inputs zero; CROP: only the first half of the
  // outputs is used (those stages run on the vector ALUs, see split_stage)
  template <bool INV, bool ZHI = false, bool CROP = false>
  __device__ __forceinline__ void run(float2 (&v)[Shape<L>::E], float2 *line, float2 *wave_lines,
                                      int lane) {
    fft_line_split<L, INV, MODE, ZHI, CROP>(v, tw, ops, wave_lines, lane);
  }
};
// Lengths 32..512 of the form 16 B: the two-factor matrix-core engine
// (fft_mfma.h), whose matrix stages exchange no data through LDS.
template <int L, int MODE> struct LineEngine<L, MODE, 2> {
  MfmaLine<L, MODE> m;
  __device__ __forceinline__ void init(const float2 *tab, int lane) { m.init(tab, lane); }
  template <bool INV, bool ZHI = false, bool CROP = false>
  __device__ __forceinline__ void run(float2 (&v)[Shape<L>::E], float2 *line, float2 *wave_lines,
                                      int lane) {
    m.template run<INV, ZHI, CROP>(v, wave_lines, lane);
  }
};
template <int L> struct LineEngine<L, MODE_FP32, 0> {
  Twiddles<L> tw;
  __device__ __forceinline__ void init(const float2 *tab, int lane) { tw.load(tab, lane % kT<L>); }
  // (a cropped output needs nothing here: unstored outputs are dead code)
  template <bool INV, bool ZHI = false, bool CROP = false>
  __device__ __forceinline__ void run(float2 (&v)[Shape<L>::E], float2 *line, float2 *wave_lines,
                                      int lane) {
    fft_line<L, INV, ZHI>(v, tw, line, lane % kT<L>);
  }
};

// Direct layouts of the two-factor engine for lengths with 8 elements per
// lane (32 ... 512, powers of two): a pass moves data straight between HBM
// (or its LDS tile) and the engine's operand layouts, with no canonical
// exchange around the transform.  Register i of a lane is element
// `*_index(lane, i)` of wavefront line `*_line(lane, i)` (-1: not an
// element, e.g. the zero-padded half), for the forward input, the spectrum
// (forward output = inverse input) and the inverse output.
template <int L, int MODE> struct Direct {
  static constexpr bool ON = engine_kind<L, MODE>() == 2 && Shape<L>::E == 8;
  using Eng = MfmaLine<L, MODE == MODE_FP32 ? MODE_SPLIT_FP16 : MODE>;
  static constexpr int KB = Eng::KB, P = Eng::P, NB = Eng::NB;
  __device__ __forceinline__ static int blk(int i) { return i / (4 * KB); }
  __device__ __forceinline__ static int kb(int i) { return (i / 4) % KB; }
  __device__ __forceinline__ static int in_line(int lane, int i) { return blk(i) * P + Eng::in_line(lane, kb(i), i % 4); }
  template <bool ZHI> __device__ __forceinline__ static int in_index(int lane, int i) {
    return Eng::template in_index<ZHI>(lane, kb(i), i % 4);
  }
  __device__ __forceinline__ static int spec_line(int lane, int i) { return blk(i) * P + Eng::spec_line(lane, kb(i)); }
  __device__ __forceinline__ static int spec_index(int lane, int i) { return Eng::spec_index(lane, kb(i), i % 4); }
  __device__ __forceinline__ static int out_line(int lane, int i) { return blk(i) * P + Eng::out_line(lane, kb(i), i % 4); }
  template <bool CROP> __device__ __forceinline__ static int out_index(int lane, int i) {
    return Eng::template out_index<CROP>(lane, kb(i), i % 4);
  }
  // forward (v in the input layout -> spectrum) or inverse (spectrum ->
  // output layout) of the wavefront's blocks, unnormalized, in registers
  template <bool INV, bool ZHI, bool CROP>
  __device__ __forceinline__ static void transform(const Eng &e, float2 (&v)[8], int lane) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      float2 x[KB][4];
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) x[k][l] = v[(b * KB + k) * 4 + l];
      int s[KB][4];
      if constexpr (INV) e.template inverse<CROP>(x, s, lane);
      else e.template forward<ZHI>(x, s, lane);
      Eng::unscale(x, s);
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int l = 0; l < 4; ++l) v[(b * KB + k) * 4 + l] = x[k][l];
    }
  }
};

// The matrix-core engine reads its twiddles by index for every line; they
// come from a copy of the length-L table in LDS, staged once per workgroup,
// so the per-line lookups do not compete with the pass's HBM streams in the
// vector memory pipeline.  (The float32 engine keeps each lane's twiddles in
// registers.)
template <int L, int MODE> struct TwiddleStage {
  static constexpr bool ON = engine_kind<L, MODE>() == 2;
  __device__ __forceinline__ static const float2 *stage(float2 *lds, const float2 *tab, int tid, int nt) {
    if constexpr (ON) {
      for (int n = tid; n < L; n += nt) lds[n] = tab[n];
      __syncthreads();
      return lds;
    } else {
      return tab;
    }
  }
};

// Non-temporal hints, chosen by measurement on the 512-length passes (whole
// solve, 2.62k -> 2.68k solves/s): every store of a pass output streams, and
// so do the tiled loads (128-byte row segments of W lines); contiguous line
// loads keep ordinary loads (streaming them cost 4-9%).  A streaming store
// makes its own pass slower and the next one faster: the 256 MB last-level
// cache then holds no dirty lines that the next pass would have to evict.
typedef float psn_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_stream(float2 *p, float2 v) {
  __builtin_nontemporal_store(*reinterpret_cast<const psn_f2v *>(&v), reinterpret_cast<psn_f2v *>(p));
}
__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
// A store of an output whose lanes cover SEG contiguous bytes per row or
// line in one instruction.  Streaming pieces shorter than a 128-byte cache
// line leaves them unmerged on their way to HBM (a 96-length line written
// 16 bytes at a time ran at 0.85 TB/s), so those take ordinary stores, which
// the L2 gathers into whole lines.
template <int SEG, typename TE> __device__ __forceinline__ void st_out(TE *p, TE v) {
  if constexpr (SEG >= 128) st_stream(p, v);
  else *p = v;
}
__device__ __forceinline__ float2 ld_stream(const float2 *p) {
  const psn_f2v v = __builtin_nontemporal_load(reinterpret_cast<const psn_f2v *>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }

// Workgroups are dispatched round-robin over the 8 XCDs of the chip
// (workgroup b runs on XCD b % 8, each XCD with its own L2).  With `xcd` set
// (grid a multiple of 8), workgroup b takes the virtual index that gives
// each XCD a contiguous run of tiles per round: XCD x's j-th workgroup gets
// x * (G / 8) + j, so neighbouring tiles, which read neighbouring row
// segments, share an L2.  The autotuner decides per pass whether it pays.
__device__ __forceinline__ int block_order(int xcd) {
  const int b = blockIdx.x, G = gridDim.x;
  return xcd ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

// A ROWS x W tile moved between HBM (rows at stride `sl`, W consecutive
// elements per row) and LDS (row stride LD) by all NT threads, through
// registers so the HBM side can be issued early.
template <int ROWS, int W, int NT, int LD, typename TE> struct TileRegs {
  static constexpr int N = ROWS * W, PF = (N + NT - 1) / NT;
  TE r[PF];
  __device__ __forceinline__ void load(const TE *__restrict__ base, int sl, int ncols,
                                       int tid) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int idx = tid + p * NT;
      const int row = idx / W, col = idx % W;
      if (idx < N && col < ncols) r[p] = ld_stream(&base[row * sl + col]);
    }
  }
  __device__ __forceinline__ void to_lds(TE *tile, int tid) const {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int idx = tid + p * NT;
      if (idx < N) tile[(idx / W) * LD + (idx % W)] = r[p];
    }
  }
};

template <int ROWS, int W, int NT, int LD, typename TE>
__device__ __forceinline__ void tile_store(TE *__restrict__ base, int sl, int ncols,
                                           const TE *tile, int tid) {
  for (int idx = tid; idx < ROWS * W; idx += NT) {
    const int row = idx / W, col = idx % W;
    if (col < ncols) st_out<W * int(sizeof(TE))>(&base[row * sl + col], tile[row * LD + col]);
  }
}

struct TileCoord {
  int a0, ncols, b, solve;
};

__device__ __forceinline__ TileCoord tile_coord(const PassParams &a, int tile, int W) {
  TileCoord c;
  c.solve = tile / a.tiles_per_solve;
  const int rem = tile - c.solve * a.tiles_per_solve;
  c.a0 = (rem % a.tiles_per_batch) * W;
  c.b = rem / a.tiles_per_batch;
  c.ncols = min(W, a.ext_tile - c.a0);
  return c;
}

// ------------------------------------------------------------- P2 / P4
template <int L, bool INV, bool IN_TILED, bool OUT_TILED, bool PC, int MODE, int TS>
__global__ __launch_bounds__((Geo<L, TS>::NT)) void c2c_kernel(PassParams a) {
  using C = Geo<L, TS>;
  constexpr int E = C::E, T = C::T, LPW = C::LPW, NT = C::NT, W = C::G, LD = W + 1;
  constexpr bool PAD = !INV && PC, CROP = INV && PC;
  constexpr int ROWS_IN = PAD ? L / 2 : L, ROWS_OUT = CROP ? L / 2 : L;
  constexpr int LDS_F2 = c2c_lds_f2<L, TS>();
  __shared__ float2 smem[LDS_F2];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / T, t = lane % T;
  const int c = wave * LPW + g;
  float2 *xch = smem + c * C::SLOTS;

  float2 *wave_lines = smem + wave * LPW * C::SLOTS;
  LineEngine<L, MODE> eng;
  __shared__ float2 tw_lds[TwiddleStage<L, MODE>::ON ? L : 1];
  eng.init(TwiddleStage<L, MODE>::stage(tw_lds, a.tw, tid, NT), lane);

  using D = Direct<L, MODE>;
  TileRegs<ROWS_IN, W, NT, LD, float2> pf;
  float2 vn[E];
  auto fetch = [&](int tile) {
    const TileCoord q = tile_coord(a, tile, W);
    const float2 *__restrict__ in = static_cast<const float2 *>(a.in[q.solve]);
    if constexpr (IN_TILED) {
      pf.load(in + q.b * a.in_sb + q.a0, a.in_sl, q.ncols, tid);
    } else if constexpr (D::ON) {
      // straight into the engine's input (forward) or spectrum (inverse) layout
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int lc = wave * LPW + (INV ? D::spec_line(lane, i) : D::in_line(lane, i));
        const int n = INV ? D::spec_index(lane, i) : D::template in_index<PAD>(lane, i);
        vn[i] = (n >= 0 && lc < q.ncols) ? in[(q.a0 + lc) * a.in_st + q.b * a.in_sb + n] : make_float2(0.f, 0.f);
      }
    } else {
      const bool ok = c < q.ncols;
      const float2 *line = in + (q.a0 + c) * a.in_st + q.b * a.in_sb;
#pragma unroll
      for (int i = 0; i < E; ++i)
        vn[i] = ((!PAD || i < E / 2) && ok) ? line[t + T * i] : make_float2(0.f, 0.f);
    }
  };

  int tile = block_order(a.xcd);
  if (tile < a.ntiles) fetch(tile);
  while (tile < a.ntiles) {
    const TileCoord q = tile_coord(a, tile, W);
    const int next = tile + gridDim.x;
    float2 v[E];
    __syncthreads();  // the previous tile is done with smem
    if constexpr (IN_TILED) {
      pf.to_lds(smem, tid);
      __syncthreads();
      if constexpr (D::ON) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int lc = wave * LPW + (INV ? D::spec_line(lane, i) : D::in_line(lane, i));
          const int n = INV ? D::spec_index(lane, i) : D::template in_index<PAD>(lane, i);
          v[i] = (n >= 0 && lc < q.ncols) ? smem[n * LD + lc] : make_float2(0.f, 0.f);
        }
      } else {
        const bool ok = c < q.ncols;  // columns past a ragged edge hold stale LDS
#pragma unroll
        for (int i = 0; i < E; ++i)
          v[i] = ((!PAD || i < E / 2) && ok) ? smem[(t + T * i) * LD + c] : make_float2(0.f, 0.f);
      }
      if (next < a.ntiles) fetch(next);
      __syncthreads();  // the tile region becomes exchange space
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = vn[i];
      if (next < a.ntiles) fetch(next);
    }

    if constexpr (D::ON) {
      D::template transform<INV, PAD, CROP>(eng.m, v, lane);
    } else {
      eng.template run<INV, PAD, CROP>(v, xch, wave_lines, lane);
    }

    if constexpr (OUT_TILED) {
      __syncthreads();  // every line is done exchanging
      if constexpr (D::ON) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int lc = wave * LPW + (INV ? D::out_line(lane, i) : D::spec_line(lane, i));
          const int n = INV ? D::template out_index<CROP>(lane, i) : D::spec_index(lane, i);
          if (n >= 0) smem[n * LD + lc] = v[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i)
          if (!CROP || i < E / 2) smem[(t + T * i) * LD + c] = v[i];
      }
      __syncthreads();
      tile_store<ROWS_OUT, W, NT, LD>(static_cast<float2 *>(a.out[q.solve]) + q.b * a.out_sb + q.a0,
                                      a.out_sl, q.ncols, smem, tid);
    } else if constexpr (D::ON) {
      float2 *out = static_cast<float2 *>(a.out[q.solve]);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int lc = wave * LPW + (INV ? D::out_line(lane, i) : D::spec_line(lane, i));
        const int n = INV ? D::template out_index<CROP>(lane, i) : D::spec_index(lane, i);
        // 16 lanes cover 16 consecutive elements (128 bytes) of one line
        if (n >= 0 && lc < q.ncols) st_out<128>(&out[(q.a0 + lc) * a.out_st + q.b * a.out_sb + n], v[i]);
      }
    } else {
      if (c < q.ncols) {
        float2 *line = static_cast<float2 *>(a.out[q.solve]) + (q.a0 + c) * a.out_st + q.b * a.out_sb;
#pragma unroll
        for (int i = 0; i < E; ++i)
          if (!CROP || i < E / 2) st_out<T * 8>(&line[t + T * i], v[i]);
      }
    }
    tile = next;
  }
}

// ------------------------------------------------------------------ P1
template <int L, bool IN_TILED, bool PAD, int MODE, int TS>
__global__ __launch_bounds__((Geo<L, TS>::NT)) void r2c_kernel(PassParams a) {
  using C = Geo<L, TS>;
  constexpr int E = C::E, T = C::T, LPW = C::LPW, NT = C::NT, W = 2 * C::G;
  constexpr int LDR = W + 2, LDC = W + 1;  // real tile (floats), complex tile (float2)
  constexpr int ROWS_IN = PAD ? L / 2 : L, ROWS_OUT = L / 2 + 1;
  constexpr int LDS_F2 = r2c_lds_f2<L, TS, PAD>();
  __shared__ float2 smem[LDS_F2];
  float *smem_f = reinterpret_cast<float *>(smem);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / T, t = lane % T;
  const int c = wave * LPW + g;  // complex line: real lines 2c, 2c + 1
  float2 *xch = smem + c * C::SLOTS;

  float2 *wave_lines = smem + wave * LPW * C::SLOTS;
  LineEngine<L, MODE> eng;
  __shared__ float2 tw_lds[TwiddleStage<L, MODE>::ON ? L : 1];
  eng.init(TwiddleStage<L, MODE>::stage(tw_lds, a.tw, tid, NT), lane);

  using D = Direct<L, MODE>;
  TileRegs<ROWS_IN, W, NT, LDR, float> pf;
  float2 vn[E];
  auto fetch = [&](int tile) {
    const TileCoord q = tile_coord(a, tile, W);
    const float *__restrict__ in = static_cast<const float *>(a.in[q.solve]);
    if constexpr (IN_TILED) {
      pf.load(in + q.b * a.in_sb + q.a0, a.in_sl, q.ncols, tid);
    } else if constexpr (D::ON) {
      // real lines 2 lc and 2 lc + 1 as one complex line, in the engine's
      // input layout
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int lc = wave * LPW + D::in_line(lane, i);
        const int n = D::template in_index<PAD>(lane, i);
        const float *l0 = in + (q.a0 + 2 * lc) * a.in_st + q.b * a.in_sb;
        vn[i].x = (n >= 0 && 2 * lc < q.ncols) ? l0[n] : 0.f;
        vn[i].y = (n >= 0 && 2 * lc + 1 < q.ncols) ? l0[a.in_st + n] : 0.f;
      }
    } else {
      const bool ok0 = 2 * c < q.ncols, ok1 = 2 * c + 1 < q.ncols;
      const float *l0 = in + (q.a0 + 2 * c) * a.in_st + q.b * a.in_sb;
      const float *l1 = l0 + a.in_st;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const bool live = !PAD || i < E / 2;
        vn[i].x = (live && ok0) ? l0[t + T * i] : 0.f;
        vn[i].y = (live && ok1) ? l1[t + T * i] : 0.f;
      }
    }
  };

  int tile = block_order(a.xcd);
  if (tile < a.ntiles) fetch(tile);
  while (tile < a.ntiles) {
    const TileCoord q = tile_coord(a, tile, W);
    const int next = tile + gridDim.x;
    float2 v[E];
    __syncthreads();
    if constexpr (IN_TILED) {
      pf.to_lds(smem_f, tid);
      __syncthreads();
      if constexpr (D::ON) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int lc = wave * LPW + D::in_line(lane, i);
          const int n = D::template in_index<PAD>(lane, i);
          const float2 x = n >= 0 ? *reinterpret_cast<const float2 *>(smem_f + n * LDR + 2 * lc)
                                  : make_float2(0.f, 0.f);
          v[i] = make_float2(2 * lc < q.ncols ? x.x : 0.f, 2 * lc + 1 < q.ncols ? x.y : 0.f);
        }
      } else {
        const bool ok0 = 2 * c < q.ncols, ok1 = 2 * c + 1 < q.ncols;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const float2 x = (!PAD || i < E / 2)
                               ? *reinterpret_cast<const float2 *>(smem_f + (t + T * i) * LDR + 2 * c)
                               : make_float2(0.f, 0.f);
          v[i] = make_float2(ok0 ? x.x : 0.f, ok1 ? x.y : 0.f);
        }
      }
      if (next < a.ntiles) fetch(next);
      __syncthreads();
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = vn[i];
      if (next < a.ntiles) fetch(next);
    }

    // separate the two real lines: needs Z[L - k] from the mirrored lane
    if constexpr (D::ON) {
      D::template transform<false, PAD, false>(eng.m, v, lane);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int k = D::spec_index(lane, i);
        if (k >= 0) wave_lines[D::spec_line(lane, i) * C::SLOTS + lds_pad(k)] = v[i];
      }
      wave_lds_fence();
#pragma unroll
      for (int i = 0; i <= E / 2; ++i) v[i] = xch[lds_pad(t + T * i < L ? t + T * i : 0)];
    } else {
      eng.template run<false, PAD>(v, xch, wave_lines, lane);
#pragma unroll
      for (int i = 0; i < E; ++i) xch[lds_pad(t + T * i)] = v[i];
      wave_lds_fence();
    }
    float2 x0[E / 2 + 1], x1[E / 2 + 1];
#pragma unroll
    for (int i = 0; i <= E / 2; ++i) {
      const int k = t + T * i;
      const int km = (k == 0) ? 0 : L - k;
      const float2 z = v[i];
      const float2 zr = xch[lds_pad(km < L ? km : 0)];
      x0[i] = make_float2(0.5f * (z.x + zr.x), 0.5f * (z.y - zr.y));
      x1[i] = make_float2(0.5f * (z.y + zr.y), 0.5f * (zr.x - z.x));
    }
    __syncthreads();  // every line is done with its exchange region
#pragma unroll
    for (int i = 0; i <= E / 2; ++i) {
      const int k = t + T * i;
      if (i < E / 2 || t == 0) {
        smem[k * LDC + 2 * c] = x0[i];
        smem[k * LDC + 2 * c + 1] = x1[i];
      }
    }
    __syncthreads();
    tile_store<ROWS_OUT, W, NT, LDC>(static_cast<float2 *>(a.out[q.solve]) + q.b * a.out_sb + q.a0,
                                     a.out_sl, q.ncols, smem, tid);
    tile = next;
  }
}

// ------------------------------------------------------------------ P5
template <int L, bool OUT_TILED, bool CROP, int MODE, int TS>
__global__ __launch_bounds__((Geo<L, TS>::NT)) void c2r_kernel(PassParams a) {
  using C = Geo<L, TS>;
  constexpr int E = C::E, T = C::T, LPW = C::LPW, NT = C::NT, W = 2 * C::G;
  constexpr int LDR = W + 2, LDC = W + 1;
  constexpr int ROWS_IN = L / 2 + 1, ROWS_OUT = CROP ? L / 2 : L;
  constexpr int LDS_F2 = c2r_lds_f2<L, TS, CROP>();
  __shared__ float2 smem[LDS_F2];
  float *smem_f = reinterpret_cast<float *>(smem);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / T, t = lane % T;
  const int c = wave * LPW + g;
  float2 *xch = smem + c * C::SLOTS;

  float2 *wave_lines = smem + wave * LPW * C::SLOTS;
  LineEngine<L, MODE> eng;
  __shared__ float2 tw_lds[TwiddleStage<L, MODE>::ON ? L : 1];
  eng.init(TwiddleStage<L, MODE>::stage(tw_lds, a.tw, tid, NT), lane);

  using D = Direct<L, MODE>;
  TileRegs<ROWS_IN, W, NT, LDC, float2> pf;
  int tile = block_order(a.xcd);
  if (tile < a.ntiles) {
    const TileCoord q = tile_coord(a, tile, W);
    pf.load(static_cast<const float2 *>(a.in[q.solve]) + q.b * a.in_sb + q.a0, a.in_sl, q.ncols, tid);
  }
  while (tile < a.ntiles) {
    const TileCoord q = tile_coord(a, tile, W);
    const int next = tile + gridDim.x;
    float2 v[E];
    __syncthreads();
    pf.to_lds(smem, tid);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) {
      // register i holds spectrum index k of complex line lc (the engine's
      // input layout, or lane t's strided elements)
      const int lc = D::ON ? wave * LPW + D::spec_line(lane, i) : c;
      const int k = D::ON ? D::spec_index(lane, i) : t + T * i;
      const bool ok0 = k >= 0 && 2 * lc < q.ncols, ok1 = k >= 0 && 2 * lc + 1 < q.ncols;
      const bool direct = k <= L / 2;
      const int kk = k < 0 ? 0 : direct ? k : L - k;
      float2 x0 = ok0 ? smem[kk * LDC + 2 * lc] : make_float2(0.f, 0.f);
      float2 x1 = ok1 ? smem[kk * LDC + 2 * lc + 1] : make_float2(0.f, 0.f);
      if (kk == 0 || kk == L / 2) {
        // DC and Nyquist coefficients of a real line are real
        x0.y = 0.f;
        x1.y = 0.f;
      }
      // Z = X_a + i X_b, using X[k] = conj(X[L - k]) above L/2
      v[i] = direct ? make_float2(x0.x - x1.y, x0.y + x1.x) : make_float2(x0.x + x1.y, x1.x - x0.y);
    }
    if (next < a.ntiles) {
      const TileCoord qn = tile_coord(a, next, W);
      pf.load(static_cast<const float2 *>(a.in[qn.solve]) + qn.b * a.in_sb + qn.a0, a.in_sl, qn.ncols,
              tid);
    }
    __syncthreads();

    if constexpr (D::ON) {
      D::template transform<true, false, CROP>(eng.m, v, lane);
    } else {
      eng.template run<true, false, CROP>(v, xch, wave_lines, lane);
    }

    if constexpr (OUT_TILED) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int lc = D::ON ? wave * LPW + D::out_line(lane, i) : c;
        const int n = D::ON ? D::template out_index<CROP>(lane, i) : ((!CROP || i < E / 2) ? t + T * i : -1);
        if (n >= 0) *reinterpret_cast<float2 *>(smem_f + n * LDR + 2 * lc) = v[i];
      }
      __syncthreads();
      tile_store<ROWS_OUT, W, NT, LDR>(static_cast<float *>(a.out[q.solve]) + q.b * a.out_sb + q.a0,
                                       a.out_sl, q.ncols, smem_f, tid);
    } else if constexpr (D::ON) {
      float *out = static_cast<float *>(a.out[q.solve]);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int lc = wave * LPW + D::out_line(lane, i);
        const int n = D::template out_index<CROP>(lane, i);
        float *l0 = out + (q.a0 + 2 * lc) * a.out_st + q.b * a.out_sb;
        // 16 lanes cover 64 contiguous bytes of each real line
        if (n >= 0 && 2 * lc < q.ncols) st_out<64>(&l0[n], v[i].x);
        if (n >= 0 && 2 * lc + 1 < q.ncols) st_out<64>(&l0[a.out_st + n], v[i].y);
      }
    } else {
      const bool ok0 = 2 * c < q.ncols, ok1 = 2 * c + 1 < q.ncols;
      float *l0 = static_cast<float *>(a.out[q.solve]) + (q.a0 + 2 * c) * a.out_st + q.b * a.out_sb;
      float *l1 = l0 + a.out_st;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        if (!CROP || i < E / 2) {
          if (ok0) st_out<T * 4>(&l0[t + T * i], v[i].x);
          if (ok1) st_out<T * 4>(&l1[t + T * i], v[i].y);
        }
      }
    }
    tile = next;
  }
}

// ------------------------------------------------------------------ P3
struct ConvParams {
  float2 *data;       // A2 of the first solve, lines along r contiguous
  long long solve_stride;  // elements between the A2 arrays of consecutive solves
  const float *kf;    // [k_p][k_q'][k_r'] float32, 1/(S1 S2 S3) folded in
  const float2 *tw;
  int st_q, st_p;     // element strides of line (k_p, k_q)
  int S_q;
  int kq_half;        // S_q/2 + 1
  int H;              // number of k_p planes
  int nrows;          // H * kq_half kernel rows per solve
  int nsolve;
  int xcd;            // 1: XCD-blocked workgroup order (block_order)
};

constexpr int kConvWaves = 4;

// One kernel row (k_p, k_q') serves the lines k_q = k_q' and S_q - k_q'
// (K^F is even in k_q); the mirror line re-reads the row from cache.  Each
// line group walks its rows in order with two line buffers: the next line
// (and its kernel values) is loaded while the current one is transformed.
// The walk is wavefront-uniform (a group without work transforms the first
// line of the array and stores nothing) so matrix-core stages always run on
// whole wavefronts.  With one line per wavefront the walk is scalar.
// 24-element lanes: two wavefronts per SIMD (see the single line buffer below)
// The fused fp16 matrix-core conv (one line per wavefront, two transformed
// back to back) is latency-bound: at least three wavefronts per SIMD (it
// fits 125 registers; bf16 needs more).
template <int L, int MODE> constexpr int conv_min_waves() {
  return Shape<L>::E >= 24 ? 2 : (MODE == MODE_SPLIT_FP16 && engine_kind<L, MODE>() == 2 && kT<L> == 64) ? 3 : 1;
}

template <int L, bool PC, int MODE>
__global__ __launch_bounds__(kConvWaves * 64)
__attribute__((amdgpu_waves_per_eu(conv_min_waves<L, MODE>()))) void conv_kernel(ConvParams a) {
  constexpr int E = Shape<L>::E, T = L / E, LPW = 64 / T, KR = L / 2 + 1;
  constexpr int SLOTS = line_lds_slots<L>();
  __shared__ float2 smem[kConvWaves * LPW * SLOTS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane / T, t = lane % T;
  float2 *xch = smem + (wave * LPW + g) * SLOTS;
  float2 *wave_lines = smem + wave * LPW * SLOTS;

  // (the table is staged before idle wavefronts leave: all reach the barrier)
  __shared__ float2 tw_lds[TwiddleStage<L, MODE>::ON ? L : 1];
  const float2 *tw = TwiddleStage<L, MODE>::stage(tw_lds, a.tw, tid, kConvWaves * 64);
  const int row0 = (block_order(a.xcd) * kConvWaves + wave) * LPW + g;
  if (!__any(row0 < a.nrows * a.nsolve)) return;  // whole wavefront idle

  LineEngine<L, MODE> eng;
  eng.init(tw, lane);

  // rows are (solve, k_p, k_q') in mixed radix; walk them with carries
  const int stride = gridDim.x * kConvWaves * LPW;
  const int dsolve = stride / a.nrows, dr = stride % a.nrows;
  const int dkp = dr / a.kq_half, dkq = dr % a.kq_half;
  int solve = row0 / a.nrows;
  const int r0 = row0 % a.nrows;
  int kp = r0 / a.kq_half, kqf = r0 % a.kq_half, rep = 0;

  struct Item {
    float2 v[E];
    float k[E];
    float2 *line;
    bool live;
  };
  // One line per wavefront on the two-factor matrix-core engine: the line
  // is loaded straight into the engine's operand layout and the kernel
  // values into its spectrum layout, so the fused transform exchanges
  // nothing through LDS.
  constexpr bool FUSED = engine_kind<L, MODE>() == 2 && LPW == 1;
  using Eng = MfmaLine<L, MODE == MODE_FP32 ? MODE_SPLIT_FP16 : MODE>;
  auto fetch = [&](Item &it) {
    it.live = solve < a.nsolve;
    const int kq = rep == 0 ? kqf : a.S_q - kqf;
    it.line = a.data + (it.live ? solve * a.solve_stride + (kp * a.st_p + kq * a.st_q) : 0);
    const float *krow = a.kf + (it.live ? (kp * a.kq_half + kqf) * KR : 0);
    if constexpr (FUSED) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int n = Eng::template in_index<PC>(lane, i / 4, i % 4);
        it.v[i] = n >= 0 ? it.line[n] : make_float2(0.f, 0.f);
        const int k = Eng::spec_index(lane, i / 4, i % 4);  // 0 <= k < L
        it.k[i] = krow[k <= L / 2 ? k : L - k];
      }
    } else {
      // K^F is even along r: element k >= L/2 takes row entry L - k (i >= E/2
      // holds exactly those k, and k = L/2 reads the same entry either way)
      const float *kup = krow + t, *kdown = krow + (L - t);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int k = t + T * i;
        it.k[i] = i < E / 2 ? kup[T * i] : kdown[-T * i];
        // the padding half: never read by the float32 first stage
        it.v[i] = (!PC || i < E / 2) ? it.line[k] : make_float2(0.f, 0.f);
      }
    }
  };
  auto advance = [&]() {
    const bool pair = kqf != 0 && 2 * kqf != a.S_q;
    if (rep == 0 && pair) {
      rep = 1;
    } else {
      rep = 0;
      kqf += dkq;
      kp += dkp;
      solve += dsolve;
      if (kqf >= a.kq_half) {
        kqf -= a.kq_half;
        ++kp;
      }
      if (kp >= a.H) {
        kp -= a.H;
        ++solve;
      }
    }
  };
  auto process = [&](Item &it) {
    if constexpr (FUSED) {
      constexpr int KB = Eng::KB;
      float2 x[KB][4];
      float kv[KB][4];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        x[i / 4][i % 4] = it.v[i];
        kv[i / 4][i % 4] = it.k[i];
      }
      eng.m.template conv<PC>(x, kv, lane);
      if (it.live) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int n = Eng::template out_index<PC>(lane, i / 4, i % 4);
          if (n >= 0) st_out<128>(&it.line[n], x[i / 4][i % 4]);  // 16 lanes: 128 contiguous bytes
        }
      }
    } else {
      eng.template run<false, PC>(it.v, xch, wave_lines, lane);
#pragma unroll
      for (int i = 0; i < E; ++i) it.v[i] = make_float2(it.v[i].x * it.k[i], it.v[i].y * it.k[i]);
      eng.template run<true, false, PC>(it.v, xch, wave_lines, lane);
      if (it.live) {
#pragma unroll
        for (int i = 0; i < E; ++i)
          if (!PC || i < E / 2) st_out<T * 8>(&it.line[t + T * i], it.v[i]);
      }
    }
  };

  Item A;
  fetch(A);
  advance();
  if constexpr (FUSED && MODE == MODE_SPLIT_FP16) {
    // two lines per step, transformed back to back: independent matrix-core
    // and vector chains for the scheduler to interleave (fp16 conv at
    // L = 512: 161 -> 155 us per launch; the bf16 conv, with three products
    // per product and more registers, ran slower this way and keeps the
    // alternating walk below)
    Item B;
    fetch(B);
    advance();
    while (true) {
      process(A);
      process(B);
      if (!__any(B.live)) break;
      fetch(A);
      advance();
      fetch(B);
      advance();
      if (!__any(A.live)) break;
    }
  } else if constexpr (E >= 24) {
    // 24 elements per lane: two items would need about 260 registers and
    // leave one wavefront per SIMD; one item, two wavefronts per SIMD
    while (true) {
      process(A);
      fetch(A);
      advance();
      if (!__any(A.live)) break;
    }
  } else {
    Item B;
    while (true) {
      fetch(B);
      advance();
      process(A);
      if (!__any(B.live)) break;
      fetch(A);
      advance();
      process(B);
      if (!__any(A.live)) break;
    }
  }
}

// ------------------------------------------------------------ launchers
namespace {

int device_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

PassParams make_params(const Pass &P, const PassIO &io, const float2 *tw, int W) {
  PassParams a;
  for (int j = 0; j < kMaxBatch; ++j) {
    a.in[j] = j < io.count ? io.in[j] : nullptr;
    a.out[j] = j < io.count ? io.out[j] : nullptr;
  }
  a.tw = tw;
  a.in_sl = int(P.in_s[0]);
  a.in_st = int(P.in_s[1]);
  a.in_sb = int(P.in_s[2]);
  a.out_sl = int(P.out_s[0]);
  a.out_st = int(P.out_s[1]);
  a.out_sb = int(P.out_s[2]);
  a.ext_tile = P.ext_tile;
  a.tiles_per_batch = (P.ext_tile + W - 1) / W;
  a.tiles_per_solve = a.tiles_per_batch * P.ext_batch;
  a.ntiles = a.tiles_per_solve * io.count;
  a.xcd = 0;
  return a;
}

// persistent grid: as many workgroups as fit on the device at once
template <typename K>
int persistent_grid(K kernel, int threads, int ntiles) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const long long cap = (long long)device_cu_count() * per_cu;
  return int(ntiles < cap ? ntiles : cap);
}

template <int L, int MODE, bool INV, bool IT, bool OT, bool PC, int TS>
hipError_t launch_c2c_ts(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
  using C = Geo<L, TS>;
  PassParams a = make_params(P, io, tw, C::G);
  auto k = c2c_kernel<L, INV, IT, OT, PC, MODE, TS>;
  const int grid = persistent_grid(k, C::NT, a.ntiles);
  if (grid <= 0) return hipSuccess;
  a.xcd = ((P.tile_sel >> 2) & 1) && grid % 8 == 0;
  hipLaunchKernelGGL(k, dim3(grid), dim3(C::NT), 0, s, a);
  return hipGetLastError();
}

template <int L, int MODE, bool IT, bool PAD, int TS>
hipError_t launch_r2c_ts(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
  using C = Geo<L, TS>;
  PassParams a = make_params(P, io, tw, 2 * C::G);
  auto k = r2c_kernel<L, IT, PAD, MODE, TS>;
  const int grid = persistent_grid(k, C::NT, a.ntiles);
  if (grid <= 0) return hipSuccess;
  a.xcd = ((P.tile_sel >> 2) & 1) && grid % 8 == 0;
  hipLaunchKernelGGL(k, dim3(grid), dim3(C::NT), 0, s, a);
  return hipGetLastError();
}

template <int L, int MODE, bool OT, bool CROP, int TS>
hipError_t launch_c2r_ts(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
  using C = Geo<L, TS>;
  PassParams a = make_params(P, io, tw, 2 * C::G);
  auto k = c2r_kernel<L, OT, CROP, MODE, TS>;
  const int grid = persistent_grid(k, C::NT, a.ntiles);
  if (grid <= 0) return hipSuccess;
  a.xcd = ((P.tile_sel >> 2) & 1) && grid % 8 == 0;
  hipLaunchKernelGGL(k, dim3(grid), dim3(C::NT), 0, s, a);
  return hipGetLastError();
}

// The pass's tile schedule selects the kernel variant, in every precision; a
// schedule that does not fit runs schedule 0.
#define PSN_TILE_DISPATCH(LAUNCH, FITS, ...)                                   \
  {                                                                            \
    switch (P.tile_sel & 3) {                                                  \
      case 1: if constexpr (FITS(1)) return LAUNCH<__VA_ARGS__, 1>(P, io, tw, s); break; \
      case 2: if constexpr (FITS(2)) return LAUNCH<__VA_ARGS__, 2>(P, io, tw, s); break; \
      case 3: if constexpr (FITS(3)) return LAUNCH<__VA_ARGS__, 3>(P, io, tw, s); break; \
      default: break;                                                          \
    }                                                                          \
  }                                                                            \
  return LAUNCH<__VA_ARGS__, 0>(P, io, tw, s);

template <int L, int MODE, bool INV, bool IT, bool OT, bool PC>
hipError_t launch_c2c(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
#define PSN_FITS(T) (c2c_lds_f2<L, T>() <= kLdsLimitF2 && tile_distinct<L, T>())
  PSN_TILE_DISPATCH(launch_c2c_ts, PSN_FITS, L, MODE, INV, IT, OT, PC)
#undef PSN_FITS
}

template <int L, int MODE, bool IT, bool PAD>
hipError_t launch_r2c(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
#define PSN_FITS(T) (r2c_lds_f2<L, T, PAD>() <= kLdsLimitF2 && tile_distinct<L, T>())
  PSN_TILE_DISPATCH(launch_r2c_ts, PSN_FITS, L, MODE, IT, PAD)
#undef PSN_FITS
}

template <int L, int MODE, bool OT, bool CROP>
hipError_t launch_c2r(const Pass &P, const PassIO &io, const float2 *tw, hipStream_t s) {
#define PSN_FITS(T) (c2r_lds_f2<L, T, CROP>() <= kLdsLimitF2 && tile_distinct<L, T>())
  PSN_TILE_DISPATCH(launch_c2r_ts, PSN_FITS, L, MODE, OT, CROP)
#undef PSN_FITS
}
#undef PSN_TILE_DISPATCH

template <int L, int MODE, bool PC>
hipError_t launch_conv(const Pass &P, const PassIO &io, const float2 *tw, const float *kf,
                       int S_q, hipStream_t s) {
  ConvParams a;
  a.data = static_cast<float2 *>(io.out[0]);
  a.solve_stride = io.conv_stride;
  a.nsolve = io.count;
  a.kf = kf;
  a.tw = tw;
  a.st_q = int(P.in_s[1]);
  a.st_p = int(P.in_s[2]);
  a.S_q = S_q;
  a.kq_half = S_q / 2 + 1;
  a.H = P.ext_batch;
  a.nrows = P.ext_batch * a.kq_half;
  constexpr int LPW = 64 / (L / Shape<L>::E);
  const long long groups_per_block = (long long)kConvWaves * LPW;
  const long long need = ((long long)a.nrows * a.nsolve + groups_per_block - 1) / groups_per_block;
  auto k = conv_kernel<L, PC, MODE>;
  const int blocks = persistent_grid(k, kConvWaves * 64, int(need < (1 << 30) ? need : (1 << 30)));
  if (blocks <= 0) return hipSuccess;
  a.xcd = ((P.tile_sel >> 2) & 1) && blocks % 8 == 0;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(kConvWaves * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <int L, int MODE>
hipError_t launch_for_mode(const Pass &P, const PassIO &io, const float2 *tw, const float *kf,
                           int S_q, hipStream_t s) {
  const bool it = P.in_tiled, ot = P.out_tiled;
  switch (P.kind) {
    case KIND_R2C:
      if (it) return P.pad ? launch_r2c<L, MODE, true, true>(P, io, tw, s)
                           : launch_r2c<L, MODE, true, false>(P, io, tw, s);
      return P.pad ? launch_r2c<L, MODE, false, true>(P, io, tw, s)
                   : launch_r2c<L, MODE, false, false>(P, io, tw, s);
    case KIND_FWD:
      if (it) return P.pad ? launch_c2c<L, MODE, false, true, true, true>(P, io, tw, s)
                           : launch_c2c<L, MODE, false, true, true, false>(P, io, tw, s);
      return P.pad ? launch_c2c<L, MODE, false, false, true, true>(P, io, tw, s)
                   : launch_c2c<L, MODE, false, false, true, false>(P, io, tw, s);
    case KIND_CONV:
      return P.pad ? launch_conv<L, MODE, true>(P, io, tw, kf, S_q, s)
                   : launch_conv<L, MODE, false>(P, io, tw, kf, S_q, s);
    case KIND_INV:
      if (ot) return P.crop ? launch_c2c<L, MODE, true, true, true, true>(P, io, tw, s)
                            : launch_c2c<L, MODE, true, true, true, false>(P, io, tw, s);
      return P.crop ? launch_c2c<L, MODE, true, true, false, true>(P, io, tw, s)
                    : launch_c2c<L, MODE, true, true, false, false>(P, io, tw, s);
    case KIND_C2R:
      if (ot) return P.crop ? launch_c2r<L, MODE, true, true>(P, io, tw, s)
                            : launch_c2r<L, MODE, true, false>(P, io, tw, s);
      return P.crop ? launch_c2r<L, MODE, false, true>(P, io, tw, s)
                    : launch_c2r<L, MODE, false, false>(P, io, tw, s);
  }
  return hipErrorInvalidValue;
}

#if defined(PSN_PLANE_ONLY)
// ------------------------------------------------------- small-grid plane
// P2, P3 and P4 for one k_p plane at a time, with the plane held in LDS:
// for a small grid the plane after the q transform (S_q x N_r complex) fits,
// so the three passes become one launch and the intermediate A2 never
// reaches HBM.  Phase A transforms the N_r q-lines of the plane from A1 into
// the LDS plane, phase B runs the conv along r on its S_q rows in place, and
// phase C transforms the q-lines back into A1 (which doubles as A4: every
// plane reads all its elements before it writes any, and planes are
// disjoint).  Each line's arithmetic is that of the three separate passes.
struct PlaneParams {
  float2 *data[kMaxBatch];  // A1 of each solve: read in phase A, overwritten in phase C
  const float2 *twq, *twr;
  const float *kf;          // [k_p][k_q'][k_r'] float32, 1/(S1 S2 S3) folded in
  int s_r, s_p;             // A1 element strides along r and p (q-lines are contiguous)
  int H;                    // planes per solve
  int kq_half;              // S_q/2 + 1
  int nplanes;              // H * solves
};

template <int LQ, int LR, bool PADQ, bool PADR> struct PlaneGeo {
  static constexpr int EQ = Shape<LQ>::E, TQ = LQ / EQ, LPWQ = 64 / TQ;
  static constexpr int ER = Shape<LR>::E, TR = LR / ER, LPWR = 64 / TR;
  static constexpr int NQ = PADQ ? LQ / 2 : LQ, NR = PADR ? LR / 2 : LR;
  static constexpr int PLD = NR + 1;  // plane row stride (float2), padded
  static constexpr int XQ = LPWQ * line_lds_slots<LQ>(), XR = LPWR * line_lds_slots<LR>();
  static constexpr int XW = XQ > XR ? XQ : XR;  // exchange slots per wavefront
  // wavefronts: enough for the larger phase (N_r q-lines, or L_q r-rows) in
  // one round, at most 8, and 4 where 8 would not fit the LDS
  static constexpr int NEED_A = (NR + LPWQ - 1) / LPWQ, NEED_B = (LQ + LPWR - 1) / LPWR;
  static constexpr int NEED = NEED_A > NEED_B ? NEED_A : NEED_B;
  static constexpr int NW8 = NEED < 8 ? NEED : 8;
  static constexpr int NW = (LQ * PLD + NW8 * XW) * 8 <= 150 * 1024 ? NW8 : (NW8 < 4 ? NW8 : 4);
  static constexpr int LDS_F2 = LQ * PLD + NW * XW;
};

template <int LQ, int LR, bool PADQ, bool PADR, int MODE>
__global__ __launch_bounds__((PlaneGeo<LQ, LR, PADQ, PADR>::NW * 64)) void plane_kernel(PlaneParams a) {
  using C = PlaneGeo<LQ, LR, PADQ, PADR>;
  constexpr int EQ = C::EQ, TQ = C::TQ, LPWQ = C::LPWQ, ER = C::ER, TR = C::TR, LPWR = C::LPWR;
  constexpr int NR = C::NR, PLD = C::PLD, NW = C::NW, KR = LR / 2 + 1;
  __shared__ float2 smem[C::LDS_F2];
  float2 *plane = smem;
  float2 *xbase = smem + LQ * PLD;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int gq = lane / TQ, tq = lane % TQ, gr = lane / TR, tr = lane % TR;
  // this wavefront's line regions (the split engine works on all of them
  // together) and this line group's own
  float2 *xw = xbase + wave * C::XW;
  float2 *xq = xw + gq * line_lds_slots<LQ>();
  float2 *xr = xw + gr * line_lds_slots<LR>();

  LineEngine<LQ, MODE> engq;
  engq.init(a.twq, lane);
  LineEngine<LR, MODE> engr;
  engr.init(a.twr, lane);

  for (int pl = blockIdx.x; pl < a.nplanes; pl += gridDim.x) {
    const int solve = pl / a.H, kp = pl % a.H;
    float2 *base = a.data[solve] + kp * a.s_p;
    // A: forward along q of the N_r lines (zero-padded half never loaded)
    for (int r0 = 0; r0 < NR; r0 += NW * LPWQ) {
      const int r = r0 + wave * LPWQ + gq;
      const bool ok = r < NR;
      const float2 *line = base + (ok ? r : 0) * a.s_r;
      float2 v[EQ];
#pragma unroll
      for (int i = 0; i < EQ; ++i)
        v[i] = ((!PADQ || i < EQ / 2) && ok) ? line[tq + TQ * i] : make_float2(0.f, 0.f);
      engq.template run<false, PADQ>(v, xq, xw, lane);
      if (ok) {
#pragma unroll
        for (int i = 0; i < EQ; ++i) plane[(tq + TQ * i) * PLD + r] = v[i];
      }
    }
    __syncthreads();
    // B: along r: forward, times K^F (even in k_q: row min(k_q, S_q - k_q)),
    // inverse, crop; in place in the plane
    for (int q0 = 0; q0 < LQ; q0 += NW * LPWR) {
      const int kq = q0 + wave * LPWR + gr;
      const bool ok = kq < LQ;
      const int kqf = ok ? (kq <= LQ / 2 ? kq : LQ - kq) : 0;
      const float *krow = a.kf + (kp * a.kq_half + kqf) * KR;
      float2 *row = plane + (ok ? kq : 0) * PLD;
      float2 v[ER];
#pragma unroll
      for (int i = 0; i < ER; ++i)
        v[i] = (!PADR || i < ER / 2) ? row[tr + TR * i] : make_float2(0.f, 0.f);
      engr.template run<false, PADR>(v, xr, xw, lane);
#pragma unroll
      for (int i = 0; i < ER; ++i) {
        const float kv = i < ER / 2 ? krow[tr + TR * i] : krow[LR - tr - TR * i];
        v[i] = make_float2(v[i].x * kv, v[i].y * kv);
      }
      engr.template run<true, false, PADR>(v, xr, xw, lane);
      if (ok) {
#pragma unroll
        for (int i = 0; i < ER; ++i)
          if (!PADR || i < ER / 2) row[tr + TR * i] = v[i];
      }
    }
    __syncthreads();
    // C: inverse along q, crop, back into A1
    for (int r0 = 0; r0 < NR; r0 += NW * LPWQ) {
      const int r = r0 + wave * LPWQ + gq;
      const bool ok = r < NR;
      float2 v[EQ];
#pragma unroll
      for (int i = 0; i < EQ; ++i) v[i] = plane[(tq + TQ * i) * PLD + (ok ? r : 0)];
      engq.template run<true, false, PADQ>(v, xq, xw, lane);
      if (ok) {
        float2 *line = base + r * a.s_r;
#pragma unroll
        for (int i = 0; i < EQ; ++i)
          if (!PADQ || i < EQ / 2) st_out<TQ * 8>(&line[tq + TQ * i], v[i]);
      }
    }
    __syncthreads();  // the plane is free for the next one
  }
}

namespace {
template <int LQ, int LR, bool PADQ, bool PADR, int MODE>
hipError_t launch_plane_t(const PlaneParams &a, hipStream_t s) {
  auto k = plane_kernel<LQ, LR, PADQ, PADR, MODE>;
  constexpr int NT = PlaneGeo<LQ, LR, PADQ, PADR>::NW * 64;
  const int grid = persistent_grid(k, NT, a.nplanes);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}
}  // namespace

// launch_plane's per-precision half (each precision is its own object); the
// caller has checked plane_available
template <int MODE>
hipError_t launch_plane_for_mode(const Geometry &g, const PassIO &io, const float2 *twq,
                                 const float2 *twr, const float *kf, hipStream_t s) {
  const Pass &P2 = g.pass[1];
  PlaneParams a;
  for (int j = 0; j < kMaxBatch; ++j) a.data[j] = j < io.count ? static_cast<float2 *>(io.out[j]) : nullptr;
  a.twq = twq;
  a.twr = twr;
  a.kf = kf;
  a.s_r = int(P2.in_s[1]);
  a.s_p = int(P2.in_s[2]);
  a.H = P2.ext_batch;
  a.kq_half = P2.L / 2 + 1;
  a.nplanes = a.H * io.count;
  const int LQ = P2.L, LR = g.pass[2].L;
  const bool pq = P2.pad, pr = g.pass[2].pad;
#define PSN_X(a_, b_, c_, d_) \
  if (LQ == a_ && LR == b_ && pq == c_ && pr == d_) return launch_plane_t<a_, b_, c_, d_, MODE>(a, s);
  PSN_PLANE_CASES(PSN_X)
#undef PSN_X
  return hipErrorInvalidValue;
}
template hipError_t launch_plane_for_mode<PSN_ONLY_MODE>(const Geometry &, const PassIO &,
                                                         const float2 *, const float2 *,
                                                         const float *, hipStream_t);
#endif  // PSN_PLANE_ONLY

#if defined(PSN_ONLY_LENGTH) && defined(PSN_ONLY_MODE)
template hipError_t launch_for_mode<PSN_ONLY_LENGTH, PSN_ONLY_MODE>(const Pass &, const PassIO &,
                                                                    const float2 *, const float *,
                                                                    int, hipStream_t);
#endif

#else  // PSN_DISPATCH_ONLY

hipError_t launch_pass(const Pass &P, const PassIO &io, const float2 *tw, const float *kf,
                       int S_q, int mode, hipStream_t s) {
  if (io.count < 1 || io.count > kMaxBatch) return hipErrorInvalidValue;
  if (mode < MODE_FP32 || mode > MODE_SPLIT_BF16) return hipErrorInvalidValue;
  // shapes the layouts promise (checked here so no kernel ever runs on a
  // layout it was not written for)
  if (P.kind == KIND_R2C && !P.out_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_FWD && !P.out_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_INV && !P.in_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_C2R && !P.in_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_CONV && (P.in_tiled || P.out_tiled)) return hipErrorInvalidValue;
  switch (P.L) {
#define PSN_CASE(LL)                                                           \
  case LL:                                                                     \
    if (mode == MODE_SPLIT_FP16) return launch_for_mode<LL, MODE_SPLIT_FP16>(P, io, tw, kf, S_q, s); \
    if (mode == MODE_SPLIT_BF16) return launch_for_mode<LL, MODE_SPLIT_BF16>(P, io, tw, kf, S_q, s); \
    return launch_for_mode<LL, MODE_FP32>(P, io, tw, kf, S_q, s);
    PSN_CASE(4) PSN_CASE(6) PSN_CASE(8) PSN_CASE(12) PSN_CASE(16) PSN_CASE(24) PSN_CASE(32)
    PSN_CASE(48) PSN_CASE(64) PSN_CASE(96) PSN_CASE(128) PSN_CASE(192) PSN_CASE(256)
    PSN_CASE(384) PSN_CASE(512) PSN_CASE(768) PSN_CASE(1024)
#undef PSN_CASE
  }
  return hipErrorInvalidValue;
}

int pass_tile_lines(const Pass &P, int sched, int mode) {
  if (sched < 0 || sched >= kSchedules) return 0;
  const int ts = sched & 3;  // the XCD-order bit does not change the tile
  switch (P.L) {
#define PSN_CASE(LL) \
  case LL: return tile_lines_of<LL>(P, ts);
    PSN_CASE(4) PSN_CASE(6) PSN_CASE(8) PSN_CASE(12) PSN_CASE(16) PSN_CASE(24) PSN_CASE(32)
    PSN_CASE(48) PSN_CASE(64) PSN_CASE(96) PSN_CASE(128) PSN_CASE(192) PSN_CASE(256)
    PSN_CASE(384) PSN_CASE(512) PSN_CASE(768) PSN_CASE(1024)
#undef PSN_CASE
  }
  return 0;
}

bool plane_available(const Geometry &g, int mode) {
  if (mode < MODE_FP32 || mode > MODE_SPLIT_BF16) return false;
  return plane_geometry_ok(g);
}

hipError_t launch_plane(const Geometry &g, int mode, const PassIO &io, const float2 *twq,
                        const float2 *twr, const float *kf, hipStream_t s) {
  if (io.count < 1 || io.count > kMaxBatch || !plane_available(g, mode)) return hipErrorInvalidValue;
  if (mode == MODE_SPLIT_FP16) return launch_plane_for_mode<MODE_SPLIT_FP16>(g, io, twq, twr, kf, s);
  if (mode == MODE_SPLIT_BF16) return launch_plane_for_mode<MODE_SPLIT_BF16>(g, io, twq, twr, kf, s);
  return launch_plane_for_mode<MODE_FP32>(g, io, twq, twr, kf, s);
}

#endif  // PSN_DISPATCH_ONLY

}  // namespace psn
