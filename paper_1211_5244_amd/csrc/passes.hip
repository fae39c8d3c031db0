// passes.hip - the five passes of one solve (paper, Section 3).
//
//   P1 R2C    real-to-complex along p of the density, zero-padded half
//             skipped (spread_X + 1DFFT_X of the paper's step list)
//   P2 FWD    forward along q (transpose/spread_Y + 1DFFT_Y)
//   P3 CONV   forward along r, times K^F, inverse along r, crop
//             (spread_Z + 1DFFT_Z + kernel multiplication + inverse_1DFFT_Z +
//             compactification_Z, with the kernel stored in pass order so no
//             final transpose is needed)
//   P4 INV    inverse along q, crop (compactification_Y + transpose)
//   P5 C2R    complex-to-real along p, crop (inverse_1DFFT_X +
//             compactification_X)
//
// The paper's separate transpose/spread/compaction kernels do not exist here:
// zero padding happens in registers at load time, crops at store time, and
// the transposes are the LDS staging of tiled sides (plan.cpp picks layouts
// so every pass has at most one strided side per array, read or written as
// rows of W consecutive lines).  Each HBM array is read and written once
// per pass.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "kernels.h"

namespace psn {

template <int L>
hipError_t launch_for_length(const Pass &P, const void *in, void *out, const float2 *tw,
                             const float *kf, int S_q, hipStream_t s);

#if !defined(PSN_DISPATCH_ONLY)

struct PassParams {
  const void *in;
  void *out;
  const float2 *tw;
  long long in_sl, in_st, in_sb;
  long long out_sl, out_st, out_sb;
  int ext_tile;
  int tiles_per_batch;
  int ntiles;
};

template <int L> struct TileCfg {
  static constexpr int E = Shape<L>::E, T = L / E, LPW = 64 / T;
  static constexpr int NW = LPW >= 16 ? 1 : 16 / LPW;  // waves per workgroup
  static constexpr int W = NW * LPW;                    // lines per tile
  static constexpr int NTHREADS = NW * 64;
  static constexpr int SLOTS = line_lds_slots<L>();
  static constexpr int LD = W + 1;  // row stride of a staged tile (elements)
  static constexpr int TILE_F2 = (L + 1) * LD;
  static constexpr int XCH_F2 = W * SLOTS;
  static constexpr int LDS_F2 = TILE_F2 > XCH_F2 ? TILE_F2 : XCH_F2;
};

// KIND: KIND_R2C, KIND_FWD, KIND_INV or KIND_C2R.  PC: pad (R2C/FWD) or
// crop (INV/C2R) along the line axis.
template <int L, int KIND, bool IN_TILED, bool OUT_TILED, bool PC>
__global__ __launch_bounds__(TileCfg<L>::NTHREADS) void pass_kernel(PassParams a) {
  using C = TileCfg<L>;
  constexpr int E = C::E, T = C::T, LPW = C::LPW, W = C::W, LD = C::LD, NT = C::NTHREADS;
  constexpr bool REAL_IN = KIND == KIND_R2C;
  constexpr bool REAL_OUT = KIND == KIND_C2R;
  constexpr bool INV = KIND == KIND_INV || KIND == KIND_C2R;
  constexpr bool PAD = !INV && PC;
  constexpr bool CROP = INV && PC;
  constexpr int ROWS_IN = KIND == KIND_C2R ? L / 2 + 1 : (PAD ? L / 2 : L);
  constexpr int ROWS_OUT = KIND == KIND_R2C ? L / 2 + 1 : (CROP ? L / 2 : L);

  __shared__ float2 smem[C::LDS_F2];
  float *smem_f = reinterpret_cast<float *>(smem);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / T, t = lane % T;
  const int c = wave * LPW + g;  // my line within the tile
  float2 *xch = smem + c * C::SLOTS;

  Twiddles<L> tw;
  tw.load(a.tw, t);

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int a0 = (tile % a.tiles_per_batch) * W;
    const long long b = tile / a.tiles_per_batch;
    const int ncols = min(W, a.ext_tile - a0);
    const bool valid = c < ncols;
    float2 v[E];

    __syncthreads();  // the previous tile is done with smem
    if constexpr (IN_TILED) {
      // rows of ncols consecutive lines; a.in_st == 1
      if constexpr (REAL_IN) {
        const float *in = static_cast<const float *>(a.in) + b * a.in_sb + a0;
        for (int idx = tid; idx < ROWS_IN * W; idx += NT) {
          const int row = idx / W, col = idx % W;
          if (col < ncols) smem_f[row * LD + col] = in[row * a.in_sl + col];
        }
      } else {
        const float2 *in = static_cast<const float2 *>(a.in) + b * a.in_sb + a0;
        for (int idx = tid; idx < ROWS_IN * W; idx += NT) {
          const int row = idx / W, col = idx % W;
          if (col < ncols) smem[row * LD + col] = in[row * a.in_sl + col];
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int k = t + T * i;
        if constexpr (REAL_IN) {
          v[i] = (!PAD || i < E / 2) ? make_float2(smem_f[k * LD + c], 0.f) : make_float2(0.f, 0.f);
        } else if constexpr (KIND == KIND_C2R) {
          // Hermitian half X[0..L/2]; X[k] = conj(X[L-k]) above L/2
          if (i < E / 2) {
            v[i] = smem[k * LD + c];
          } else {
            const bool direct = (k == L / 2);
            const float2 x = smem[(direct ? k : L - k) * LD + c];
            v[i] = direct ? x : make_float2(x.x, -x.y);
          }
        } else {
          v[i] = (!PAD || i < E / 2) ? smem[k * LD + c] : make_float2(0.f, 0.f);
        }
      }
      __syncthreads();  // the tile region becomes exchange space
    } else {
      // whole lines; a.in_sl == 1
      const long long base = (long long)(a0 + c) * a.in_st + b * a.in_sb;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int k = t + T * i;
        if ((!PAD || i < E / 2) && valid) {
          if constexpr (REAL_IN) v[i] = make_float2(static_cast<const float *>(a.in)[base + k], 0.f);
          else v[i] = static_cast<const float2 *>(a.in)[base + k];
        } else {
          v[i] = make_float2(0.f, 0.f);
        }
      }
      static_assert(KIND != KIND_C2R || IN_TILED, "C2R reads a staged tile");
    }

    fft_line<L, INV>(v, tw, xch, t);

    if constexpr (OUT_TILED) {
      __syncthreads();  // every line is done exchanging
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int k = t + T * i;
        bool keep;
        if constexpr (KIND == KIND_R2C) keep = (i < E / 2) || (i == E / 2 && t == 0);
        else keep = !CROP || i < E / 2;
        if (keep) {
          if constexpr (REAL_OUT) smem_f[k * LD + c] = v[i].x;
          else smem[k * LD + c] = v[i];
        }
      }
      __syncthreads();
      if constexpr (REAL_OUT) {
        float *out = static_cast<float *>(a.out) + b * a.out_sb + a0;
        for (int idx = tid; idx < ROWS_OUT * W; idx += NT) {
          const int row = idx / W, col = idx % W;
          if (col < ncols) out[row * a.out_sl + col] = smem_f[row * LD + col];
        }
      } else {
        float2 *out = static_cast<float2 *>(a.out) + b * a.out_sb + a0;
        for (int idx = tid; idx < ROWS_OUT * W; idx += NT) {
          const int row = idx / W, col = idx % W;
          if (col < ncols) out[row * a.out_sl + col] = smem[row * LD + col];
        }
      }
    } else {
      static_assert(KIND != KIND_R2C, "R2C writes a staged tile");
      if (valid) {
        const long long base = (long long)(a0 + c) * a.out_st + b * a.out_sb;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int k = t + T * i;
          if (!CROP || i < E / 2) {
            if constexpr (REAL_OUT) static_cast<float *>(a.out)[base + k] = v[i].x;
            else static_cast<float2 *>(a.out)[base + k] = v[i];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- P3
struct ConvParams {
  float2 *data;       // A2, lines along r contiguous
  const float *kf;    // [k_p][k_q'][k_r'] float32, 1/(S1 S2 S3) folded in
  const float2 *tw;
  long long st_q, st_p;  // element strides of line (k_p, k_q)
  int S_q;
  int kq_half;        // S_q/2 + 1
  long long nrows;    // H * kq_half kernel rows
};

constexpr int kConvWaves = 4;

template <int L, bool PC>
__global__ __launch_bounds__(kConvWaves * 64) void conv_kernel(ConvParams a) {
  constexpr int E = Shape<L>::E, T = L / E, LPW = 64 / T, KR = L / 2 + 1;
  constexpr int SLOTS = line_lds_slots<L>();
  __shared__ float2 smem[kConvWaves * LPW * SLOTS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / T, t = lane % T;
  float2 *xch = smem + (wave * LPW + g) * SLOTS;

  Twiddles<L> tw;
  tw.load(a.tw, t);

  const long long ngroups = (long long)gridDim.x * kConvWaves * LPW;
  // One kernel row (k_p, k_q') serves the lines k_q = k_q' and S_q - k_q':
  // K^F is even in k_q, so the row is read from HBM once for both.
  for (long long row = ((long long)blockIdx.x * kConvWaves + wave) * LPW + g; row < a.nrows;
       row += ngroups) {
    const int kp = int(row / a.kq_half);
    const int kqf = int(row % a.kq_half);
    float kv[E];
    const float *krow = a.kf + row * KR;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = t + T * i;
      kv[i] = krow[k <= L / 2 ? k : L - k];
    }
    const int nrep = (kqf == 0 || 2 * kqf == a.S_q) ? 1 : 2;
    for (int rep = 0; rep < nrep; ++rep) {
      const int kq = rep == 0 ? kqf : a.S_q - kqf;
      float2 *line = a.data + kp * a.st_p + kq * a.st_q;
      float2 v[E];
#pragma unroll
      for (int i = 0; i < E; ++i)
        v[i] = (!PC || i < E / 2) ? line[t + T * i] : make_float2(0.f, 0.f);
      fft_line<L, false>(v, tw, xch, t);
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = make_float2(v[i].x * kv[i], v[i].y * kv[i]);
      fft_line<L, true>(v, tw, xch, t);
#pragma unroll
      for (int i = 0; i < E; ++i)
        if (!PC || i < E / 2) line[t + T * i] = v[i];
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

template <int L, int KIND, bool IT, bool OT, bool PC>
hipError_t launch_tiled(const Pass &P, const void *in, void *out, const float2 *tw,
                        hipStream_t s) {
  using C = TileCfg<L>;
  PassParams a;
  a.in = in;
  a.out = out;
  a.tw = tw;
  a.in_sl = P.in_s[0];
  a.in_st = P.in_s[1];
  a.in_sb = P.in_s[2];
  a.out_sl = P.out_s[0];
  a.out_st = P.out_s[1];
  a.out_sb = P.out_s[2];
  a.ext_tile = P.ext_tile;
  a.tiles_per_batch = (P.ext_tile + C::W - 1) / C::W;
  const long long nt = (long long)a.tiles_per_batch * P.ext_batch;
  a.ntiles = int(nt);
  const int lds_bytes = C::LDS_F2 * 8;
  const int per_cu = lds_bytes > 0 ? (160 * 1024) / lds_bytes : 8;
  const long long cap = (long long)device_cu_count() * (per_cu > 0 ? per_cu : 1) * 4;
  const int grid = int(nt < cap ? nt : cap);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((pass_kernel<L, KIND, IT, OT, PC>), dim3(grid), dim3(C::NTHREADS), 0, s, a);
  return hipGetLastError();
}

template <int L, bool PC>
hipError_t launch_conv(const Pass &P, void *data, const float2 *tw, const float *kf, int S_q,
                       hipStream_t s) {
  ConvParams a;
  a.data = static_cast<float2 *>(data);
  a.kf = kf;
  a.tw = tw;
  a.st_q = P.in_s[1];
  a.st_p = P.in_s[2];
  a.S_q = S_q;
  a.kq_half = S_q / 2 + 1;
  a.nrows = (long long)P.ext_batch * a.kq_half;
  constexpr int LPW = 64 / (L / Shape<L>::E);
  const long long groups_per_block = (long long)kConvWaves * LPW;
  long long blocks = (a.nrows + groups_per_block - 1) / groups_per_block;
  const long long cap = (long long)device_cu_count() * 8;
  if (blocks > cap) blocks = cap;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((conv_kernel<L, PC>), dim3(int(blocks)), dim3(kConvWaves * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <int L>
hipError_t launch_for_length(const Pass &P, const void *in, void *out, const float2 *tw,
                             const float *kf, int S_q, hipStream_t s) {
  const bool it = P.in_tiled, ot = P.out_tiled;
  switch (P.kind) {
    case KIND_R2C:
      if (it) return P.pad ? launch_tiled<L, KIND_R2C, true, true, true>(P, in, out, tw, s)
                           : launch_tiled<L, KIND_R2C, true, true, false>(P, in, out, tw, s);
      return P.pad ? launch_tiled<L, KIND_R2C, false, true, true>(P, in, out, tw, s)
                   : launch_tiled<L, KIND_R2C, false, true, false>(P, in, out, tw, s);
    case KIND_FWD:
      if (it) return P.pad ? launch_tiled<L, KIND_FWD, true, true, true>(P, in, out, tw, s)
                           : launch_tiled<L, KIND_FWD, true, true, false>(P, in, out, tw, s);
      return P.pad ? launch_tiled<L, KIND_FWD, false, true, true>(P, in, out, tw, s)
                   : launch_tiled<L, KIND_FWD, false, true, false>(P, in, out, tw, s);
    case KIND_CONV:
      return P.pad ? launch_conv<L, true>(P, out, tw, kf, S_q, s)
                   : launch_conv<L, false>(P, out, tw, kf, S_q, s);
    case KIND_INV:
      if (ot) return P.crop ? launch_tiled<L, KIND_INV, true, true, true>(P, in, out, tw, s)
                            : launch_tiled<L, KIND_INV, true, true, false>(P, in, out, tw, s);
      return P.crop ? launch_tiled<L, KIND_INV, true, false, true>(P, in, out, tw, s)
                    : launch_tiled<L, KIND_INV, true, false, false>(P, in, out, tw, s);
    case KIND_C2R:
      if (ot) return P.crop ? launch_tiled<L, KIND_C2R, true, true, true>(P, in, out, tw, s)
                            : launch_tiled<L, KIND_C2R, true, true, false>(P, in, out, tw, s);
      return P.crop ? launch_tiled<L, KIND_C2R, true, false, true>(P, in, out, tw, s)
                    : launch_tiled<L, KIND_C2R, true, false, false>(P, in, out, tw, s);
  }
  return hipErrorInvalidValue;
}

#if defined(PSN_ONLY_LENGTH)
template hipError_t launch_for_length<PSN_ONLY_LENGTH>(const Pass &, const void *, void *,
                                                       const float2 *, const float *, int,
                                                       hipStream_t);
#endif

#else  // PSN_DISPATCH_ONLY

hipError_t launch_pass(const Pass &P, const void *in, void *out, const float2 *tw,
                       const float *kf, int S_q, hipStream_t s) {
  // shapes the layouts promise (checked here so no kernel ever runs on a
  // layout it was not written for)
  if (P.kind == KIND_R2C && !P.out_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_FWD && !P.out_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_INV && !P.in_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_C2R && !P.in_tiled) return hipErrorInvalidValue;
  if (P.kind == KIND_CONV && (P.in_tiled || P.out_tiled)) return hipErrorInvalidValue;
  switch (P.L) {
#define PSN_CASE(LL) \
  case LL: return launch_for_length<LL>(P, in, out, tw, kf, S_q, s);
    PSN_CASE(4) PSN_CASE(6) PSN_CASE(8) PSN_CASE(12) PSN_CASE(16) PSN_CASE(24) PSN_CASE(32)
    PSN_CASE(48) PSN_CASE(64) PSN_CASE(96) PSN_CASE(128) PSN_CASE(192) PSN_CASE(256)
    PSN_CASE(384) PSN_CASE(512) PSN_CASE(768) PSN_CASE(1024)
#undef PSN_CASE
  }
  return hipErrorInvalidValue;
}

#endif  // PSN_DISPATCH_ONLY

}  // namespace psn
