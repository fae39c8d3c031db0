// queue.hip - the persistent batched solve: one launch, a pass-ordered work
// queue, per-(solve, pass) completion counters (protocol in queue.h).
//
// The engine is generic in the line length: a tile of C complex lines sits
// in LDS and each radix stage (2, 3, 4 or 8, any order, chosen per length by
// the batch autotuner) is a Stockham step between two LDS buffers.  The
// passes are those of the grouped launches (paper, Section 3): P1 packs two
// real lines per complex line and separates their spectra, P2/P4 transform
// along q, P3 transforms along r, multiplies by K^F and transforms back, P5
// rebuilds two real lines from their Hermitian halves.  Zero padding is
// applied at load (and the first stage skips the zero half), crops at store;
// pencils that are all zero are never loaded (the pass extents cover only
// the nonzero ones).
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "kernels.h"
#include "queue.h"

namespace psn {
namespace {

// LDS slot of complex element i of a tile: one pad slot per 32.
__device__ __forceinline__ int qx(int i) { return i + (i >> 5); }
constexpr int kQSlots = kQMaxTile + kQMaxTile / 32;
constexpr int kQTwSlots = 1024;  // the longest line's twiddle table

__device__ __forceinline__ float2 fzero() { return make_float2(0.f, 0.f); }

// x / d and x % d for d = 2^shift (three = 0) or 3 * 2^shift (three = 1):
// 0xAAAAAAAB / 2^33 rounds up 1/3 closely enough to be exact for every
// 32-bit x.
__device__ __forceinline__ int qdiv(int x, int shift, int three) {
  const unsigned y = unsigned(x) >> shift;
  return int(three ? __umulhi(y, 0xAAAAAAABu) >> 1 : y);
}

// f(c, j) for c < 2^c_log2, j < nj, spread over the workgroup's threads.
// line_fast: consecutive threads take consecutive lines c (the side whose
// tile of lines is contiguous); otherwise they walk along a line, 64 at a
// time (fewer for short lines).
template <typename F>
__device__ __forceinline__ void q_for(int c_log2, int nj, bool line_fast, F &&f) {
  const int tid = threadIdx.x;
  if (line_fast) {
    const int lc = c_log2 < 8 ? c_log2 : 8;
    const int c0 = tid & ((1 << lc) - 1), j0 = tid >> lc;
    for (int j = j0; j < nj; j += kQThreads >> lc)
      for (int c = c0; c < (1 << c_log2); c += 1 << lc) f(c, j);
  } else {
    int lj = 6;
    while (lj > 0 && (1 << (lj - 1)) >= nj) --lj;  // 2^lj >= nj, at most 64
    const int j0 = tid & ((1 << lj) - 1), c0 = tid >> lj;
    for (int c = c0; c < (1 << c_log2); c += kQThreads >> lj)
      for (int j = j0; j < nj; j += 1 << lj) f(c, j);
  }
}

// The fields of an item's pass that its tiles use, as 32-bit values in
// registers (every array is below 2^31 elements).
struct QTile {
  int in_s[3], out_s[3];
  int kind, L, n_in, n_out, pad, ext_tile, W, tiles_a, c_log2, nrad;
};

// The stage tables of the item's transform, staged in LDS with its twiddles
// (indexed by stage at run time, they would otherwise live in scratch).
struct QStages {
  int rad[kQMaxRadices], ns_shift[kQMaxRadices], ns_three[kQMaxRadices], tw_step[kQMaxRadices];
};

// One radix-R Stockham stage over the tile: butterfly j of line c reads
// src[c][j + m L/R] and writes dst[c][(j / NS) NS R + j % NS + m NS], with
// twiddles w^(k m) = tw[k m step], k = j % NS, from the LDS table.
template <int R, bool INV>
__device__ __forceinline__ void q_stage_r(const float2 *src, float2 *dst, const QTile &P, const QStages &st,
                                          int s, bool zhi, const float2 *tw) {
  const int L = P.L, Lr = L / R;
  const int sh = st.ns_shift[s], th = st.ns_three[s], step = st.tw_step[s];
  const bool first = s == 0;
  q_for(P.c_log2, Lr, false, [&](int c, int j) {
    const int base = c * L;
    const int q = first ? j : qdiv(j, sh, th);
    const int k = first ? 0 : j - q * ((th ? 3 : 1) << sh);
    float2 x[R];
    if (zhi && R % 2 == 0) {
#pragma unroll
      for (int m = 0; m < R / 2; ++m) x[m] = src[qx(base + j + m * Lr)];
#pragma unroll
      for (int m = R / 2; m < R; ++m) x[m] = fzero();
      if constexpr (R % 2 == 0) dft<R, INV, true>(x);
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m) x[m] = src[qx(base + j + m * Lr)];
      if (!first) {
#pragma unroll
        for (int m = 1; m < R; ++m) x[m] = cmul_tw<INV>(x[m], tw[k * m * step]);
      }
      dft<R, INV, false>(x);
    }
    const int ns = first ? 1 : ((th ? 3 : 1) << sh);
    const int o = base + q * ns * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) dst[qx(o + m * ns)] = x[m];
  });
}

// The whole line transform of the tile in buf[cur] (result in buf[cur] on
// return, cur updated).  zhi: the upper half of every input line is zero
// (the first stage, which has no twiddles, skips it).
template <bool INV>
__device__ void q_fft(float2 (*buf)[kQSlots], int &cur, const QTile &P, const QStages &st, bool zhi,
                      const float2 *tw) {
  for (int s = 0; s < P.nrad; ++s) {
    const int R = st.rad[s];
    const bool z = zhi && s == 0;
    const float2 *src = buf[cur];
    float2 *dst = buf[cur ^ 1];
    switch (R) {
      case 2: q_stage_r<2, INV>(src, dst, P, st, s, z, tw); break;
      case 3: q_stage_r<3, INV>(src, dst, P, st, s, false, tw); break;
      case 4: q_stage_r<4, INV>(src, dst, P, st, s, z, tw); break;
      default: q_stage_r<8, INV>(src, dst, P, st, s, z, tw); break;
    }
    cur ^= 1;
    __syncthreads();
  }
}

// Offset of element j of tile line a, batch b on one side of a pass (every
// array is below 2^31 elements, so the sum of these non-negative terms fits).
__device__ __forceinline__ int q_off(const int *s, int j, int a, int b) {
  return j * s[0] + a * s[1] + b * s[2];
}

// One tile: load, transform, store.  Arrays by pass kind: P1 rho -> a1,
// P2 a1 -> a2, P3 a2 -> a2, P4 a2 -> a1, P5 a1 -> V.  tw: the pass's twiddle
// table in LDS.
__device__ void q_tile(float2 (*buf)[kQSlots], const float2 *tw, const QStages &st,
                       const float *__restrict__ kf, int S_q, int kq_half, const QTile &P,
                       const QSolve &S, int tile) {
  const int ta = tile % P.tiles_a, b = tile / P.tiles_a, a0 = ta * P.W;
  const int L = P.L, cl = P.c_log2;
  const bool in_line = P.in_s[0] == 1, out_line = P.out_s[0] == 1;
  int cur = 0;
  float2 *X = buf[0];

  if (P.kind == KIND_R2C) {
    // real lines 2c and 2c + 1 as the real and imaginary parts of line c
    const float *__restrict__ in = S.rho;
    q_for(cl + 1, L, !in_line, [&](int w, int j) {
      const int a = a0 + w;
      const float v = (a < P.ext_tile && j < P.n_in) ? in[q_off(P.in_s, j, a, b)] : 0.f;
      reinterpret_cast<float *>(&X[qx((w >> 1) * L + j)])[w & 1] = v;
    });
  } else if (P.kind == KIND_C2R) {
    // Z = X_a + i X_b from the Hermitian halves of lines 2c and 2c + 1 (the
    // imaginary parts of the k = 0 and k = L/2 terms are not part of a real
    // line's spectrum and are dropped)
    const float2 *__restrict__ in = S.a1;
    const int h = L / 2;
    q_for(cl, L, !in_line, [&](int c, int j) {
      const int a = a0 + 2 * c;
      float2 z = fzero();
      if (a < P.ext_tile) {
        const int m = j <= h ? j : L - j;
        float2 xa = in[q_off(P.in_s, m, a, b)];
        float2 xb = a + 1 < P.ext_tile ? in[q_off(P.in_s, m, a + 1, b)] : fzero();
        if (m == 0 || m == h) { xa.y = 0.f; xb.y = 0.f; }
        z = j <= h ? make_float2(xa.x - xb.y, xa.y + xb.x) : make_float2(xa.x + xb.y, xb.x - xa.y);
      }
      X[qx(c * L + j)] = z;
    });
  } else {
    const float2 *__restrict__ in = P.kind == KIND_FWD ? S.a1 : S.a2;
    q_for(cl, L, !in_line, [&](int c, int j) {
      const int a = a0 + c;
      X[qx(c * L + j)] = (a < P.ext_tile && j < P.n_in) ? in[q_off(P.in_s, j, a, b)] : fzero();
    });
  }
  __syncthreads();

  if (P.kind == KIND_INV || P.kind == KIND_C2R) q_fft<true>(buf, cur, P, st, false, tw);
  else q_fft<false>(buf, cur, P, st, P.pad != 0, tw);

  if (P.kind == KIND_CONV) {
    // times K^F (even along q and r): row (k_p, min(k_q, S_q - k_q))
    float2 *Y = buf[cur];
    const int KR = L / 2 + 1;
    q_for(cl, L, false, [&](int c, int j) {
      const int kq = a0 + c;
      if (kq < P.ext_tile) {
        const int kqf = kq <= S_q - kq ? kq : S_q - kq;
        const float kv = kf[(b * kq_half + kqf) * KR + (j <= L - j ? j : L - j)];
        const float2 v = Y[qx(c * L + j)];
        Y[qx(c * L + j)] = make_float2(v.x * kv, v.y * kv);
      }
    });
    __syncthreads();
    q_fft<true>(buf, cur, P, st, false, tw);
  }

  const float2 *Y = buf[cur];
  if (P.kind == KIND_R2C) {
    // X_a[k] = (Z[k] + conj Z[L-k]) / 2, X_b[k] = (Z[k] - conj Z[L-k]) / (2i)
    float2 *__restrict__ out = S.a1;
    q_for(cl + 1, P.n_out, !out_line, [&](int w, int k) {
      const int a = a0 + w;
      if (a < P.ext_tile) {
        const int c = w >> 1;
        const float2 zk = Y[qx(c * L + k)], zl = Y[qx(c * L + (k == 0 ? 0 : L - k))];
        const float2 v = (w & 1) ? make_float2(0.5f * (zk.y + zl.y), 0.5f * (zl.x - zk.x))
                                 : make_float2(0.5f * (zk.x + zl.x), 0.5f * (zk.y - zl.y));
        out[q_off(P.out_s, k, a, b)] = v;
      }
    });
  } else if (P.kind == KIND_C2R) {
    float *__restrict__ out = S.V;
    q_for(cl + 1, P.n_out, !out_line, [&](int w, int j) {
      const int a = a0 + w;
      if (a < P.ext_tile) {
        const float2 z = Y[qx((w >> 1) * L + j)];
        out[q_off(P.out_s, j, a, b)] = (w & 1) ? z.y : z.x;
      }
    });
  } else {
    float2 *__restrict__ out = P.kind == KIND_INV ? S.a1 : S.a2;
    q_for(cl, P.n_out, !out_line, [&](int c, int j) {
      const int a = a0 + c;
      if (a < P.ext_tile) out[q_off(P.out_s, j, a, b)] = Y[qx(c * L + j)];
    });
  }
  __syncthreads();  // the tile buffers are free again
}

// Makes the workgroup's stores visible at agent scope: every wavefront
// writes its own stores back from the XCD's L2 (release fence) and waits for
// that write-back to finish (the fence alone may leave it in flight), then
// the barrier orders all of them before wave 0's counter adds.
__device__ __forceinline__ void q_release_all() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Counts the held items complete: one add per item and one per level (wave 0
// only, after q_release_all).
__device__ __forceinline__ void q_count(const QParams &a, const int *pend, int npend, int level) {
  const int lane = threadIdx.x;
  unsigned *segc = a.state + kQStateHeader;
  if (lane < npend) __hip_atomic_fetch_add(&segc[pend[lane]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (lane == 0)
    __hip_atomic_fetch_add(&a.state[kQLevel + level], unsigned(npend), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single-lane work sits in branches that are uniform per wavefront (wave 0):
// a branch on the loop-invariant threadIdx.x == 0 around the dequeue and the
// release would let the compiler give lane 0 a loop of its own around the
// barriers, which the other lanes of its wavefront would then run alone.
__global__ __launch_bounds__(kQThreads) void queue_kernel(QParams a) {
  __shared__ float2 buf[2][kQSlots];
  __shared__ float2 tw[kQTwSlots];
  __shared__ QStages st;
  __shared__ int s_item, s_full;
  __shared__ int s_pend[kQPending];
  const int tid = threadIdx.x;
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < 64;
  const unsigned one = tid == 0 ? 1u : 0u;
  unsigned *state = a.state;
  unsigned *segc = state + kQStateHeader;

  int npend = 0, pend_level = 0, acq_level = -1;
  const float2 *tw_src = nullptr;  // the table staged in tw
  for (;;) {
    if (wave0) {
      const unsigned got = __hip_atomic_fetch_add(&state[kQHead], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tid == 0) s_item = int(got);
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= a.nitems) break;
    const int si = q_find_seg(a.segs, a.nseg, item);
    const QSeg sg = a.segs[si];
    const int k = sg.pass;

    if (q_must_flush(npend, pend_level, k)) {
      q_release_all();
      if (wave0) q_count(a, s_pend, npend, pend_level);
      npend = 0;
    }
    if (q_must_wait(k, acq_level)) {
      if (wave0) {
        const int dep = q_dep_seg(si, a.nsolve);
        const unsigned need_seg = unsigned(a.segs[dep].count), need_lvl = unsigned(a.level_items[k - 1]);
        int full = 0;
        for (unsigned spins = 0;; ++spins) {
          if (__hip_atomic_load(&state[kQLevel + k - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need_lvl) {
            full = 1;
            break;
          }
          if (__hip_atomic_load(&segc[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need_seg) break;
          if (__hip_atomic_load(&state[kQAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          if (spins >= a.spin_limit) {
            __hip_atomic_fetch_or(&state[kQError], kQErrSpin * one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&state[kQAbort], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        // invalidate this XCD's L2 (and the compute unit's L1) for every
        // wavefront of the workgroup: the barrier below orders their loads
        // after it
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
        if (tid == 0) s_full = full;
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_full)) acq_level = k - 1;
    }

    // the item's descriptors as values: read once, not again after every
    // store (which the compiler could not tell apart from them)
    const QSolve S = a.solves[sg.solve];
    const QPass &Pg = a.geoms[S.geom].pass[k];
    QTile P;  // the scalar fields (the stage tables go to LDS)
    for (int i = 0; i < 3; ++i) {
      P.in_s[i] = int(Pg.in_s[i]);
      P.out_s[i] = int(Pg.out_s[i]);
    }
    P.kind = Pg.kind; P.L = Pg.L; P.n_in = Pg.n_in; P.n_out = Pg.n_out; P.pad = Pg.pad;
    P.ext_tile = Pg.ext_tile; P.W = Pg.W; P.tiles_a = Pg.tiles_a; P.c_log2 = Pg.c_log2;
    P.nrad = Pg.nrad;
    const float2 *ptw = Pg.tw;
    const int G = Pg.G, ntiles = Pg.ntiles;
    const float *kf = a.geoms[S.geom].kf;
    const int S_q = a.geoms[S.geom].S_q, kq_half = a.geoms[S.geom].kq_half;
    if (ptw != tw_src) {  // (uniform: the tile loops end with a barrier)
      for (int i = tid; i < P.L; i += kQThreads) tw[i] = ptw[i];
      if (tid < P.nrad) {
        st.rad[tid] = Pg.rad[tid];
        st.ns_shift[tid] = Pg.ns_shift[tid];
        st.ns_three[tid] = Pg.ns_three[tid];
        st.tw_step[tid] = Pg.tw_step[tid];
      }
      tw_src = ptw;
      __syncthreads();
    }
    const int t0 = (item - sg.first) * G;
    const int t1 = min(t0 + G, ntiles);
    for (int t = t0; t < t1; ++t) q_tile(buf, tw, st, kf, S_q, kq_half, P, S, t);

    if (tid == 0) s_pend[npend] = si;
    ++npend;
    pend_level = k;
  }
  if (npend > 0) {
    q_release_all();
    if (wave0) q_count(a, s_pend, npend, pend_level);
  }
  if (wave0) {
    // the last workgroup out returns the counters to zero for the next launch
    const unsigned done = __hip_atomic_fetch_add(&state[kQExit], one, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    const int last = __builtin_amdgcn_readfirstlane(done) == gridDim.x - 1;
    if (last) {
      for (int i = tid; i < a.nseg; i += 64) __hip_atomic_store(&segc[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tid < kQLevels) __hip_atomic_store(&state[kQLevel + tid], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tid == 0) {
        __hip_atomic_store(&state[kQHead], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[kQAbort], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[kQExit], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

}  // namespace

hipError_t launch_queue(const QParams &a, int grid, hipStream_t stream) {
  if (grid < 1 || a.nitems < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(queue_kernel, dim3(grid), dim3(kQThreads), 0, stream, a);
  return hipGetLastError();
}

hipError_t queue_occupancy(int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, queue_kernel, kQThreads, 0);
}

}  // namespace psn
