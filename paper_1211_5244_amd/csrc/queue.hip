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

__device__ __forceinline__ float2 fzero() { return make_float2(0.f, 0.f); }

// One radix-R butterfly of a Stockham stage with span NS over the lines of
// a tile: reads src[c][j + m L/R], writes dst[c][(j / NS) NS R + j % NS + m NS].
template <int R, bool INV, bool ZHI>
__device__ __forceinline__ void q_bfly(const float2 *src, float2 *dst, int c, int j, int L, int NS,
                                       const float2 *__restrict__ tw) {
  const int Lr = L / R, k = j % NS, base = c * L;
  float2 x[R];
#pragma unroll
  for (int m = 0; m < R; ++m) x[m] = (ZHI && m >= R / 2) ? fzero() : src[qx(base + j + m * Lr)];
  if (NS > 1) {
    const int step = L / (NS * R);
#pragma unroll
    for (int m = 1; m < R; ++m) x[m] = cmul_tw<INV>(x[m], tw[k * m * step]);
  }
  dft<R, INV, ZHI>(x);
  const int o = base + (j / NS) * NS * R + k;
#pragma unroll
  for (int m = 0; m < R; ++m) dst[qx(o + m * NS)] = x[m];
}

template <int R, bool INV>
__device__ __forceinline__ void q_stage_r(const float2 *src, float2 *dst, int C, int L, int NS,
                                          bool zhi, const float2 *__restrict__ tw) {
  const int Lr = L / R, nb = C * Lr;
  for (int idx = threadIdx.x; idx < nb; idx += kQThreads) {
    const int c = idx / Lr, j = idx - c * Lr;
    if (zhi) q_bfly<R, INV, true>(src, dst, c, j, L, NS, tw);
    else q_bfly<R, INV, false>(src, dst, c, j, L, NS, tw);
  }
}

// The whole line transform of the tile in buf[cur] (result in buf[cur] on
// return, cur updated).  zhi: the upper half of every input line is zero.
template <bool INV>
__device__ void q_fft(float2 (*buf)[kQSlots], int &cur, const QPass &P, int C, bool zhi) {
  int NS = 1;
  for (int s = 0; s < P.nrad; ++s) {
    const int R = P.rad[s];
    const bool z = zhi && s == 0;
    const float2 *src = buf[cur];
    float2 *dst = buf[cur ^ 1];
    switch (R) {
      case 2: q_stage_r<2, INV>(src, dst, C, P.L, NS, z, P.tw); break;
      case 3: q_stage_r<3, INV>(src, dst, C, P.L, NS, false, P.tw); break;
      case 4: q_stage_r<4, INV>(src, dst, C, P.L, NS, z, P.tw); break;
      default: q_stage_r<8, INV>(src, dst, C, P.L, NS, z, P.tw); break;
    }
    cur ^= 1;
    NS *= R;
    __syncthreads();
  }
}

// Index of element j, tile line w, batch b on one side of a pass.
__device__ __forceinline__ long long q_off(const long long *s, int j, int a, int b) {
  return j * s[0] + a * s[1] + (long long)b * s[2];
}

// One tile: load, transform, store.  Arrays by pass kind: P1 rho -> a1,
// P2 a1 -> a2, P3 a2 -> a2, P4 a2 -> a1, P5 a1 -> V.
__device__ void q_tile(float2 (*buf)[kQSlots], const QGeom &Gm, const QPass &P, const QSolve &S,
                       int tile) {
  const int tid = threadIdx.x;
  const int ta = tile % P.tiles_a, b = tile / P.tiles_a, a0 = ta * P.W;
  const int C = P.C, L = P.L;
  const bool in_line = P.in_s[0] == 1, out_line = P.out_s[0] == 1;
  int cur = 0;
  float2 *X = buf[0];

  if (P.kind == KIND_R2C) {
    // real lines 2c and 2c + 1 as the real and imaginary parts of line c
    const float *in = S.rho;
    const int W = 2 * C, n = W * L;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int w, j;
      if (in_line) { w = idx / L; j = idx - w * L; }
      else { j = idx / W; w = idx - j * W; }
      const int a = a0 + w;
      const float v = (a < P.ext_tile && j < P.n_in) ? in[q_off(P.in_s, j, a, b)] : 0.f;
      reinterpret_cast<float *>(&X[qx((w >> 1) * L + j)])[w & 1] = v;
    }
  } else if (P.kind == KIND_C2R) {
    // Z = X_a + i X_b from the Hermitian halves of lines 2c and 2c + 1 (the
    // imaginary parts of the k = 0 and k = L/2 terms are not part of a real
    // line's spectrum and are dropped)
    const float2 *in = S.a1;
    const int n = C * L, h = L / 2;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int c, j;
      if (in_line) { c = idx / L; j = idx - c * L; }
      else { j = idx / C; c = idx - j * C; }
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
    }
  } else {
    const float2 *in = P.kind == KIND_FWD ? S.a1 : S.a2;
    const int n = C * L;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int c, j;
      if (in_line) { c = idx / L; j = idx - c * L; }
      else { j = idx / C; c = idx - j * C; }
      const int a = a0 + c;
      X[qx(c * L + j)] = (a < P.ext_tile && j < P.n_in) ? in[q_off(P.in_s, j, a, b)] : fzero();
    }
  }
  __syncthreads();

  const bool zhi = P.pad != 0;
  if (P.kind == KIND_INV || P.kind == KIND_C2R) q_fft<true>(buf, cur, P, C, false);
  else q_fft<false>(buf, cur, P, C, zhi);

  if (P.kind == KIND_CONV) {
    // times K^F (even along q and r): row (k_p, min(k_q, S_q - k_q))
    float2 *Y = buf[cur];
    const int KR = L / 2 + 1, n = C * L;
    for (int idx = tid; idx < n; idx += kQThreads) {
      const int c = idx / L, j = idx - c * L;
      const int kq = a0 + c;
      if (kq < P.ext_tile) {
        const int kqf = kq <= Gm.S_q - kq ? kq : Gm.S_q - kq;
        const float kv = Gm.kf[(long long)(b * Gm.kq_half + kqf) * KR + (j <= L - j ? j : L - j)];
        const float2 v = Y[qx(idx)];
        Y[qx(idx)] = make_float2(v.x * kv, v.y * kv);
      }
    }
    __syncthreads();
    q_fft<true>(buf, cur, P, C, false);
  }

  const float2 *Y = buf[cur];
  if (P.kind == KIND_R2C) {
    // X_a[k] = (Z[k] + conj Z[L-k]) / 2, X_b[k] = (Z[k] - conj Z[L-k]) / (2i)
    float2 *out = S.a1;
    const int W = 2 * C, H = P.n_out, n = W * H;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int w, k;
      if (out_line) { w = idx / H; k = idx - w * H; }
      else { k = idx / W; w = idx - k * W; }
      const int a = a0 + w;
      if (a < P.ext_tile) {
        const int c = w >> 1;
        const float2 zk = Y[qx(c * L + k)], zl = Y[qx(c * L + (k == 0 ? 0 : L - k))];
        const float2 v = (w & 1) ? make_float2(0.5f * (zk.y + zl.y), 0.5f * (zl.x - zk.x))
                                 : make_float2(0.5f * (zk.x + zl.x), 0.5f * (zk.y - zl.y));
        out[q_off(P.out_s, k, a, b)] = v;
      }
    }
  } else if (P.kind == KIND_C2R) {
    float *out = S.V;
    const int W = 2 * C, n = W * P.n_out;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int w, j;
      if (out_line) { w = idx / P.n_out; j = idx - w * P.n_out; }
      else { j = idx / W; w = idx - j * W; }
      const int a = a0 + w;
      if (a < P.ext_tile) {
        const float2 z = Y[qx((w >> 1) * L + j)];
        out[q_off(P.out_s, j, a, b)] = (w & 1) ? z.y : z.x;
      }
    }
  } else {
    float2 *out = P.kind == KIND_INV ? S.a1 : S.a2;
    const int n = C * P.n_out;
    for (int idx = tid; idx < n; idx += kQThreads) {
      int c, j;
      if (out_line) { c = idx / P.n_out; j = idx - c * P.n_out; }
      else { j = idx / C; c = idx - j * C; }
      const int a = a0 + c;
      if (a < P.ext_tile) out[q_off(P.out_s, j, a, b)] = Y[qx(c * L + j)];
    }
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
  __shared__ int s_item, s_full;
  __shared__ int s_pend[kQPending];
  const int tid = threadIdx.x;
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < 64;
  const unsigned one = tid == 0 ? 1u : 0u;
  unsigned *state = a.state;
  unsigned *segc = state + kQStateHeader;

  int npend = 0, pend_level = 0, acq_level = -1;
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

    const QSolve S = a.solves[sg.solve];
    const QGeom &Gm = a.geoms[S.geom];
    const QPass &P = Gm.pass[k];
    const int t0 = (item - sg.first) * P.G;
    const int t1 = min(t0 + P.G, P.ntiles);
    for (int t = t0; t < t1; ++t) q_tile(buf, Gm, P, S, t);

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
