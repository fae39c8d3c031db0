// queue.h - the persistent batched solve: one launch runs every pass of every
// solve of a batch, taking work items from a pass-ordered device queue
// (paper, Section 5: many densities per run; the passes are those of
// Section 3).  Shared by the device kernel (queue.hip) and the host
// simulation of the completion protocol (api.cpp).
//
// Items.  A solve's pass k is split into tiles of C complex lines; G tiles
// form one item.  The queue holds the items of every (solve, pass) segment
// in level order: all pass-0 segments (solve 0, 1, ...), then all pass-1
// segments, and so on.  A workgroup takes the next item with one atomic add.
//
// Dependencies.  An item of pass k > 0 of solve s reads what pass k - 1 of s
// wrote, so it may start once every item of segment (s, k - 1) is complete.
// Every such item sits earlier in the queue, so it was taken by a running
// workgroup before this one; a workgroup only waits on items of a lower
// level than any it holds (see the flush rule), so waits form no cycle and
// every wait ends without any assumption on how many workgroups are
// resident.
//
// Completion.  Each XCD has its own L2, so a result is visible to another
// workgroup only after an agent-scope release by its writer (an L2 write-
// back) and an agent-scope acquire by its reader (an L2 invalidate).  A
// release per item would stall every workgroup of the XCD once per item, so
// a workgroup holds its completed items and releases them together (one
// release, then one counter add per held item) when it takes an item of a
// higher level, when its list is full, or when the queue is empty.  A reader
// acquires once per item until the whole level below is complete; after one
// acquire that observed the complete level it reads that level freely.
//
// Every wait is bounded by a spin limit; running out sets a sticky error bit
// (the batch's results are then undefined) and an abort word that ends every
// other wait of the launch at once, so the kernel still ends promptly.  The
// last workgroup to leave returns the counters (not the error bits) to zero
// for the next launch.
#pragma once

#include <hip/hip_runtime.h>

namespace psn {

constexpr int kQThreads = 256;      // threads of a queue workgroup
constexpr int kQMaxTile = 2048;     // complex elements of one tile buffer
constexpr int kQMaxRadices = 12;
constexpr int kQPending = 32;       // completed items a workgroup holds before a release
constexpr int kQLevels = 5;
constexpr int kQRadixChoices = 3;

// state words: [0] head, [1] workgroups done, [2] sticky error bits (kept
// until the host reads them), [3] abort (set with an error: every later wait
// of the launch gives up at once), [4 .. 8] completed items per level,
// [16 ..] completed items per segment
constexpr int kQHead = 0, kQExit = 1, kQError = 2, kQAbort = 3, kQLevel = 4;
constexpr int kQStateHeader = 16;
constexpr unsigned kQErrSpin = 1u;  // a bounded wait ran out

// One pass of one geometry as the queue engine runs it.  Element j of line
// (a, b) sits at j*s[0] + a*s[1] + b*s[2] on each side; a side is either
// line-contiguous (s[0] == 1) or tile-contiguous (s[1] == 1).
struct QPass {
  const float2 *tw;              // exp(-2 pi i n / L), n < L
  long long in_s[3], out_s[3];
  int kind, L, n_in, n_out;
  int pad;                       // input holds the lower half only
  int ext_tile, ext_batch;
  int C;                         // complex lines per tile
  int W;                         // tile-axis lines per tile (2C for the real passes)
  int tiles_a;                   // tiles along the tile axis
  int ntiles;                    // tiles_a * ext_batch
  int G;                         // tiles per item
  int c_log2;                    // log2 C (C is a power of two)
  int nrad;
  int rad[kQMaxRadices];         // radices of the line transform, first stage first
  // per stage: span NS = product of the earlier radices as NS = 2^ns_shift
  // * (ns_three ? 3 : 1), and the twiddle step L / (NS R)
  int ns_shift[kQMaxRadices], ns_three[kQMaxRadices], tw_step[kQMaxRadices];
};

struct QGeom {
  QPass pass[kQLevels];
  const float *kf;               // float32 K^F in pass order, 1/(S1 S2 S3) folded in
  int S_q, kq_half;
};

struct QSolve {
  const float *rho;
  float *V;
  float2 *a1, *a2;
  int geom;
  int pad_;
};

// Items first .. first + count - 1 are segment (solve, pass).  Segment index
// = pass * nsolve + solve.
struct QSeg {
  int first, count, solve, pass;
};

struct QParams {
  const QGeom *geoms;
  const QSolve *solves;
  const QSeg *segs;
  unsigned *state;
  int nsolve, nseg, nitems;
  int level_items[kQLevels];
  unsigned spin_limit;
};

// ------------------------------------------------- protocol rules
// The segment holding item `it` (segments sorted by `first`, none empty).
__host__ __device__ inline int q_find_seg(const QSeg *segs, int nseg, int it) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
// Held items must be released before taking an item of level k.
__host__ __device__ inline bool q_must_flush(int npend, int pend_level, int k) {
  return npend > 0 && (pend_level < k || npend >= kQPending);
}
// An item of level k needs a wait (and an acquire) unless this workgroup has
// already acquired the complete level k - 1.
__host__ __device__ inline bool q_must_wait(int k, int acq_level) { return k > 0 && acq_level < k - 1; }
// The segment an item of segment `si` waits on.
__host__ __device__ inline int q_dep_seg(int si, int nsolve) { return si - nsolve; }

// Radices of a length-L line transform (L = 2^a 3^b, b <= 1, 4 <= L <= 1024)
// for radix choice `sel`: 0 the stages of the grouped float32 kernels'
// compiled shape (Shape<L> of the line FFT), so a queue solve at choice 0
// computes every butterfly as they do and gives their results bit for bit;
// 1 radix-4 stages (then 2, then 3); 2 the stages of choice 0 in reverse
// order.  Returns the count, 0 for an unsupported L or sel.
__host__ __device__ inline int q_radices(int L, int sel, int *rad) {
  if (L < 4 || L > 1024 || sel < 0 || sel >= kQRadixChoices) return 0;
  int m = L, three = 0;
  if (m % 3 == 0) { three = 1; m /= 3; }
  int e = 0;
  while ((m & 1) == 0) { m >>= 1; ++e; }
  if (m != 1) return 0;
  int n = 0;
  if (sel == 1) {
    for (; e >= 2; e -= 2) rad[n++] = 4;
    if (e) rad[n++] = 2;
    if (three) rad[n++] = 3;
    return n;
  }
  // the compiled shapes: radix-8 stages, then the rest of the power of two
  // as one radix (two radix-4 stages at 1024), then 3 before a final 2
  if (L == 1024) {
    rad[n++] = 8; rad[n++] = 8; rad[n++] = 4; rad[n++] = 4;
  } else {
    for (; e >= 3; e -= 3) rad[n++] = 8;
    if (e == 2) rad[n++] = 4;
    if (three) rad[n++] = 3;
    if (e == 1) rad[n++] = 2;
  }
  if (sel == 2)
    for (int i = 0, j = n - 1; i < j; ++i, --j) {
      const int t = rad[i]; rad[i] = rad[j]; rad[j] = t;
    }
  return n;
}

}  // namespace psn
