// kernels.h - host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace psn {

// Most solves one pass launch covers (their array bases travel as kernel
// arguments).
constexpr int kMaxBatch = 64;

// Arrays of the solves one launch covers, all of the same geometry.
struct PassIO {
  int count = 0;                    // 1..kMaxBatch
  const void *in[kMaxBatch] = {};   // per-solve input array
  void *out[kMaxBatch] = {};        // per-solve output array
  long long conv_stride = 0;        // conv pass: elements between the A2 arrays of
                                    // consecutive solves (out[0] is the first)
};

// One pass on `stream` for io.count solves: reads io.in[j], writes io.out[j]
// (complex intermediates are float2, density and potential float).  `tw` is
// the table exp(-2 pi i n / L), n = 0..L-1, of the pass's length; `kf` the
// float32 K^F in pass order (conv pass only).  `mode` selects float32
// radix stages (0) or split-precision matrix-core radix-8 stages (1: fp16
// hi+lo, 2: bf16 three-way).  Returns a hipError_t.
hipError_t launch_pass(const Pass &P, const PassIO &io, const float2 *tw, const float *kf,
                       int S_q, int mode, hipStream_t stream);

// Pass schedules (P.tile_sel = 0..kSchedules-1): bits 0-1 select the tile
// width of a tiled pass (kTileSchedules choices; the conv pass has none),
// bit 2 the XCD-blocked workgroup order, and bit 3 (conv pass only) runs
// passes 1-3 as the small-grid plane kernel.  pass_tile_lines gives the
// complex lines per workgroup tile of schedule `sched` for pass P in
// `mode`, or 0 where its tile width is not compiled (it then runs as width 0).
constexpr int kTileSchedules = 4;
constexpr int kSchedules = 16;
constexpr int kPlaneBit = 8;
int pass_tile_lines(const Pass &P, int sched, int mode);

// Small grids: passes 1-3 (forward q, conv r, inverse q) as one launch that
// keeps each k_p plane in LDS.  plane_available tells whether geometry g has
// a compiled plane kernel in `mode`; launch_plane runs it on the A1 arrays
// io.out[j] in place (A1 doubles as A4), with the q and r twiddle tables and
// the float32 K^F of the pass order.  launch_plane_for_mode is its
// per-precision half (each precision compiled in its own object).
bool plane_available(const Geometry &g, int mode);
hipError_t launch_plane(const Geometry &g, int mode, const PassIO &io, const float2 *twq,
                        const float2 *twr, const float *kf, hipStream_t stream);
template <int MODE>
hipError_t launch_plane_for_mode(const Geometry &g, const PassIO &io, const float2 *twq,
                                 const float2 *twr, const float *kf, hipStream_t stream);

// float64 K^F octant of the default Green's function (layout of the C ABI:
// k1 fastest), built in place in `kf64` using `tmp` (same size) as scratch.
// cos_tabs[j]: device table cos(2 pi n / S_j), n = 0..S_j-1, for each axis.
hipError_t launch_kernel_build(const Geometry &g, double h, double *kf64, double *tmp,
                               const double *const cos_tabs[3], hipStream_t stream);

// float64 K^F octant of the free-boundary Green's function on Deslauriers-
// Dubuc interpolating scaling functions of even order 8..32 (fully free
// geometries), written to `kf64`.  `scratch` (device, at least
// isf_table_bytes(g)) holds the quadrature nodes and per-node DCT tables; the
// node records are copied there with a blocking copy, the kernels are
// enqueued on `stream`.  hipErrorInvalidValue for an order out of range or
// too little scratch.
size_t isf_table_bytes(const Geometry &g);
hipError_t launch_isf_build(const Geometry &g, double h, int order, double *kf64, void *scratch,
                            size_t scratch_bytes, const double *const cos_tabs[3],
                            hipStream_t stream);

// float32 K^F in pass order [k_p][k_q'][k_r'] with 1/(S1 S2 S3) folded in,
// from the float64 octant.
hipError_t launch_kernel_permute(const Geometry &g, const double *kf64, float *kf32,
                                 hipStream_t stream);

// partial sums of (v - ref)^2 and ref^2 in float64: writes 2*blocks doubles
// to `partials`; blocks is the returned count (<= max_blocks).
hipError_t launch_rel_l2_partials(const float *v, const double *ref, size_t count,
                                  double *partials, int max_blocks, int *blocks,
                                  hipStream_t stream);

// The same residual with its partial sums in the library's static device
// scratch and the result, ||v - ref|| / ||ref||, written to device memory
// `out`: no allocation, no host wait.  Calls that overlap on one device
// share the scratch and race.
hipError_t launch_rel_l2_noalloc(const float *v, const double *ref, size_t count, double *out,
                                 hipStream_t stream);

// The persistent batched solve (queue.h): one launch of `grid` workgroups
// on `stream`; queue_occupancy gives the workgroups per compute unit that
// fit at once.
struct QParams;
hipError_t launch_queue(const QParams &a, int grid, hipStream_t stream);
hipError_t queue_occupancy(int *blocks_per_cu);

}  // namespace psn
