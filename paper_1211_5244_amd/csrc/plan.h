// plan.h - host-side geometry of a solve: axis order, pass descriptors,
// intermediate layouts, workspace size and byte model.  No HIP calls.
#pragma once

#include <cstddef>
#include <string>

namespace psn {

// FFT lengths with a compiled kernel shape (2^a 3^b, 4..1024).
bool supported_length(int S);

enum PassKind { KIND_R2C = 0, KIND_FWD = 1, KIND_CONV = 2, KIND_INV = 3, KIND_C2R = 4 };

// One pass = a batch of 1D transforms along `line_axis`.  Lines are indexed
// by (a, b): a runs along `tile_axis` (consecutive lines of one workgroup
// tile), b along `batch_axis`.  Element j of line (a, b) of an array sits at
// j*s[0] + a*s[1] + b*s[2].  A side is "tiled" when s[1] == 1 (the tile of
// lines is contiguous, staged through LDS) and "line" when s[0] == 1 (each
// line is contiguous and read straight into registers).
struct Pass {
  int kind = 0;
  int line_axis = 0, tile_axis = 0, batch_axis = 0;
  int L = 0;      // FFT length along the line axis
  int n_in = 0;   // valid input values per line (zero padding above it)
  int n_out = 0;  // values written per line
  int ext_tile = 0, ext_batch = 0;
  long long in_s[3] = {0, 0, 0}, out_s[3] = {0, 0, 0};
  bool in_tiled = false, out_tiled = false;
  bool pad = false;   // input holds L/2 values (free axis before its transform)
  bool crop = false;  // only the first L/2 outputs are kept (free axis after inverse)
  int tile_sel = 0;   // tile schedule of a tiled pass (0 = default; see the autotuner)
};

struct Geometry {
  int n[3] = {0, 0, 0};
  int S[3] = {0, 0, 0};
  unsigned bc = 0;
  int order[3] = {0, 1, 2};  // forward axis order p, q, r
  int t1 = 1;                // fastest axis of the first intermediate
  int H = 0;                 // S_p / 2 + 1
  long long a1_elems = 0;    // complex elements of intermediate A1 (= A4)
  long long a2_elems = 0;    // complex elements of intermediate A2 (= A3)
  size_t a1_bytes = 0, a2_bytes = 0, ws_bytes = 0;
  double alg_bytes = 0;
  long long kf_octant = 0;   // float64 octant values (S1/2+1)(S2/2+1)(S3/2+1)
  long long kf_internal = 0; // float32 values H (S_q/2+1) (S_r/2+1)
  Pass pass[5];
};

// Fills g for the given problem, with the minimum-byte axis order or, if
// force_order is not null, that forward order (p, q, r).  Returns 0 or a
// negative POISSON_E_* code with a message in err.
int build_geometry(int n1, int n2, int n3, unsigned bc, Geometry &g, std::string &err,
                   const int *force_order = nullptr);

// Minimum HBM bytes of one solve for axis order (p, q, r) (five passes, each
// reading and writing its data once, plus the float32 K^F octant).
double algorithmic_bytes(const int n[3], const int S[3], const int order[3]);

// The small-grid plane kernel's compiled (L_q, L_r, padded q, padded r)
// combinations: periodic, free and wire cubes and surface grids (q
// periodic, r free), lengths up to 128.
#define PSN_PLANE_CASES(X)                                                      \
  X(32, 32, false, false) X(48, 48, false, false) X(64, 64, false, false)       \
  X(96, 96, false, false) X(128, 128, false, false)                             \
  X(64, 64, true, true) X(96, 96, true, true) X(128, 128, true, true)          \
  X(32, 64, false, true) X(48, 96, false, true) X(64, 128, false, true)        \
  X(96, 192, false, true) X(128, 256, false, true)

// Whether geometry g can run passes 1-3 as the plane kernel: a compiled
// (L_q, L_r) case whose q-lines are contiguous in A1 and are written back
// where they were read (A4 = A1), one k_p plane of N_r lines per p index.
bool plane_geometry_ok(const Geometry &g);

// Minimum HBM bytes of one solve that runs passes 1-3 as the plane kernel:
// the intermediate A2 stays in LDS, so only the density, A1 (written by
// pass 0, read and rewritten by the plane kernel, read by pass 4), the
// potential and the K^F octant move.
double algorithmic_bytes_plane(const Geometry &g);

}  // namespace psn
