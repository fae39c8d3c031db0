// plan.cpp - axis order, layouts and pass descriptors of a solve.
//
// Section 3 of the paper: with S_j = N_j B_j, the forward transform along the
// first axis touches N_q N_r rows, the second S_p N_r rows, the third S_p S_q
// rows, so putting free axes last (periodic first) minimizes the work; the
// inverse runs the axes in reverse and crops each free axis after its
// transform.  The first forward axis is real-to-complex and keeps
// H = S_p/2 + 1 coefficients.  The paper's explicit transposes between steps
// are replaced here by the choice of layouts: every pass reads and writes
// HBM once, with one side either line-contiguous or a contiguous tile of
// lines staged through LDS.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "../../include/poisson.h"

namespace psn {

bool supported_length(int S) {
  static const int ok[] = {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  for (int v : ok)
    if (v == S) return true;
  return false;
}

double algorithmic_bytes(const int n[3], const int S[3], const int order[3]) {
  const int p = order[0], q = order[1], r = order[2];
  const double H = S[p] / 2 + 1;
  const double grid = double(n[0]) * n[1] * n[2];
  return 8.0 * grid                          // rho in, V out (float32)
         + 32.0 * H * n[q] * n[r]            // A1: P1 write, P2 read, P4 write, P5 read
         + 32.0 * H * S[q] * n[r]            // A2: P2 write, P3 read + write, P4 read
         + 4.0 * H * (S[q] / 2 + 1) * (S[r] / 2 + 1);  // K^F octant, float32, once
}

bool plane_geometry_ok(const Geometry &g) {
  const Pass &P2 = g.pass[1], &P4 = g.pass[3];
  if (P2.in_s[0] != 1 || P4.out_s[0] != 1) return false;  // q-lines contiguous in A1
  const int LQ = P2.L, LR = g.pass[2].L;
  const bool pq = P2.pad, pr = g.pass[2].pad;
  if (P4.out_s[1] != P2.in_s[1] || P4.out_s[2] != P2.in_s[2] || P4.ext_tile != P2.ext_tile ||
      P4.ext_batch != P2.ext_batch || P2.ext_batch != g.H || P2.ext_tile != (pr ? LR / 2 : LR))
    return false;
#define PSN_X(a, b, c, d) if (LQ == a && LR == b && pq == c && pr == d) return true;
  PSN_PLANE_CASES(PSN_X)
#undef PSN_X
  return false;
}

double algorithmic_bytes_plane(const Geometry &g) {
  const int p = g.order[0], q = g.order[1], r = g.order[2];
  const double H = g.S[p] / 2 + 1;
  const double grid = double(g.n[0]) * g.n[1] * g.n[2];
  return 8.0 * grid + 32.0 * H * g.n[q] * g.n[r] + 4.0 * H * (g.S[q] / 2 + 1) * (g.S[r] / 2 + 1);
}

namespace {

// strides (elements) per physical axis for an array whose axes, fastest
// first, are f0, f1, f2 with extents ext[axis]
void strides_of(const int fast[3], const long long ext[3], long long st[3]) {
  long long s = 1;
  for (int k = 0; k < 3; ++k) {
    st[fast[k]] = s;
    s *= ext[fast[k]];
  }
}

void set_side(const long long st[3], int line_axis, int tile_axis, int batch_axis, long long out[3]) {
  out[0] = st[line_axis];
  out[1] = st[tile_axis];
  out[2] = st[batch_axis];
}

int third_axis(int a, int b) { return 3 - a - b; }

}  // namespace

int build_geometry(int n1, int n2, int n3, unsigned bc, Geometry &g, std::string &err,
                   const int *force_order) {
  g = Geometry();
  const int n[3] = {n1, n2, n3};
  if (bc > 7u) {
    err = "bc_mask must be in 0..7";
    return POISSON_E_ARG;
  }
  for (int j = 0; j < 3; ++j) {
    if (n[j] < 2 || n[j] > 1024) {
      err = "grid sizes must be in 2..1024";
      return POISSON_E_ARG;
    }
  }
  for (int j = 0; j < 3; ++j) {
    g.n[j] = n[j];
    g.S[j] = n[j] * (((bc >> j) & 1u) ? 2 : 1);
    if (!supported_length(g.S[j])) {
      char buf[160];
      std::snprintf(buf, sizeof buf,
                    "FFT length S_%d = %d is not of the form 2^a or 3*2^a in 4..1024", j + 1, g.S[j]);
      err = buf;
      return POISSON_E_UNSUPPORTED;
    }
  }
  g.bc = bc;

  // Axis order: minimum byte model (periodic first, free last); ties go to
  // the order whose first axis is x (contiguous density rows), then to the
  // lexicographically first permutation.
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int best = -1;
  double best_bytes = 0;
  for (int k = 0; k < 6; ++k) {
    const double b = algorithmic_bytes(g.n, g.S, perms[k]);
    const bool better = best < 0 || b < best_bytes * (1 - 1e-12) ||
                        (std::fabs(b - best_bytes) <= 1e-12 * best_bytes && perms[k][0] == 0 &&
                         perms[best][0] != 0);
    if (better) {
      best = k;
      best_bytes = b;
    }
  }
  if (force_order) {
    // a caller-chosen order (the axis-order study of Section 3): any
    // permutation of 0, 1, 2
    const int *o = force_order;
    if (o[0] < 0 || o[0] > 2 || o[1] < 0 || o[1] > 2 || o[2] < 0 || o[2] > 2 || o[0] == o[1] ||
        o[0] == o[2] || o[1] == o[2]) {
      err = "axis_order must be a permutation of 0, 1, 2";
      return POISSON_E_ARG;
    }
    for (int k = 0; k < 6; ++k)
      if (perms[k][0] == o[0] && perms[k][1] == o[1] && perms[k][2] == o[2]) best = k;
    best_bytes = algorithmic_bytes(g.n, g.S, perms[best]);
  }
  const int p = perms[best][0], q = perms[best][1], r = perms[best][2];
  g.order[0] = p;
  g.order[1] = q;
  g.order[2] = r;
  g.H = g.S[p] / 2 + 1;
  g.alg_bytes = best_bytes;
  // fastest axis of A1/A4: the second transform axis when the first is x
  // (then P2 reads and P4 writes whole lines); otherwise x, so the first pass
  // reads tiles of consecutive x.
  g.t1 = (p == 0) ? q : 0;
  const int t1 = g.t1;

  const bool fp = (bc >> p) & 1u, fq = (bc >> q) & 1u, fr = (bc >> r) & 1u;
  const int H = g.H;

  // extents of every array along each physical axis
  long long ext_grid[3] = {n[0], n[1], n[2]};
  long long ext_a1[3];
  ext_a1[p] = H;
  ext_a1[q] = n[q];
  ext_a1[r] = n[r];
  long long ext_a2[3];
  ext_a2[p] = H;
  ext_a2[q] = g.S[q];
  ext_a2[r] = n[r];

  long long st_grid[3], st_a1[3], st_a2[3];
  {
    const int f[3] = {0, 1, 2};
    strides_of(f, ext_grid, st_grid);
  }
  {
    // A1/A4: t1 fastest, then p, then the remaining axis
    const int o1 = third_axis(t1, p);
    const int f[3] = {t1, p, o1};
    strides_of(f, ext_a1, st_a1);
  }
  {
    // A2/A3: r fastest, then q, then p
    const int f[3] = {r, q, p};
    strides_of(f, ext_a2, st_a2);
  }
  g.a1_elems = ext_a1[0] * ext_a1[1] * ext_a1[2];
  g.a2_elems = ext_a2[0] * ext_a2[1] * ext_a2[2];
  auto round256 = [](size_t b) { return (b + 255) / 256 * 256; };
  g.a1_bytes = round256(size_t(g.a1_elems) * 8);
  g.a2_bytes = round256(size_t(g.a2_elems) * 8);
  g.ws_bytes = g.a1_bytes + g.a2_bytes;
  g.kf_octant = (long long)(g.S[0] / 2 + 1) * (g.S[1] / 2 + 1) * (g.S[2] / 2 + 1);
  g.kf_internal = (long long)H * (g.S[q] / 2 + 1) * (g.S[r] / 2 + 1);

  // P1: real-to-complex along p (tile axis t1)
  {
    Pass &P = g.pass[0];
    P.kind = KIND_R2C;
    P.line_axis = p;
    P.tile_axis = t1;
    P.batch_axis = third_axis(p, t1);
    P.L = g.S[p];
    P.n_in = n[p];
    P.n_out = H;
    P.pad = fp;
    P.ext_tile = int(ext_a1[P.tile_axis]);
    P.ext_batch = int(ext_a1[P.batch_axis]);
    set_side(st_grid, P.line_axis, P.tile_axis, P.batch_axis, P.in_s);
    set_side(st_a1, P.line_axis, P.tile_axis, P.batch_axis, P.out_s);
  }
  // P2: forward along q, tiles along r (A2 is r-fastest)
  {
    Pass &P = g.pass[1];
    P.kind = KIND_FWD;
    P.line_axis = q;
    P.tile_axis = r;
    P.batch_axis = p;
    P.L = g.S[q];
    P.n_in = n[q];
    P.n_out = g.S[q];
    P.pad = fq;
    P.ext_tile = n[r];
    P.ext_batch = H;
    set_side(st_a1, q, r, p, P.in_s);
    set_side(st_a2, q, r, p, P.out_s);
  }
  // P3: forward along r, times K^F, inverse along r, crop; lines (q, p)
  {
    Pass &P = g.pass[2];
    P.kind = KIND_CONV;
    P.line_axis = r;
    P.tile_axis = q;
    P.batch_axis = p;
    P.L = g.S[r];
    P.n_in = n[r];
    P.n_out = n[r];
    P.pad = fr;
    P.crop = fr;
    P.ext_tile = g.S[q];
    P.ext_batch = H;
    set_side(st_a2, r, q, p, P.in_s);
    set_side(st_a2, r, q, p, P.out_s);
  }
  // P4: inverse along q, crop, tiles along r
  {
    Pass &P = g.pass[3];
    P.kind = KIND_INV;
    P.line_axis = q;
    P.tile_axis = r;
    P.batch_axis = p;
    P.L = g.S[q];
    P.n_in = g.S[q];
    P.n_out = n[q];
    P.crop = fq;
    P.ext_tile = n[r];
    P.ext_batch = H;
    set_side(st_a2, q, r, p, P.in_s);
    set_side(st_a1, q, r, p, P.out_s);
  }
  // P5: complex-to-real along p, crop, tiles along t1
  {
    Pass &P = g.pass[4];
    P.kind = KIND_C2R;
    P.line_axis = p;
    P.tile_axis = t1;
    P.batch_axis = third_axis(p, t1);
    P.L = g.S[p];
    P.n_in = H;
    P.n_out = n[p];
    P.crop = fp;
    P.ext_tile = n[P.tile_axis];
    P.ext_batch = n[P.batch_axis];
    set_side(st_a1, P.line_axis, P.tile_axis, P.batch_axis, P.in_s);
    set_side(st_grid, P.line_axis, P.tile_axis, P.batch_axis, P.out_s);
  }
  for (int k = 0; k < 5; ++k) {
    Pass &P = g.pass[k];
    P.in_tiled = (P.in_s[0] != 1);
    P.out_tiled = (P.out_s[0] != 1);
    // every side is either line-contiguous or tile-contiguous
    if ((P.in_tiled && P.in_s[1] != 1) || (P.out_tiled && P.out_s[1] != 1)) {
      err = "internal error: pass layout is neither line- nor tile-contiguous";
      return POISSON_E_STATE;
    }
  }
  return POISSON_OK;
}

}  // namespace psn
