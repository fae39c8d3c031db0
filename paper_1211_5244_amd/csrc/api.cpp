// api.cpp - the C ABI of libpoisson (declared in include/poisson.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <atomic>
#include <chrono>
#include <random>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "../../include/poisson.h"
#include "kernels.h"
#include "plan.h"
#include "queue.h"

using psn::Geometry;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(e == hipErrorOutOfMemory ? POISSON_E_NOMEM : POISSON_E_HIP, m);
}

// Runs a call with the plan's device current and restores the caller's.
struct DeviceScope {
  int prev = -1;
  bool ok = true;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define PSN_TRY_HIP(call, what)                 \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

}  // namespace

struct poisson_plan_s {
  Geometry g;
  double h = 0;
  int precision = POISSON_FP32;
  int device = 0;
  float2 *tw[3] = {nullptr, nullptr, nullptr};     // per physical axis (shared by equal lengths)
  double *cos_tab[3] = {nullptr, nullptr, nullptr};
  std::vector<void *> owned;                        // every device buffer the plan allocated
  double *kf64 = nullptr;
  float *kf32 = nullptr;
  void *ws = nullptr;
  bool own_ws = false;
  bool auto_ws = true;  // allocate a workspace when the kernel is set
  bool kernel_ready = false;
  // host-buffer solves: two device grids and two copy streams (created on
  // first use, default priority)
  float *io[2] = {nullptr, nullptr};
  hipStream_t h2d = nullptr, d2h = nullptr;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_solved[2] = {nullptr, nullptr},
             ev_out[2] = {nullptr, nullptr};
};

struct poisson_batch_s {
  std::vector<poisson_plan_t> plans;        // unique problems
  std::vector<int> which;                   // solve i uses plans[which[i]]
  std::vector<std::vector<int>> members;    // per plan: its solves, in order
  std::vector<int> chunk;                   // per plan: solves per launch
  double chunk_mb = 384.0;                  // intermediates budget of one launch
  void *ws = nullptr;                       // ws_lanes regions of ws_bytes each
  size_t ws_bytes = 0;                      // one stream's region
  int ws_lanes = 1;
  int lanes = 1;                            // concurrent streams of a solve
  std::vector<hipStream_t> side;            // the batch's own streams (lanes - 1 used)
  std::vector<hipEvent_t> events;           // fork event, then one join event per side stream
  int device = 0;
  // the persistent schedule (float32): one launch over a pass-ordered queue
  int mode = POISSON_BATCH_GROUPED;
  std::map<int, int> q_radix;               // radix choice per line length (absent: 0)
  int q_tile = psn::kQMaxTile;              // complex elements per tile
  int q_item_kb = 512;                      // target bytes (in + out) per work item
  unsigned q_spin = 1u << 20;               // bound of every wait (about a second of polls)
  bool q_dirty = true;                      // descriptors to rebuild before the next launch
  void *q_desc = nullptr;                   // geometries, solve table, segments
  size_t q_desc_bytes = 0;
  unsigned *q_state = nullptr;              // queue counters (zero between launches)
  void *q_ws = nullptr;                     // every solve's intermediates
  size_t q_ws_bytes = 0;
  std::vector<psn::QSolve> q_solves;        // host copy of the device solve table
  psn::QParams q_params{};
  int q_grid = 0;
};

namespace {

constexpr int kMaxLanes = 4;  // concurrent streams of a batch solve (GPU_MAX_HW_QUEUES is 4)
constexpr int kDefaultLanes = 4;

int check_precision(int precision) {
  if (precision == POISSON_FP32 || precision == POISSON_SPLIT_FP16 ||
      precision == POISSON_SPLIT_BF16)
    return POISSON_OK;
  return fail(POISSON_E_ARG, "precision must be POISSON_FP32, POISSON_SPLIT_FP16 or POISSON_SPLIT_BF16");
}

int plan_alloc(poisson_plan_t P, void **ptr, size_t bytes, const char *what) {
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_fail(e, what);
  }
  P->owned.push_back(p);
  *ptr = p;
  return POISSON_OK;
}

void plan_free_all(poisson_plan_t P) {
  for (void *p : P->owned) (void)hipFree(p);
  P->owned.clear();
  for (hipEvent_t *e : {&P->ev_start, &P->ev_end, &P->ev_in[0], &P->ev_in[1], &P->ev_solved[0],
                        &P->ev_solved[1], &P->ev_out[0], &P->ev_out[1]})
    if (*e) (void)hipEventDestroy(*e), *e = nullptr;
  if (P->h2d) (void)hipStreamDestroy(P->h2d), P->h2d = nullptr;
  if (P->d2h) (void)hipStreamDestroy(P->d2h), P->d2h = nullptr;
}

// Device grids, copy streams and events of the host-buffer solves.
int ensure_host_io(poisson_plan_t P) {
  if (P->io[1]) return POISSON_OK;
  const size_t bytes = sizeof(float) * size_t(P->g.n[0]) * P->g.n[1] * P->g.n[2];
  for (int b = 0; b < 2; ++b) {
    if (P->io[b]) continue;
    void *p = nullptr;
    int rc = plan_alloc(P, &p, bytes, "hipMalloc(host-solve grid)");
    if (rc) return rc;
    P->io[b] = static_cast<float *>(p);
  }
  if (!P->h2d) PSN_TRY_HIP(hipStreamCreateWithFlags(&P->h2d, hipStreamNonBlocking), "hipStreamCreate");
  if (!P->d2h) PSN_TRY_HIP(hipStreamCreateWithFlags(&P->d2h, hipStreamNonBlocking), "hipStreamCreate");
  for (hipEvent_t *e : {&P->ev_start, &P->ev_end, &P->ev_in[0], &P->ev_in[1], &P->ev_solved[0],
                        &P->ev_solved[1], &P->ev_out[0], &P->ev_out[1]})
    if (!*e) PSN_TRY_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
  return POISSON_OK;
}

int ensure_workspace(poisson_plan_t P) {
  if (P->ws || !P->auto_ws) return POISSON_OK;
  void *p = nullptr;
  int rc = plan_alloc(P, &p, P->g.ws_bytes, "hipMalloc(workspace)");
  if (rc) return rc;
  P->ws = p;
  P->own_ws = true;
  return POISSON_OK;
}

// exp(-2 pi i n / L), n = 0..L-1, evaluated in long double, rounded once
std::vector<float2> twiddle_table(int L) {
  std::vector<float2> t(L);
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int n = 0; n < L; ++n) {
    const long double a = two_pi * n / L;
    t[n] = make_float2(float(std::cos(a)), float(-std::sin(a)));
  }
  return t;
}

std::vector<double> cosine_table(int S) {
  std::vector<double> t(S);
  const long double two_pi = 6.283185307179586476925286766559L;
  for (int n = 0; n < S; ++n) t[n] = double(std::cos(two_pi * n / S));
  return t;
}

// Solves per launch for each plan of B under an intermediates budget of
// budget_mb MiB (at least 1, at most kMaxBatch); returns the workspace the
// largest chunk needs.
size_t batch_chunks(poisson_batch_t B, double budget_mb, std::vector<int> &chunk) {
  const size_t budget = size_t(budget_mb * 1024.0 * 1024.0);
  size_t ws = 0;
  chunk.clear();
  for (size_t u = 0; u < B->plans.size(); ++u) {
    const size_t per = B->plans[u]->g.ws_bytes;
    size_t c = per > 0 ? budget / per : 1;
    if (c < 1) c = 1;
    if (c > size_t(psn::kMaxBatch)) c = psn::kMaxBatch;
    if (c > B->members[u].size()) c = B->members[u].size();
    chunk.push_back(int(c));
    ws = std::max(ws, c * per);
  }
  B->chunk_mb = budget_mb;
  return ws;
}

// ------------------------------------------------ tuned-schedule cache
// A text file of tuned schedules, one line per problem and device kind:
//   v1 <arch> <CUs> <n1> <n2> <n3> <bc> <precision> <p> <q> <r> : <s1> .. <s5>
// poisson_plan_tune writes its result there and new plans of the same
// problem start from it, so a process need not tune again.  The file is
// advisory: unreadable files, unknown lines and schedules the library does
// not compile are ignored.
std::mutex g_cache_mutex;
std::string g_cache_path;
bool g_cache_path_set = false;

std::string cache_path_locked() {
  if (!g_cache_path_set) {
    g_cache_path_set = true;
    if (const char *e = std::getenv("POISSON_TUNE_CACHE")) g_cache_path = e;
  }
  return g_cache_path;
}

std::string cache_key(const poisson_plan_s *P) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    cus = prop.multiProcessorCount;
  }
  std::ostringstream k;
  k << "v1 " << arch << ' ' << cus << ' ' << P->g.n[0] << ' ' << P->g.n[1] << ' ' << P->g.n[2]
    << ' ' << P->g.bc << ' ' << P->precision << ' ' << P->g.order[0] << ' ' << P->g.order[1]
    << ' ' << P->g.order[2];
  return k.str();
}

// Makes room for `lanes` workspace regions of `per_lane` bytes (waits for
// stream s before replacing the allocation).  A failed allocation keeps the
// old one.
int batch_reserve(poisson_batch_t B, size_t per_lane, int lanes, hipStream_t s) {
  if (per_lane <= B->ws_bytes && lanes <= B->ws_lanes) return POISSON_OK;
  per_lane = std::max(per_lane, B->ws_bytes);
  lanes = std::max(lanes, B->ws_lanes);
  PSN_TRY_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, per_lane * size_t(lanes));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_fail(e, "hipMalloc(batch workspace)");
  }
  if (B->ws) (void)hipFree(B->ws);
  B->ws = p;
  B->ws_bytes = per_lane;
  B->ws_lanes = lanes;
  return POISSON_OK;
}

// The batch's side streams (default priority) and fork/join events for
// `lanes` concurrent streams, created once.
int batch_streams(poisson_batch_t B, int lanes) {
  while (int(B->side.size()) < lanes - 1) {
    hipStream_t st = nullptr;
    PSN_TRY_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    B->side.push_back(st);
  }
  while (int(B->events.size()) < lanes) {
    hipEvent_t ev = nullptr;
    PSN_TRY_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    B->events.push_back(ev);
  }
  return POISSON_OK;
}

// Whether schedule `sched` (tile width in bits 0-1, XCD order in bit 2) is
// compiled for pass k of plan P.  The conv pass has no tile width.
bool schedule_valid(poisson_plan_t P, int k, int sched) {
  if (sched < 0 || sched >= psn::kSchedules) return false;
  if (k == psn::KIND_CONV)
    return (sched & 3) == 0 && (!(sched & psn::kPlaneBit) || psn::plane_available(P->g, P->precision));
  if (sched & psn::kPlaneBit) return false;
  return psn::pass_tile_lines(P->g.pass[k], sched, P->precision) > 0;
}

// Starts plan P from its cached schedule, if the cache has one the library
// compiles.
void cache_apply(poisson_plan_t P) {
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  const std::string path = cache_path_locked();
  if (path.empty()) return;
  std::ifstream in(path);
  if (!in) return;
  const std::string key = cache_key(P);
  std::string line;
  while (std::getline(in, line)) {
    const size_t colon = line.find(" : ");
    if (colon == std::string::npos || line.compare(0, colon, key) != 0 || colon != key.size()) continue;
    std::istringstream vals(line.substr(colon + 3));
    int sel[5];
    bool ok = true;
    for (int k = 0; k < 5 && ok; ++k) ok = bool(vals >> sel[k]) && schedule_valid(P, k, sel[k]);
    if (ok)
      for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = sel[k];
  }
}

// Records plan P's schedule in the cache (replacing its line), through a
// temporary file renamed over the old one.
void cache_store(poisson_plan_t P) {
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  const std::string path = cache_path_locked();
  if (path.empty()) return;
  const std::string key = cache_key(P);
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (in && std::getline(in, line))
      if (line.compare(0, key.size() + 3, key + " : ") != 0 && !line.empty()) keep.push_back(line);
  }
  std::ostringstream mine;
  mine << key << " :";
  for (int k = 0; k < 5; ++k) mine << ' ' << P->g.pass[k].tile_sel;
  keep.push_back(mine.str());
  const std::string tmp = path + ".tmp." + std::to_string(long(getpid()));
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;
    for (const std::string &l : keep) out << l << '\n';
    if (!out) return;
  }
  (void)std::rename(tmp.c_str(), path.c_str());
}

int finish_kernel(poisson_plan_t P, hipStream_t s) {
  hipError_t e = psn::launch_kernel_permute(P->g, P->kf64, P->kf32, s);
  if (e != hipSuccess) return hip_fail(e, "K^F permute launch");
  P->kernel_ready = true;
  return POISSON_OK;
}

// Enqueues the float64 build of the default K^F and its float32 permuted
// copy on stream s.  The DCT ping-pong's float64 scratch (one octant) lives
// in `scratch`, a workspace the solves use between builds: the workspace of
// a solve always has room for it (S_q/2+1 <= S_q and S_r/2+1 <= N_r+1, so
// the octant is at most the A2 array plus S_q H complex values of A1).
int build_kernel_into(poisson_plan_t P, void *scratch, size_t scratch_bytes, hipStream_t s) {
  const size_t need = sizeof(double) * size_t(P->g.kf_octant);
  if (!scratch || scratch_bytes < need)
    return fail(POISSON_E_STATE, "no workspace to build K^F in (poisson_set_workspace first)");
  const double *tabs[3] = {P->cos_tab[0], P->cos_tab[1], P->cos_tab[2]};
  hipError_t e = psn::launch_kernel_build(P->g, P->h, P->kf64, static_cast<double *>(scratch), tabs, s);
  if (e != hipSuccess) return hip_fail(e, "K^F build");
  return finish_kernel(P, s);
}

}  // namespace

extern "C" {

const char *poisson_last_error(void) { return g_last_error.c_str(); }

int poisson_plan_describe(int n1, int n2, int n3, unsigned bc_mask, int precision,
                          int axis_order[3], int S[3], size_t *workspace_bytes,
                          double *alg_bytes) {
  return poisson_plan_describe_ordered(n1, n2, n3, bc_mask, precision, nullptr, axis_order, S,
                                       workspace_bytes, alg_bytes, nullptr);
}

int poisson_plan_describe_ordered(int n1, int n2, int n3, unsigned bc_mask, int precision,
                                  const int force_order[3], int axis_order[3], int S[3],
                                  size_t *workspace_bytes, double *alg_bytes, long long rows[3]) {
  try {
    Geometry g;
    std::string err;
    int rc = psn::build_geometry(n1, n2, n3, bc_mask, g, err, force_order);
    if (rc) return fail(rc, err);
    rc = check_precision(precision);
    if (rc) return rc;
    const int p = g.order[0], q = g.order[1], r = g.order[2];
    const long long R[3] = {(long long)g.n[q] * g.n[r], (long long)g.S[p] * g.n[r],
                            (long long)g.S[p] * g.S[q]};
    for (int j = 0; j < 3; ++j) {
      if (axis_order) axis_order[j] = g.order[j];
      if (S) S[j] = g.S[j];
      if (rows) rows[j] = R[j];
    }
    if (workspace_bytes) *workspace_bytes = g.ws_bytes;
    if (alg_bytes) *alg_bytes = g.alg_bytes;
    return POISSON_OK;
  } catch (...) {
    return fail(POISSON_E_STATE, "unexpected exception");
  }
}

int poisson_plan_rows(int n1, int n2, int n3, unsigned bc_mask, long long rows[3],
                      int lengths[3]) {
  try {
    Geometry g;
    std::string err;
    int rc = psn::build_geometry(n1, n2, n3, bc_mask, g, err);
    if (rc) return fail(rc, err);
    const int p = g.order[0], q = g.order[1], r = g.order[2];
    const long long R[3] = {(long long)g.n[q] * g.n[r], (long long)g.S[p] * g.n[r],
                            (long long)g.S[p] * g.S[q]};
    const int Ls[3] = {g.S[p], g.S[q], g.S[r]};
    for (int k = 0; k < 3; ++k) {
      if (rows) rows[k] = R[k];
      if (lengths) lengths[k] = Ls[k];
    }
    return POISSON_OK;
  } catch (...) {
    return fail(POISSON_E_STATE, "unexpected exception");
  }
}

int poisson_plan(poisson_plan_t *out, int n1, int n2, int n3, unsigned bc_mask, double h,
                 int precision) {
  return poisson_plan_ordered(out, n1, n2, n3, bc_mask, h, precision, nullptr);
}

int poisson_plan_ordered(poisson_plan_t *out, int n1, int n2, int n3, unsigned bc_mask, double h,
                         int precision, const int axis_order[3]) {
  try {
    if (!out) return fail(POISSON_E_ARG, "out is NULL");
    *out = nullptr;
    if (!(h > 0.0) || !std::isfinite(h)) return fail(POISSON_E_ARG, "spacing h must be positive and finite");
    Geometry g;
    std::string err;
    int rc = psn::build_geometry(n1, n2, n3, bc_mask, g, err, axis_order);
    if (rc) return fail(rc, err);
    rc = check_precision(precision);
    if (rc) return rc;

    poisson_plan_t P = new (std::nothrow) poisson_plan_s();
    if (!P) return fail(POISSON_E_NOMEM, "host allocation failed");
    P->g = g;
    P->h = h;
    P->precision = precision;
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) {
      delete P;
      return hip_fail(e, "hipGetDevice");
    }
    auto cleanup = [&](int code) {
      plan_free_all(P);
      delete P;
      return code;
    };
    // twiddle and cosine tables, one per distinct length
    for (int j = 0; j < 3; ++j) {
      int same = -1;
      for (int k = 0; k < j; ++k)
        if (g.S[k] == g.S[j]) same = k;
      if (same >= 0) {
        P->tw[j] = P->tw[same];
        P->cos_tab[j] = P->cos_tab[same];
        continue;
      }
      void *p = nullptr;
      if ((rc = plan_alloc(P, &p, sizeof(float2) * g.S[j], "hipMalloc(twiddles)"))) return cleanup(rc);
      P->tw[j] = static_cast<float2 *>(p);
      std::vector<float2> t = twiddle_table(g.S[j]);
      e = hipMemcpy(p, t.data(), sizeof(float2) * t.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemcpy(twiddles)"));
      if ((rc = plan_alloc(P, &p, sizeof(double) * g.S[j], "hipMalloc(cosines)"))) return cleanup(rc);
      P->cos_tab[j] = static_cast<double *>(p);
      std::vector<double> c = cosine_table(g.S[j]);
      e = hipMemcpy(p, c.data(), sizeof(double) * c.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return cleanup(hip_fail(e, "hipMemcpy(cosines)"));
    }
    void *p = nullptr;
    if ((rc = plan_alloc(P, &p, sizeof(double) * g.kf_octant, "hipMalloc(K^F float64)"))) return cleanup(rc);
    P->kf64 = static_cast<double *>(p);
    if ((rc = plan_alloc(P, &p, sizeof(float) * g.kf_internal, "hipMalloc(K^F float32)"))) return cleanup(rc);
    P->kf32 = static_cast<float *>(p);
    cache_apply(P);
    *out = P;
    return POISSON_OK;
  } catch (...) {
    return fail(POISSON_E_STATE, "unexpected exception");
  }
}

int poisson_plan_info(poisson_plan_t P, int axis_order[3], int S[3], size_t *workspace_bytes,
                      double *alg_bytes) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  for (int j = 0; j < 3; ++j) {
    if (axis_order) axis_order[j] = P->g.order[j];
    if (S) S[j] = P->g.S[j];
  }
  if (workspace_bytes) *workspace_bytes = P->g.ws_bytes;
  if (alg_bytes) *alg_bytes = P->g.alg_bytes;
  return POISSON_OK;
}

int poisson_set_workspace(poisson_plan_t P, void *dev_ptr, size_t bytes) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (dev_ptr && bytes < P->g.ws_bytes)
    return fail(POISSON_E_ARG, "workspace smaller than poisson_plan_describe's workspace_bytes");
  if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) % 256) != 0)
    return fail(POISSON_E_ARG, "workspace must be 256-byte aligned");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  if (P->own_ws && P->ws) {
    PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    for (size_t i = 0; i < P->owned.size(); ++i) {
      if (P->owned[i] == P->ws) {
        (void)hipFree(P->ws);
        P->owned.erase(P->owned.begin() + i);
        break;
      }
    }
  }
  P->ws = dev_ptr;
  P->own_ws = false;
  return POISSON_OK;
}

int poisson_kernel_set(poisson_plan_t P, const double *kf, int is_device_ptr) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (!kf) return fail(POISSON_E_ARG, "K^F pointer is NULL");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  int rc = ensure_workspace(P);
  if (rc) return rc;
  PSN_TRY_HIP(hipMemcpy(P->kf64, kf, sizeof(double) * P->g.kf_octant,
                        is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice),
              "hipMemcpy(K^F)");
  rc = finish_kernel(P, nullptr);
  if (rc) return rc;
  PSN_TRY_HIP(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
  return POISSON_OK;
}

int poisson_kernel_build(poisson_plan_t P, void *stream) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  int rc = ensure_workspace(P);
  if (rc) return rc;
  return build_kernel_into(P, P->ws, P->ws ? P->g.ws_bytes : 0, static_cast<hipStream_t>(stream));
}

int poisson_kernel_build_isf(poisson_plan_t P, int order, void *stream) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (order < 8 || order > 32 || order % 2)
    return fail(POISSON_E_ARG, "interpolation order must be even, 8 to 32");
  if ((P->g.bc & 7u) == 0u)
    return fail(POISSON_E_UNSUPPORTED, "ISF kernels need at least one free axis");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  int rc = ensure_workspace(P);  // as poisson_kernel_build: solves need it
  if (rc) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = psn::isf_table_bytes(P->g);
  void *scratch = nullptr;
  PSN_TRY_HIP(hipMalloc(&scratch, bytes), "hipMalloc(ISF tables)");
  const double *tabs[3] = {P->cos_tab[0], P->cos_tab[1], P->cos_tab[2]};
  hipError_t e = psn::launch_isf_build(P->g, P->h, order, P->kf64, scratch, bytes, tabs, s);
  rc = e == hipSuccess ? finish_kernel(P, s) : hip_fail(e, "ISF K^F build");
  if (rc == POISSON_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
  } else {
    (void)hipStreamSynchronize(s);
  }
  (void)hipFree(scratch);
  return rc;
}

int poisson_kernel_get(poisson_plan_t P, double *host) {
  if (!P || !host) return fail(POISSON_E_ARG, "NULL argument");
  if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "no K^F has been set or built");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  PSN_TRY_HIP(hipMemcpy(host, P->kf64, sizeof(double) * P->g.kf_octant, hipMemcpyDeviceToHost),
              "hipMemcpy(K^F to host)");
  return POISSON_OK;
}

}  // extern "C"

namespace {

// Enqueue passes first..last for `count` solves of plan P whose
// intermediates live in `ws`: count A1 arrays, then count A2 arrays.
int enqueue_passes(poisson_plan_t P, int count, const float *const *rho, float *const *V,
                   void *ws, int first, int last, hipStream_t s) {
  const Geometry &g = P->g;
  char *base = static_cast<char *>(ws);
  char *a1 = base;
  char *a2 = base + size_t(count) * g.a1_bytes;
  const int p = g.order[0], q = g.order[1], r = g.order[2];
  const float2 *tws[5] = {P->tw[p], P->tw[q], P->tw[r], P->tw[q], P->tw[p]};
  // small grids: passes 1-3 as one plane kernel (schedule bit of pass 2)
  const bool plane = (g.pass[2].tile_sel & psn::kPlaneBit) && first <= 1 && last >= 3 &&
                     psn::plane_available(g, P->precision);
  for (int k = first; k <= last; ++k) {
    if (plane && k >= 1 && k <= 3) {
      if (k == 1) {
        psn::PassIO io;
        io.count = count;
        for (int j = 0; j < count; ++j) io.out[j] = a1 + size_t(j) * g.a1_bytes;
        hipError_t e = psn::launch_plane(g, P->precision, io, P->tw[q], P->tw[r], P->kf32, s);
        if (e != hipSuccess) return hip_fail(e, "plane launch");
      }
      continue;
    }
    psn::PassIO io;
    io.count = count;
    io.conv_stride = (long long)(g.a2_bytes / sizeof(float2));
    for (int j = 0; j < count; ++j) {
      void *A1 = a1 + size_t(j) * g.a1_bytes;
      void *A2 = a2 + size_t(j) * g.a2_bytes;
      switch (k) {
        case 0: io.in[j] = rho[j]; io.out[j] = A1; break;
        case 1: io.in[j] = A1; io.out[j] = A2; break;
        case 2: io.in[j] = A2; io.out[j] = A2; break;
        case 3: io.in[j] = A2; io.out[j] = A1; break;
        default: io.in[j] = A1; io.out[j] = V[j]; break;
      }
    }
    hipError_t e = psn::launch_pass(g.pass[k], io, tws[k], P->kf32, g.S[q], P->precision, s);
    if (e != hipSuccess) return hip_fail(e, "pass launch");
  }
  return POISSON_OK;
}

// ----------------------------------------------- persistent batch schedule
// Queue descriptor of pass k of plan P (radix choice and tile shape from B).
int queue_pass(poisson_batch_t B, poisson_plan_t P, int k, psn::QPass &Q) {
  const Geometry &g = P->g;
  const psn::Pass &pp = g.pass[k];
  const int axis[5] = {g.order[0], g.order[1], g.order[2], g.order[1], g.order[0]};
  Q = psn::QPass{};
  Q.tw = P->tw[axis[k]];
  for (int i = 0; i < 3; ++i) {
    Q.in_s[i] = pp.in_s[i];
    Q.out_s[i] = pp.out_s[i];
  }
  Q.kind = pp.kind;
  Q.L = pp.L;
  Q.n_in = pp.n_in;
  Q.n_out = pp.n_out;
  Q.pad = pp.pad ? 1 : 0;
  Q.ext_tile = pp.ext_tile;
  Q.ext_batch = pp.ext_batch;
  // C: the largest power of two with C L <= tile (at least 1)
  Q.c_log2 = 0;
  while ((2 << Q.c_log2) * pp.L <= B->q_tile) ++Q.c_log2;
  Q.C = 1 << Q.c_log2;
  const bool real = pp.kind == psn::KIND_R2C || pp.kind == psn::KIND_C2R;
  Q.W = real ? 2 * Q.C : Q.C;
  Q.tiles_a = (Q.ext_tile + Q.W - 1) / Q.W;
  Q.ntiles = Q.tiles_a * Q.ext_batch;
  const double tile_bytes = double(Q.C) * pp.L * 16.0;  // complex lines in and out
  Q.G = std::max(1, int(B->q_item_kb * 1024.0 / tile_bytes));
  auto it = B->q_radix.find(pp.L);
  Q.nrad = psn::q_radices(pp.L, it == B->q_radix.end() ? 0 : it->second, Q.rad);
  if (Q.nrad == 0) return fail(POISSON_E_STATE, "internal error: no radix decomposition");
  int ns = 1;
  for (int st = 0; st < Q.nrad; ++st) {
    int m = ns, sh = 0;
    Q.ns_three[st] = m % 3 == 0 ? 1 : 0;
    if (Q.ns_three[st]) m /= 3;
    while (m > 1) { m >>= 1; ++sh; }
    Q.ns_shift[st] = sh;
    Q.tw_step[st] = pp.L / (ns * Q.rad[st]);
    ns *= Q.rad[st];
  }
  // element offsets are 32-bit on the device
  const long long big = (1LL << 31) - 1;
  for (int i = 0; i < 3; ++i)
    if (std::llabs(Q.in_s[i]) > big || std::llabs(Q.out_s[i]) > big)
      return fail(POISSON_E_UNSUPPORTED, "array too large for the queue schedule");
  return POISSON_OK;
}

// (Re)builds the queue's descriptors, counters and workspace.  Waits for the
// device: descriptors in use by an earlier launch are replaced.
int queue_build(poisson_batch_t B) {
  const int ns = int(B->which.size()), nplan = int(B->plans.size());
  std::vector<psn::QGeom> geoms(nplan);
  for (int u = 0; u < nplan; ++u) {
    poisson_plan_t P = B->plans[u];
    for (int k = 0; k < 5; ++k) {
      int rc = queue_pass(B, P, k, geoms[u].pass[k]);
      if (rc) return rc;
    }
    geoms[u].kf = P->kf32;
    geoms[u].S_q = P->g.S[P->g.order[1]];
    geoms[u].kq_half = geoms[u].S_q / 2 + 1;
  }
  const int nseg = psn::kQLevels * ns;
  std::vector<psn::QSeg> segs(nseg);
  psn::QParams &a = B->q_params;
  a = psn::QParams{};
  long long first = 0;
  for (int k = 0; k < psn::kQLevels; ++k)
    for (int i = 0; i < ns; ++i) {
      const psn::QPass &Q = geoms[B->which[i]].pass[k];
      const int cnt = (Q.ntiles + Q.G - 1) / Q.G;
      segs[k * ns + i] = {int(first), cnt, i, k};
      first += cnt;
      a.level_items[k] += cnt;
    }
  if (first >= (1LL << 30)) return fail(POISSON_E_UNSUPPORTED, "batch too large for the queue schedule");
  // every solve's intermediates, 256-byte aligned
  std::vector<size_t> off(ns);
  size_t ws = 0;
  for (int i = 0; i < ns; ++i) {
    off[i] = ws;
    ws += B->plans[B->which[i]]->g.ws_bytes;
  }
  auto align = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t geo_b = align(sizeof(psn::QGeom) * nplan), sol_b = align(sizeof(psn::QSolve) * ns),
               seg_b = align(sizeof(psn::QSeg) * nseg);
  PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  auto grow = [&](void **ptr, size_t &have, size_t need, const char *what) -> int {
    if (have >= need && *ptr) return POISSON_OK;
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    have = 0;
    hipError_t e = hipMalloc(ptr, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      hip_fail(e, what);
      return e == hipErrorOutOfMemory ? POISSON_E_NOMEM : POISSON_E_HIP;
    }
    have = need;
    return POISSON_OK;
  };
  int rc = grow(&B->q_desc, B->q_desc_bytes, geo_b + sol_b + seg_b, "hipMalloc(queue descriptors)");
  if (rc) return rc;
  rc = grow(&B->q_ws, B->q_ws_bytes, std::max<size_t>(ws, 256), "hipMalloc(queue workspace)");
  if (rc) return rc;
  if (!B->q_state) {
    void *st = nullptr;
    size_t have = 0;
    rc = grow(&st, have, sizeof(unsigned) * (psn::kQStateHeader + nseg), "hipMalloc(queue counters)");
    if (rc) return rc;
    B->q_state = static_cast<unsigned *>(st);
    PSN_TRY_HIP(hipMemset(B->q_state, 0, have), "hipMemset(queue counters)");
  }
  char *d = static_cast<char *>(B->q_desc);
  PSN_TRY_HIP(hipMemcpy(d, geoms.data(), sizeof(psn::QGeom) * nplan, hipMemcpyHostToDevice),
              "hipMemcpy(queue geometries)");
  PSN_TRY_HIP(hipMemcpy(d + geo_b + sol_b, segs.data(), sizeof(psn::QSeg) * nseg, hipMemcpyHostToDevice),
              "hipMemcpy(queue segments)");
  B->q_solves.assign(ns, psn::QSolve{});
  char *wsb = static_cast<char *>(B->q_ws);
  for (int i = 0; i < ns; ++i) {
    const Geometry &g = B->plans[B->which[i]]->g;
    B->q_solves[i].geom = B->which[i];
    B->q_solves[i].a1 = reinterpret_cast<float2 *>(wsb + off[i]);
    B->q_solves[i].a2 = reinterpret_cast<float2 *>(wsb + off[i] + g.a1_bytes);
  }
  // the solve table goes up with the first solve's arrays
  a.geoms = reinterpret_cast<const psn::QGeom *>(d);
  a.solves = reinterpret_cast<const psn::QSolve *>(d + geo_b);
  a.segs = reinterpret_cast<const psn::QSeg *>(d + geo_b + sol_b);
  a.state = B->q_state;
  a.nsolve = ns;
  a.nseg = nseg;
  a.nitems = int(first);
  int per_cu = 0, cus = 0;
  PSN_TRY_HIP(psn::queue_occupancy(&per_cu), "queue occupancy");
  PSN_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device),
              "hipDeviceGetAttribute");
  B->q_grid = std::max(1, std::min(a.nitems, std::max(1, per_cu) * cus));
  B->q_dirty = false;
  return POISSON_OK;
}

int queue_solve(poisson_batch_t B, const float *const *rho, float *const *V, hipStream_t s) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  PSN_TRY_HIP(hipStreamIsCapturing(s, &cap), "hipStreamIsCapturing");
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (B->q_dirty) {
    if (capturing)
      return fail(POISSON_E_STATE, "queue schedule changed: run one solve outside graph capture first");
    int rc = queue_build(B);
    if (rc) return rc;
  }
  const int ns = int(B->which.size());
  bool changed = false;
  for (int i = 0; i < ns && !changed; ++i)
    changed = B->q_solves[i].rho != rho[i] || B->q_solves[i].V != V[i];
  if (changed) {
    if (capturing)
      return fail(POISSON_E_STATE, "new arrays: run one solve with them outside graph capture first");
    PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");  // the table may be in use
    for (int i = 0; i < ns; ++i) {
      B->q_solves[i].rho = rho[i];
      B->q_solves[i].V = V[i];
    }
    PSN_TRY_HIP(hipMemcpy(const_cast<psn::QSolve *>(B->q_params.solves), B->q_solves.data(),
                          sizeof(psn::QSolve) * ns, hipMemcpyHostToDevice),
                "hipMemcpy(queue solve table)");
  }
  B->q_params.spin_limit = B->q_spin;
  hipError_t e = psn::launch_queue(B->q_params, B->q_grid, s);
  if (e != hipSuccess) return hip_fail(e, "queue launch");
  return POISSON_OK;
}

}  // namespace

extern "C" {

int poisson_solve(poisson_plan_t P, const float *rho, float *V, void *stream) {
  return poisson_solve_passes(P, rho, V, 0, 4, stream);
}

int poisson_solve_passes(poisson_plan_t P, const float *rho, float *V, int first, int last,
                         void *stream) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (first < 0 || last > 4 || first > last) return fail(POISSON_E_ARG, "pass range must satisfy 0 <= first <= last <= 4");
  if (!rho || !V) return fail(POISSON_E_ARG, "rho or V is NULL");
  if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "no K^F has been set or built");
  if (!P->ws) return fail(POISSON_E_STATE, "no workspace");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return enqueue_passes(P, 1, &rho, &V, P->ws, first, last, s);
}

int poisson_solve_host(poisson_plan_t P, const float *rho_host, float *V_host, void *stream) {
  return poisson_solve_host_many(P, 1, &rho_host, &V_host, stream);
}

int poisson_solve_host_many(poisson_plan_t P, int count, const float *const *rho_host,
                            float *const *V_host, void *stream) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (count < 1 || !rho_host || !V_host) return fail(POISSON_E_ARG, "empty request or NULL array");
  for (int i = 0; i < count; ++i)
    if (!rho_host[i] || !V_host[i]) return fail(POISSON_E_ARG, "host pointer " + std::to_string(i) + " is NULL");
  if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "no K^F has been set or built");
  if (!P->ws) return fail(POISSON_E_STATE, "no workspace");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  int rc = ensure_host_io(P);
  if (rc) return rc;
  hipStream_t cs = static_cast<hipStream_t>(stream);
  const size_t bytes = sizeof(float) * size_t(P->g.n[0]) * P->g.n[1] * P->g.n[2];
  // the copy streams start after the caller's earlier work (including an
  // earlier call's last copies, which the caller's stream waited for)
  PSN_TRY_HIP(hipEventRecord(P->ev_start, cs), "hipEventRecord");
  PSN_TRY_HIP(hipStreamWaitEvent(P->h2d, P->ev_start, 0), "hipStreamWaitEvent");
  PSN_TRY_HIP(hipStreamWaitEvent(P->d2h, P->ev_start, 0), "hipStreamWaitEvent");
  for (int i = 0; i < count; ++i) {
    const int b = i & 1;
    float *buf = P->io[b];
    // buffer b is free once its previous result has left the device
    if (i >= 2) PSN_TRY_HIP(hipStreamWaitEvent(P->h2d, P->ev_out[b], 0), "hipStreamWaitEvent");
    PSN_TRY_HIP(hipMemcpyAsync(buf, rho_host[i], bytes, hipMemcpyHostToDevice, P->h2d),
                "hipMemcpyAsync(density to device)");
    PSN_TRY_HIP(hipEventRecord(P->ev_in[b], P->h2d), "hipEventRecord");
    PSN_TRY_HIP(hipStreamWaitEvent(cs, P->ev_in[b], 0), "hipStreamWaitEvent");
    const float *r = buf;
    rc = enqueue_passes(P, 1, &r, &buf, P->ws, 0, 4, cs);
    if (rc) return rc;
    PSN_TRY_HIP(hipEventRecord(P->ev_solved[b], cs), "hipEventRecord");
    PSN_TRY_HIP(hipStreamWaitEvent(P->d2h, P->ev_solved[b], 0), "hipStreamWaitEvent");
    PSN_TRY_HIP(hipMemcpyAsync(V_host[i], buf, bytes, hipMemcpyDeviceToHost, P->d2h),
                "hipMemcpyAsync(potential to host)");
    PSN_TRY_HIP(hipEventRecord(P->ev_out[b], P->d2h), "hipEventRecord");
  }
  // the caller's stream completes after the last copy to the host
  PSN_TRY_HIP(hipEventRecord(P->ev_end, P->d2h), "hipEventRecord");
  PSN_TRY_HIP(hipStreamWaitEvent(cs, P->ev_end, 0), "hipStreamWaitEvent");
  return POISSON_OK;
}

int poisson_plan_destroy(poisson_plan_t P) {
  if (!P) return POISSON_OK;
  {
    DeviceScope ds(P->device);
    (void)hipDeviceSynchronize();
    plan_free_all(P);
  }
  delete P;
  return POISSON_OK;
}

int poisson_batch_create(poisson_batch_t *out, int count, const int *n, const unsigned *bc_mask,
                         const double *h, int precision) {
  try {
    if (!out) return fail(POISSON_E_ARG, "out is NULL");
    *out = nullptr;
    if (count <= 0 || !n || !bc_mask || !h) return fail(POISSON_E_ARG, "empty batch or NULL array");
    int rc = check_precision(precision);
    if (rc) return rc;
    // validate every entry before allocating anything
    for (int i = 0; i < count; ++i) {
      Geometry g;
      std::string err;
      rc = psn::build_geometry(n[3 * i], n[3 * i + 1], n[3 * i + 2], bc_mask[i], g, err);
      if (rc) return fail(rc, "batch entry " + std::to_string(i) + ": " + err);
      if (!(h[i] > 0.0) || !std::isfinite(h[i]))
        return fail(POISSON_E_ARG, "batch entry " + std::to_string(i) + ": bad spacing");
    }
    poisson_batch_t B = new (std::nothrow) poisson_batch_s();
    if (!B) return fail(POISSON_E_NOMEM, "host allocation failed");
    auto cleanup = [&](int code) {
      std::string msg = g_last_error;
      for (auto *pp : B->plans) poisson_plan_destroy(pp);
      if (B->ws) (void)hipFree(B->ws);
      for (hipStream_t st : B->side) (void)hipStreamDestroy(st);
      for (hipEvent_t ev : B->events) (void)hipEventDestroy(ev);
      delete B;
      return fail(code, msg);
    };
    (void)hipGetDevice(&B->device);
    std::map<std::tuple<int, int, int, unsigned, double>, int> index;
    for (int i = 0; i < count; ++i) {
      auto key = std::make_tuple(n[3 * i], n[3 * i + 1], n[3 * i + 2], bc_mask[i], h[i]);
      auto it = index.find(key);
      if (it == index.end()) {
        poisson_plan_t P = nullptr;
        rc = poisson_plan(&P, n[3 * i], n[3 * i + 1], n[3 * i + 2], bc_mask[i], h[i], precision);
        if (rc) return cleanup(rc);
        P->auto_ws = false;  // the batch owns one workspace for every chunk
        it = index.emplace(key, int(B->plans.size())).first;
        B->plans.push_back(P);
        B->members.emplace_back();
      }
      B->which.push_back(it->second);
      B->members[it->second].push_back(i);
    }
    // Solves per launch: as many as keep a chunk's intermediates within the
    // budget, at most kMaxBatch.  Larger chunks mean fewer, fuller launches;
    // on the 512-solve mixed batch 384 MiB measured fastest (96 MiB, which
    // would keep a chunk in the 256 MB last-level cache, was 17% slower).
    // poisson_batch_tune picks the budget on the device.
    double budget_mb = 384.0;
    if (const char *env = std::getenv("POISSON_BATCH_CHUNK_MB")) {
      const double v = std::atof(env);
      if (v > 0) budget_mb = v;
    }
    B->ws_bytes = batch_chunks(B, budget_mb, B->chunk);
    // concurrent streams: 4 by default (the 512-solve mixed batch ran 10%
    // faster in float32 and 20% faster in split fp16 than on one stream)
    B->lanes = B->ws_lanes = kDefaultLanes;
    rc = batch_streams(B, B->lanes);
    if (rc) return cleanup(rc);
    hipError_t e = hipMalloc(&B->ws, B->ws_bytes * size_t(B->ws_lanes));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      B->ws = nullptr;
      hip_fail(e, "hipMalloc(batch workspace)");
      return cleanup(e == hipErrorOutOfMemory ? POISSON_E_NOMEM : POISSON_E_HIP);
    }
    *out = B;
    return POISSON_OK;
  } catch (...) {
    return fail(POISSON_E_STATE, "unexpected exception");
  }
}

int poisson_batch_kernel_build(poisson_batch_t B, void *stream) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  DeviceScope ds(B->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the batch's device");
  // the batch workspace holds at least one solve of every distinct problem
  for (auto *P : B->plans) {
    int rc = build_kernel_into(P, B->ws, B->ws_bytes, static_cast<hipStream_t>(stream));
    if (rc) return rc;
  }
  return POISSON_OK;
}

int poisson_batch_kernel_build_isf(poisson_batch_t B, int order, void *stream) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  if (order < 8 || order > 32 || order % 2)
    return fail(POISSON_E_ARG, "interpolation order must be even, 8 to 32");
  for (size_t u = 0; u < B->plans.size(); ++u)
    if ((B->plans[u]->g.bc & 7u) == 0u)
      return fail(POISSON_E_UNSUPPORTED, "ISF kernels need at least one free axis (distinct problem " +
                                             std::to_string(u) + " is periodic)");
  for (auto *P : B->plans) {
    int rc = poisson_kernel_build_isf(P, order, stream);
    if (rc) return rc;
  }
  return POISSON_OK;
}

int poisson_batch_solve(poisson_batch_t B, const float *const *rho, float *const *V, void *stream) {
  if (!B || !rho || !V) return fail(POISSON_E_ARG, "NULL argument");
  for (size_t i = 0; i < B->which.size(); ++i)
    if (!rho[i] || !V[i]) return fail(POISSON_E_ARG, "batch entry " + std::to_string(i) + ": NULL pointer");
  for (auto *P : B->plans)
    if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "batch kernels not built");
  DeviceScope ds(B->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the batch's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (B->mode == POISSON_BATCH_QUEUE) return queue_solve(B, rho, V, s);
  // the chunks: up to chunk[u] solves of plan u per launch
  struct Chunk {
    int u, start, cnt;
    double cost;
  };
  std::vector<Chunk> chunks;
  for (size_t u = 0; u < B->plans.size(); ++u) {
    const std::vector<int> &m = B->members[u];
    const int c = B->chunk[u];
    for (size_t start = 0; start < m.size(); start += size_t(c)) {
      const int cnt = int(std::min(m.size() - start, size_t(c)));
      chunks.push_back({int(u), int(start), cnt, B->plans[u]->g.alg_bytes * cnt});
    }
  }
  const int lanes = std::min(B->lanes, int(chunks.size()));
  // each chunk to a stream: largest first, to the stream with the fewest
  // algorithmic bytes so far (a solve's result does not depend on it)
  std::vector<int> lane_of(chunks.size(), 0);
  if (lanes > 1) {
    std::vector<int> order(chunks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return chunks[a].cost > chunks[b].cost; });
    std::vector<double> load(lanes, 0.0);
    for (int i : order) {
      const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
      lane_of[i] = l;
      load[l] += chunks[i].cost;
    }
    PSN_TRY_HIP(hipEventRecord(B->events[0], s), "hipEventRecord(fork)");
    for (int l = 1; l < lanes; ++l)
      PSN_TRY_HIP(hipStreamWaitEvent(B->side[l - 1], B->events[0], 0), "hipStreamWaitEvent(fork)");
  }
  std::vector<const float *> r(psn::kMaxBatch);
  std::vector<float *> v(psn::kMaxBatch);
  for (size_t i = 0; i < chunks.size(); ++i) {
    const Chunk &ch = chunks[i];
    const std::vector<int> &m = B->members[ch.u];
    for (int j = 0; j < ch.cnt; ++j) {
      r[j] = rho[m[ch.start + j]];
      v[j] = V[m[ch.start + j]];
    }
    const int l = lane_of[i];
    hipStream_t st = l == 0 ? s : B->side[l - 1];
    void *ws = static_cast<char *>(B->ws) + size_t(l) * B->ws_bytes;
    int rc = enqueue_passes(B->plans[ch.u], ch.cnt, r.data(), v.data(), ws, 0, 4, st);
    if (rc) return rc;
  }
  for (int l = 1; l < lanes; ++l) {
    PSN_TRY_HIP(hipEventRecord(B->events[l], B->side[l - 1]), "hipEventRecord(join)");
    PSN_TRY_HIP(hipStreamWaitEvent(s, B->events[l], 0), "hipStreamWaitEvent(join)");
  }
  return POISSON_OK;
}

int poisson_batch_set_streams(poisson_batch_t B, int streams) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  if (streams < 1 || streams > kMaxLanes) return fail(POISSON_E_ARG, "streams must be 1 to 4");
  DeviceScope ds(B->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the batch's device");
  PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  int rc = batch_streams(B, streams);
  if (rc) return rc;
  rc = batch_reserve(B, B->ws_bytes, streams, nullptr);
  if (rc) return rc;
  B->lanes = streams;
  return POISSON_OK;
}

int poisson_batch_get_streams(poisson_batch_t B, int *streams) {
  if (!B || !streams) return fail(POISSON_E_ARG, "NULL argument");
  *streams = B->lanes;
  return POISSON_OK;
}

int poisson_batch_destroy(poisson_batch_t B) {
  if (!B) return POISSON_OK;
  {
    DeviceScope ds(B->device);
    (void)hipDeviceSynchronize();
    if (B->ws) (void)hipFree(B->ws);
    if (B->q_desc) (void)hipFree(B->q_desc);
    if (B->q_state) (void)hipFree(B->q_state);
    if (B->q_ws) (void)hipFree(B->q_ws);
    for (hipStream_t st : B->side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : B->events) (void)hipEventDestroy(ev);
  }
  for (auto *P : B->plans) poisson_plan_destroy(P);
  delete B;
  return POISSON_OK;
}

int poisson_batch_set_mode(poisson_batch_t B, int mode) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  if (mode != POISSON_BATCH_GROUPED && mode != POISSON_BATCH_QUEUE)
    return fail(POISSON_E_ARG, "mode must be POISSON_BATCH_GROUPED or POISSON_BATCH_QUEUE");
  if (mode == POISSON_BATCH_QUEUE && B->plans[0]->precision != POISSON_FP32)
    return fail(POISSON_E_UNSUPPORTED, "the queue schedule runs float32 batches only");
  B->mode = mode;
  return POISSON_OK;
}

int poisson_batch_get_mode(poisson_batch_t B, int *mode) {
  if (!B || !mode) return fail(POISSON_E_ARG, "NULL argument");
  *mode = B->mode;
  return POISSON_OK;
}

int poisson_queue_radices(int length, int radix_sel, int radices[12]) {
  if (!radices) return fail(POISSON_E_ARG, "radices is NULL");
  if (!psn::supported_length(length)) return fail(POISSON_E_UNSUPPORTED, "length not supported");
  const int n = psn::q_radices(length, radix_sel, radices);
  if (n == 0) return fail(POISSON_E_ARG, "radix choice must be 0, 1 or 2");
  return n;
}

int poisson_batch_set_queue_radix(poisson_batch_t B, int length, int radix_sel) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  int rad[psn::kQMaxRadices];
  if (!psn::supported_length(length)) return fail(POISSON_E_UNSUPPORTED, "length not supported");
  if (psn::q_radices(length, radix_sel, rad) == 0) return fail(POISSON_E_ARG, "radix choice must be 0, 1 or 2");
  B->q_radix[length] = radix_sel;
  B->q_dirty = true;
  return POISSON_OK;
}

int poisson_batch_get_queue_radix(poisson_batch_t B, int length, int *radix_sel) {
  if (!B || !radix_sel) return fail(POISSON_E_ARG, "NULL argument");
  auto it = B->q_radix.find(length);
  *radix_sel = it == B->q_radix.end() ? 0 : it->second;
  return POISSON_OK;
}

int poisson_batch_set_queue_shape(poisson_batch_t B, int tile_elems, int item_kb) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  if (tile_elems < 64 || tile_elems > psn::kQMaxTile || (tile_elems & (tile_elems - 1)))
    return fail(POISSON_E_ARG, "tile_elems must be a power of two, 64 to 2048");
  if (item_kb < 1 || item_kb > (1 << 20)) return fail(POISSON_E_ARG, "item_kb must be 1 to 2^20");
  B->q_tile = tile_elems;
  B->q_item_kb = item_kb;
  B->q_dirty = true;
  return POISSON_OK;
}

int poisson_batch_set_queue_spin(poisson_batch_t B, unsigned spin_limit) {
  if (!B) return fail(POISSON_E_ARG, "batch is NULL");
  if (spin_limit == 0) return fail(POISSON_E_ARG, "spin_limit must be positive");
  B->q_spin = spin_limit;
  return POISSON_OK;
}

int poisson_batch_queue_status(poisson_batch_t B, unsigned *flags) {
  if (!B || !flags) return fail(POISSON_E_ARG, "NULL argument");
  *flags = 0;
  if (!B->q_state) return POISSON_OK;
  DeviceScope ds(B->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the batch's device");
  PSN_TRY_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  PSN_TRY_HIP(hipMemcpy(flags, B->q_state + psn::kQError, sizeof(unsigned), hipMemcpyDeviceToHost),
              "hipMemcpy(queue flags)");
  PSN_TRY_HIP(hipMemset(B->q_state + psn::kQError, 0, sizeof(unsigned)), "hipMemset(queue flags)");
  return POISSON_OK;
}

// Host simulation of the queue protocol (queue.h): `workers` threads play
// workgroups over segments of seg_items[pass * nsolve + solve] items with the
// same ordering, flush and wait rules as the device kernel, and check that
// every item of a dependency segment had finished its work when a dependent
// item passed its wait, that every item ran once and that the counters end at
// zero.  fault (for tests of the checks): 1 skips the flush before a higher
// level, 2 marks an item complete before its work.
int poisson_queue_simulate(int nsolve, const int *seg_items, int workers, int fault, unsigned seed,
                           long long stats[4]) {
  if (nsolve < 1 || !seg_items || workers < 1 || workers > 256 || fault < 0 || fault > 2)
    return fail(POISSON_E_ARG, "bad simulation arguments");
  const int nseg = psn::kQLevels * nsolve;
  std::vector<psn::QSeg> segs(nseg);
  long long level_items[psn::kQLevels] = {0, 0, 0, 0, 0};
  long long first = 0;
  for (int k = 0; k < psn::kQLevels; ++k)
    for (int i = 0; i < nsolve; ++i) {
      const int cnt = seg_items[k * nsolve + i];
      if (cnt < 1) return fail(POISSON_E_ARG, "every segment needs at least one item");
      segs[k * nsolve + i] = {int(first), cnt, i, k};
      first += cnt;
      level_items[k] += cnt;
    }
  if (first > (1 << 24)) return fail(POISSON_E_ARG, "too many items to simulate");
  const unsigned nitems = unsigned(first);
  std::atomic<unsigned> head{0}, exitc{0}, err{0};
  std::vector<std::atomic<unsigned>> lvl(psn::kQLevels), segc(nseg), work(nseg), taken(nitems);
  for (auto &x : lvl) x = 0;
  for (auto &x : segc) x = 0;
  for (auto &x : work) x = 0;
  for (auto &x : taken) x = 0;
  std::atomic<long long> waits{0}, flushes{0}, violations{0}, timeouts{0};
  auto worker = [&](int id) {
    std::mt19937 rng(seed * 7919u + unsigned(id));
    int npend = 0, pend_level = 0, acq_level = -1;
    int pend[psn::kQPending];
    auto flush = [&] {
      for (int j = 0; j < npend; ++j) segc[pend[j]].fetch_add(1);
      lvl[pend_level].fetch_add(unsigned(npend));
      flushes.fetch_add(1);
      npend = 0;
    };
    for (;;) {
      const unsigned item = head.fetch_add(1);
      if (item >= nitems) break;
      taken[item].fetch_add(1);
      const int si = psn::q_find_seg(segs.data(), nseg, int(item));
      const int k = segs[si].pass;
      // fault 1 releases lower-level items only after the wait below
      if (psn::q_must_flush(npend, pend_level, k) && (fault != 1 || pend_level == k)) flush();
      if (psn::q_must_wait(k, acq_level)) {
        const int dep = psn::q_dep_seg(si, nsolve);
        bool full = false;
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
          if (lvl[k - 1].load() >= level_items[k - 1]) { full = true; break; }
          if (segc[dep].load() >= unsigned(segs[dep].count)) break;
          if (err.load() || std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(500)) {
            err.fetch_or(1u);
            timeouts.fetch_add(1);
            break;
          }
          std::this_thread::yield();
        }
        waits.fetch_add(1);
        if (full) acq_level = k - 1;
      }
      if (k > 0 && work[si - nsolve].load() != unsigned(segs[si - nsolve].count)) violations.fetch_add(1);
      if (fault == 2) {
        segc[si].fetch_add(1);
        lvl[k].fetch_add(1);
      }
      if (fault == 2) std::this_thread::sleep_for(std::chrono::milliseconds(5));
      else if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
      work[si].fetch_add(1);
      if (fault != 2) {
        if (npend > 0 && pend_level != k) flush();  // (only under fault 1: a list holds one level)
        pend[npend++] = si;
        pend_level = k;
      }
    }
    if (npend > 0) flush();
    if (exitc.fetch_add(1) == unsigned(workers - 1)) {
      for (auto &x : segc) x = 0;
      for (auto &x : lvl) x = 0;
      head = 0;
      exitc = 0;
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int w = 0; w < workers; ++w) pool.emplace_back(worker, w);
  } catch (...) {
    for (auto &t : pool) t.join();
    return fail(POISSON_E_STATE, "cannot start simulation threads");
  }
  for (auto &t : pool) t.join();
  if (stats) {
    stats[0] = waits.load();
    stats[1] = flushes.load();
    stats[2] = violations.load();
    stats[3] = timeouts.load();
  }
  for (unsigned i = 0; i < nitems; ++i)
    if (taken[i].load() != 1u) return fail(POISSON_E_STATE, "simulation: an item ran " + std::to_string(taken[i].load()) + " times");
  if (violations.load()) return fail(POISSON_E_STATE, "simulation: an item started before its dependency finished");
  if (err.load()) return fail(POISSON_E_STATE, "simulation: a wait ran out");
  for (auto &x : segc)
    if (x.load()) return fail(POISSON_E_STATE, "simulation: counters not reset");
  if (head.load() || exitc.load()) return fail(POISSON_E_STATE, "simulation: queue head not reset");
  return POISSON_OK;
}

// ------------------------------------------------------------- autotuner

int poisson_plan_set_schedule(poisson_plan_t P, const int tile_sel[5]) {
  if (!P || !tile_sel) return fail(POISSON_E_ARG, "NULL argument");
  for (int k = 0; k < 5; ++k) {
    if (tile_sel[k] < 0 || tile_sel[k] >= psn::kSchedules)
      return fail(POISSON_E_ARG, "schedule out of range");
    if (!schedule_valid(P, k, tile_sel[k]))
      return fail(POISSON_E_UNSUPPORTED,
                  "schedule " + std::to_string(tile_sel[k]) + " is not compiled for pass " +
                      std::to_string(k) + " of this plan");
  }
  for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = tile_sel[k];
  return POISSON_OK;
}

int poisson_batch_set_schedule(poisson_batch_t B, const int tile_sel[5]) {
  if (!B || !tile_sel) return fail(POISSON_E_ARG, "NULL argument");
  for (size_t u = 0; u < B->plans.size(); ++u)
    for (int k = 0; k < 5; ++k) {
      if (tile_sel[k] < 0 || tile_sel[k] >= psn::kSchedules)
        return fail(POISSON_E_ARG, "schedule out of range");
      if (!schedule_valid(B->plans[u], k, tile_sel[k]))
        return fail(POISSON_E_UNSUPPORTED,
                    "schedule " + std::to_string(tile_sel[k]) + " is not compiled for pass " +
                        std::to_string(k) + " of distinct problem " + std::to_string(u));
    }
  for (auto *P : B->plans)
    for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = tile_sel[k];
  return POISSON_OK;
}

int poisson_batch_get_schedule(poisson_batch_t B, int index, int tile_sel[5]) {
  if (!B || !tile_sel) return fail(POISSON_E_ARG, "NULL argument");
  if (index < 0 || index >= int(B->which.size()))
    return fail(POISSON_E_ARG, "solve index " + std::to_string(index) + " out of range");
  const poisson_plan_t P = B->plans[B->which[index]];
  for (int k = 0; k < 5; ++k) tile_sel[k] = P->g.pass[k].tile_sel;
  return POISSON_OK;
}

int poisson_plan_get_schedule(poisson_plan_t P, int tile_sel[5], int tile_lines[5]) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  for (int k = 0; k < 5; ++k) {
    const psn::Pass &pass = P->g.pass[k];
    if (tile_sel) tile_sel[k] = pass.tile_sel;
    if (tile_lines)
      tile_lines[k] = k == psn::KIND_CONV ? 0 : psn::pass_tile_lines(pass, pass.tile_sel, P->precision);
  }
  return POISSON_OK;
}

}  // extern "C"

namespace {

// Best (over two rounds) mean time in ms of one `enqueue()` over `reps`
// back-to-back calls on stream s, after one warm-up call.
template <typename F> int time_enqueue(F &&enqueue, hipStream_t s, int reps, double *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  PSN_TRY_HIP(hipEventCreate(&e0), "hipEventCreate");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  double best = INFINITY;
  int rc = enqueue();
  for (int round = 0; round < 2 && rc == POISSON_OK; ++round) {
    e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && rc == POISSON_OK && e == hipSuccess; ++i) rc = enqueue();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess && rc == POISSON_OK) rc = hip_fail(e, "timing events");
    if (rc == POISSON_OK) best = std::min(best, double(t) / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return rc;
}

// Picks each pass's schedule for `count` solves of plan P run together
// (arrays rho/V, intermediates in ws) by coordinate descent over the passes
// (pass 2 first and last):
// a candidate is timed as whole solves, so that what one pass leaves in the
// caches (or evicts) for the next is part of its cost; it replaces the
// current choice only when the solve gets at least 1% faster.  pass_ms (may
// be null) receives the final schedule's per-pass times, from events between
// the passes of whole solves.
int tune_plan_passes(poisson_plan_t P, int count, const float *const *rho, float *const *V,
                     void *ws, hipStream_t s, int reps, double *pass_ms) {
  auto solve = [&] { return enqueue_passes(P, count, rho, V, ws, 0, 4, s); };
  int start[5];
  for (int k = 0; k < 5; ++k) start[k] = P->g.pass[k].tile_sel;
  // a failure leaves the schedules as they were
  auto restore = [&](int code) {
    for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = start[k];
    return code;
  };
  double best = 0;
  int rc = time_enqueue(solve, s, reps, &best);
  if (rc) return rc;
  // small solves are launch-bound and noisy: time at least ~2 ms per round
  if (best > 0) reps = std::max(reps, std::min(1000, int(std::ceil(2.0 / best))));
  rc = time_enqueue(solve, s, reps, &best);
  if (rc) return restore(rc);
  const double start_ms = best;
  // pass 2 first and again last: its plane-kernel choice decides whether
  // passes 1 and 3 run at all, and so which schedules of the others pay
  for (int k : {2, 0, 1, 3, 4, 2}) {
    psn::Pass &pass = P->g.pass[k];
    const int keep = pass.tile_sel;
    int best_sel = keep;
    for (int sel = 0; sel < psn::kSchedules; ++sel) {
      if (sel == keep || !schedule_valid(P, k, sel)) continue;
      pass.tile_sel = sel;
      double t = 0;
      rc = time_enqueue(solve, s, reps, &t);
      if (rc) return restore(rc);
      if (t < 0.99 * best) {
        best = t;
        best_sel = sel;
      }
    }
    pass.tile_sel = best_sel;
  }
  // keep the new schedule only if it still beats the starting one when both
  // are timed again now, alternately, best of two each (one slow window,
  // e.g. a clock change, must not decide)
  bool changed = false;
  for (int k = 0; k < 5; ++k) changed = changed || P->g.pass[k].tile_sel != start[k];
  if (changed) {
    int tuned[5];
    for (int k = 0; k < 5; ++k) tuned[k] = P->g.pass[k].tile_sel;
    double t_tuned = INFINITY, t_start = INFINITY;
    for (int round = 0; round < 2; ++round) {
      double t = 0;
      for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = tuned[k];
      if ((rc = time_enqueue(solve, s, reps, &t))) return restore(rc);
      t_tuned = std::min(t_tuned, t);
      for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = start[k];
      if ((rc = time_enqueue(solve, s, reps, &t))) return restore(rc);
      t_start = std::min(t_start, t);
    }
    const bool keep = t_tuned < 0.99 * std::min(t_start, start_ms);
    for (int k = 0; k < 5; ++k) P->g.pass[k].tile_sel = keep ? tuned[k] : start[k];
  }
  if (!pass_ms) return POISSON_OK;
  hipEvent_t ev[6] = {};
  for (auto &e : ev) {
    hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      for (auto &f : ev)
        if (f) (void)hipEventDestroy(f);
      return hip_fail(he, "hipEventCreate");
    }
  }
  // the launches the chosen schedule runs: five passes, or with the plane
  // kernel pass 0, passes 1-3 as one launch (reported as pass 1) and pass 4
  const bool plane = (P->g.pass[2].tile_sel & psn::kPlaneBit) && psn::plane_available(P->g, P->precision);
  const int ranges[5][2] = {{0, 0}, {1, 1}, {2, 2}, {3, 3}, {4, 4}};
  const int plane_ranges[3][2] = {{0, 0}, {1, 3}, {4, 4}};
  const int plane_slot[3] = {0, 1, 4};
  const int nl = plane ? 3 : 5;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int r = 0; r < reps && rc == POISSON_OK; ++r) {
    hipError_t he = hipEventRecord(ev[0], s);
    for (int k = 0; k < nl && he == hipSuccess && rc == POISSON_OK; ++k) {
      const int *rg = plane ? plane_ranges[k] : ranges[k];
      rc = enqueue_passes(P, count, rho, V, ws, rg[0], rg[1], s);
      if (rc == POISSON_OK) he = hipEventRecord(ev[k + 1], s);
    }
    if (he == hipSuccess) he = hipEventSynchronize(ev[nl]);
    for (int k = 0; k < nl && he == hipSuccess; ++k) {
      float t = 0.f;
      he = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
      acc[plane ? plane_slot[k] : k] += t;
    }
    if (he != hipSuccess && rc == POISSON_OK) rc = hip_fail(he, "timing events");
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 5; ++k) pass_ms[k] = acc[k] / reps;
  return rc;
}

}  // namespace

extern "C" {

int poisson_plan_tune(poisson_plan_t P, const float *rho, float *V, int reps, double pass_ms[5],
                      void *stream) {
  if (!P) return fail(POISSON_E_ARG, "plan is NULL");
  if (!rho || !V) return fail(POISSON_E_ARG, "rho or V is NULL");
  if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "no K^F has been set or built");
  if (!P->ws) return fail(POISSON_E_STATE, "no workspace");
  DeviceScope ds(P->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the plan's device");
  if (reps <= 0) reps = 10;
  const int rc = tune_plan_passes(P, 1, &rho, &V, P->ws, static_cast<hipStream_t>(stream), reps, pass_ms);
  if (rc == POISSON_OK) cache_store(P);
  return rc;
}

int poisson_set_tune_cache(const char *path) {
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  g_cache_path_set = true;
  g_cache_path = path ? path : "";
  return POISSON_OK;
}

int poisson_batch_tune(poisson_batch_t B, const float *const *rho, float *const *V, int reps,
                       double *chunk_mb, void *stream) {
  if (!B || !rho || !V) return fail(POISSON_E_ARG, "NULL argument");
  for (size_t i = 0; i < B->which.size(); ++i)
    if (!rho[i] || !V[i]) return fail(POISSON_E_ARG, "batch entry " + std::to_string(i) + ": NULL pointer");
  for (auto *P : B->plans)
    if (!P->kernel_ready) return fail(POISSON_E_NO_KERNEL, "batch kernels not built");
  DeviceScope ds(B->device);
  if (!ds.ok) return fail(POISSON_E_HIP, "cannot select the batch's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (reps <= 0) reps = 5;
  B->mode = POISSON_BATCH_GROUPED;  // steps 1-3 tune the grouped launches
  // 1. tile schedules of every plan, timed on its first chunk
  std::vector<const float *> r(psn::kMaxBatch);
  std::vector<float *> v(psn::kMaxBatch);
  for (size_t u = 0; u < B->plans.size(); ++u) {
    const std::vector<int> &m = B->members[u];
    const int cnt = std::min(int(m.size()), B->chunk[u]);
    for (int j = 0; j < cnt; ++j) {
      r[j] = rho[m[j]];
      v[j] = V[m[j]];
    }
    int rc = tune_plan_passes(B->plans[u], cnt, r.data(), v.data(), B->ws, s, reps, nullptr);
    if (rc) return rc;
  }
  // 2. the intermediates budget of one launch, timed on the whole batch; a
  // failure restores the chunking it started from (a grown workspace stays)
  const std::vector<int> chunk0 = B->chunk;
  const double mb0 = B->chunk_mb;
  auto restore = [&](int code) {
    B->chunk = chunk0;
    B->chunk_mb = mb0;
    return code;
  };
  std::vector<double> budgets = {B->chunk_mb};  // the current budget first
  for (double mb : {32.0, 64.0, 96.0, 128.0, 192.0, 256.0, 384.0, 512.0})
    if (mb != B->chunk_mb) budgets.push_back(mb);
  double best_mb = B->chunk_mb, best = INFINITY;
  {
    for (double mb : budgets) {
      std::vector<int> chunk;
      const size_t need = batch_chunks(B, mb, chunk);
      if (batch_reserve(B, need, B->lanes, s) != POISSON_OK)
        continue;  // a budget that does not fit is not a candidate
      B->chunk = chunk;
      double t = 0;
      int rc = time_enqueue([&] { return poisson_batch_solve(B, rho, V, stream); }, s, reps, &t);
      if (rc) return restore(rc);
      if (t < 0.99 * best) {
        best = t;
        best_mb = mb;
      }
    }
  }
  (void)batch_chunks(B, best_mb, B->chunk);
  if (chunk_mb) *chunk_mb = best_mb;
  // 3. concurrent streams, timed on the whole batch at that budget
  {
    const int lanes0 = B->lanes;
    int best_lanes = lanes0;
    best = INFINITY;
    for (int lanes = 1; lanes <= kMaxLanes; ++lanes) {
      int rc = batch_streams(B, lanes);
      if (rc) return rc;
      if (batch_reserve(B, B->ws_bytes, lanes, s) != POISSON_OK) break;
      B->lanes = lanes;
      double t = 0;
      rc = time_enqueue([&] { return poisson_batch_solve(B, rho, V, stream); }, s, reps, &t);
      if (rc) {
        B->lanes = lanes0;
        return rc;
      }
      if (t < 0.99 * best) {
        best = t;
        best_lanes = lanes;
      }
    }
    B->lanes = best_lanes;
  }
  // 4. float32: the persistent schedule, radix choice per line length
  // (coordinate descent over the lengths), then the tile and item size; it
  // becomes the batch's schedule only if it beats the grouped launches
  if (B->plans[0]->precision == POISSON_FP32) {
    double grouped = INFINITY;
    int rc = time_enqueue([&] { return poisson_batch_solve(B, rho, V, stream); }, s, reps, &grouped);
    if (rc) return rc;
    B->mode = POISSON_BATCH_QUEUE;
    auto timed = [&](double *t) {
      return time_enqueue([&] { return poisson_batch_solve(B, rho, V, stream); }, s, reps, t);
    };
    double qbest = INFINITY;
    rc = timed(&qbest);
    if (rc) {
      B->mode = POISSON_BATCH_GROUPED;
      return rc;
    }
    std::vector<int> lengths;
    for (auto *P : B->plans)
      for (int k = 0; k < 5; ++k)
        if (std::find(lengths.begin(), lengths.end(), P->g.pass[k].L) == lengths.end())
          lengths.push_back(P->g.pass[k].L);
    std::sort(lengths.begin(), lengths.end());
    for (int L : lengths) {
      auto it = B->q_radix.find(L);
      const int cur = it == B->q_radix.end() ? 0 : it->second;
      int keep = cur;
      int rad[psn::kQMaxRadices];
      const int n0 = psn::q_radices(L, cur, rad);
      for (int sel = 0; sel < psn::kQRadixChoices; ++sel) {
        if (sel == cur) continue;
        int other[psn::kQMaxRadices];
        const int n1 = psn::q_radices(L, sel, other);
        if (n1 == n0 && std::equal(rad, rad + n0, other)) continue;  // the same stages
        B->q_radix[L] = sel;
        B->q_dirty = true;
        double t = 0;
        rc = timed(&t);
        if (rc) {
          B->mode = POISSON_BATCH_GROUPED;
          return rc;
        }
        if (t < 0.99 * qbest) {
          qbest = t;
          keep = sel;
        }
      }
      B->q_radix[L] = keep;
      B->q_dirty = true;
    }
    const int kb0 = B->q_item_kb, tile0 = B->q_tile;
    int best_kb = kb0, best_tile = tile0;
    for (int tile : {1024, 2048})
      for (int kb : {128, 512, 2048}) {
        if (kb == kb0 && tile == tile0) continue;
        B->q_item_kb = kb;
        B->q_tile = tile;
        B->q_dirty = true;
        double t = 0;
        rc = timed(&t);
        if (rc) {
          B->mode = POISSON_BATCH_GROUPED;
          return rc;
        }
        if (t < 0.99 * qbest) {
          qbest = t;
          best_kb = kb;
          best_tile = tile;
        }
      }
    B->q_item_kb = best_kb;
    B->q_tile = best_tile;
    B->q_dirty = true;
    B->mode = qbest < grouped ? POISSON_BATCH_QUEUE : POISSON_BATCH_GROUPED;
  }
  return POISSON_OK;
}

int poisson_rel_l2(const float *v, const double *ref, size_t count, double *out, void *stream) {
  if (!v || !ref || !out || count == 0) return fail(POISSON_E_ARG, "NULL argument or empty input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int max_blocks = 1024;
  double *partials = nullptr;
  PSN_TRY_HIP(hipMalloc(&partials, sizeof(double) * 2 * max_blocks), "hipMalloc(partials)");
  int blocks = 0;
  hipError_t e = psn::launch_rel_l2_partials(v, ref, count, partials, max_blocks, &blocks, s);
  std::vector<double> host(2 * max_blocks);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), partials, sizeof(double) * 2 * blocks,
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(partials);
  if (e != hipSuccess) return hip_fail(e, "relative L2 norm");
  double num = 0, den = 0;
  for (int b = 0; b < blocks; ++b) {
    num += host[2 * b];
    den += host[2 * b + 1];
  }
  *out = den > 0 ? std::sqrt(num / den) : (num > 0 ? INFINITY : 0.0);
  return POISSON_OK;
}

int poisson_rel_l2_noalloc(const float *v, const double *ref, size_t count, double *out_dev,
                           void *stream) {
  if (!v || !ref || !out_dev || count == 0) return fail(POISSON_E_ARG, "NULL argument or empty input");
  hipError_t e = psn::launch_rel_l2_noalloc(v, ref, count, out_dev, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "relative L2 norm (static scratch)");
  return POISSON_OK;
}

}  // extern "C"
