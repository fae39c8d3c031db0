// kernel_build.hip - float64 setup and check kernels: the Green's-function
// octant K^F, its float32 pass-order copy, and the float64 residual norm.
//
// The paper takes its kernels from the BigDFT solver it accelerates and
// cites, for free, wire and surface BCs, kernels it does not write out
// (Section 2).  The family built here: spectral on periodic axes
// (k_j = 2 pi f_j / (S_j h), kappa^2 = sum of periodic k_j^2) and, along the
// d free axes, h^d times the Green's function of (lap_d - kappa^2) sampled at
// the grid offsets, with origin weights that keep the trapezoidal rule
// fourth-order accurate; then the DFT along the free axes.  For an even
// sequence on S points that DFT is a DCT-I over the S/2+1 unique samples,
// which is what this file evaluates, as plain float64 sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "kernels.h"

namespace psn {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
// -(value of the analytically continued sum of 1/|m| over Z^3 without 0)
constexpr double kCoulombOrigin = 2.837297479480619;

// K0(x) for x > 0 from K0(x) = int_0^inf exp(-x cosh t) dt by the trapezoidal
// rule, which converges geometrically for this integrand (analytic in the
// strip |Im t| < pi/2).  The step shrinks with x so the e^x growth of the
// integrand inside the strip stays below float64 resolution; exp(-x) is
// factored out so the sum itself never underflows.
__device__ double bessel_k0(double x) {
  const double step = fmin(0.25, (kPi * kPi) / (x + 40.0));
  double sum = 0.5;
  for (int j = 1; j < 4096; ++j) {
    const double sh = sinh(0.5 * j * step);
    const double e = 2.0 * x * sh * sh;  // x (cosh t - 1)
    if (e > 40.0) break;
    sum += exp(-e);
  }
  return step * sum * exp(-x);
}

struct BuildParams {
  int S[3];
  int O[3];  // octant extents S_j/2 + 1
  unsigned bc;
  double h;
  double c2;  // ln(2 sqrt(pi) / Gamma(1/4)^2)
};

// Mixed-representation samples on the octant: offsets m_j along free axes,
// frequencies f_j along periodic axes.
__global__ void sample_kernel(BuildParams p, double *out) {
  const long long n = (long long)p.O[0] * p.O[1] * p.O[2];
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i1 = int(idx % p.O[0]);
    const int i2 = int((idx / p.O[0]) % p.O[1]);
    const int i3 = int(idx / ((long long)p.O[0] * p.O[1]));
    const int ii[3] = {i1, i2, i3};
    double kappa2 = 0.0, m2 = 0.0;
    int d = 0;
    for (int j = 0; j < 3; ++j) {
      if ((p.bc >> j) & 1u) {
        m2 += double(ii[j]) * ii[j];
        ++d;
      } else {
        const double k = 2.0 * kPi * ii[j] / (p.S[j] * p.h);
        kappa2 += k * k;
      }
    }
    const double h = p.h;
    const double kappa = sqrt(kappa2);
    double val;
    if (d == 0) {
      val = kappa2 > 0.0 ? -1.0 / kappa2 : 0.0;
    } else if (d == 1) {
      const double r = h * sqrt(m2);
      if (m2 == 0.0) {
        // the |y|/2 kink at the node: Euler-Maclaurin correction h^2/12
        val = (kappa > 0.0 ? -h / (2.0 * kappa) : 0.0) + h * h / 12.0;
      } else {
        val = kappa > 0.0 ? -h * exp(-kappa * r) / (2.0 * kappa) : 0.5 * h * r;
      }
    } else if (d == 2) {
      const double r = h * sqrt(m2);
      const double w = h * h / (2.0 * kPi);
      if (m2 == 0.0) {
        val = w * (kappa > 0.0 ? log(0.5 * kappa * h) + kEulerGamma + p.c2 : log(h) + p.c2);
      } else {
        val = kappa > 0.0 ? -w * bessel_k0(kappa * r) : w * log(r);
      }
    } else {
      val = m2 == 0.0 ? -(h * h / (4.0 * kPi)) * kCoulombOrigin : -(h * h) / (4.0 * kPi * sqrt(m2));
    }
    out[idx] = val;
  }
}

// DCT-I along one axis of the octant: out[k] = sum_m w_m in[m] cos(2 pi k m / S),
// w_0 = w_{S/2} = 1, otherwise 2 (the full-length DFT of an even sequence).
__global__ void dct1_axis_kernel(const double *in, double *out, int O0, int O1, int O2, int axis,
                                 int S, const double *cos_tab) {
  const long long n = (long long)O0 * O1 * O2;
  const int O[3] = {O0, O1, O2};
  const long long stride = axis == 0 ? 1 : (axis == 1 ? (long long)O0 : (long long)O0 * O1);
  const int M = O[axis];
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int ii[3] = {int(idx % O0), int((idx / O0) % O1), int(idx / ((long long)O0 * O1))};
    const int k = ii[axis];
    const long long base = idx - (long long)k * stride;
    double acc = 0.0;
    for (int m = 0; m < M; ++m) {
      const double w = (m == 0 || 2 * m == S) ? 1.0 : 2.0;
      acc += w * in[base + m * stride] * cos_tab[(long long)k * m % S];
    }
    out[idx] = acc;
  }
}

struct PermuteParams {
  int O[3];        // octant extents per physical axis
  int order[3];    // p, q, r
  int E[3];        // internal extents: H, S_q/2+1, S_r/2+1
  double scale;    // 1 / (S1 S2 S3)
};

__global__ void permute_kernel(PermuteParams p, const double *kf64, float *kf32) {
  const long long n = (long long)p.E[0] * p.E[1] * p.E[2];
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int kr = int(idx % p.E[2]);
    const int kq = int((idx / p.E[2]) % p.E[1]);
    const int kp = int(idx / ((long long)p.E[2] * p.E[1]));
    int k[3];
    k[p.order[0]] = kp;
    k[p.order[1]] = kq;
    k[p.order[2]] = kr;
    const long long src = k[0] + (long long)p.O[0] * (k[1] + (long long)p.O[1] * k[2]);
    kf32[idx] = float(kf64[src] * p.scale);
  }
}

constexpr int kNormThreads = 256;

__global__ __launch_bounds__(kNormThreads) void rel_l2_kernel(const float *v, const double *ref,
                                                              size_t count, double *partials) {
  __shared__ double s_num[kNormThreads], s_den[kNormThreads];
  double num = 0.0, den = 0.0;
  for (size_t i = blockIdx.x * (size_t)kNormThreads + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kNormThreads) {
    const double r = ref[i];
    const double d = double(v[i]) - r;
    num += d * d;
    den += r * r;
  }
  s_num[threadIdx.x] = num;
  s_den[threadIdx.x] = den;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_num[threadIdx.x] += s_num[threadIdx.x + w];
      s_den[threadIdx.x] += s_den[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s_num[0];
    partials[2 * blockIdx.x + 1] = s_den[0];
  }
}

int grid_for(long long n, int threads) {
  long long g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : int(g);
}

}  // namespace

hipError_t launch_kernel_build(const Geometry &g, double h, double *kf64, double *tmp,
                               const double *const cos_tabs[3], hipStream_t s) {
  BuildParams p;
  for (int j = 0; j < 3; ++j) {
    p.S[j] = g.S[j];
    p.O[j] = g.S[j] / 2 + 1;
  }
  p.bc = g.bc;
  p.h = h;
  p.c2 = std::log(2.0) + 0.5 * std::log(kPi) - 2.0 * std::lgamma(0.25);
  const long long n = (long long)p.O[0] * p.O[1] * p.O[2];
  const int threads = 256;
  // sample into whichever buffer leaves the result in kf64 after the DCTs
  int nfree = 0;
  for (int j = 0; j < 3; ++j) nfree += (g.bc >> j) & 1u;
  double *cur = (nfree % 2 == 0) ? kf64 : tmp;
  double *other = (cur == kf64) ? tmp : kf64;
  hipLaunchKernelGGL(sample_kernel, dim3(grid_for(n, threads)), dim3(threads), 0, s, p, cur);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int j = 0; j < 3; ++j) {
    if (!((g.bc >> j) & 1u)) continue;
    hipLaunchKernelGGL(dct1_axis_kernel, dim3(grid_for(n, threads)), dim3(threads), 0, s,
                       (const double *)cur, other, p.O[0], p.O[1], p.O[2], j, p.S[j], cos_tabs[j]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double *t = cur;
    cur = other;
    other = t;
  }
  return hipSuccess;
}

hipError_t launch_kernel_permute(const Geometry &g, const double *kf64, float *kf32,
                                 hipStream_t s) {
  PermuteParams p;
  for (int j = 0; j < 3; ++j) {
    p.O[j] = g.S[j] / 2 + 1;
    p.order[j] = g.order[j];
  }
  p.E[0] = g.H;
  p.E[1] = g.S[g.order[1]] / 2 + 1;
  p.E[2] = g.S[g.order[2]] / 2 + 1;
  p.scale = 1.0 / (double(g.S[0]) * g.S[1] * g.S[2]);
  const long long n = (long long)p.E[0] * p.E[1] * p.E[2];
  hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, kf64, kf32);
  return hipGetLastError();
}

// ------------------------------------------- allocation-free residual
// The per-block partial sums of the allocation-free residual live in this
// file-scope device array (16 KiB, held by every device the library runs
// on until the process ends).  In host code `scratch` names a host-side
// stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int kScratchBlocks = 1024;
static __device__ __align__(256) double scratch[2 * kScratchBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// device's first call).
hipError_t scratch_address(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Sum of the block partials in block order (the order the host sum of
// poisson_rel_l2 uses), then sqrt(num / den) with the same zero cases.
__global__ void rel_l2_final_kernel(const double *partials, int blocks, double *out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int b = 0; b < blocks; ++b) {
    num += partials[2 * b];
    den += partials[2 * b + 1];
  }
  *out = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? HUGE_VAL : 0.0);
}

}  // namespace

hipError_t launch_rel_l2_noalloc(const float *v, const double *ref, size_t count, double *out,
                                 hipStream_t s) {
  double *partials = nullptr;
  hipError_t e = scratch_address(&partials);
  if (e != hipSuccess) return e;
  int blocks = 0;
  e = launch_rel_l2_partials(v, ref, count, partials, kScratchBlocks, &blocks, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rel_l2_final_kernel, dim3(1), dim3(64), 0, s, (const double *)partials, blocks,
                     out);
  return hipGetLastError();
}

hipError_t launch_rel_l2_partials(const float *v, const double *ref, size_t count,
                                  double *partials, int max_blocks, int *blocks, hipStream_t s) {
  long long b = (long long)((count + kNormThreads - 1) / kNormThreads);
  if (b > max_blocks) b = max_blocks;
  if (b < 1) b = 1;
  *blocks = int(b);
  hipLaunchKernelGGL(rel_l2_kernel, dim3(int(b)), dim3(kNormThreads), 0, s, v, ref, count,
                     partials);
  return hipGetLastError();
}

}  // namespace psn
