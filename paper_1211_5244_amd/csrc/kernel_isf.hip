// kernel_isf.hip - float64 free-boundary K^F on interpolating scaling
// functions, the kernel family of the BigDFT solver the paper implements
// (Section 2 and the start of Section 3 take their kernels from it).
//
// The grid values of the density are read as the coefficients of an
// expansion in Deslauriers-Dubuc interpolating scaling functions phi of even
// order m (8 to 32), so the potential at the grid points is the convolution
// of Eq. 2 with (lap V = rho)
//   K(i) = -(h^2 / 4 pi) I(i),   I(i) = int phi(u1) phi(u2) phi(u3) / |i - u| d^3u.
// 1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt separates the integral,
//   I(i) = (2/sqrt(pi)) int_0^inf g(t, i1) g(t, i2) g(t, i3) dt,
//   g(t, n) = int phi(u) exp(-t^2 (n - u)^2) du,
// and with it the DFT over the padded grid (S = 2N on every axis): K^F is the
// t integral of the product of the three 1-D DCT-Is of g.  So the 3-D kernel
// is never formed in real space.
//
// The t integral: 16-point Gauss-Legendre panels of unit length in
// s = ln t from t = 1e-12 to 4096.  Below 1e-12 every g is 1 to 1e-20 and
// the piece is 2e-12/sqrt(pi) everywhere in real space, which is prod(S)
// times that at k = 0.  Above 4096 only the origin keeps a term,
// (2/sqrt(pi)) int (sqrt(pi)/t)^3 dt = pi/4096^2, constant in k.
//
// g(t, n) is the projection of the Gaussian f(u) = exp(-t^2 u^2) onto the
// shifted scaling functions, through the refinement relation
// phi(x) = sum_k a_k phi(2x - k), a_k = phi(k/2): with
// c_j[n] = 2^j int phi(2^j u - n) f(u) du,
//   c_j[n] = 1/2 sum_k a_k c_{j+1}[2n + k],   g(t, n) = c_0[n],
// started at a level J fine enough that c_J[p] = f(p 2^-J): phi's moments 1
// to m-1 vanish, so that error falls like (t 2^-J)^m; J is the smallest level
// with 2^J >= c t, c = max(32, 2^ceil(64/m)).  f is symmetric, so each level
// is stored for n >= 0 only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace psn {

namespace {

constexpr double kIsfTMin = 1e-12;
constexpr double kIsfTMax = 4096.0;
constexpr int kIsfGauss = 16;           // Gauss-Legendre points per panel
constexpr int kIsfMaxTaps = 63;         // a_k, |k| <= m - 1 <= 31
constexpr int kIsfBuf = 4096;           // doubles per cascade level in LDS
constexpr int kIsfThreads = 256;

struct IsfNode {
  double t;   // Gaussian parameter
  double w;   // quadrature weight, (2/sqrt(pi)) t dt/ds times the panel weight
  double wt;  // the plain weight of dt (t dt/ds times the panel weight)
  int J;      // starting dyadic level (0: g is the sample exp(-t^2 n^2))
  int P;      // level-J samples kept for 0 <= p <= P
};

struct IsfParams {
  int O[3];               // octant extents S_j/2 + 1
  int S[3];
  int m;                  // interpolation order
  int omax;               // max O_j
  int row;                // one node's DCT row: O[0] + O[1] + O[2] (+ O[f1m])
  int free_mask;          // axes whose DCT rows are made
  int f1m;                // axis of the DCT of 1 - g (one free axis), else -1
  double a[kIsfMaxTaps];  // a_k at index k + m - 1
};

// Deslauriers-Dubuc refinement filter a_k = phi(k/2), |k| <= m - 1: a_0 = 1,
// a_k = 0 for even k != 0, and for odd k = 2l + 1 the value at l + 1/2 of
// the degree m-1 Lagrange polynomial through the integer nodes
// l - m/2 + 1 .. l + m/2 that is 1 at node 0 and 0 at the others (phi
// interpolates delta_0 at the integers).
void dd_filter(int m, double *a) {
  const int M = m / 2;
  for (int k = -(m - 1); k <= m - 1; ++k) {
    long double v = 0.0L;
    if (k == 0) {
      v = 1.0L;
    } else if (k % 2 != 0) {
      const int l = (k - 1) / 2;  // exact: k - 1 is even
      const int lo = l - M + 1, hi = l + M;
      if (lo <= 0 && 0 <= hi) {
        v = 1.0L;
        const long double x = l + 0.5L;
        for (int node = lo; node <= hi; ++node)
          if (node != 0) v *= (x - node) / (0.0L - node);
      }
    }
    a[k + m - 1] = double(v);
  }
}

// n-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, long double *x, long double *w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) {
        // derivative at the converged root
        p0 = 1.0L;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0L);
        break;
      }
    }
    x[i] = z;
    w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

std::vector<IsfNode> isf_nodes(int m) {
  long double x[kIsfGauss], w[kIsfGauss];
  gauss_legendre(kIsfGauss, x, w);
  const long double a = logl(kIsfTMin), b = logl(kIsfTMax);
  const int panels = int(ceill(b - a));
  const long double L = (b - a) / panels;
  const long double two_over_sqrt_pi = 1.128379167095512573896158903121545172L;
  const double c = std::max(32.0, std::ldexp(1.0, (64 + m - 1) / m));
  std::vector<IsfNode> out;
  for (int k = 0; k < panels; ++k)
    for (int i = 0; i < kIsfGauss; ++i) {
      const long double s = a + L * (k + (x[i] + 1.0L) / 2.0L);
      const long double t = expl(s);
      IsfNode nd;
      nd.t = double(t);
      nd.w = double(two_over_sqrt_pi * t * w[i] * L / 2.0L);
      nd.wt = double(t * w[i] * L / 2.0L);
      int J = 0;
      while (std::ldexp(1.0, J) < c * nd.t) ++J;
      nd.J = J;
      nd.P = J ? int(std::floor(7.0 * std::ldexp(1.0, J) / nd.t)) : 0;
      out.push_back(nd);
    }
  return out;
}

// One workgroup per node: g(t, n) by the cascade, then its DCT-I along each
// axis, DCT_j(k) = sum_{n <= S_j/2} w_n g(t, n) cos(2 pi k n / S_j), w_n = 1
// at n = 0 and n = S_j/2, otherwise 2 (the DFT of the even extension).
__global__ __launch_bounds__(kIsfThreads) void isf_table_kernel(IsfParams p, const IsfNode *nodes,
                                                                const double *cos0,
                                                                const double *cos1,
                                                                const double *cos2, double *table) {
  __shared__ double buf[2][kIsfBuf];
  const IsfNode nd = nodes[blockIdx.x];
  const int tid = threadIdx.x;
  int cur = 0, R;
  if (nd.J == 0) {
    R = p.omax - 1;
    for (int n = tid; n <= R; n += kIsfThreads) buf[0][n] = exp(-(nd.t * n) * (nd.t * n));
  } else {
    R = nd.P;
    for (int q = tid; q <= R; q += kIsfThreads) {
      const double u = nd.t * ldexp(double(q), -nd.J);
      buf[0][q] = exp(-u * u);
    }
    const int m = p.m;
    for (int j = nd.J - 1; j >= 0; --j) {
      __syncthreads();
      const double *src = buf[cur];
      double *dst = buf[cur ^ 1];
      const int Rn = (R + m - 1) / 2;
      for (int n = tid; n <= Rn; n += kIsfThreads) {
        double acc = 0.0;
        for (int k = -(m - 1); k <= m - 1; ++k) {
          if (k != 0 && (k & 1) == 0) continue;
          int x = 2 * n + k;
          x = x < 0 ? -x : x;
          if (x <= R) acc += p.a[k + m - 1] * src[x];
        }
        dst[n] = 0.5 * acc;
      }
      cur ^= 1;
      R = Rn;
    }
  }
  __syncthreads();
  const double *g = buf[cur];
  double *row = table + (size_t)blockIdx.x * p.row;
  const double *cs[3] = {cos0, cos1, cos2};
  int off = 0;
  for (int d = 0; d < 3; ++d) {
    const int O = p.O[d], S = p.S[d];
    const int top = min(R, O - 1);
    if ((p.free_mask >> d) & 1) {
      for (int k = tid; k < O; k += kIsfThreads) {
        double acc = 0.0;
        for (int n = 0; n <= top; ++n) {
          const double wn = (n == 0 || 2 * n == S) ? 1.0 : 2.0;
          acc += wn * g[n] * cs[d][(long long)k * n % S];
        }
        row[off + k] = acc;
      }
    }
    off += O;
  }
  if (p.f1m >= 0) {
    // the DCT of 1 - g along the one free axis: g is 0 past R, and where g
    // is the sample exp(-t^2 n^2), 1 - g is -expm1(-t^2 n^2) (no cancellation)
    const int d = p.f1m, O = p.O[d], S = p.S[d];
    for (int k = tid; k < O; k += kIsfThreads) {
      double acc = 0.0;
      for (int n = 0; n < O; ++n) {
        const double wn = (n == 0 || 2 * n == S) ? 1.0 : 2.0;
        const double x = nd.t * n;
        const double omg = nd.J == 0 ? -expm1(-x * x) : (n <= R ? 1.0 - g[n] : 1.0);
        acc += wn * omg * cs[d][(long long)k * n % S];
      }
      row[off + k] = acc;
    }
  }
}

// Surface and wire problems: one workgroup per periodic wave-number pair
// (surface) or wave number (wire), kappa^2 the sum of the periodic k_j^2,
// k_j = 2 pi f_j / (S_j h), a = kappa h / 2.  Along the free axes
//   surface, kappa > 0: -(h^2 / (2 sqrt pi)) int DCT g(t) exp(-a^2/t^2) dt / t^2
//   surface, kappa = 0:  (h^2 / (2 sqrt pi)) int DCT (1 - g(t)) dt / t^2
//   wire, kappa > 0:    -(h^2 / (2 pi)) int DCT g(t) DCT g(t) exp(-a^2/t^2) dt / t
//   wire, kappa = 0:     (h^2 / (2 pi)) [(ln h + int exp(-t^2) dt / t) prod S_f at k = 0
//                                        - int DCT g(t) DCT g(t) dt / t]
// (the transforms of the ISF integrals of exp(-kappa|y|)/(2 kappa), |y|/2,
// K0(kappa r)/(2 pi) and ln(r)/(2 pi)), plus the end pieces: -h^2/(4 T^2)
// from the origin above T in every case; for the surface at kappa = 0 also
// the 1 of 1 - g above T (S_f / T at k = 0) and below the panels
// (t_min DCT(n^2)).  The node weights of the workgroup's kappa sit in LDS.
constexpr int kIsfMaxNodes = 1024;
__global__ __launch_bounds__(kIsfThreads) void isf_assemble_mixed_kernel(
    IsfParams p, const IsfNode *nodes, int count, const double *table, double h,
    double wire_const, const double *dct_n2, double *out) {
  __shared__ double wk[kIsfMaxNodes];
  const double pi = 3.14159265358979323846;
  int fr[2], nf = 0, per[2], np = 0;
  for (int d = 0; d < 3; ++d) {
    if ((p.free_mask >> d) & 1) fr[nf++] = d;
    else per[np++] = d;
  }
  // this workgroup's periodic octant indices
  int kp[2] = {0, 0};
  {
    int b = blockIdx.x;
    for (int i = 0; i < np; ++i) {
      kp[i] = b % p.O[per[i]];
      b /= p.O[per[i]];
    }
  }
  double kappa2 = 0.0;
  for (int i = 0; i < np; ++i) {
    const double k = 2.0 * pi * kp[i] / (p.S[per[i]] * h);
    kappa2 += k * k;
  }
  const double a2 = 0.25 * kappa2 * h * h;
  const bool zero = kappa2 == 0.0;
  for (int q = threadIdx.x; q < count; q += kIsfThreads) {
    const double t = nodes[q].t, wt = nodes[q].wt;
    if (nf == 1) wk[q] = zero ? wt / (t * t) : wt * exp(-a2 / (t * t)) / (t * t);
    else wk[q] = zero ? wt / t : wt * exp(-a2 / (t * t)) / t;
  }
  __syncthreads();
  const double Tm = kIsfTMax;
  long long stride[3] = {1, p.O[0], (long long)p.O[0] * p.O[1]};
  long long base = 0;
  for (int i = 0; i < np; ++i) base += kp[i] * stride[per[i]];
  int off[3];
  off[0] = 0;
  off[1] = p.O[0];
  off[2] = p.O[0] + p.O[1];
  const int extra = p.O[0] + p.O[1] + p.O[2];
  if (nf == 1) {
    const int f = fr[0], O = p.O[f];
    const double c = h * h / (2.0 * sqrt(pi));
    for (int k = threadIdx.x; k < O; k += kIsfThreads) {
      double acc = 0.0;
      if (zero) {
        for (int q = 0; q < count; ++q) acc += wk[q] * table[(size_t)q * p.row + extra + k];
        acc += kIsfTMin * dct_n2[k];
        if (k == 0) acc += double(p.S[f]) / Tm;
        acc = c * acc;
      } else {
        for (int q = 0; q < count; ++q) acc += wk[q] * table[(size_t)q * p.row + off[f] + k];
        acc = -c * acc;
      }
      out[base + k * stride[f]] = acc - h * h / (4.0 * Tm * Tm);
    }
  } else {
    const int f0 = fr[0], f1 = fr[1], O0 = p.O[f0], O1 = p.O[f1];
    const double c = h * h / (2.0 * pi);
    for (int e = threadIdx.x; e < O0 * O1; e += kIsfThreads) {
      const int k0 = e % O0, k1 = e / O0;
      double acc = 0.0;
      for (int q = 0; q < count; ++q) {
        const double *row = table + (size_t)q * p.row;
        acc += wk[q] * row[off[f0] + k0] * row[off[f1] + k1];
      }
      if (zero) {
        acc = -acc;
        if (e == 0) acc += wire_const * double(p.S[f0]) * double(p.S[f1]);
        acc = c * acc;
      } else {
        acc = -c * acc;
      }
      out[base + k0 * stride[f0] + k1 * stride[f1]] = acc - h * h / (4.0 * Tm * Tm);
    }
  }
}

// K^F(k) = pref (sum over nodes w DCT_1(k1) DCT_2(k2) DCT_3(k3) + tails):
// the origin's t > 4096 term (constant in k) and, at k = 0, prod(S) times
// the t < 1e-12 constant.
__global__ void isf_assemble_kernel(IsfParams p, const IsfNode *nodes, int count,
                                    const double *table, double pref, double tail_all,
                                    double tail_k0, double *out) {
  const long long total = (long long)p.O[0] * p.O[1] * p.O[2];
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int k1 = int(idx % p.O[0]);
    const int k2 = int((idx / p.O[0]) % p.O[1]);
    const int k3 = int(idx / ((long long)p.O[0] * p.O[1]));
    double acc = 0.0;
    for (int q = 0; q < count; ++q) {
      const double *row = table + (size_t)q * p.row;
      acc += nodes[q].w * row[k1] * row[p.O[0] + k2] * row[p.O[0] + p.O[1] + k3];
    }
    acc += tail_all;
    if (idx == 0) acc += tail_k0;
    out[idx] = pref * acc;
  }
}

}  // namespace

size_t isf_table_bytes(const Geometry &g) {
  const size_t nodes = isf_nodes(16).size();
  size_t row = 0, omax = 0;
  for (int j = 0; j < 3; ++j) {
    row += size_t(g.S[j] / 2 + 1);
    omax = std::max(omax, size_t(g.S[j] / 2 + 1));
  }
  row += omax;  // the DCT of 1 - g (one free axis)
  // the node records, the DCT of n^2, then the DCT rows
  return nodes * sizeof(IsfNode) + 256 + omax * sizeof(double) + 256 + nodes * row * sizeof(double);
}

hipError_t launch_isf_build(const Geometry &g, double h, int order, double *kf64, void *scratch,
                            size_t scratch_bytes, const double *const cos_tabs[3],
                            hipStream_t s) {
  if (order < 8 || order > 32 || order % 2 || scratch_bytes < isf_table_bytes(g))
    return hipErrorInvalidValue;
  const unsigned fm = g.bc & 7u;
  const int nfree = int(fm & 1u) + int((fm >> 1) & 1u) + int((fm >> 2) & 1u);
  if (nfree == 0) return hipErrorInvalidValue;
  IsfParams p;
  p.m = order;
  p.omax = 0;
  p.row = 0;
  p.free_mask = int(fm);
  p.f1m = -1;
  for (int j = 0; j < 3; ++j) {
    p.S[j] = g.S[j];
    p.O[j] = g.S[j] / 2 + 1;
    p.omax = std::max(p.omax, p.O[j]);
    p.row += p.O[j];
    if (nfree == 1 && ((fm >> j) & 1u)) p.f1m = j;
  }
  if (p.f1m >= 0) p.row += p.O[p.f1m];
  if (p.omax > kIsfBuf) return hipErrorInvalidValue;
  dd_filter(order, p.a);
  const std::vector<IsfNode> nodes = isf_nodes(order);
  if (int(nodes.size()) > kIsfMaxNodes) return hipErrorInvalidValue;
  for (const IsfNode &nd : nodes)
    if (nd.P >= kIsfBuf) return hipErrorInvalidValue;
  char *base = static_cast<char *>(scratch);
  IsfNode *dnodes = reinterpret_cast<IsfNode *>(base);
  const size_t node_bytes = (nodes.size() * sizeof(IsfNode) + 255) / 256 * 256;
  double *dct_n2 = reinterpret_cast<double *>(base + node_bytes);
  const size_t n2_bytes = (size_t(p.omax) * sizeof(double) + 255) / 256 * 256;
  double *table = reinterpret_cast<double *>(base + node_bytes + n2_bytes);
  // blocking copies: the host arrays live on this function's stack
  hipError_t e = hipMemcpy(dnodes, nodes.data(), nodes.size() * sizeof(IsfNode),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  if (p.f1m >= 0) {
    // DCT-I of n^2 along the free axis (the small-t piece of the surface
    // kernel at kappa = 0), in long double
    const int f = p.f1m, O = p.O[f], S = p.S[f];
    std::vector<double> v(O);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < O; ++k) {
      long double acc = 0.0L;
      for (int n = 0; n < O; ++n) {
        const long double wn = (n == 0 || 2 * n == S) ? 1.0L : 2.0L;
        acc += wn * (long double)n * n * cosl(two_pi * (long double)((long long)k * n % S) / S);
      }
      v[k] = double(acc);
    }
    e = hipMemcpy(dct_n2, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(isf_table_kernel, dim3(unsigned(nodes.size())), dim3(kIsfThreads), 0, s, p,
                     (const IsfNode *)dnodes, cos_tabs[0], cos_tabs[1], cos_tabs[2], table);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nfree < 3) {
    // one workgroup per periodic octant index (pair)
    long long groups = 1;
    long double wire_const = logl((long double)h);
    for (int j = 0; j < 3; ++j)
      if (!((fm >> j) & 1u)) groups *= p.O[j];
    for (const IsfNode &nd : nodes)
      wire_const += (long double)nd.wt * expl(-(long double)nd.t * nd.t) / nd.t;
    hipLaunchKernelGGL(isf_assemble_mixed_kernel, dim3(unsigned(groups)), dim3(kIsfThreads), 0, s,
                       p, (const IsfNode *)dnodes, int(nodes.size()), (const double *)table, h,
                       double(wire_const), (const double *)dct_n2, kf64);
    return hipGetLastError();
  }
  const double pi = 3.14159265358979323846;
  const double pref = -(h * h) / (4.0 * pi);
  const double tail_all = pi / (kIsfTMax * kIsfTMax);
  const double tail_k0 =
      2.0 * kIsfTMin / std::sqrt(pi) * double(g.S[0]) * double(g.S[1]) * double(g.S[2]);
  const long long total = (long long)p.O[0] * p.O[1] * p.O[2];
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(isf_assemble_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p,
                     (const IsfNode *)dnodes, int(nodes.size()), (const double *)table, pref,
                     tail_all, tail_k0, kf64);
  return hipGetLastError();
}

}  // namespace psn
