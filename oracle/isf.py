"""Free-boundary Green's function on interpolating scaling functions (ISF).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper implements the Poisson solver of the BigDFT package and takes its
kernels from it (Section 2, first paragraph of Section 3).  That solver's
free-boundary kernel reads the grid values of the density as the
coefficients of an expansion in interpolating scaling functions:

    rho(r) = sum_j rho_j phi3(r/h - j),   phi3(u) = phi(u1) phi(u2) phi(u3),

with phi the Deslauriers-Dubuc interpolating scaling function of even order
m.  The potential of that density at the grid points is the discrete
convolution of Eq. 2, V_i = sum_j K(i - j) rho_j, with (lap V = rho, so the
Green's function is -1/(4 pi r))

    K(i) = -(h^2 / 4 pi) I(i),   I(i) = int phi3(u) / |i - u| d^3u.

Steps, each a plain definition or a quadrature of one:

1. phi.  Deslauriers-Dubuc subdivision: values at the integers are delta_0;
   each halving of the spacing keeps the old values and sets every new
   midpoint to the value, at that midpoint, of the degree m-1 polynomial
   through the m nearest old values (Lagrange interpolation).  The values at
   the dyadic points are exact and never change at later levels.
2. 1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt separates the integral:
   I(i) = (2/sqrt(pi)) int_0^inf g(t, i1) g(t, i2) g(t, i3) dt, with
   g(t, n) = int phi(u) exp(-t^2 (n - u)^2) du.
3. g by the trapezoidal rule on the dyadic grid of level J:
   g = 2^-J sum_p phi(p 2^-J) exp(-t^2 (n - p 2^-J)^2).  phi's Fourier
   transform vanishes to order m at every nonzero multiple of 2 pi (it
   reproduces polynomials of degree < m), so the rule's aliasing error for a
   Gaussian of width 1/t falls like (t 2^-J)^m.  J is the smallest level
   with 2^J >= c_m t, c_m = max(16, 2^ceil(64/m)), which keeps that factor
   at or below 2^-64; measured, the values then agree with those of four
   times finer grids to rounding.  Orders 8 to 32 are served (lower orders
   would need far finer grids).  At J = 0 the rule is the sample
   exp(-t^2 n^2) itself.
4. The t integral in three parts:
   - t <= t_lo = 1/c_m (J = 0): the integrand is exp(-t^2 |i|^2), whose
     integral is erf(t_lo |i|) sqrt(pi) / (2 |i|) (and t_lo at i = 0);
   - t_lo <= t <= 4096: Gauss-Legendre panels in s = ln t (16 points per
     unit panel; the integrand is analytic and varies on a unit scale in s);
   - t >= 4096: g(t, n) = (sqrt(pi)/t) (phi(n) + O(t^-2)), so only the
     origin keeps a term, pi / 4096^2, with an error of order 4096^-4.
   The tests check each split point and the panels by moving or refining
   them.
5. K^F: the even extension of K to the padded grid S_j = 2 N_j (Section 3),
   and its whole-grid FFT, as `greens.kernel_fourier` does for the sampled
   kernel.
"""

from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import scipy.fft
from scipy import special

T_MAX = 4096.0         # upper end; the origin tail beyond is pi / T_MAX^2
PANEL = 1.0            # panel length in s = ln t
GL_POINTS = 16         # Gauss-Legendre points per panel
ORDERS = range(8, 33, 2)  # interpolation orders served by the kernel
GAUSS_CUT = 7.0        # exp(-t^2 x^2) is dropped beyond t |x| = 7 (e^-49)


def dd_midpoint_weights(order):
    """Deslauriers-Dubuc subdivision weights, exact rationals: the Lagrange
    weights of the nodes -M+1 .. M (M = order/2) at x = 1/2, in node order.
    A new midpoint between old points k and k+1 is sum_l w_l f(k + l)."""
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    M = order // 2
    nodes = list(range(-M + 1, M + 1))
    weights = []
    for l in nodes:
        w = Fraction(1)
        for k in nodes:
            if k != l:
                w *= (Fraction(1, 2) - k) / (l - k)
        weights.append(w)
    return nodes, weights


_PHI_CACHE = {}


def isf_values(order, level):
    """phi(p 2^-level) for p = -(order-1) 2^level .. (order-1) 2^level by
    subdivision from the integer values delta_0 (phi vanishes outside
    [-(order-1), order-1])."""
    key = (order, level)
    if key in _PHI_CACHE:
        return _PHI_CACHE[key]
    nodes, weights = dd_midpoint_weights(order)
    w = [float(x) for x in weights]
    M = order // 2
    R = order - 1
    vals = np.zeros(2 * R + 1)
    vals[R] = 1.0
    for _ in range(level):
        n = vals.size
        ext = np.concatenate([np.zeros(M), vals, np.zeros(M)])
        mid = np.zeros(n - 1)
        for wl, l in zip(w, nodes):
            mid += wl * ext[M + l: M + l + n - 1]
        new = np.empty(2 * n - 1)
        new[0::2] = vals
        new[1::2] = mid
        vals = new
    _PHI_CACHE[key] = vals
    return vals


def level_factor(order):
    """c_m = max(16, 2^ceil(64/m)): the dyadic grid spacing is at most
    1/(c_m t)."""
    return max(16, 2 ** -(-64 // order))


def dyadic_level(t, order, factor=None):
    """Smallest J >= 0 with 2^J >= c t (c = level_factor(order) unless given)."""
    c = level_factor(order) if factor is None else factor
    J = 0
    while 2.0 ** J < c * t:
        J += 1
    return J


def gauss_integrals(order, t, nmax, factor=None):
    """g(t, n) = int phi(u) exp(-t^2 (n-u)^2) du for n = 0 .. nmax, by the
    trapezoidal rule on the dyadic grid of level dyadic_level(t, order)."""
    J = dyadic_level(t, order, factor)
    n = np.arange(nmax + 1)
    if J == 0:
        return np.exp(-(t * n) ** 2)
    phi = isf_values(order, J)
    R = order - 1
    step = 2.0 ** -J
    out = np.zeros(nmax + 1)
    reach = GAUSS_CUT / t
    for k in range(min(nmax, int(R + reach) + 1) + 1):
        # grid points u = p step within reach of k and inside the support
        lo = max(-R * 2 ** J, math.ceil((k - reach) / step))
        hi = min(R * 2 ** J, math.floor((k + reach) / step))
        if lo > hi:
            continue
        p = np.arange(lo, hi + 1)
        u = p * step
        out[k] = step * np.sum(phi[p + R * 2 ** J] * np.exp(-(t * (k - u)) ** 2))
    return out


def quadrature_nodes(t_lo, t_hi=T_MAX, panel=PANEL, points=GL_POINTS):
    """Gauss-Legendre panels in s = ln t on [ln t_lo, ln t_hi]: nodes t and
    weights for int f(t) dt = int f(e^s) e^s ds."""
    x, w = np.polynomial.legendre.leggauss(points)
    a, b = math.log(t_lo), math.log(t_hi)
    K = max(1, math.ceil((b - a) / panel - 1e-12))
    L = (b - a) / K
    s = np.concatenate([a + L * (k + (x + 1.0) / 2.0) for k in range(K)])
    ws = np.concatenate([w * L / 2.0 for _ in range(K)])
    t = np.exp(s)
    return t, ws * t


def coulomb_integrals(order, offsets_shape, t_lo=None, t_hi=T_MAX, panel=PANEL,
                      points=GL_POINTS):
    """I(i) = int phi3(u) / |i - u| d^3u for 0 <= i_j <= offsets_shape[j]-1,
    array shape (n3, n2, n1) with i1 fastest."""
    if order not in ORDERS:
        raise ValueError("interpolation order must be even, 8 to 32")
    if t_lo is None:
        t_lo = 1.0 / level_factor(order)
    o1, o2, o3 = offsets_shape
    t, w = quadrature_nodes(t_lo, t_hi, panel, points)
    nmax = max(o1, o2, o3) - 1
    G = np.array([gauss_integrals(order, tq, nmax) for tq in t])
    W = (2.0 / math.sqrt(math.pi)) * w
    i1, i2, i3 = np.arange(o1), np.arange(o2), np.arange(o3)
    r = np.sqrt(i3[:, None, None] ** 2 + i2[None, :, None] ** 2 + i1[None, None, :] ** 2
                ).astype(np.float64)
    # t <= t_lo: (2/sqrt(pi)) int_0^t_lo exp(-t^2 r^2) dt
    safe = np.where(r > 0, r, 1.0)
    I = np.where(r > 0, special.erf(t_lo * safe) / safe, 2.0 * t_lo / math.sqrt(math.pi))
    # the panels: sum over nodes q of W_q g(t_q, i3) g(t_q, i2) g(t_q, i1),
    # as one matrix product over q
    A = (G[:, :o3][:, :, None] * G[:, :o2][:, None, :]).reshape(t.size, o3 * o2)
    I += (A.T @ (W[:, None] * G[:, :o1])).reshape(o3, o2, o1)
    # t >= t_hi: the origin's (2/sqrt(pi)) int (sqrt(pi)/t)^3 dt
    I[0, 0, 0] += math.pi / t_hi ** 2
    return I


def isf_kernel_real(n, h, order=16, **quad):
    """K(i) = -(h^2/4pi) I(i) on the octant 0 <= i_j <= N_j, shape
    (N3+1, N2+1, N1+1)."""
    shape = (n[0] + 1, n[1] + 1, n[2] + 1)
    return -(h * h / (4.0 * math.pi)) * coulomb_integrals(order, shape, **quad)


def isf_kernel_fourier(n, h, order=16, half=False, **quad):
    """K^F of the fully free problem on the padded grid S_j = 2 N_j, real
    float64: the even extension of the real-space octant (K_pad[j] =
    K(min(j, S - j)) per axis) and its whole-grid FFT.  Shape (S3, S2, S1),
    or with half=True the real-input half spectrum (S3, S2, S1/2+1), which is
    all `solve` reads."""
    K = isf_kernel_real(n, h, order, **quad)
    S = tuple(2 * x for x in n)
    for axis, Sx in ((2, S[0]), (1, S[1]), (0, S[2])):
        j = np.arange(Sx)
        K = np.take(K, np.minimum(j, Sx - j), axis=axis)
    fft = scipy.fft.rfftn if half else scipy.fft.fftn
    kf = fft(K, workers=os.cpu_count() or 1)
    del K
    if float(np.abs(kf.imag).max()) > 1e-9 * float(np.abs(kf.real).max()):
        raise AssertionError("kernel is not even: K^F has an imaginary part")
    return np.ascontiguousarray(kf.real)


def isf_kernel_octant(n, h, order=16, kf=None, **quad):
    """The unique octant 0 <= k_j <= S_j/2 of K^F (as greens.kernel_octant)."""
    if kf is None:
        kf = isf_kernel_fourier(n, h, order, half=True, **quad)
    return np.ascontiguousarray(kf[: n[2] + 1, : n[1] + 1, : n[0] + 1])


# ------------------------------------------------------------ mixed BCs
# Surface (one free axis) and wire (two free axes) problems: along the
# periodic axes the kernel stays spectral, k_j = 2 pi f_j / (S_j h) and
# kappa^2 = sum of periodic k_j^2 (the same reading as the sampled kernels),
# and along the free axes the Green's function of (lap_d - kappa^2) is
# integrated against the scaling functions, as in the free case:
#   d = 1:  G(y) = -exp(-kappa |y|) / (2 kappa),  |y|/2 at kappa = 0;
#   d = 2:  G(r) = -K0(kappa r) / (2 pi),          ln(r) / (2 pi) at kappa = 0,
# K_kappa(n) = h^d int phi_d(u) G(h (n - u)) d^d u.  Gaussian integrals
# separate them again (tau = h t, a = kappa h / 2):
#   exp(-kappa|y|)/(2 kappa) = (1/(2 sqrt pi)) int exp(-y^2 t^2 - kappa^2/(4 t^2)) dt / t^2,
#   |y|                      = (1/sqrt pi)     int (1 - exp(-y^2 t^2)) dt / t^2,
#   K0(kappa r)              =                 int exp(-r^2 t^2 - kappa^2/(4 t^2)) dt / t,
#   ln r                     =                 int (exp(-t^2) - exp(-r^2 t^2)) dt / t,
# so with g(tau, n) of the free case
#   d = 1, kappa > 0:  K = -(h^2 / (2 sqrt pi)) int g(tau, n) exp(-a^2/tau^2) dtau / tau^2
#   d = 1, kappa = 0:  K =  (h^2 / (2 sqrt pi)) int (1 - g(tau, n)) dtau / tau^2
#   d = 2, kappa > 0:  K = -(h^2 / (2 pi)) int g(tau, i) g(tau, j) exp(-a^2/tau^2) dtau / tau
#   d = 2, kappa = 0:  K =  (h^2 / (2 pi)) [ln h + int (exp(-tau^2) - g(tau, i) g(tau, j)) dtau / tau].
# Quadrature: the same Gauss-Legendre panels in ln tau, from MIXED_TAU_LO to
# T_MAX; below, the integrands are their small-tau forms (n^2 tau_lo for
# d = 1 at kappa = 0, negligible otherwise); above, only the origin keeps a
# term (g ~ sqrt(pi)/tau there): -1/(4 T^2) times h^2 in every case, plus
# h^2/(2 sqrt pi) / T for d = 1 at kappa = 0.  1 - g is formed as -expm1 where
# g is the sample exp(-tau^2 n^2), so small tau loses nothing to cancellation.

MIXED_TAU_LO = 1e-9


def _free_kernel_1d(order, kappa_h, nfree, nodes):
    """h^-2 K_kappa(n), n = 0 .. nfree, for one free axis."""
    t, w, G, OneMinusG = nodes
    n = np.arange(nfree + 1, dtype=np.float64)
    c = 1.0 / (2.0 * math.sqrt(math.pi))
    if kappa_h > 0.0:
        a2 = (0.5 * kappa_h) ** 2
        wk = w * np.exp(-a2 / t ** 2) / t ** 2
        out = -c * (wk @ G[:, : nfree + 1])
    else:
        out = c * ((w / t ** 2) @ OneMinusG[:, : nfree + 1])
        out += c * (n ** 2 * MIXED_TAU_LO + 1.0 / T_MAX)   # below the panels; above: the 1 of 1 - g
        out[0] += c * (-math.sqrt(math.pi) / (2.0 * T_MAX ** 2))
    out[0] += -0.25 / T_MAX ** 2 if kappa_h > 0.0 else 0.0
    return out


def _free_kernel_2d(order, kappa_h, n1, n2, h, nodes):
    """h^-2 K_kappa(i, j), i = 0 .. n1 (fastest), j = 0 .. n2: shape (n2+1, n1+1)."""
    t, w, G, _ = nodes
    c = 1.0 / (2.0 * math.pi)
    A, B = G[:, : n2 + 1], G[:, : n1 + 1]
    if kappa_h > 0.0:
        a2 = (0.5 * kappa_h) ** 2
        wk = w * np.exp(-a2 / t ** 2) / t
        out = -c * ((A * wk[:, None]).T @ B)
    else:
        const = math.log(h) + float(np.sum(w * np.exp(-t ** 2) / t))
        out = c * (const - (A * (w / t)[:, None]).T @ B)
    out[0, 0] += -0.25 / T_MAX ** 2
    return out


def _mixed_nodes(order, nmax):
    t, w = quadrature_nodes(MIXED_TAU_LO, T_MAX, PANEL, GL_POINTS)
    G = np.array([gauss_integrals(order, tq, nmax) for tq in t])
    n = np.arange(nmax + 1, dtype=np.float64)
    OneMinusG = np.array([-np.expm1(-(tq * n) ** 2) if dyadic_level(tq, order) == 0 else 1.0 - G[q]
                          for q, tq in enumerate(t)])
    return t, w, G, OneMinusG


def isf_mixed_kernel_fourier(n, bc_mask, h, order=16, half=False):
    """K^F for surface (one free axis) and wire (two free axes) problems on
    the padded grid (S3, S2, S1) (half=True: the half spectrum along x): the
    mixed representation (periodic axes in Fourier, free axes as the ISF
    kernel at offsets min(j, S_j - j)), then the FFT along the free axes."""
    if order not in ORDERS:
        raise ValueError("interpolation order must be even, 8 to 32")
    free = [j for j in range(3) if (bc_mask >> j) & 1]
    per = [j for j in range(3) if not (bc_mask >> j) & 1]
    if len(free) not in (1, 2):
        raise ValueError("one or two free axes")
    S = [n[j] * (2 if j in free else 1) for j in range(3)]
    nodes = _mixed_nodes(order, max(n[j] for j in free))
    # periodic wave numbers of every mode and the distinct kappa h values
    ks = [2.0 * math.pi * np.fft.fftfreq(S[j], d=1.0 / S[j]) / (S[j] * h) for j in per]
    grids = np.meshgrid(*ks, indexing="ij")
    kappa_h = np.sqrt(sum(k ** 2 for k in grids)) * h
    uniq, inv = np.unique(kappa_h, return_inverse=True)  # +-f give bitwise equal kappa
    inv = inv.reshape(kappa_h.shape)
    if len(free) == 1:
        (f,) = free
        tabs = np.array([_free_kernel_1d(order, float(kh), n[f], nodes) for kh in uniq])
        idx = np.minimum(np.arange(S[f]), S[f] - np.arange(S[f]))
        vals = h * h * tabs[:, idx]                     # (kappa, S_f)
        mixed_pf = vals[inv]                            # (S_per0, S_per1, S_f)
        order_axes = per + [f]
    else:
        f0, f1 = free
        tabs = np.array([_free_kernel_2d(order, float(kh), n[f0], n[f1], h, nodes) for kh in uniq])
        i0 = np.minimum(np.arange(S[f0]), S[f0] - np.arange(S[f0]))
        i1 = np.minimum(np.arange(S[f1]), S[f1] - np.arange(S[f1]))
        vals = h * h * tabs[:, i1][:, :, i0]            # (kappa, S_f1, S_f0)
        mixed_pf = vals[inv]                            # (S_per, S_f1, S_f0)
        order_axes = per + [f1, f0]
    # to array axes (S3, S2, S1): physical axis j is array axis 2 - j
    perm = [order_axes.index(j) for j in (2, 1, 0)]
    mixed = np.transpose(mixed_pf, perm)
    free_axes = tuple(2 - j for j in free)
    kf = scipy.fft.fftn(mixed, axes=free_axes, workers=os.cpu_count() or 1)
    if float(np.abs(kf.imag).max()) > 1e-9 * float(np.abs(kf.real).max()):
        raise AssertionError("kernel is not even: K^F has an imaginary part")
    kf = np.ascontiguousarray(kf.real)
    return kf[:, :, : S[0] // 2 + 1].copy() if half else kf
