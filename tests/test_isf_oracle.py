"""Pins of the oracle's interpolating-scaling-function (ISF) Green's
function (free BCs), each against something other than the oracle itself:
textbook filter values, exact properties of Deslauriers-Dubuc functions,
closed forms, a library quadrature, the far field of 1/r, invariance under
the quadrature's own split points and refinements, and the potential of a
Gaussian charge."""

import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import isf

H = 0.3


def test_midpoint_weights_textbook_values():
    # the four-point scheme (order 4): -1/16, 9/16, 9/16, -1/16
    nodes, w = isf.dd_midpoint_weights(4)
    assert nodes == [-1, 0, 1, 2]
    assert w == [Fraction(-1, 16), Fraction(9, 16), Fraction(9, 16), Fraction(-1, 16)]
    # order 2: the midpoint average
    assert isf.dd_midpoint_weights(2)[1] == [Fraction(1, 2), Fraction(1, 2)]
    # order 6: 3/256, -25/256, 150/256, 150/256, -25/256, 3/256
    assert isf.dd_midpoint_weights(6)[1] == [Fraction(x, 256) for x in (3, -25, 150, 150, -25, 3)]


@pytest.mark.parametrize("order", [2, 4, 8, 16, 32])
def test_midpoint_weights_reproduce_polynomials(order):
    nodes, w = isf.dd_midpoint_weights(order)
    for p in range(order):
        assert sum(wl * Fraction(l) ** p for wl, l in zip(w, nodes)) == Fraction(1, 2) ** p
    # and not the next degree: the scheme has order exactly m
    assert sum(wl * Fraction(l) ** order for wl, l in zip(w, nodes)) != Fraction(1, 2) ** order


def test_order_two_is_the_hat_function():
    level = 6
    phi = isf.isf_values(2, level)
    x = np.arange(-2 ** level, 2 ** level + 1) / 2.0 ** level
    assert np.array_equal(phi, 1.0 - np.abs(x))


@pytest.mark.parametrize("order", [8, 16, 24])
def test_scaling_function_properties(order):
    level = 7
    R = order - 1
    phi = isf.isf_values(order, level)
    step = 2.0 ** -level
    x = np.arange(-R * 2 ** level, R * 2 ** level + 1) * step
    # interpolating: phi(k) = delta_k0
    ints = phi[:: 2 ** level]
    assert ints[R] == 1.0 and np.all(ints[np.arange(ints.size) != R] == 0.0)
    # symmetric
    assert np.allclose(phi, phi[::-1], rtol=0, atol=1e-15)
    # polynomial reproduction sum_k k^p phi(x - k) = x^p at dyadic x in [0, 1)
    for frac in (0.25, 0.5, 0.875):
        k = np.arange(-R, R + 2)
        idx = np.round((frac - k) / step).astype(int) + R * 2 ** level
        ok = (idx >= 0) & (idx < phi.size)
        vals = np.where(ok, phi[np.clip(idx, 0, phi.size - 1)], 0.0)
        for p in range(0, order, 3):
            assert abs(np.sum(k.astype(float) ** p * vals) - frac ** p) <= 1e-12 * max(1, R ** p)
    # unit integral and vanishing moments 1 .. m-1 (trapezoidal rule on the
    # dyadic grid, exact for phi times polynomials of degree < m)
    assert abs(step * phi.sum() - 1.0) <= 1e-14
    for p in range(1, order):
        scale = step * np.sum(np.abs(x) ** p * np.abs(phi))
        assert abs(step * np.sum(x ** p * phi)) <= 1e-12 * scale, p
    # the m-th moment does not vanish
    assert abs(step * np.sum(x ** order * phi)) > 1e-6


@pytest.mark.parametrize("order", [8, 16, 32])
@pytest.mark.parametrize("t", [0.02, 0.3, 1.7, 12.0, 900.0])
def test_gauss_integral_sum_rule(order, t):
    """sum over all integers n of g(t, n) = int exp(-t^2 u^2) du = sqrt(pi)/t,
    since the shifted phi sum to one."""
    g = isf.gauss_integrals(order, t, 4000)
    total = g[0] + 2.0 * g[1:].sum()
    assert abs(total * t / math.sqrt(math.pi) - 1.0) <= 2e-15


@pytest.mark.parametrize("order", [8, 16])
def test_gauss_integral_limits(order):
    # wide Gaussians: g(t, n) = exp(-t^2 n^2) + O(t^m) (the m-th moment of
    # phi is the first that does not vanish)
    n = np.arange(60)
    d = [np.max(np.abs(isf.gauss_integrals(order, t, 59) - np.exp(-(t * n) ** 2)))
         for t in (0.1, 0.05)]
    assert d[1] <= 1e3 * 0.05 ** order
    if d[1] > 1e-14:
        assert 2 ** (order - 1) <= d[0] / d[1] <= 2 ** (order + 1)
    # narrow Gaussians: g(t, 0) t / sqrt(pi) -> phi(0) = 1, g(t, 1) -> phi(1) = 0
    g = isf.gauss_integrals(order, 3000.0, 3)
    assert abs(g[0] * 3000.0 / math.sqrt(math.pi) - 1.0) <= 1e-6
    assert abs(g[1]) <= 1e-6 * g[0]


@pytest.mark.parametrize("order", [8, 16, 24])
def test_gauss_integral_grid_refinement(order):
    """Four times finer dyadic grids leave g unchanged to rounding."""
    for t in (0.4, 3.0, 50.0):
        c = isf.level_factor(order)
        a = isf.gauss_integrals(order, t, 40)
        b = isf.gauss_integrals(order, t, 40, factor=4 * c)
        assert np.max(np.abs(a - b)) <= 4e-16 * np.max(np.abs(b)), t


def test_gauss_integral_hat_closed_form():
    """Order 2 (the hat): the trapezoidal rule at a fine enough level against
    scipy's adaptive quadrature of (1 - |u|) exp(-t^2 (n - u)^2)."""
    for t, n in ((0.8, 0), (0.8, 1), (2.5, 0), (2.5, 2)):
        ref, _ = integrate.quad(lambda u: (1 - abs(u)) * math.exp(-(t * (n - u)) ** 2), -1, 1,
                                points=[0.0], epsabs=1e-15, epsrel=1e-14)
        got = isf.gauss_integrals(2, t, 3, factor=2 ** 14)[n]
        assert abs(got - ref) <= 1e-8 * max(ref, 1e-3), (t, n, got, ref)


def _I(order=16, shape=(12, 12, 12), **kw):
    return isf.coulomb_integrals(order, shape, **kw)


def test_coulomb_far_field():
    """Outside the support of phi3 (radius (m-1) sqrt 3) the first m-1
    multipole moments of phi3 beyond the charge vanish, so I(i) = 1/|i| to
    the order-m term; at |i| = 10 the deviation is already tiny."""
    I = _I(16, (41, 41, 41))
    for i in [(40, 0, 0), (20, 20, 20), (40, 30, 10)]:
        r = math.sqrt(sum(x * x for x in i))
        assert abs(I[i[2], i[1], i[0]] * r - 1.0) <= 1e-14
    r = math.sqrt(10 ** 2 + 3 ** 2)
    assert abs(I[0, 3, 10] * r - 1.0) <= 1e-8
    # near the charge the smearing shows: I(0) is finite, I(1,0,0) above 1
    assert 2.0 < I[0, 0, 0] < 3.0
    assert I[0, 0, 1] > 1.0


def test_coulomb_symmetry():
    I = _I(16, (9, 9, 9))
    assert np.array_equal(I, I.transpose(1, 0, 2)) or np.allclose(I, I.transpose(1, 0, 2), rtol=1e-15)
    assert np.allclose(I, I.transpose(2, 1, 0), rtol=1e-14, atol=0)


@pytest.mark.parametrize("order", [8, 16])
def test_coulomb_quadrature_split_points_and_panels(order):
    """Moving the lower split, the upper cut-off or halving the panels
    changes I by rounding only: the analytic end pieces (erf below, pi/T^2
    above) and the panels are consistent."""
    base = _I(order, (9, 9, 9))
    c = isf.level_factor(order)
    for kw in ({"t_lo": 0.5 / c}, {"t_hi": 16384.0}, {"panel": 0.5}, {"points": 24}):
        other = _I(order, (9, 9, 9), **kw)
        assert np.max(np.abs(other - base) / base) <= 1e-13, kw


def test_coulomb_orders_converge_to_each_other():
    """Higher orders smear the unit charge over wider, smoother functions;
    far from the charge all orders give 1/|i| and near it they differ."""
    a = _I(16, (24, 24, 24))
    b = _I(24, (24, 24, 24))
    r = math.sqrt(23 ** 2 * 3)
    assert abs(a[23, 23, 23] - b[23, 23, 23]) <= 1e-12 / r
    assert abs(a[0, 0, 0] - b[0, 0, 0]) > 1e-6


def test_orders_served():
    with pytest.raises(ValueError):
        isf.coulomb_integrals(6, (4, 4, 4))
    with pytest.raises(ValueError):
        isf.coulomb_integrals(9, (4, 4, 4))


def _gaussian_case(n, sigma_h):
    x = np.arange(n) * H
    c = (n - 1) / 2 * H
    r = np.sqrt((x[None, None, :] - c) ** 2 + (x[None, :, None] - c) ** 2
                + (x[:, None, None] - c) ** 2)
    s = sigma_h * H
    rho = np.exp(-r ** 2 / (2 * s * s)) / (2 * math.pi * s * s) ** 1.5
    V = -special.erf(r / (math.sqrt(2) * s)) / (4 * math.pi * r)
    return rho, V


def test_gaussian_potential_converges_at_high_order():
    """The ISF kernel solves a Gaussian charge far more accurately than the
    sampled kernel with the fourth-order origin weight, and its error falls
    fast with sigma/h (the interpolation order, not the origin correction,
    sets the rate)."""
    n = 32
    kf_isf = isf.isf_kernel_fourier((n, n, n), H, 16)
    kf_def = oracle.kernel_fourier((n, n, n), 7, H)
    errs = {}
    for sig in (1.0, 2.0):
        rho, V = _gaussian_case(n, sig)
        e_isf = np.max(np.abs(oracle.solve(rho, 7, H, kf=kf_isf) - V)) / np.max(np.abs(V))
        e_def = np.max(np.abs(oracle.solve(rho, 7, H, kf=kf_def) - V)) / np.max(np.abs(V))
        errs[sig] = (e_isf, e_def)
        assert e_isf * 10 <= e_def, (sig, e_isf, e_def)
    assert errs[2.0][0] <= 1e-6
    assert errs[1.0][0] / errs[2.0][0] >= 2 ** 7


def test_isf_kernel_fourier_is_real_even_and_octant_consistent():
    n = (12, 8, 10)
    kf = isf.isf_kernel_fourier(n, H, 16)
    assert kf.shape == (20, 16, 24)
    # even in every axis: kf[k] = kf[S - k]
    for axis in range(3):
        S = kf.shape[axis]
        idx = (-np.arange(S)) % S
        assert np.allclose(kf, np.take(kf, idx, axis=axis), rtol=0, atol=1e-12 * np.abs(kf).max())
    octant = isf.isf_kernel_octant(n, H, 16, kf=kf)
    assert octant.shape == (11, 9, 13)
    # the half-spectrum route gives the same octant
    half = isf.isf_kernel_fourier(n, H, 16, half=True)
    assert half.shape == (20, 16, 13)
    assert np.allclose(isf.isf_kernel_octant(n, H, 16), octant, rtol=0,
                       atol=1e-13 * np.abs(octant).max())
    # k = 0 is the sum of the padded real-space kernel
    K = isf.isf_kernel_real(n, H, 16)
    w = [np.where((np.arange(o) == 0) | (np.arange(o) == o - 1), 1.0, 2.0) for o in K.shape]
    total = np.einsum("cba,c,b,a->", K, w[0], w[1], w[2])
    assert abs(octant[0, 0, 0] - total) <= 1e-12 * abs(total)


# ------------------------------------------------------------ mixed BCs
import sys as _sys
_sys.path.insert(0, __import__("os").path.dirname(__file__))
from closed_forms import (gaussian1, grid_axes, line_potential_kappa,  # noqa: E402
                          line_potential_kappa0, mesh, sheet_potential)


def _surface_case(N, a, kernel):
    h = H * 32 / N
    n = (N, N, N)
    x, y, z = grid_axes(n, h)
    L = N * h
    k = 2 * math.pi * a / L
    rho = np.cos(k * x)[None, None, :] * gaussian1(y, 0.5 * L, 0.9)[None, :, None] * np.ones((N, 1, 1))
    want = (np.cos(k * x)[None, None, :] * sheet_potential(y, 0.5 * L, 0.9, k)[None, :, None]
            * np.ones((N, 1, 1)))
    kf = isf.isf_mixed_kernel_fourier(n, 2, h, 16, half=True) if kernel == "isf" else None
    return oracle.rel_l2(oracle.solve(rho, 2, h, kf=kf), want)


def _wire_case(N, mode, kernel):
    h = H * 32 / N
    n = (N, N, N)
    X, Y, Z = mesh(n, h)
    L = N * h
    r = np.sqrt((X - L / 2) ** 2 + (Y - L / 2) ** 2)
    g2 = np.exp(-r ** 2 / (2 * 0.81)) / (2 * math.pi * 0.81)
    if mode == 0:
        rho, want = g2, line_potential_kappa0(r, 0.9)
    else:
        k = 2 * math.pi * mode / L
        rho = np.cos(k * Z) * g2
        want = np.cos(k * Z) * line_potential_kappa(r[0], 0.9, k)[None]
    kf = isf.isf_mixed_kernel_fourier(n, 3, h, 16, half=True) if kernel == "isf" else None
    return oracle.rel_l2(oracle.solve(rho, 3, h, kf=kf), want)


@pytest.mark.parametrize("a", [0, 1, 5])
def test_isf_surface_sheet_potential(a):
    """Surface BCs (y free): cos(2 pi a x/L) g(y) against the closed form.
    The ISF kernel stays at the 1e-7 level up to the high mode a = 5 (kappa h
    = 0.98), where the sampled kernel's small-kappa h origin weight leaves
    about 1e-3."""
    e16, e32 = _surface_case(16, a, "isf"), _surface_case(32, a, "isf")
    assert e32 <= 4e-7, (a, e32)
    assert e16 / e32 >= 4, (a, e16, e32)
    assert _surface_case(32, a, "sampled") >= 10 * e32


@pytest.mark.parametrize("mode", [0, 1, 4])
def test_isf_wire_line_potential(mode):
    """Wire BCs (z periodic): a Gaussian line charge, uniform (kappa = 0) or
    cos-modulated up to kappa h = 0.79, against the radial closed forms."""
    e16, e32 = _wire_case(16, mode, "isf"), _wire_case(32, mode, "isf")
    assert e32 <= 4e-7, (mode, e32)
    assert e16 / e32 >= 4, (mode, e16, e32)
    assert _wire_case(32, mode, "sampled") >= 10 * e32


def test_isf_surface_kappa0_far_field_exact():
    """|y|/2 against phi: int phi(u) |n - u| du = |n| exactly once the
    support of phi lies on one side of n (phi's first moment vanishes)."""
    nodes = isf._mixed_nodes(16, 40)
    K = isf._free_kernel_1d(16, 0.0, 40, nodes)
    n = np.arange(41)
    far = n >= 15
    assert np.max(np.abs(K[far] - 0.5 * n[far]) / (0.5 * n[far])) <= 1e-13
    # and the kappa > 0 kernel tends to the sampled -exp(-kappa h n)/(2 kappa h)
    kh = 0.05
    Kk = isf._free_kernel_1d(16, kh, 40, nodes)
    want = -np.exp(-kh * n) / (2 * kh)
    assert np.max(np.abs(Kk[far] - want[far]) / np.abs(want[far])) <= 1e-12


def test_isf_wire_kappa0_far_field():
    nodes = isf._mixed_nodes(16, 40)
    K = isf._free_kernel_2d(16, 0.0, 40, 40, H, nodes)
    for i, j in ((40, 0), (30, 30), (25, 36)):
        r = math.hypot(i, j)
        want = (math.log(H) + math.log(r)) / (2 * math.pi)
        assert abs(K[j, i] - want) <= 1e-12 * abs(want), (i, j)


@pytest.mark.parametrize("bc", [2, 3, 5])
def test_isf_mixed_quadrature_split_points(bc):
    """Moving the lower end of the panels, raising the cut-off or halving
    the panels leaves the mixed K^F unchanged to rounding."""
    n = (8, 12, 6)
    base = isf.isf_mixed_kernel_fourier(n, bc, H, 16)
    scale = np.abs(base).max()
    for attr, val in (("MIXED_TAU_LO", 1e-11), ("T_MAX", 16384.0), ("PANEL", 0.5)):
        old = getattr(isf, attr)
        setattr(isf, attr, val)
        try:
            other = isf.isf_mixed_kernel_fourier(n, bc, H, 16)
        finally:
            setattr(isf, attr, old)
        assert np.max(np.abs(other - base)) <= 1e-12 * scale, attr


def test_isf_mixed_rejects_free_and_periodic():
    with pytest.raises(ValueError):
        isf.isf_mixed_kernel_fourier((8, 8, 8), 7, H)
    with pytest.raises(ValueError):
        isf.isf_mixed_kernel_fourier((8, 8, 8), 0, H)
