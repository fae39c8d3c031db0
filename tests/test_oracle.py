"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes
from brute force on tiny grids, a closed-form potential, a lattice constant
computed by Ewald summation, a library routine for a special case, or an
invariant of the convolution (paper, Section 2, Eqs. 1-3).
"""

import math

import numpy as np
import pytest

import oracle
from closed_forms import (cosine_mode, epstein_cubic_half, gaussian1, gaussian3,
                          gaussian3_potential, grid_axes, line_potential_kappa,
                          line_potential_kappa0, mesh, sheet_potential)

H = 0.3
ALL_MASKS = list(range(8))


def _rand_rho(n, bc, seed):
    rng = np.random.default_rng(seed)
    rho = rng.standard_normal((n[2], n[1], n[0]))
    if bc == 0:
        rho -= rho.mean()
    return rho


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("bc", ALL_MASKS)
@pytest.mark.parametrize("n", [(6, 8, 12), (5, 3, 4), (16, 16, 16)])
def test_solve_equals_direct_sum(n, bc):
    """Eq. 2 evaluated term by term equals the padded-FFT solve (Eq. 3 with
    zero padding on free axes) on small non-cubic grids, odd sizes included."""
    rho = _rand_rho(n, bc, 10 * bc + n[0])
    V = oracle.solve(rho, bc, H)
    B = oracle.brute_force(rho, bc, H)
    assert oracle.rel_l2(V, B) < 1e-12


def test_direct_sum_free_32cube():
    """The small fully free workload (32^3, about 1e9 pair terms)."""
    from densities import workload_density
    n, bc, rho = workload_density("free32")
    rho = rho.astype(np.float32).astype(np.float64)
    V = oracle.solve(rho, bc, H)
    B = oracle.brute_force(rho, bc, H)
    assert oracle.rel_l2(V, B) < 1e-12


def test_free_kernel_is_plain_coulomb_sum():
    """For free BCs the direct sum uses the sampled -h^2/(4 pi |m|) with no
    spectral step at all: check the kernel values themselves."""
    n = (4, 5, 6)
    K = oracle.real_space_kernel(n, 7, H)
    S = oracle.padded_shape(n, 7)
    for (a, b, c) in [(1, 0, 0), (0, 2, 0), (0, 0, 3), (1, 2, 3), (3, 9, 11), (4, 5, 6)]:
        m = (min(a, S[0] - a), min(b, S[1] - b), min(c, S[2] - c))
        want = -H * H / (4 * math.pi * math.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2))
        assert K[c, b, a] == pytest.approx(want, rel=1e-14)
    assert K[0, 0, 0] == pytest.approx(-(H * H / (4 * math.pi)) * 2.837297479480619, rel=1e-14)


# ------------------------------------------------------------- lattice constants
def test_coulomb_origin_constant_is_ewald_value():
    """c3 is minus the Epstein zeta value of the cubic lattice (Ewald sum)."""
    assert epstein_cubic_half() == pytest.approx(-oracle.C3_COULOMB_ORIGIN, abs=1e-12)


def test_log_origin_constant():
    """c2 = ln(2 sqrt(pi) / Gamma(1/4)^2), from the gamma function."""
    from scipy.special import gamma
    assert oracle.C2_LOG_ORIGIN == pytest.approx(
        math.log(2 * math.sqrt(math.pi) / gamma(0.25) ** 2), abs=1e-14)


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,freqs", [((16, 16, 16), (1, 2, 3)), ((12, 8, 24), (2, 1, 5)),
                                     ((8, 6, 10), (4, 3, 5))])
def test_periodic_cosine_mode_is_exact(n, freqs):
    """Spectral periodic kernel: V^F = -rho^F/|k|^2 exactly, Nyquist modes included."""
    rho, want = cosine_mode(n, H, freqs)
    V = oracle.solve(rho, 0, H)
    assert np.max(np.abs(V - want)) < 1e-13 * np.max(np.abs(want))


def _free_gauss_err(N, n_shape=None):
    h = H * 32 / N
    n = n_shape or (N, N, N)
    L = [ni * h for ni in n]
    c = (L[0] / 2, L[1] / 2, L[2] / 2)
    rho = gaussian3(n, h, c, 0.9)
    return oracle.rel_l2(oracle.solve(rho, 7, h), gaussian3_potential(n, h, c, 0.9))


def test_free_gaussian_potential_fourth_order():
    """Free BCs reproduce the potential -erf(r/sqrt2 s)/(4 pi r) of a Gaussian
    with error O(h^4): a dropped origin constant gives O(h^2)."""
    e16, e32 = _free_gauss_err(16), _free_gauss_err(32)
    assert e32 < 3e-5
    assert math.log2(e16 / e32) > 3.7


def test_free_gaussian_noncubic_off_center():
    h = 0.3
    # the box keeps every center >= 5.5 sigma from the faces, so the cut-off
    # tails of the Gaussian stay below the discretization error
    n = (36, 40, 44)
    c = (0.48 * 36 * h, 0.53 * 40 * h, 0.5 * 44 * h + 0.11)
    rho = gaussian3(n, h, c, 0.9, q=-0.7)
    err = oracle.rel_l2(oracle.solve(rho, 7, h), gaussian3_potential(n, h, c, 0.9, q=-0.7))
    assert err < 3e-5


def _surface_err(N, a, n_other=(None, None)):
    h = H * 32 / N
    n = (N, N, N)
    x, y, z = grid_axes(n, h)
    L = N * h
    k = 2 * math.pi * a / L
    prof = gaussian1(y, 0.5 * L, 0.9)
    rho = np.cos(k * x)[None, None, :] * prof[None, :, None] * np.ones((N, 1, 1))
    want = np.cos(k * x)[None, None, :] * sheet_potential(y, 0.5 * L, 0.9, k)[None, :, None] * np.ones((N, 1, 1))
    return oracle.rel_l2(oracle.solve(rho, 2, h), want)


@pytest.mark.parametrize("a", [0, 1])
def test_surface_sheet_potential_fourth_order(a):
    """Surface BCs (y free): rho = cos(2 pi a x/L) g(y) gives cos(..) u(y) with
    u the 1-D modified-Helmholtz (a > 0) or |y|/2 (a = 0) convolution."""
    e16, e32 = _surface_err(16, a), _surface_err(32, a)
    assert e32 < 3e-5
    assert math.log2(e16 / e32) > 3.7


def test_surface_free_axis_x_noncubic():
    """Free axis x, periodic y and z, non-cubic: pins the axis bookkeeping.
    (The origin weight is a small-kappa h expansion, so the mode is kept at
    kappa h = 0.26; at kappa h ~ 1 the error grows to ~1e-3.)"""
    h = 0.3
    n = (40, 24, 8)
    x, y, z = grid_axes(n, h)
    Ly = n[1] * h
    k = 2 * math.pi * 1 / Ly
    prof = gaussian1(x, 0.5 * n[0] * h, 1.2)
    rho = np.cos(k * y)[None, :, None] * prof[None, None, :] * np.ones((n[2], 1, 1))
    want = (np.cos(k * y)[None, :, None] * sheet_potential(x, 0.5 * n[0] * h, 1.2, k)[None, None, :]
            * np.ones((n[2], 1, 1)))
    assert oracle.rel_l2(oracle.solve(rho, 1, h), want) < 3e-5


def _wire_err(N, kappa_mode):
    h = H * 32 / N
    n = (N, N, N)
    X, Y, Z = mesh(n, h)
    L = N * h
    c = L / 2
    r = np.sqrt((X - c) ** 2 + (Y - c) ** 2)
    g2 = np.exp(-r ** 2 / (2 * 0.81)) / (2 * math.pi * 0.81)
    if kappa_mode == 0:
        want = line_potential_kappa0(r, 0.9)
        rho = g2
    else:
        k = 2 * math.pi * kappa_mode / L
        rho = np.cos(k * Z) * g2
        want = np.cos(k * Z) * line_potential_kappa(r[0], 0.9, k)[None]
    return oracle.rel_l2(oracle.solve(rho, 3, h), want)


@pytest.mark.parametrize("mode", [0, 1])
def test_wire_line_potential_fourth_order(mode):
    """Wire BCs (z periodic): a Gaussian line charge, uniform (kappa = 0,
    ln r + E1/2) or cos-modulated (kappa > 0, K0/I0 radial integral)."""
    e16, e32 = _wire_err(16, mode), _wire_err(32, mode)
    assert e32 < 6e-5
    assert math.log2(e16 / e32) > 3.7


# ------------------------------------------------------------ special cases
@pytest.mark.parametrize("n", [(8, 12, 6), (16, 16, 16)])
def test_periodic_equals_textbook_spectral_solve(n):
    rho = _rand_rho(n, 0, 3)
    F = np.fft.fftn(rho)
    k2 = 0
    for j, ax in ((0, 2), (1, 1), (2, 0)):
        kj = 2 * np.pi * np.fft.fftfreq(n[j], d=H)
        shape = [1, 1, 1]
        shape[ax] = n[j]
        k2 = k2 + kj.reshape(shape) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        Vf = np.where(k2 > 0, -F / k2, 0)
    want = np.fft.ifftn(Vf).real
    assert oracle.rel_l2(oracle.solve(rho, 0, H), want) < 1e-13


def test_free_axis_profile_is_linear_convolution():
    """A density varying only along a free x axis (y, z periodic) is the
    kappa = 0 mode: V is np.convolve with the kernel h^2|m|/2, origin h^2/12."""
    n = (20, 4, 6)
    rng = np.random.default_rng(7)
    prof = rng.standard_normal(n[0])
    rho = np.broadcast_to(prof[None, None, :], (n[2], n[1], n[0]))
    m = np.arange(-(n[0] - 1), n[0])
    k = H * H * np.abs(m) / 2.0
    k[n[0] - 1] = H * H / 12.0
    want = np.convolve(prof, k)[n[0] - 1: 2 * n[0] - 1]
    V = oracle.solve(rho, 1, H)
    assert np.max(np.abs(V - want[None, None, :])) < 1e-12 * np.max(np.abs(want))


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("bc", ALL_MASKS)
def test_linearity_and_self_adjointness(bc):
    n = (8, 6, 10)
    r1, r2 = _rand_rho(n, bc, 1), _rand_rho(n, bc, 2)
    V1, V2 = oracle.solve(r1, bc, H), oracle.solve(r2, bc, H)
    V12 = oracle.solve(2.5 * r1 - 0.5 * r2, bc, H)
    assert oracle.rel_l2(V12, 2.5 * V1 - 0.5 * V2) < 1e-13
    a, b = np.vdot(r1, V2), np.vdot(r2, V1)
    assert abs(a - b) < 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("bc", ALL_MASKS)
def test_mirror_symmetry(bc):
    """K is even in every axis: mirroring the density mirrors the potential
    (periodic axes mirror as i -> -i mod N, free axes as i -> N-1-i)."""
    n = (8, 6, 10)
    rho = _rand_rho(n, bc, 11)
    V = oracle.solve(rho, bc, H)
    for j in range(3):
        ax = 2 - j
        if (bc >> j) & 1:
            flip = lambda a: np.flip(a, axis=ax)  # noqa: E731
        else:
            flip = lambda a: np.roll(np.flip(a, axis=ax), 1, axis=ax)  # noqa: E731
        assert oracle.rel_l2(oracle.solve(flip(rho), bc, H), flip(V)) < 1e-12


@pytest.mark.parametrize("bc", ALL_MASKS)
def test_translation(bc):
    """Rolling along a periodic axis commutes with the solve; on a free axis
    a density supported away from the end shifts with its potential."""
    n = (10, 8, 12)
    rho = _rand_rho(n, bc, 5)
    for j in range(3):
        ax = 2 - j
        if (bc >> j) & 1:
            sl = [slice(None)] * 3
            sl[ax] = slice(n[j] - 3, None)
            r = rho.copy()
            r[tuple(sl)] = 0.0
            if bc == 0:
                r -= r.mean()
            V = oracle.solve(r, bc, H)
            Vs = oracle.solve(np.roll(r, 3, axis=ax), bc, H)
            keep = [slice(None)] * 3
            keep[ax] = slice(3, None)
            keep0 = [slice(None)] * 3
            keep0[ax] = slice(0, n[j] - 3)
            assert oracle.rel_l2(Vs[tuple(keep)], V[tuple(keep0)]) < 1e-12
        else:
            V = oracle.solve(rho, bc, H)
            Vs = oracle.solve(np.roll(rho, 3, axis=ax), bc, H)
            assert oracle.rel_l2(Vs, np.roll(V, 3, axis=ax)) < 1e-12


# ------------------------------------------------------------------ the octant
@pytest.mark.parametrize("bc", ALL_MASKS)
def test_kernel_is_real_even_and_octant_complete(bc):
    n = (6, 5, 4)
    kf = oracle.kernel_fourier(n, bc, H)
    S = oracle.padded_shape(n, bc)
    for ax, Sj in ((2, S[0]), (1, S[1]), (0, S[2])):
        idx = (-np.arange(Sj)) % Sj
        scale = np.max(np.abs(kf))
        assert np.max(np.abs(np.take(kf, idx, axis=ax) - kf)) < 1e-14 * scale
    oct_ = oracle.kernel_octant(n, bc, H, kf)
    assert oct_.shape == (S[2] // 2 + 1, S[1] // 2 + 1, S[0] // 2 + 1)
    # rebuild the full grid from the octant by folding k -> min(k, S - k)
    f = [np.minimum(np.arange(Sj), Sj - np.arange(Sj)) for Sj in S]
    full = oct_[f[2][:, None, None], f[1][None, :, None], f[0][None, None, :]]
    assert np.max(np.abs(full - kf)) < 1e-14 * np.max(np.abs(kf))
