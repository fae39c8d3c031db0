"""Closed-form potentials that pin the oracle's Green's functions.

Each function returns the exact continuum solution of lap V = rho (paper,
Eq. 1) for a density whose discrete samples the tests feed to the oracle.
They are derived from the mathematics, not from the oracle's code: the
oracle is checked against them, never the reverse.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special


def grid_axes(n, h):
    """Coordinates x_i = i h along each axis, as (x, y, z) 1-D arrays."""
    return [np.arange(ni) * h for ni in n]


def mesh(n, h):
    x, y, z = grid_axes(n, h)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def gaussian3(n, h, center, sigma, q=1.0):
    X, Y, Z = mesh(n, h)
    r2 = (X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2
    return q * (2 * math.pi * sigma ** 2) ** -1.5 * np.exp(-r2 / (2 * sigma ** 2))


def gaussian3_potential(n, h, center, sigma, q=1.0):
    """Free space: V = -q erf(r / (sqrt(2) sigma)) / (4 pi r)."""
    X, Y, Z = mesh(n, h)
    r = np.sqrt((X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2)
    safe = np.where(r == 0, 1.0, r)
    v = -q * special.erf(safe / (math.sqrt(2) * sigma)) / (4 * math.pi * safe)
    v0 = -q * math.sqrt(2.0 / math.pi) / (4 * math.pi * sigma)
    return np.where(r == 0, v0, v)


def cosine_mode(n, h, freqs):
    """rho = prod_j cos(2 pi a_j x_j / L_j) on a periodic box; returns
    (rho, V) with V = -rho / |k|^2."""
    X, Y, Z = mesh(n, h)
    L = [ni * h for ni in n]
    k = [2 * math.pi * a / Lj for a, Lj in zip(freqs, L)]
    rho = np.cos(k[0] * X) * np.cos(k[1] * Y) * np.cos(k[2] * Z)
    return rho, -rho / (k[0] ** 2 + k[1] ** 2 + k[2] ** 2)


def gaussian1(y, c, sigma):
    return np.exp(-((y - c) ** 2) / (2 * sigma ** 2)) / (math.sqrt(2 * math.pi) * sigma)


def sheet_potential(y, c, sigma, kappa):
    """Solution of u'' - kappa^2 u = g for the unit 1-D Gaussian g(y - c),
    decaying (kappa > 0) or the |y|/2 convolution (kappa = 0)."""
    s = y - c
    if kappa == 0.0:
        return 0.5 * (s * special.erf(s / (math.sqrt(2) * sigma))
                      + sigma * math.sqrt(2 / math.pi) * np.exp(-s * s / (2 * sigma ** 2)))
    # -(1/(4 kappa)) exp(kappa^2 sigma^2 / 2) [e^{-kappa s} erfc((kappa sigma^2 - s)/(sqrt2 sigma))
    #                                          + e^{kappa s} erfc((kappa sigma^2 + s)/(sqrt2 sigma))]
    a = kappa * sigma ** 2
    b = math.sqrt(2) * sigma
    # combine exponentials in log space to stay finite
    t1 = np.exp(0.5 * kappa ** 2 * sigma ** 2 - kappa * s) * special.erfc((a - s) / b)
    t2 = np.exp(0.5 * kappa ** 2 * sigma ** 2 + kappa * s) * special.erfc((a + s) / b)
    return -(t1 + t2) / (4 * kappa)


def line_potential_kappa0(r, sigma, q=1.0):
    """2-D Gaussian line charge q (2 pi sigma^2)^-1 exp(-r^2 / 2 sigma^2):
    V = (q / 2 pi) [ln r + E1(r^2 / 2 sigma^2) / 2]."""
    safe = np.where(r == 0, 1.0, r)
    v = (q / (2 * math.pi)) * (np.log(safe) + 0.5 * special.exp1(safe ** 2 / (2 * sigma ** 2)))
    # r -> 0: ln r + E1(r^2/2s^2)/2 -> (ln(2 s^2) - gamma)/2
    v0 = (q / (2 * math.pi)) * 0.5 * (math.log(2 * sigma ** 2) - np.euler_gamma)
    return np.where(r == 0, v0, v)


def epstein_cubic_half():
    """Analytic continuation of sum_{m in Z^3, m != 0} 1/|m| by Ewald
    splitting with alpha = sqrt(pi) (unit cell volume 1):
    Z = sum' erfc(sqrt(pi)|m|)/|m| + sum' exp(-pi |k|^2)/(pi |k|^2) - 2 - 1,
    where the -2 removes the self term 2 alpha / sqrt(pi) and the -1 is the
    neutralizing k = 0 term pi / alpha^2."""
    R = 6
    m = np.arange(-R, R + 1)
    M1, M2, M3 = np.meshgrid(m, m, m, indexing="ij")
    r = np.sqrt(M1 ** 2 + M2 ** 2 + M3 ** 2).astype(float)
    mask = r > 0
    real = np.sum(special.erfc(math.sqrt(math.pi) * r[mask]) / r[mask])
    recip = np.sum(np.exp(-math.pi * r[mask] ** 2) / (math.pi * r[mask] ** 2))
    return real + recip - 2.0 - 1.0


def line_potential_kappa(r_values, sigma, kappa, q=1.0):
    """Radial solution of (lap_2 - kappa^2) u = q g(r) for the 2-D Gaussian
    g = (2 pi sigma^2)^-1 exp(-r^2 / 2 sigma^2), kappa > 0, by the radial
    Green's function of the modified Helmholtz operator:
    u(r) = -[K0(kappa r) int_0^r I0(kappa s) g(s) s ds
             + I0(kappa r) int_r^inf K0(kappa s) g(s) s ds],
    integrated with adaptive quadrature (scaled Bessel functions keep the
    products finite)."""
    from scipy import integrate

    def g(s):
        return q * math.exp(-s * s / (2 * sigma ** 2)) / (2 * math.pi * sigma ** 2)

    out = {}
    upper = 12.0 * sigma
    for r in np.unique(np.asarray(r_values).ravel()):
        r = float(r)
        if r == 0.0:
            inner = 0.0
            outer = integrate.quad(lambda s: special.k0(kappa * s) * g(s) * s, 0.0, upper,
                                   epsabs=0, epsrel=1e-13, limit=400)[0]
            out[r] = -outer
            continue
        # K0(kr) I0(ks) = k0e(kr) i0e(ks) exp(k(s - r)) for s <= r
        inner = integrate.quad(
            lambda s: special.k0e(kappa * r) * special.i0e(kappa * s)
            * math.exp(kappa * (s - r)) * g(s) * s, 0.0, r,
            epsabs=0, epsrel=1e-13, limit=400)[0]
        outer = 0.0
        if r < upper:
            outer = integrate.quad(
                lambda s: special.i0e(kappa * r) * special.k0e(kappa * s)
                * math.exp(kappa * (r - s)) * g(s) * s, r, upper,
                epsabs=0, epsrel=1e-13, limit=400)[0]
        out[r] = -(inner + outer)
    return np.vectorize(lambda x: out[float(x)])(r_values)
