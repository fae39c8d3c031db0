"""Gaussian-mixture charge densities on a uniform grid.

The paper benchmarks its solver on synthetic grids of various sizes and
boundary conditions (Section 4) without fixing a density.  The densities here
are smooth, localized Gaussian clouds, the kind of input an electronic
structure code hands to its Poisson solver (Section 1).

Grid convention: point (i1, i2, i3) sits at r = (i1, i2, i3) * h; arrays are
shaped (n3, n2, n1), so axis x (index i1) is the fastest-varying one.
bc_mask bit j set means axis j has free boundary conditions; a clear bit means
periodic.  Along periodic axes every Gaussian is summed over its images
shifted by -2L..2L so the density is periodic; a fully periodic density has
its mean removed (a periodic Poisson problem needs a neutral cell).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class GaussianSpec:
    center: tuple  # (cx, cy, cz) in length units
    sigma: float   # width in length units
    charge: float  # total charge of the cloud


def draw_gaussians(n, h, count, sigma_range, seed):
    """Draw `count` Gaussians with numpy's PCG64 stream `default_rng(seed)`.

    Per Gaussian, in this order: three center coordinates uniform in
    [0.25 L_i, 0.75 L_i] (L_i = n_i h), the width uniform in
    [sigma_range[0], sigma_range[1]] grid spacings, the charge uniform in
    [-1, 1].
    """
    rng = np.random.default_rng(seed)
    lengths = [ni * h for ni in n]
    out = []
    for _ in range(count):
        c = tuple(float(rng.uniform(0.25 * L, 0.75 * L)) for L in lengths)
        s = float(rng.uniform(sigma_range[0], sigma_range[1])) * h
        q = float(rng.uniform(-1.0, 1.0))
        out.append(GaussianSpec(c, s, q))
    return out


def _axis_factor(ni, h, c, sigma, periodic):
    x = np.arange(ni, dtype=np.float64) * h
    if not periodic:
        return np.exp(-((x - c) ** 2) / (2.0 * sigma * sigma))
    L = ni * h
    f = np.zeros(ni)
    for j in range(-2, 3):
        f += np.exp(-((x - c - j * L) ** 2) / (2.0 * sigma * sigma))
    return f


def gaussian_mixture(n, bc_mask, h, gaussians):
    """Evaluate the mixture on the (n3, n2, n1) grid in float64."""
    n1, n2, n3 = n
    per = [not (bc_mask >> j) & 1 for j in range(3)]
    fx = np.stack([_axis_factor(n1, h, g.center[0], g.sigma, per[0]) for g in gaussians])
    fy = np.stack([_axis_factor(n2, h, g.center[1], g.sigma, per[1]) for g in gaussians])
    fz = np.stack([_axis_factor(n3, h, g.center[2], g.sigma, per[2]) for g in gaussians])
    amp = np.array([g.charge * (2.0 * math.pi * g.sigma ** 2) ** -1.5 for g in gaussians])
    # rho[z, y, x] = sum_g amp_g fz[g, z] fy[g, y] fx[g, x]
    zy = np.einsum("g,gz,gy->zyg", amp, fz, fy).reshape(n3 * n2, len(gaussians))
    rho = (zy @ fx).reshape(n3, n2, n1)
    if bc_mask & 7 == 0:
        rho -= rho.mean()
    return rho


# Named synthetic workloads.  Each entry fixes grid, boundary conditions,
# spacing and the Gaussian recipe; `seed` seeds the Gaussian draw.
BC_FREE, BC_WIRE_Z, BC_SURFACE_Y, BC_PERIODIC = 7, 3, 2, 0

WORKLOADS = {
    # fully free 32^3 (padded 64^3): small enough for the CPU oracle in seconds
    "free32": dict(n=(32, 32, 32), bc=BC_FREE, gaussians=3, sigma=(1.5, 3.0), seed=1),
    # 128^3, one entry per boundary-condition class
    "free128": dict(n=(128, 128, 128), bc=BC_FREE, gaussians=8, sigma=(1.0, 6.0), seed=2),
    "wire128": dict(n=(128, 128, 128), bc=BC_WIRE_Z, gaussians=8, sigma=(1.0, 6.0), seed=2),
    "surface128": dict(n=(128, 128, 128), bc=BC_SURFACE_Y, gaussians=8, sigma=(1.0, 6.0), seed=2),
    "periodic128": dict(n=(128, 128, 128), bc=BC_PERIODIC, gaussians=8, sigma=(1.0, 6.0), seed=2),
    # fully free 256^3 (padded 512^3): the throughput workload
    "free256": dict(n=(256, 256, 256), bc=BC_FREE, gaussians=32, sigma=(1.0, 6.0), seed=3),
    # mixed BCs with non-cubic grids and a factor 3 in the FFT lengths
    "wire192x192x384": dict(n=(192, 192, 384), bc=BC_WIRE_Z, gaussians=64, sigma=(1.0, 6.0), seed=4),
    "surface384x192x384": dict(n=(384, 192, 384), bc=BC_SURFACE_Y, gaussians=64, sigma=(1.0, 6.0), seed=4),
}

SPACING = 0.3


def workload_density(name, h=SPACING):
    """Return (n, bc_mask, rho_float64) for a named workload."""
    w = WORKLOADS[name]
    gs = draw_gaussians(w["n"], h, w["gaussians"], w["sigma"], w["seed"])
    return w["n"], w["bc"], gaussian_mixture(w["n"], w["bc"], h, gs)


BATCH_EDGES = (32, 48, 64, 96, 128)
BATCH_BCS = (BC_FREE, BC_WIRE_Z, BC_SURFACE_Y, BC_PERIODIC)


def batch_workload(count=512, composition_seed=4999, h=SPACING):
    """Mixed batch of cubic solves: edge uniform over BATCH_EDGES, boundary
    conditions uniform over the four classes, 4 Gaussians with widths in
    [1.5, 3] spacings; density i is seeded with 5000 + i.

    Returns a list of (n, bc_mask, seed)."""
    rng = np.random.default_rng(composition_seed)
    edges = rng.integers(0, len(BATCH_EDGES), size=count)
    bcs = rng.integers(0, len(BATCH_BCS), size=count)
    out = []
    for i in range(count):
        e = BATCH_EDGES[int(edges[i])]
        out.append(((e, e, e), BATCH_BCS[int(bcs[i])], 5000 + i))
    return out


def batch_density(n, bc_mask, seed, h=SPACING):
    gs = draw_gaussians(n, h, 4, (1.5, 3.0), seed)
    return gaussian_mixture(n, bc_mask, h, gs)
