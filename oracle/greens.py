"""Green's-function kernels of the discrete Poisson convolution, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper writes the solution as a convolution of the density with a Green's
function K (Section 2, Eq. 2) that becomes a pointwise product in Fourier
space (Eq. 3); free axes are zero padded to twice their length so the
circular convolution of the FFT does not wrap around (Section 2), giving FFT
lengths S_j = N_j B_j with B_j = 1 (periodic) or 2 (free) (Section 3).  Which
Green's function goes with each mix of boundary conditions is only cited, not
written out (Section 2 cites the free-space and the surface/wire kernels).
This module fixes one reading, and every test pins it against closed-form
potentials:

* Poisson's equation is taken literally as lap V = rho (Eq. 1), so the
  free-space Green's function is G(r) = -1/(4 pi r) and the periodic kernel is
  -1/|k|^2.
* Periodic axes are handled spectrally: for wave numbers k_j = 2 pi f_j / L_j
  (signed integer frequency f_j, L_j = S_j h) put kappa^2 = sum of k_j^2 over
  the periodic axes.  Along the d free axes the kernel is then the Green's
  function of (lap_d - kappa^2) in d dimensions, sampled on the grid and
  multiplied by the cell volume h^d:

    d = 0 (periodic): K^F = -1/kappa^2, and K^F = 0 for the k = 0 mode.
    d = 1 (surface):  G = -exp(-kappa r)/(2 kappa);  kappa = 0: G = r/2.
    d = 2 (wire):     G = -K0(kappa r)/(2 pi);       kappa = 0: G = ln(r)/(2 pi).
    d = 3 (free):     G = -1/(4 pi r).

* The singular (or kinked) origin sample gets the weight that makes the
  trapezoidal rule accurate to O(h^4) for smooth densities:
    d = 1: h G(0) + h^2/12 (the derivative jump of |y|/2 is 1, and the
           Euler-Maclaurin correction for a kink at a node is h^2/12 times it);
    d = 2: (h^2 / 2 pi) (ln(kappa h / 2) + gamma + c2), kappa = 0:
           (h^2 / 2 pi) (ln h + c2), with c2 = ln(2 sqrt(pi) / Gamma(1/4)^2);
    d = 3: -(h^2 / 4 pi) c3, with c3 = 2.837297479480619, minus the value of
           the simple-cubic lattice sum of 1/|m| continued analytically (the
           corrected trapezoidal rule for a 1/r singularity).
* The padded kernel is even in every axis; on a free axis the offset of
  index m is min(m, S - m), so the sample at m = S/2 = N is G(N h) (it never
  reaches the cropped output, since |i - j| <= N - 1 there).
* K^F = DFT over the free axes of that mixed (real space on free axes,
  Fourier on periodic axes) array, unnormalized; the inverse transform of the
  solve carries 1/prod(S).  K^F is real and even, so its unique part is the
  octant 0 <= k_j <= S_j/2.

Arrays are shaped (S3, S2, S1): axis x (index 1 in the paper's notation) is
the last, fastest array axis.
"""

from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft
from scipy import special

EULER_GAMMA = 0.57721566490153286061
# ln(2 sqrt(pi) / Gamma(1/4)^2): origin constant of the 2-D logarithmic kernel
C2_LOG_ORIGIN = math.log(2.0) + 0.5 * math.log(math.pi) - 2.0 * math.lgamma(0.25)
# minus the analytically continued lattice sum of 1/|m| over Z^3 \ {0}
C3_COULOMB_ORIGIN = 2.837297479480619


def padded_shape(n, bc_mask):
    """FFT lengths S_j = N_j B_j, B_j = 2 on free axes (Section 3)."""
    return tuple(int(n[j]) * (2 if (bc_mask >> j) & 1 else 1) for j in range(3))


def _axis_view(j, values):
    # axis j of the problem (0 = x) is array axis 2 - j
    shape = [1, 1, 1]
    shape[2 - j] = values.shape[0]
    return values.reshape(shape)


def _free_offsets(S):
    m = np.arange(S, dtype=np.float64)
    return np.minimum(m, S - m)


def _wavenumbers(S, h):
    f = np.fft.fftfreq(S, d=1.0 / S)  # signed integer frequencies
    return 2.0 * math.pi * f / (S * h)


def mixed_kernel(n, bc_mask, h):
    """Kernel in the mixed representation on the padded grid (S3, S2, S1):
    real-space samples times h^d along free axes, Fourier along periodic
    axes.  For fully periodic BCs this already is K^F."""
    S = padded_shape(n, bc_mask)
    free = [bool((bc_mask >> j) & 1) for j in range(3)]
    d = sum(free)
    shape = (S[2], S[1], S[0])
    kappa2 = np.zeros(shape)
    m2 = np.zeros(shape)
    for j in range(3):
        if free[j]:
            m2 = m2 + _axis_view(j, _free_offsets(S[j])) ** 2
        else:
            kappa2 = kappa2 + _axis_view(j, _wavenumbers(S[j], h)) ** 2
    kappa2 = np.broadcast_to(kappa2, shape)
    m2 = np.broadcast_to(m2, shape)
    kappa = np.sqrt(kappa2)
    origin = m2 == 0.0
    pos = kappa > 0.0
    out = np.empty(shape)

    if d == 0:
        with np.errstate(divide="ignore"):
            out = np.where(pos, -1.0 / np.where(pos, kappa2, 1.0), 0.0)
        return out

    r = h * np.sqrt(m2)
    safe_r = np.where(origin, 1.0, r)
    safe_k = np.where(pos, kappa, 1.0)
    if d == 1:
        g = np.where(pos, -np.exp(-safe_k * r) / (2.0 * safe_k), 0.5 * r)
        out = h * g
        org = h * np.where(pos, -1.0 / (2.0 * safe_k), 0.0) + h * h / 12.0
        out = np.where(origin, org, out)
    elif d == 2:
        g = np.where(pos, -special.k0(safe_k * safe_r) / (2.0 * math.pi),
                     np.log(safe_r) / (2.0 * math.pi))
        out = h * h * g
        org = np.where(pos,
                       np.log(safe_k * h / 2.0) + EULER_GAMMA + C2_LOG_ORIGIN,
                       math.log(h) + C2_LOG_ORIGIN) * (h * h / (2.0 * math.pi))
        out = np.where(origin, org, out)
    else:
        out = -h * h / (4.0 * math.pi * np.sqrt(np.where(origin, 1.0, m2)))
        out = np.where(origin, -(h * h / (4.0 * math.pi)) * C3_COULOMB_ORIGIN, out)
    return np.ascontiguousarray(out)


def kernel_fourier(n, bc_mask, h):
    """K^F on the whole padded grid, shape (S3, S2, S1), real float64."""
    mixed = mixed_kernel(n, bc_mask, h)
    free_axes = tuple(2 - j for j in range(3) if (bc_mask >> j) & 1)
    if not free_axes:
        return mixed
    kf = scipy.fft.fftn(mixed, axes=free_axes, workers=os.cpu_count() or 1)
    scale = max(1.0, float(np.abs(kf.real).max()))
    if float(np.abs(kf.imag).max()) > 1e-9 * scale:
        raise AssertionError("kernel is not even: K^F has an imaginary part")
    return np.ascontiguousarray(kf.real)


def kernel_octant(n, bc_mask, h, kf=None):
    """The unique octant 0 <= k_j <= S_j/2 of K^F, shape
    (S3/2+1, S2/2+1, S1/2+1), k1 fastest."""
    S = padded_shape(n, bc_mask)
    if kf is None:
        kf = kernel_fourier(n, bc_mask, h)
    return np.ascontiguousarray(kf[: S[2] // 2 + 1, : S[1] // 2 + 1, : S[0] // 2 + 1])
