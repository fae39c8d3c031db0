"""Plain FP64 Poisson solve and brute-force direct sum.

TEST INFRASTRUCTURE ONLY (see the package docstring).

`solve` is the method's result by its definition (Section 2, Eqs. 2-3, and
the padding S_j = N_j B_j of Section 3): pad the density with zeros to the
FFT lengths, take the whole-grid DFT, multiply by K^F, invert, keep the first
N_j points of every axis.  It uses no zero-skipping, axis order or fusion.

`brute_force` evaluates the real-space convolution of Eq. 2 term by term,
V[i] = sum_j K_pad[(i - j) mod S] rho[j], with the padded kernel put into real
space by explicit cosine sums (no FFT), for tiny grids only.
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .greens import kernel_fourier, mixed_kernel, padded_shape


def _shape_n(rho):
    n3, n2, n1 = rho.shape
    return (n1, n2, n3)


def solve(rho, bc_mask, h, kf=None, workers=None):
    """V = crop(IDFT_S(K^F * DFT_S(pad(rho)))) in float64; rho is (n3, n2, n1)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = _shape_n(rho)
    S = padded_shape(n, bc_mask)
    if kf is None:
        kf = kernel_fourier(n, bc_mask, h)
    if workers is None:
        workers = os.cpu_count() or 1
    padded = np.zeros((S[2], S[1], S[0]))
    padded[: n[2], : n[1], : n[0]] = rho
    spec = scipy.fft.rfftn(padded, workers=workers)
    # the half spectrum of a real array keeps k1 in [0, S1/2]
    spec *= kf[:, :, : S[0] // 2 + 1]
    V = scipy.fft.irfftn(spec, s=padded.shape, workers=workers)
    return np.ascontiguousarray(V[: n[2], : n[1], : n[0]])


def _inverse_dft_real_axis(arr, axis):
    """Explicit inverse DFT along one axis of a real, even spectrum:
    x[m] = (1/S) sum_f X[f] cos(2 pi f m / S)."""
    S = arr.shape[axis]
    f = np.arange(S)
    c = np.cos(2.0 * np.pi * np.outer(f, f) / S) / S
    moved = np.moveaxis(arr, axis, -1)
    return np.moveaxis(moved @ c, -1, axis)


def real_space_kernel(n, bc_mask, h):
    """K_pad on the padded grid in real space.  Free axes are sampled
    directly; periodic axes are taken from spectral to real space by an
    explicit cosine sum (the spectral kernel is real and even)."""
    K = mixed_kernel(n, bc_mask, h)
    for j in range(3):
        if not (bc_mask >> j) & 1:
            K = _inverse_dft_real_axis(K, 2 - j)
    return K


def brute_force(rho, bc_mask, h, kpad=None):
    """Direct sum of Eq. 2 over all source points (O(N^2) work)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = _shape_n(rho)
    S = padded_shape(n, bc_mask)
    if kpad is None:
        kpad = real_space_kernel(n, bc_mask, h)
    dx = (np.arange(n[0])[:, None] - np.arange(n[0])[None, :]) % S[0]
    dy = (np.arange(n[1])[:, None] - np.arange(n[1])[None, :]) % S[1]
    dz = (np.arange(n[2])[:, None] - np.arange(n[2])[None, :]) % S[2]
    V = np.empty(rho.shape)
    for i3 in range(n[2]):
        # block[j3, i2, j2, i1, j1] = K_pad[dz[i3, j3], dy[i2, j2], dx[i1, j1]]
        block = kpad[dz[i3][:, None, None, None, None],
                     dy[None, :, :, None, None],
                     dx[None, None, None, :, :]]
        V[i3] = np.einsum("cbBaA,cBA->ba", block, rho, optimize=True)
    return V


def rel_l2(v, ref):
    """||v - ref||_2 / ||ref||_2 accumulated in float64."""
    v = np.asarray(v, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
