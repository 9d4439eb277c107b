"""Discrete Fourier transforms written out as sums (the definition).

Oracle (test infrastructure only).

Convention (the estimator does not depend on it): forward
X[k] = sum_j x[j] exp(-2 pi i j k / P), unnormalised; inverse
x[j] = P^-1 sum_k X[k] exp(+2 pi i j k / P) per axis.  This is the discrete
counterpart of the continuous transform with kernel e^{-i w x} and inverse
factor 1/(4 pi^2) used in the Plancherel equalities of Sec. 4 (Lemma 1).
"""
from __future__ import annotations

import numpy as np


def dft_matrix(p: int, inverse: bool = False):
    """W[k, j] = exp(-+2 pi i j k / P) with the angle reduced exactly via (j k mod P)."""
    j = np.arange(p)
    jk = np.outer(j, j) % p
    ang = 2.0 * np.pi * jk / p
    w = np.cos(ang) + (1j if inverse else -1j) * np.sin(ang)
    return w / p if inverse else w


def dft_axis(x, axis: int, inverse: bool = False):
    """Apply the 1D DFT sum along one axis."""
    x = np.asarray(x, dtype=np.complex128)
    w = dft_matrix(x.shape[axis], inverse)
    return np.moveaxis(np.tensordot(w, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def dft3(x, inverse: bool = False):
    """3D DFT as the iterated 1D sums (separable, O(P^4))."""
    y = x
    for ax in range(3):
        y = dft_axis(y, ax, inverse)
    return y


def dft3_full(x, inverse: bool = False):
    """3D DFT as one direct sum over all P^3 points for every output (O(P^6)).
    For tiny grids only."""
    x = np.asarray(x, dtype=np.complex128)
    pz, py, px = x.shape
    kz, ky, kx = np.meshgrid(np.arange(pz), np.arange(py), np.arange(px), indexing="ij")
    kz, ky, kx = kz.ravel(), ky.ravel(), kx.ravel()
    phase = (np.outer(kz, kz) % pz) / pz + (np.outer(ky, ky) % py) / py + (np.outer(kx, kx) % px) / px
    sgn = 1.0 if inverse else -1.0
    w = np.exp(sgn * 2j * np.pi * phase)
    out = w @ x.ravel()
    if inverse:
        out = out / (pz * py * px)
    return out.reshape(x.shape)
