"""Features of the alpha predictor: radial spectral energy of the padded data.

Oracle (test infrastructure only).  The paper has no predictor; this is the
definition the HIP path is checked against.

For every point k of the P^3 spectrum, with signed frequencies
m_i = k_i (k_i <= P_i/2) or k_i - P_i, the normalised radius is
rho = sqrt(u/3), u = sum_i (2 m_i / P_i)^2 in [0, 3], and the bin is
b = min(63, floor(64 rho)).  The bin is decided exactly in integers:
b is the largest b <= 63 with 3 b^2 L <= 4096 U, where L = lcm(P)^2 and
U = u L = sum_i 4 m_i^2 (lcm(P)/P_i)^2.

E_b = sum over bin b of |f^(k)|^2 (f^ = DFT3 of the zero-padded data),
x_b = log10(E_b / mean_b(E_b) + 1e-30) for b < 64 and x_64 = log10(delta/||F||).
"""
from __future__ import annotations

import math

import numpy as np

NBINS = 64


def _signed(p):
    k = np.arange(p, dtype=np.int64)
    return np.where(k <= p // 2, k, k - p)


def bin_index(pshape):
    """Integer bin of every spectral point, shape pshape (z, y, x)."""
    pz, py, px = pshape
    lc = math.lcm(pz, py, px)
    L = lc * lc
    mz, my, mx = _signed(pz), _signed(py), _signed(px)
    U = (4 * mz * mz * (lc // pz) ** 2)[:, None, None] + (4 * my * my * (lc // py) ** 2)[None, :, None] \
        + (4 * mx * mx * (lc // px) ** 2)[None, None, :]
    b = np.floor(64.0 * np.sqrt(U / (3.0 * L))).astype(np.int64)
    b = np.where(3 * (b + 1) ** 2 * L <= 4096 * U, b + 1, b)
    b = np.where(3 * b * b * L > 4096 * U, b - 1, b)
    return np.minimum(b, NBINS - 1)


def radial_energy(fhat):
    b = bin_index(fhat.shape)
    e = (fhat.real ** 2 + fhat.imag ** 2)
    return np.bincount(b.ravel(), weights=e.ravel(), minlength=NBINS)[:NBINS]


def features(F_pad_hat, delta, F_norm):
    E = radial_energy(F_pad_hat)
    x = np.empty(NBINS + 1)
    x[:NBINS] = np.log10(E / E.mean() + 1e-30)
    x[NBINS] = math.log10(delta / F_norm)
    return x, E
