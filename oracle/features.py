"""Features of the alpha predictor: spectral energy of the padded data by the
level of the kernel's spectrum.

Oracle (test infrastructure only).  The paper has no predictor; this is the
definition the HIP path is checked against.

The Tikhonov filter acts on each spectral point through s = |k^|^2 alone
(Sec. 3-4: u^ = conj(k^) f^ / (s + alpha)), so the features sort the data's
energy by that quantity.  With s_max = max s over the P^3 box, the level of
a point is

    b = number of j in 1..63 with s >= s_max 10^((j - 64)/4),

i.e. floor(4 log10(s / s_max)) + 64 clipped to [0, 63]: quarter-decade
levels, b = 63 for the points within a quarter decade of s_max and b = 0 for
s < s_max 1e-15.75 (zeros of the spectrum included).  The thresholds are
fixed numbers, decided by comparison (no logarithm of s is taken).

E_b = sum over level b of |f^(k)|^2 (f^ = DFT3 of the zero-padded data),
x_b = log10(E_b / mean_b(E_b) + 1e-30) for b < 64 and x_64 = log10(delta/||F||).
"""
from __future__ import annotations

import math

import numpy as np

NBINS = 64


def thresholds(smax: float):
    """s_max 10^((j - 64)/4) for j = 1..63, increasing."""
    return np.array([smax * 10.0 ** ((j - 64) / 4.0) for j in range(1, NBINS)])


def level_index(s, smax: float):
    """Level of every spectral point (same shape as s)."""
    return np.searchsorted(thresholds(smax), np.asarray(s, dtype=np.float64), side="right").astype(np.int64)


def level_energy(fhat, s, smax: float):
    b = level_index(s, smax)
    e = fhat.real ** 2 + fhat.imag ** 2
    return np.bincount(b.ravel(), weights=e.ravel(), minlength=NBINS)[:NBINS]


def features(F_pad_hat, delta, F_norm, s, smax=None):
    """The 65 features of data whose padded spectrum is F_pad_hat, for a
    kernel with s = |k^|^2 on the same box (s_max its maximum by default)."""
    if smax is None:
        smax = float(np.max(s))
    E = level_energy(F_pad_hat, s, smax)
    x = np.empty(NBINS + 1)
    x[:NBINS] = np.log10(E / E.mean() + 1e-30)
    x[NBINS] = math.log10(delta / F_norm)
    return x, E
