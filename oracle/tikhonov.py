"""Tikhonov regularisation of the circulant-embedded operator.

Oracle (test infrastructure only).

The regularising algorithm R_alpha of Sec. 3 (family of Eq. (11)) is Tikhonov's
method, named in Sec. 4 as admissible for Algorithm 1.  Here it is applied to
the circulant embedding C of the discretised operator on the zero-padded P^3
box (the three-axis analogue of the paper's per-frequency systems, Eq. (14)):

    zeta_pad(alpha) = argmin_u ||C u - E_Y F||^2 + alpha_abs ||u||^2,
    zeta(alpha)     = zeta_pad restricted to R's index block [0,n)^3,
    r(alpha)        = (C zeta_pad - E_Y F) restricted to Y's index block,

where alpha_abs is the Tikhonov parameter of the functional in the L2 norms of
Sec. 3 (the cell-volume weights on both sides cancel, so alpha_abs = alpha
for any cell size).  With ``relative=True`` the given alpha is scaled by max |k^|^2
(relative to the squared operator norm of C) instead.

``dense_tikhonov`` solves the normal equations (C^T C + alpha_abs I) u = C^T E_Y F
with C assembled as a matrix and a Cholesky factorisation -- no transform.
``solve_spectral`` is the same minimiser through the DFT, where C is diagonal:
u^ = conj(k^) f^ / (|k^|^2 + alpha_abs).

Other regularising algorithms (Sec. 5 names standard and iterated Tikhonov
and truncated SVD as the ones applied to the per-frequency systems), on the
same circulant embedding, with s = |k^|^2 and q = alpha/(s + alpha):

* iterated Tikhonov of order m: u_0 = 0, u_j = argmin ||C u - f||^2 +
  alpha ||u - u_{j-1}||^2, j = 1..m; spectrally u^ = conj(k^) f^ (1 - q^m)/s
  = conj(k^) f^ sum_{j<m} q^j / (s + alpha), residual -q^m f^ (m = 1 is
  Tikhonov).  ``dense_iterated`` runs the m normal-equation solves.
* truncated SVD with cut alpha: the singular values of C are |k^|, so the
  modes with s >= alpha are inverted, u^ = conj(k^) f^ / s, and the others
  dropped; residual 0 on kept modes and -f^ on dropped ones.
  ``dense_tsvd`` uses the SVD of the assembled matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .geometry import Geom
from .operator import pad

TIKHONOV, ITERATED, TSVD = 0, 1, 2


def kernel_spectrum(k):
    """k^ = DFT3(k) (FP64), s = |k^|^2 and s_max."""
    khat = np.fft.fftn(k)
    s = (khat * khat.conj()).real
    return khat, s, float(s.max())


def spectral_filter(khat, fhat, alpha_abs: float, method: int = TIKHONOV, order: int = 1):
    """Minimiser and residual spectra on the whole box for box data with spectrum f^:
    Tikhonov u^ = conj(k^) f^ / (s + a) and (C u - f)^ = k^ u^ - f^ = -a f^ / (s + a);
    iterated Tikhonov and truncated SVD as in the module docstring."""
    s = (khat * khat.conj()).real
    a = alpha_abs
    if method == TIKHONOV:
        return khat.conj() * fhat / (s + a), -a * fhat / (s + a)
    if method == ITERATED:
        q = a / (s + a)
        g = sum(q ** j for j in range(order)) / (s + a)
        return khat.conj() * fhat * g, -(q ** order) * fhat
    if method == TSVD:
        keep = s >= a
        inv = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
        return khat.conj() * fhat * inv, np.where(keep, 0.0, -1.0) * fhat
    raise ValueError(f"unknown method {method}")


def alpha_abs(khat, alpha: float, relative: bool) -> float:
    return float(alpha) * (float((khat * khat.conj()).real.max()) if relative else 1.0)


def solve_box(khat, f_box, alpha: float, relative: bool = False):
    """Tikhonov minimiser for data given on the whole P^3 box (no restriction)."""
    a = alpha_abs(khat, alpha, relative)
    uhat, rhat = spectral_filter(khat, np.fft.fftn(f_box), a)
    return np.fft.ifftn(uhat), np.fft.ifftn(rhat)


def solve_spectral(g: Geom, khat, F, alpha: float, relative: bool = False, method: int = TIKHONOV,
                   order: int = 1):
    """Regularised estimate at alpha (Tikhonov unless ``method`` says otherwise);
    returns zeta on R, r on Y and their norms."""
    a = alpha_abs(khat, alpha, relative)
    fhat = np.fft.fftn(pad(g, np.asarray(F, dtype=np.float64)))
    uhat, rhat = spectral_filter(khat, fhat, a, method, order)
    zpad = np.fft.ifftn(uhat)
    rpad = np.fft.ifftn(rhat)
    n = g.shape
    zeta = zpad.real[: n[0], : n[1], : n[2]]
    r = rpad.real[: n[0], : n[1], : n[2]]
    return dict(
        zeta=zeta, r=r, alpha_abs=a,
        zeta_norm=float(np.sqrt(np.sum(zeta * zeta))),
        r_norm=float(np.sqrt(np.sum(r * r))),
        r_full=float(np.sqrt(np.sum(rpad.real ** 2))),
        imag_max=float(max(np.abs(zpad.imag).max(), np.abs(rpad.imag).max())),
    )


def full_box_slope(g: Geom, khat, F, alpha: float, relative: bool = False) -> float:
    """Slope d ln ||C zeta_pad - E_Y F|| / d log10 alpha of the whole-box
    Tikhonov residual (used by the learned search's first secant step; not in
    the paper).  The residual spectrum is -e f^ with e = a / (s + a), and
    de / d ln a = e (1 - e), so by Parseval

        d ln ||r_box|| / d ln a = sum e^2 (1 - e) |f^|^2 / sum e^2 |f^|^2,

    times ln 10 per decade of alpha."""
    a = alpha_abs(khat, alpha, relative)
    fhat = np.fft.fftn(pad(g, np.asarray(F, dtype=np.float64)))
    s = (khat * khat.conj()).real
    e = a / (s + a)
    q = e * e * (fhat * fhat.conj()).real
    return float(np.log(10.0) * np.sum(q * (1.0 - e)) / np.sum(q))


def circulant_matrix(k):
    """C[p, q] = k[(p - q) mod P] over the flattened P^3 box (x fastest)."""
    P = k.shape
    n = k.size
    C = np.empty((n, n))
    col = 0
    for qz in range(P[0]):
        for qy in range(P[1]):
            for qx in range(P[2]):
                C[:, col] = np.roll(k, (qz, qy, qx), axis=(0, 1, 2)).ravel()
                col += 1
    return C


def dense_tikhonov(g: Geom, k, F, alpha_abs: float):
    """Normal-equation solve with an explicit matrix (P^3 <= ~4096 unknowns)."""
    C = circulant_matrix(k)
    f = pad(g, np.asarray(F, dtype=np.float64)).ravel()
    A = C.T @ C + alpha_abs * np.eye(C.shape[0])
    u = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), C.T @ f)
    res = (C @ u - f).reshape(k.shape)
    u = u.reshape(k.shape)
    n = g.shape
    return dict(zeta_pad=u, zeta=u[: n[0], : n[1], : n[2]], r=res[: n[0], : n[1], : n[2]], r_full=res)


def _restrict(g: Geom, C, u, f, k):
    res = (C @ u - f).reshape(k.shape)
    u = u.reshape(k.shape)
    n = g.shape
    return dict(zeta_pad=u, zeta=u[: n[0], : n[1], : n[2]], r=res[: n[0], : n[1], : n[2]], r_full=res)


def dense_iterated(g: Geom, k, F, alpha_abs: float, order: int):
    """Iterated Tikhonov by its definition: ``order`` normal-equation solves
    (C^T C + alpha I) u_j = C^T f + alpha u_{j-1} from u_0 = 0, explicit matrix."""
    C = circulant_matrix(k)
    f = pad(g, np.asarray(F, dtype=np.float64)).ravel()
    fac = scipy.linalg.cho_factor(C.T @ C + alpha_abs * np.eye(C.shape[0]))
    u = np.zeros_like(f)
    for _ in range(order):
        u = scipy.linalg.cho_solve(fac, C.T @ f + alpha_abs * u)
    return _restrict(g, C, u, f, k)


def dense_tsvd(g: Geom, k, F, cut: float):
    """Truncated SVD of the explicit matrix: singular triplets with sigma^2 >= cut."""
    C = circulant_matrix(k)
    f = pad(g, np.asarray(F, dtype=np.float64)).ravel()
    U, S, Vt = np.linalg.svd(C)
    keep = S * S >= cut
    u = Vt[keep].T @ ((U[:, keep].T @ f) / S[keep])
    return _restrict(g, C, u, f, k)
