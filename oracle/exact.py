"""Tikhonov's method for the exact discrete operator A: L2(R) -> L2(Y) (the
midpoint quadrature of Eq. (8); the unknown lives on R and the residual on
Y, nothing on a padded box):

    zeta(alpha) = argmin ||A zeta - F||^2_Y + alpha ||zeta||^2_R,
    i.e. (A^T A + alpha I) zeta = A^T F,

the regularised normal solution of Sec. 3 (Sec. 4: Tikhonov's method as a
regularising algorithm) without the circulant embedding's extra freedom on
the padded box.  alpha in the functional's L2 units (cell-volume weights
cancel, as for the other forms).

Oracle (test infrastructure only).

* ``forward`` / ``adjoint``: A through the circulant embedding, A^T through
  the same table with the conjugate spectrum (real kernel table: correlation).
* ``adjoint_direct``: A^T r as the plain sum over Y's cells, K at cell-centre
  differences.
* ``dense_exact``: the normal equations with A assembled column by column
  from the direct quadrature sum (tiny grids).
* ``cg_exact``: conjugate gradients on the normal equations with
  ``forward``/``adjoint`` (larger grids), started from zero.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geom, sample_kernel
from .operator import forward_direct, offset_table, pad


def forward(g: Geom, khat, zeta):
    return np.fft.ifftn(khat * np.fft.fftn(pad(g, zeta))).real[: g.nz, : g.ny, : g.nx]


def adjoint(g: Geom, khat, r):
    return np.fft.ifftn(khat.conj() * np.fft.fftn(pad(g, r))).real[: g.nz, : g.ny, : g.nx]


def adjoint_direct(g: Geom, r):
    """(A^T r)(x_R) = sum over Y cells y of h^2 hz K(x_y - x_R) r(y), O(n^6)."""
    r = np.asarray(r, dtype=np.float64)
    T = offset_table(g)
    nz, ny, nx = g.shape
    out = np.zeros(g.shape)
    for yz in range(nz):
        for yy in range(ny):
            for yx in range(nx):
                v = r[yz, yy, yx]
                if v == 0.0:
                    continue
                # R cell x receives T[y - x] for all x in [0, n)^3
                out += v * T[yz: yz + nz, yy: yy + ny, yx: yx + nx][::-1, ::-1, ::-1]
    return out


def dense_matrix(g: Geom):
    """A as an explicit (n^3 x n^3) matrix, one direct-quadrature column per R cell."""
    n = g.nz * g.ny * g.nx
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = forward_direct(g, e.reshape(g.shape)).ravel()
    return A


def _report(g: Geom, zeta, r, iters=0):
    return dict(zeta=zeta, r=r, zeta_norm=float(np.linalg.norm(zeta)), r_norm=float(np.linalg.norm(r)), iters=iters)


def dense_exact(g: Geom, F, alpha: float):
    A = dense_matrix(g)
    f = np.asarray(F, dtype=np.float64).ravel()
    z = np.linalg.solve(A.T @ A + alpha * np.eye(A.shape[1]), A.T @ f)
    return _report(g, z.reshape(g.shape), (A @ z - f).reshape(g.shape))


def cg_exact(g: Geom, F, alpha: float, tol: float = 1e-12, max_iter: int = 5000, khat=None):
    """CG on (A^T A + alpha I) z = A^T F until ||residual of the normal
    equations|| <= tol ||A^T F||."""
    khat = np.fft.fftn(sample_kernel(g)) if khat is None else khat
    F = np.asarray(F, dtype=np.float64)
    b = adjoint(g, khat, F)
    z = np.zeros(g.shape)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    bn = np.sqrt(float(np.sum(b * b)))
    it = 0
    while it < max_iter and np.sqrt(rr) > tol * bn:
        q = adjoint(g, khat, forward(g, khat, p)) + alpha * p
        a = rr / float(np.sum(p * q))
        z += a * p
        r -= a * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return _report(g, z, forward(g, khat, z) - F, it)
