"""The forward operator A: L2(R) -> L2(Y) of the layered equation (Sec. 3, Eq. (8)).

Oracle (test infrastructure only).

(A zeta)(y) = sum over cells r of R of  h^2 hz K(x_y - x_r) zeta(r),  y a cell of Y,
the midpoint quadrature of the convolution integral of Eq. (8) with the
kernel K of Sec. 3.  Two forms:

* ``forward_direct``    -- the sum itself, K evaluated at the physical offset
                           between the two cell centres (no table, no wrap).
* ``forward_circulant`` -- the same sum through the zero-padded offset table
                           and numpy.fft (convolution theorem on the P^3 box).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geom, kernel_fn, sample_kernel


def offset_table(g: Geom):
    """h^2 hz K at every cell offset (dz, dy, dx) in (-n, n)^3, indexed [dz+nz-1][dy+ny-1][dx+nx-1]."""
    dz = np.arange(-(g.nz - 1), g.nz)[:, None, None]
    dy = np.arange(-(g.ny - 1), g.ny)[None, :, None]
    dx = np.arange(-(g.nx - 1), g.nx)[None, None, :]
    # centre of Y cell minus centre of R cell: ((dx)h, (dy)h, (D + dz)hz)
    return g.h * g.h * g.hv * kernel_fn(g.kind)(dx * g.h, dy * g.h, (g.d + dz) * g.hv)


def forward_direct(g: Geom, zeta):
    """Direct quadrature sum over every (Y cell, R cell) pair, O(n^6)."""
    zeta = np.asarray(zeta, dtype=np.float64)
    T = offset_table(g)
    nz, ny, nx = g.shape
    out = np.zeros(g.shape)
    for rz in range(nz):
        for ry in range(ny):
            for rx in range(nx):
                v = zeta[rz, ry, rx]
                if v == 0.0:
                    continue
                # Y cell y receives T[y - r] for all y in [0, n)^3
                out += v * T[nz - 1 - rz: 2 * nz - 1 - rz,
                             ny - 1 - ry: 2 * ny - 1 - ry,
                             nx - 1 - rx: 2 * nx - 1 - rx]
    return out


def pad(g: Geom, u):
    """Place an n^3 field in the corner [0,n)^3 of the zero P^3 box."""
    out = np.zeros(g.pshape, dtype=np.asarray(u).dtype)
    out[: g.nz, : g.ny, : g.nx] = u
    return out


def forward_circulant(g: Geom, zeta, k=None):
    """A zeta through the circulant embedding: IDFT(DFT(k) DFT(pad zeta)) on [0,n)^3."""
    k = sample_kernel(g) if k is None else k
    full = np.fft.ifftn(np.fft.fftn(k) * np.fft.fftn(pad(g, zeta))).real
    return full[: g.nz, : g.ny, : g.nx]


def circulant_apply(k, u):
    """(C u)[p] = sum_q k[(p - q) mod P] u[q] on the whole P^3 box, as a direct sum (tiny P)."""
    P = k.shape
    out = np.zeros(P)
    for qz in range(P[0]):
        for qy in range(P[1]):
            for qx in range(P[2]):
                v = u[qz, qy, qx]
                if v != 0.0:
                    out += v * np.roll(k, (qz, qy, qx), axis=(0, 1, 2))
    return out
