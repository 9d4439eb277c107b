"""Grids, the integral kernel, its sampled offset table, sources and V0.

Oracle (test infrastructure only).

Readings of points the paper leaves open (each also listed in the design notes):
* R and Y are horizontal layers (Sec. 3): R = cells [0,nx)x[0,ny)x[0,nz) with
  centres ((i+.5)h, (j+.5)h, (k+.5)h); Y has the same lateral cells and
  z-centres (D+k+.5)h.  R and Y are disjoint when D >= nz.
* Default gap: D = nz + ceil(nz/4).  With a source parameter q that varies the
  kernel: D_q = nz + (q+1) ceil(nz/8).
* Quadrature: midpoint rule with weight the cell volume h^2 hz (Sec. 5 names
  only "quadrature coefficients"); hz = h unless the layers are thinner
  (Sec. 6's model example), and D counts vertical cells.
* Circulant embedding: per axis P = 2n; an offset index a in [0,P) stands for
  the cell offset a (a < n) or a-P (a > P-n); the one slot a = n (P = 2n) that
  no pair of cells reaches is zero.
* Sources (Sec. 6): the ten-point cross of the model example -- the lateral
  centre and the points +-0.4 n away along x and along y -- at the two heights
  nz + G/4 and nz + 3G/4 (G = D - nz), i.e. between the layers.  A0 = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geom:
    nx: int
    ny: int
    nz: int
    h: float = 1.0
    D: float | None = None   # z-offset of Y above R in cells
    kind: int = 0            # 0: dz(1/|x|) (Eq. (6)/(8)); 1: 1/|x| (Eq. (5))
    q: int | None = None     # source parameter; None = single-kernel default gap
    hz: float | None = None  # vertical cell edge; None = h (D counts vertical cells)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def pshape(self):
        return (2 * self.nz, 2 * self.ny, 2 * self.nx)

    @property
    def hv(self) -> float:
        """Vertical cell edge."""
        return float(self.h if self.hz is None else self.hz)

    @property
    def d(self) -> float:
        if self.D is not None:
            return float(self.D)
        if self.q is None:
            return float(self.nz + math.ceil(self.nz / 4))
        return float(self.nz + (self.q + 1) * math.ceil(self.nz / 8))


def kernel_dz(x, y, z):
    """K(x,y,z) = d/dz (x^2+y^2+z^2)^(-1/2) = -z (x^2+y^2+z^2)^(-3/2)  (Sec. 3, kernel of Eq. (8))."""
    r2 = x * x + y * y + z * z
    return -z / (r2 * np.sqrt(r2))


def kernel_inv(x, y, z):
    """1/|x|, the kernel of Eq. (5) (Sec. 2)."""
    return 1.0 / np.sqrt(x * x + y * y + z * z)


def kernel_fn(kind):
    return {0: kernel_dz, 1: kernel_inv}[kind]


def offset_of_index(a, n, p):
    """Cell offset represented by circulant index a (array), and a validity mask."""
    a = np.asarray(a)
    off = np.where(a < n, a, a - p)
    valid = (a < n) | (a > p - n)
    return off, valid


def sample_kernel(g: Geom, pshape=None):
    """Wrapped offset table k[c][b][a] = h^2 hz K(off(a) h, off(b) h, (D + off(c)) hz),
    zero in slots no pair of cells reaches.  Shape (Pz, Py, Px)."""
    pz, py, px = pshape or g.pshape
    oz, vz = offset_of_index(np.arange(pz), g.nz, pz)
    oy, vy = offset_of_index(np.arange(py), g.ny, py)
    ox, vx = offset_of_index(np.arange(px), g.nx, px)
    Z = (g.d + oz)[:, None, None] * g.hv
    Y = oy[None, :, None] * g.h
    X = ox[None, None, :] * g.h
    k = g.h * g.h * g.hv * kernel_fn(g.kind)(X, Y, Z)
    mask = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    return np.where(mask, k, 0.0)


def sources(g: Geom):
    """The ten delta-source positions (physical units), shape (10, 3) as (x, y, z)."""
    G = g.d - g.nz
    cx, cy = g.nx / 2.0, g.ny / 2.0
    ax, ay = 0.4 * g.nx, 0.4 * g.ny
    pts = []
    for zc in (g.nz + G / 4.0, g.nz + 3.0 * G / 4.0):
        for (x, y) in ((cx, cy), (cx - ax, cy), (cx + ax, cy), (cx, cy - ay), (cx, cy + ay)):
            pts.append((x * g.h, y * g.h, zc * g.hv))
    return np.array(pts, dtype=np.float64)


def v0(g: Geom, A0: float = 1.0):
    """V0 at the centres of R's cells for point sources (Sec. 6):
    V0(x) = -(A0 / 4 pi) sum_l 1/|x - x_l|.  Shape (nz, ny, nx)."""
    z = (np.arange(g.nz) + 0.5)[:, None, None] * g.hv
    y = (np.arange(g.ny) + 0.5)[None, :, None] * g.h
    x = (np.arange(g.nx) + 0.5)[None, None, :] * g.h
    acc = np.zeros(g.shape)
    for (sx, sy, sz) in sources(g):
        acc += 1.0 / np.sqrt((x - sx) ** 2 + (y - sy) ** 2 + (z - sz) ** 2)
    return -(A0 / (4.0 * math.pi)) * acc
