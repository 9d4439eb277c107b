"""Shared helpers of the GPU tests: seeded instances through the oracle, and
conversions of the library's spectral layouts to the oracle's."""
import numpy as np

from oracle import synth
from oracle.geometry import Geom
from paper_1703_01216_amd import inputs


def geom(nx, ny, nz, D=None, kind=0, q=None, h=1.0, hz=None):
    return Geom(nx, ny, nz, h=h, D=D, kind=kind, q=q, hz=hz)


def instance(g: Geom, seed, delta_rel=0.01, recipe="blobs"):
    shape = g.shape
    if recipe == "blobs":
        sig = (max(1.0, min(shape) / 16), max(1.5, min(shape) / 8))
        xi = inputs.xi_blobs(shape, seed, count=3, sigma=sig)
    else:
        xi = inputs.xi_inclusions(shape, seed)
    e = inputs.noise(shape, seed)
    d = synth.make_data(g, xi, e, delta_rel)
    d["xi"] = xi
    d["noise"] = e
    return d


def octant_from_full(khat, g: Geom):
    """Oracle k^ [kz][ky][kx] -> library octant layout [kx][kz][ky], kx,ky,kz <= P/2."""
    pz, py, px = g.pshape
    o = khat[: pz // 2 + 1, : py // 2 + 1, : px // 2 + 1]
    return np.transpose(o, (2, 0, 1))


def half_spectrum(fhat, g: Geom):
    """Oracle f^ [kz][ky][kx] -> library layout [kx][kz][ky] for kx <= Px/2."""
    px = g.pshape[2]
    return np.transpose(fhat[:, :, : px // 2 + 1], (2, 0, 1))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
