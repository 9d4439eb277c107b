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


def oracle_features(g: Geom, F, delta, margin=1e-9):
    """The oracle's predictor features of data F on the geometry's sampled
    kernel, and the number of spectral points whose |k^|^2 lies within
    `margin` (relative) of a level threshold: those are the only points whose
    level two FP64 spectra of the kernel may decide differently."""
    from oracle import features
    from oracle.geometry import sample_kernel
    from oracle.operator import pad
    khat = np.fft.fftn(sample_kernel(g))
    s = (khat * khat.conj()).real
    smax = float(s.max())
    x, E = features.features(np.fft.fftn(pad(g, np.asarray(F, dtype=np.float64))), delta,
                             float(np.linalg.norm(F)), s, smax)
    thr = features.thresholds(smax)
    idx = np.clip(np.searchsorted(thr, s.ravel()), 1, len(thr) - 1)
    near = np.minimum(np.abs(s.ravel() / thr[idx - 1] - 1.0), np.abs(s.ravel() / thr[idx] - 1.0)) < margin
    return x, E, int(near.sum())
