"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This module draws random numbers and shapes them into input fields.  It holds
none of the solver's arithmetic (no kernel, no transform, no regularisation,
no potential): the contrast field xi and the raw noise draws it returns are
pushed through the paper's operator by whichever side consumes them.

Recipes (all positions in cell units, fields sampled at cell centres i+0.5):

* ``xi_blobs``     -- a sum of isotropic Gaussian blobs a*exp(-|x-c|^2/(2 s^2)).
* ``xi_inclusions``-- a mix of Gaussian blobs and axis-aligned boxes
                      a*1[|x-c|_inf <= w/2].
* ``xi_stress``    -- a smooth Gaussian background plus many sharp boxes and
                      balls with high contrast, capped below 1.
* ``noise``        -- i.i.d. standard normal draws on the data grid.

Seeds: an instance of workload ``cfg`` with index ``i`` uses seed 1000*cfg+i.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "instance_seed", "rng", "xi_blobs", "xi_inclusions", "xi_stress", "noise",
    "workload_instance",
]


def instance_seed(cfg: int, index: int) -> int:
    return 1000 * int(cfg) + int(index)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _centres(shape):
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64) + 0.5
    y = np.arange(ny, dtype=np.float64) + 0.5
    x = np.arange(nx, dtype=np.float64) + 0.5
    return z[:, None, None], y[None, :, None], x[None, None, :]


def _gauss(shape, c, s):
    z, y, x = _centres(shape)
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    return np.exp(-r2 / (2.0 * s * s))


def _box(shape, c, w):
    z, y, x = _centres(shape)
    m = (np.abs(x - c[0]) <= w / 2) & (np.abs(y - c[1]) <= w / 2) & (np.abs(z - c[2]) <= w / 2)
    return m.astype(np.float64)


def _ball(shape, c, rad):
    z, y, x = _centres(shape)
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    return (r2 <= rad * rad).astype(np.float64)


def _draw_centre(g, shape, margin_frac):
    nz, ny, nx = shape
    return np.array([g.uniform(margin_frac * n, (1 - margin_frac) * n) for n in (nx, ny, nz)])


def xi_blobs(shape, seed, count=3, amp=(0.1, 0.5), sigma=(2.0, 4.0), margin_frac=0.125):
    """Sum of ``count`` Gaussian blobs; centres uniform in the box minus a margin."""
    g = rng(seed)
    xi = np.zeros(shape, dtype=np.float64)
    for _ in range(count):
        c = _draw_centre(g, shape, margin_frac)
        a = g.uniform(*amp)
        s = g.uniform(*sigma)
        xi += a * _gauss(shape, c, s)
    return xi


def xi_inclusions(shape, seed, count=(5, 10), amp=(0.05, 0.8), margin_frac=0.125):
    """5-10 inclusions, Gaussian or box with probability 1/2 each.

    Gaussian width s ~ U[n/16, n/8], box edge w ~ U[n/10, n/4] with n the
    smallest grid extent; amplitudes ~ U[amp]."""
    g = rng(seed)
    n = min(shape)
    k = int(g.integers(count[0], count[1] + 1))
    xi = np.zeros(shape, dtype=np.float64)
    for _ in range(k):
        c = _draw_centre(g, shape, margin_frac)
        a = g.uniform(*amp)
        if g.uniform() < 0.5:
            xi += a * _gauss(shape, c, g.uniform(n / 16, n / 8))
        else:
            xi += a * _box(shape, c, g.uniform(n / 10, n / 4))
    return xi


def xi_stress(shape, seed, count=20, contrast=(0.3, 0.9), cap=0.95):
    """Smooth background 0.05+0.05*exp(-|x-m|^2/(2 (n/3)^2)) plus ``count`` sharp
    boxes/balls of contrast U[contrast], the total capped at ``cap``."""
    g = rng(seed)
    n = min(shape)
    nz, ny, nx = shape
    xi = 0.05 + 0.05 * _gauss(shape, (nx / 2, ny / 2, nz / 2), n / 3)
    for _ in range(count):
        c = _draw_centre(g, shape, 0.08)
        a = g.uniform(*contrast)
        size = g.uniform(n / 24, n / 10)
        if g.uniform() < 0.5:
            xi += a * _box(shape, c, 2 * size)
        else:
            xi += a * _ball(shape, c, size)
    return np.minimum(xi, cap)


def noise(shape, seed):
    """Standard normal draws on the data grid (stream offset from the xi draws)."""
    return rng(seed + 7_000_003).standard_normal(shape)


def workload_instance(cfg: int, index: int, n=None):
    """The synthetic instance of workload ``cfg`` (1..5) with index ``index``.

    Returns dict(shape, xi, noise, delta_rel, seed, q); q is the source
    parameter (a list of all four values for the batched workload 3).  ``n`` overrides the grid
    extent (cubic) for reduced-size tests of the same recipe.
    """
    seed = instance_seed(cfg, index)
    g = rng(seed + 13)
    if cfg == 1:
        n = n or 32
        shape = (n, n, n)
        xi = xi_blobs(shape, seed, count=3, amp=(0.1, 0.5), sigma=(2.0, 4.0), margin_frac=0.125)
        delta_rel = 0.01
    elif cfg == 2:
        n = n or 128
        shape = (n, n, n)
        xi = xi_inclusions(shape, seed)
        delta_rel = (0.01, 0.03, 0.05)[index % 3]
    elif cfg == 4:
        n = n or 256
        shape = (n, n, n)
        xi = xi_stress(shape, seed)
        delta_rel = 0.005
    elif cfg in (3, 5):
        if n is None:
            choices = (64, 96, 128, 192) if cfg == 3 else (64, 96, 128)
            if cfg == 3:
                shape = tuple(int(g.choice(choices)) for _ in range(3))
            else:
                m = int(g.choice(choices))
                shape = (m, m, m)
        else:
            shape = (n, n, n)
        xi = xi_inclusions(shape, seed)
        delta_rel = float(g.uniform(0.005, 0.05))
        q = [0, 1, 2, 3] if cfg == 3 else int(g.integers(0, 4))
        return dict(shape=shape, xi=xi, noise=noise(shape, seed), delta_rel=delta_rel, seed=seed, q=q)
    else:
        raise ValueError(f"unknown workload {cfg}")
    return dict(shape=shape, xi=xi, noise=noise(shape, seed), delta_rel=delta_rel, seed=seed, q=0)
