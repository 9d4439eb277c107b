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
    "instance_seed", "rng", "xi_blobs", "inclusion_params", "xi_inclusions", "xi_stress", "noise",
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


def inclusion_params(shape, seed, count=(5, 10), amp=(0.05, 0.8), margin_frac=0.125):
    """Parameters of 5-10 inclusions: list of (kind, centre (x,y,z), amplitude, size),
    kind "gauss" (size = s ~ U[n/16, n/8]) or "box" (size = edge w ~ U[n/10, n/4]),
    each with probability 1/2; n is the smallest grid extent."""
    g = rng(seed)
    n = min(shape)
    k = int(g.integers(count[0], count[1] + 1))
    out = []
    for _ in range(k):
        c = _draw_centre(g, shape, margin_frac)
        a = g.uniform(*amp)
        if g.uniform() < 0.5:
            out.append(("gauss", c, a, g.uniform(n / 16, n / 8)))
        else:
            out.append(("box", c, a, g.uniform(n / 10, n / 4)))
    return out


def xi_inclusions(shape, seed, count=(5, 10), amp=(0.05, 0.8), margin_frac=0.125):
    """The field of ``inclusion_params``: sum of a exp(-|x-c|^2/(2 s^2)) and a 1[|x-c|_inf <= w/2]."""
    xi = np.zeros(shape, dtype=np.float64)
    for kind, c, a, size in inclusion_params(shape, seed, count, amp, margin_frac):
        xi += a * (_gauss(shape, c, size) if kind == "gauss" else _box(shape, c, size))
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


def workload_params(cfg: int, index: int):
    """Recipe of a workload-3 or workload-5 instance without evaluating any
    field: dict(shape, inclusions, delta_rel, q, seed), the same draws as
    workload_instance.  Workload 5: grid extent n ~ U{64, 96, 128} (cubic),
    q ~ U{0..3}, delta_rel ~ U[0.5%, 5%].  Workload 3: each axis ~ U{64, 96,
    128, 192}, q = all of 0..3, delta_rel ~ U[0.5%, 5%]."""
    if cfg not in (3, 5):
        raise ValueError("parameter-only recipes exist for workloads 3 and 5")
    seed = instance_seed(cfg, index)
    g = rng(seed + 13)
    if cfg == 3:
        shape = tuple(int(g.choice((64, 96, 128, 192))) for _ in range(3))
        delta_rel = float(g.uniform(0.005, 0.05))
        return dict(shape=shape, inclusions=inclusion_params(shape, seed), delta_rel=delta_rel, q=[0, 1, 2, 3],
                    seed=seed)
    m = int(g.choice((64, 96, 128)))
    shape = (m, m, m)
    delta_rel = float(g.uniform(0.005, 0.05))
    q = int(g.integers(0, 4))
    return dict(shape=shape, inclusions=inclusion_params(shape, seed), delta_rel=delta_rel, q=q, seed=seed)


def noise_torch(shape, seed, device="cuda"):
    """Standard normal draws on the data grid from torch's generator on the
    device (for instances generated in bulk on the GPU)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 7_000_003)
    return torch.randn(shape, generator=gen, device=device, dtype=torch.float32)


def xi_torch(shape, inclusions, device="cuda"):
    """``xi_inclusions`` evaluated with torch on the device (same formula)."""
    import torch
    nz, ny, nx = shape
    z = (torch.arange(nz, device=device, dtype=torch.float32) + 0.5).view(nz, 1, 1)
    y = (torch.arange(ny, device=device, dtype=torch.float32) + 0.5).view(1, ny, 1)
    x = (torch.arange(nx, device=device, dtype=torch.float32) + 0.5).view(1, 1, nx)
    xi = torch.zeros(shape, device=device, dtype=torch.float32)
    for kind, c, a, size in inclusions:
        if kind == "gauss":
            r2 = (x - float(c[0])) ** 2 + (y - float(c[1])) ** 2 + (z - float(c[2])) ** 2
            xi += float(a) * torch.exp(-r2 / (2.0 * float(size) ** 2))
        else:
            h = float(size) / 2
            m = ((x - float(c[0])).abs() <= h) & ((y - float(c[1])).abs() <= h) & ((z - float(c[2])).abs() <= h)
            xi += float(a) * m.to(torch.float32)
    return xi


# ---------------------------------------------------------------- the model example (Sec. 6)
# R = [-10, 10]^2 x [1, 2], Y = [-10, 10]^2 x [6, 7], ten point sources at
# (0, 0), (+-8, 0), (0, +-8) and heights 3 and 5; c0 = 0.5; g(t) = e^-t
# (A0 = 1).  On n x n x nz cells: h = 20/n, hz = 1/nz, Y's bottom 5 = D hz
# above R's, so D = 5 nz; the library's default source cross (lateral centre
# and +-0.4 n, heights nz + G/4 and nz + 3G/4 with G = D - nz) lands on the
# paper's points exactly.

MODEL_C0 = 0.5


def model_geometry(n: int, nz: int):
    """dict(nx, ny, nz, h, hz, D) of the model example on n x n x nz cells."""
    return dict(nx=n, ny=n, nz=nz, h=20.0 / n, hz=1.0 / nz, D=5.0 * nz)


def model_xi(n: int, nz: int, xp=np, device=None):
    """The model solution xi(x, y, z) at R's cell centres ([nz][n][n]); the
    printed formula is garbled in two places and is read with z in a2 and a3
    and +(y + 4)^2 in the third exponent, which makes every exponent
    negative definite."""
    h, hz = 20.0 / n, 1.0 / nz
    if xp is np:
        ar = lambda m: np.arange(m, dtype=np.float64)  # noqa: E731
    else:
        ar = lambda m: xp.arange(m, dtype=xp.float64, device=device)  # noqa: E731
    x = (-10.0 + (ar(n) + 0.5) * h).reshape(1, 1, n)
    y = (-10.0 + (ar(n) + 0.5) * h).reshape(1, n, 1)
    z = (1.0 + (ar(nz) + 0.5) * hz).reshape(nz, 1, 1)
    zero = 0.0 * z
    a1 = (1.0 - 4.0 * (z - 1.5) ** 2) ** 2
    a2 = 0.4 * xp.maximum(1.0 - (z - 1.3) ** 2, zero)
    a3 = 0.2 * xp.maximum((1.0 - (z - 1.7) ** 2) ** 2, zero)
    u, v = x + 4.0, y - 5.0
    p, q = x - 4.0, y + 4.0
    return (a1 * xp.exp(-x ** 2 - 2.0 * y ** 2)
            + a2 * xp.exp(-3.0 * u ** 2 - v ** 2 + u * v)
            + a3 * xp.exp(-0.9 * (p ** 2 + q ** 2 + p * q)))


def model_noise(shape, seed: int, amplitude: float):
    """Perturbation of the data: uniform in [-amplitude, amplitude] (Sec. 6
    perturbs with a maximum of about 1e-8)."""
    return rng(seed + 11_000_017).uniform(-amplitude, amplitude, size=shape)


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
