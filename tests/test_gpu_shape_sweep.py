"""Parity sweep over grid shapes (GPU against the oracle, through the
C-ABI): every compiled transform length up to 96 on every axis (n = 2 ... 48,
so P = 4 ... 96 with the radix-3 lengths), in seeded random anisotropic
combinations, FP64 and FP32, with seeded random tile variants per pass (the
smaller tiles exist from length 64 up).  Each case: the data spectrum, the
estimate at a fixed alpha and its norms against the oracle's spectral
Tikhonov solve (FP64 1e-11, FP32 1e-5 relative)."""
import numpy as np
import pytest

from oracle import tikhonov
from oracle.geometry import sample_kernel
from oracle.operator import pad

from gpu_helpers import geom, half_spectrum, instance, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LENS = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48]


def sweep_shapes():
    rg = np.random.default_rng(2024)
    shapes = []
    for ax in range(3):
        for n in LENS:
            s = [int(rg.choice(LENS)) for _ in range(3)]
            s[ax] = n
            if tuple(s) not in shapes:
                shapes.append(tuple(s))
    return shapes


SHAPES = sweep_shapes()


@pytest.fixture(scope="module")
def fr3d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_01216_amd import fr3d as m
    return m


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_shape_sweep(fr3d, shape, precision):
    nx, ny, nz = shape
    g = geom(nx, ny, nz)
    d = instance(g, 300 + nx * 10000 + ny * 100 + nz, 0.01)
    c = fr3d.Context()
    c.load_kernel(nx, ny, nz, h=g.h, D=g.d, kind=g.kind, precision=precision)
    rg = np.random.default_rng(nx * 10000 + ny * 100 + nz + precision)
    for p in range(6):
        c.set_tile(p, int(rg.integers(0, 3 if p in (0, 1, 3, 4) else 2)))
    dt = torch.float64 if precision == 64 else torch.float32
    F = torch.tensor(np.ascontiguousarray(d["F"]), dtype=dt, device="cuda")
    Fh = F.cpu().numpy().astype(np.float64)
    print("shape", shape, "precision", precision, flush=True)
    c.set_data(F, d["delta"])
    tol = 1e-11 if precision == 64 else 1e-5
    ref_s = half_spectrum(np.fft.fftn(pad(g, Fh)), g)
    got = c.get_data_spectrum().cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    assert np.abs(got - ref_s).max() < (1e-13 if precision == 64 else 2e-6) * np.abs(ref_s).max()
    zeta = torch.empty_like(F)
    rep = c.solve_alpha(1e-3, zeta)
    ref = tikhonov.solve_spectral(g, np.fft.fftn(sample_kernel(g)), Fh, 1e-3)
    assert rel_l2(zeta.cpu().numpy().astype(np.float64), ref["zeta"]) < tol
    assert rep["residual"] == pytest.approx(ref["r_norm"], rel=tol * 10)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=tol * 10)
