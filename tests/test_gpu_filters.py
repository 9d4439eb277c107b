"""GPU parity of the regularising filters of Sec. 5 (iterated Tikhonov,
truncated SVD) in the fused prologue of the inverse z pass, through the C-ABI,
against the oracle's spectral filters (themselves pinned to explicit-matrix
normal equations and SVD)."""
import numpy as np
import pytest

from oracle import discrepancy, tikhonov
from oracle.geometry import sample_kernel

from gpu_helpers import geom, instance, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fr3d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_01216_amd import fr3d as m
    return m


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def tsvd_cut(khat, frac):
    """A cut half-way between two well separated values of s = |k^|^2."""
    s = np.unique(np.round(np.abs(khat).ravel() ** 2, 12))
    i = int(frac * len(s))
    while s[i + 1] - s[i] < 1e-6 * s[-1]:
        i += 1
    return 0.5 * (s[i] + s[i + 1])


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("method,order", [(1, 1), (1, 3), (1, 8), (2, 1)])
@pytest.mark.parametrize("shape", [(16, 12, 8), (32, 32, 32)])
def test_filter_solve_alpha(fr3d, precision, method, order, shape):
    nx, ny, nz = shape
    g = geom(nx, ny, nz)
    d = instance(g, 31, 0.02)
    khat = np.fft.fftn(sample_kernel(g))
    alpha = tsvd_cut(khat, 0.6) if method == 2 else 3e-4
    c = fr3d.Context()
    c.load_kernel(nx, ny, nz, precision=precision)
    c.set_filter(method, order)
    dt = torch.float64 if precision == 64 else torch.float32
    F = torch.tensor(d["F"], dtype=dt, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    rep = c.solve_alpha(alpha, z)
    ref = tikhonov.solve_spectral(g, khat, host(F), alpha, method=method, order=order)
    tol = 1e-11 if precision == 64 else 1e-5
    assert rel_l2(host(z), ref["zeta"]) < tol
    assert rep["residual"] == pytest.approx(ref["r_norm"], rel=10 * tol)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=10 * tol)


@pytest.mark.parametrize("method,order,K", [(1, 2, 0), (1, 4, 16), (2, 1, 0)])
def test_filter_discrepancy_fp64_matches_rule(fr3d, method, order, K):
    g = geom(16, 16, 16)
    d = instance(g, 33, 0.03)
    khat = np.fft.fftn(sample_kernel(g))
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=64)
    c.set_filter(method, order)
    F = torch.tensor(d["F"], dtype=torch.float64, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    rep = c.solve_discrepancy(z, candidates=K)

    def ev(a):
        o = tikhonov.solve_spectral(g, khat, d["F"], a, method=method, order=order)
        return o["r_norm"], o["zeta_norm"]
    ref = discrepancy.kary(ev, d["delta"], K=K) if K else discrepancy.bisection(ev, d["delta"])
    assert rep["flags"] == ref["flags"]
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    o = tikhonov.solve_spectral(g, khat, d["F"], ref["alpha"], method=method, order=order)
    assert rel_l2(host(z), o["zeta"]) < 1e-11


def test_filter_errors_and_graph_recapture(fr3d):
    g = geom(16, 16, 16)
    d = instance(g, 34, 0.02)
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=32)
    for kind, order in ((3, 1), (-1, 1), (1, 0), (1, 65)):
        with pytest.raises(fr3d.Fr3dError) as ei:
            c.set_filter(kind, order)
        assert ei.value.status == fr3d.E_INVALID
    F = torch.tensor(d["F"], dtype=torch.float32, device="cuda")
    c.set_data(F, d["delta"])
    # eager references for Tikhonov and iterated Tikhonov of order 3
    z_t, z_i = torch.empty_like(F), torch.empty_like(F)
    c.solve_alpha(1e-4, z_t)
    c.set_filter(1, 3)
    c.solve_alpha(1e-4, z_i)
    c.set_filter(0, 1)
    # with graphs: the captured evaluation follows a filter change
    c.set_graphs(True)
    z = torch.empty_like(F)
    c.solve_alpha(1e-4, z)
    torch.cuda.synchronize()
    assert np.array_equal(host(z), host(z_t))
    c.set_filter(1, 3)
    c.solve_alpha(1e-4, z)
    torch.cuda.synchronize()
    assert np.array_equal(host(z), host(z_i))
    c.set_graphs(False)
