"""GPU parity of Tikhonov for the exact restricted operator (CG on the normal
equations, through the C-ABI) against the oracle (oracle/exact.py: CG with
numpy transforms, pinned to dense normal equations and to the direct adjoint
sum).

Bars: FP64 1e-9 relative L2 (both sides iterate to 1e-12 of the
normal-equation residual; the estimate's error is that times the condition
number of A^T A + alpha I, <= 1e3 at the alphas used).  FP32: every product
with A and A^T carries FP32 rounding (~1e-7 relative), which CG turns into
an error of about 1e-7 times cond = (s_max + alpha)/alpha (s_max = max
|k^|^2 bounds ||A||^2); the bar is ten times that, at least 1e-4.
"""
import numpy as np
import pytest

from oracle import discrepancy, exact
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


def dev(a, precision):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if precision == 64 else torch.float32,
                        device="cuda")


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape,alpha", [((4, 3, 3), 1e-1), ((16, 12, 8), 1e-2), ((24, 24, 16), 3e-2)])
def test_exact_solve_against_oracle(fr3d, precision, shape, alpha):
    nx, ny, nz = shape
    g = geom(nx, ny, nz)
    d = instance(g, 61, 0.02)
    c = fr3d.Context()
    c.load_kernel(nx, ny, nz, precision=precision)
    F = dev(d["F"], precision)
    z = torch.empty_like(F)
    tol = 1e-12 if precision == 64 else 1e-6
    rep = c.solve_exact(F, alpha, z, max_iter=5000, tol=tol)
    Fh = host(F)
    ref = exact.dense_exact(g, Fh, alpha) if nx * ny * nz <= 64 else exact.cg_exact(g, Fh, alpha, tol=1e-13)
    cond = (c.get_smax() + alpha) / alpha
    bar = 1e-9 if precision == 64 else max(1e-4, 1e-6 * cond)
    assert rel_l2(host(z), ref["zeta"]) < bar
    assert rep["residual"] == pytest.approx(ref["r_norm"], rel=bar)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=bar)
    assert rep["flags"] == 0 and rep["n_evals"] > 0


def test_exact_layered_form_gives_the_same_estimate(fr3d):
    # both forms apply the same exact operator and its adjoint
    g = geom(16, 16, 12)
    d = instance(g, 62, 0.02)
    F = dev(d["F"], 64)
    out = []
    for layered_form in (False, True):
        c = fr3d.Context()
        if layered_form:
            c.load_layered(16, 16, 12, precision=64)
        else:
            c.load_kernel(16, 16, 12, precision=64)
        z = torch.empty_like(F)
        c.solve_exact(F, 1e-2, z, max_iter=5000, tol=1e-12)
        out.append(host(z))
    assert rel_l2(out[1], out[0]) < 1e-9


def test_exact_discrepancy_fp64_matches_rule(fr3d):
    g = geom(12, 12, 8)
    d = instance(g, 63, 0.05)
    khat = np.fft.fftn(sample_kernel(g))
    c = fr3d.Context()
    c.load_kernel(12, 12, 8, precision=64)
    F = dev(d["F"], 64)
    z = torch.empty_like(F)
    rep = c.solve_exact_discrepancy(F, d["delta"], z, max_iter=20000, tol=1e-12, log10_alpha_lo=-4.0)

    def ev(a):
        o = exact.cg_exact(g, d["F"], a, tol=1e-13, max_iter=20000, khat=khat)
        return o["r_norm"], o["zeta_norm"]
    ref = discrepancy.bisection(ev, d["delta"], lo=-4.0)
    assert rep["flags"] == ref["flags"]
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    o = exact.cg_exact(g, d["F"], ref["alpha"], tol=1e-13, max_iter=20000, khat=khat)
    assert rel_l2(host(z), o["zeta"]) < 1e-7


def test_exact_errors_and_iteration_limit(fr3d):
    c = fr3d.Context()
    c.load_kernel(8, 8, 8, precision=32)
    F = torch.ones((8, 8, 8), dtype=torch.float32, device="cuda")
    z = torch.empty_like(F)
    for kw in ({"max_iter": 0}, {"tol": 0.0}):
        with pytest.raises(fr3d.Fr3dError) as ei:
            c.solve_exact(F, 1e-2, z, **kw)
        assert ei.value.status == fr3d.E_INVALID
    with pytest.raises(fr3d.Fr3dError) as ei:
        c.solve_exact_discrepancy(F, 0.1, z, candidates=4)
    assert ei.value.status == fr3d.E_INVALID
    rep = c.solve_exact(F, 1e-6, z, max_iter=1, tol=1e-9)
    assert rep["flags"] == fr3d.CG_LIMIT and rep["n_evals"] == 1
    # zero data: zero estimate without iterations
    rep = c.solve_exact(torch.zeros_like(F), 1e-2, z)
    assert rep["n_evals"] == 0 and float(z.abs().max()) == 0.0
