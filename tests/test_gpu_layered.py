"""GPU parity of Algorithm 1 with per-frequency z-systems (Sec. 5, Eq. (14)),
through the C-ABI, against the oracle (oracle/layered.py, pinned to the
direct quadrature of Eq. (8) and to the explicit assembled operator).

Tolerances: the forward operator is exact quadrature (FP64 1e-12, FP32
1e-5).  Regularised estimates go through an SVD of every system, computed
by one-sided Jacobi on the device and by LAPACK in the oracle; the filter
function of A^T A is unique, and the two differ by about eps s_max / alpha
(s_max the largest squared singular value), so the FP64 bar is 1e-9 up to
s_max / alpha = 1e6 and grows in proportion beyond it; the FP32 bar is the
1e-5 of the precision split.
"""
import numpy as np
import pytest

from oracle import discrepancy, layered
from oracle.operator import forward_direct

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


def ctx_layered(fr3d, g, precision):
    c = fr3d.Context()
    c.load_layered(g.nx, g.ny, g.nz, h=g.h, D=g.d, kind=g.kind, precision=precision)
    return c


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("shape,kind", [((8, 6, 5), 0), ((6, 8, 4), 1), ((16, 16, 9), 0)])
def test_layered_forward_equals_direct_quadrature(fr3d, precision, shape, kind):
    nx, ny, nz = shape
    g = geom(nx, ny, nz, kind=kind)
    c = ctx_layered(fr3d, g, precision)
    z = np.random.default_rng(41).standard_normal(g.shape)
    zd = dev(z, precision)
    out = torch.empty_like(zd)
    c.apply_operator(zd, out)
    ref = forward_direct(g, host(zd))
    assert rel_l2(host(out), ref) < (1e-12 if precision == 64 else 1e-5)


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("method,order", [(0, 1), (1, 3), (2, 1)])
@pytest.mark.parametrize("shape", [(16, 12, 8), (16, 16, 51), (32, 32, 16)])
def test_layered_solve_alpha(fr3d, precision, method, order, shape):
    nx, ny, nz = shape
    g = geom(nx, ny, nz)
    d = instance(g, 43, 0.02)
    kt = layered.lateral_kernel_spectrum(g)
    alpha = 1e-4
    if method == 2:  # a cut half-way between two well separated squared singular values
        lam = np.unique(np.round(np.linalg.svd(layered.system_matrices(g, kt), compute_uv=False) ** 2, 10))
        i = int(0.5 * len(lam))
        while lam[i + 1] - lam[i] < 1e-6 * lam[-1]:
            i += 1
        alpha = 0.5 * (lam[i] + lam[i + 1])
    c = ctx_layered(fr3d, g, precision)
    c.set_filter(method, order)
    F = dev(d["F"], precision)
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    rep = c.solve_alpha(alpha, z)
    ref = layered.solve_layered(g, kt, host(F), alpha, method, order)
    tol = 1e-9 if precision == 64 else 1e-5
    assert rel_l2(host(z), ref["zeta"]) < tol
    assert rep["residual"] == pytest.approx(ref["r_norm"], rel=tol)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=tol)
    assert c.get_smax() == pytest.approx(float((ref["singular_values"] ** 2).max()), rel=1e-12)


@pytest.mark.parametrize("K", [0, 16])
@pytest.mark.parametrize("delta_rel", [0.01, 0.05])
def test_layered_discrepancy_fp64_matches_rule(fr3d, K, delta_rel):
    g = geom(16, 16, 12)
    d = instance(g, 44, delta_rel)
    kt = layered.lateral_kernel_spectrum(g)
    c = ctx_layered(fr3d, g, 64)
    F = dev(d["F"], 64)
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    rep = c.solve_discrepancy(z, candidates=K)

    def ev(a):
        o = layered.solve_layered(g, kt, d["F"], a)
        return o["r_norm"], o["zeta_norm"]
    ref = discrepancy.kary(ev, d["delta"], K=K) if K else discrepancy.bisection(ev, d["delta"])
    assert rep["flags"] == ref["flags"]
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    o = layered.solve_layered(g, kt, d["F"], ref["alpha"])
    # the SVD-route bar scales with the regularised system's condition s_max / alpha
    assert rel_l2(host(z), o["zeta"]) < 1e-9 * max(1.0, c.get_smax() / rep["alpha"] / 1e6)


def test_layered_batch_equals_single_and_errors(fr3d):
    g = geom(16, 12, 10)
    items = [instance(g, 50 + i, (0.01, 0.03, 0.05)[i % 3]) for i in range(4)]
    Fs = [dev(d["F"], 32) for d in items]
    deltas = [d["delta"] for d in items]
    c = ctx_layered(fr3d, g, 32)
    single = []
    for F, dl in zip(Fs, deltas):
        z = torch.empty_like(F)
        c.set_data(F, dl)
        single.append((c.solve_discrepancy(z), z))
    c.set_lanes(3)
    zs = [torch.empty_like(F) for F in Fs]
    reps = c.solve_batch(Fs, deltas, zs)
    torch.cuda.synchronize()
    for (r1, z1), r2, z2 in zip(single, reps, zs):
        assert np.array_equal(host(z1), host(z2))
        assert r1["alpha"] == r2["alpha"] and r1["n_evals"] == r2["n_evals"]
    with pytest.raises(fr3d.Fr3dError) as ei:
        c.solve_discrepancy(zs[0], use_predictor=1)
    assert ei.value.status == fr3d.E_STATE
    with pytest.raises(fr3d.Fr3dError) as ei:
        c.get_octant()
    assert ei.value.status == fr3d.E_STATE
    with pytest.raises(fr3d.Fr3dError) as ei:
        c.load_layered(16, 16, 61)
    assert ei.value.status == fr3d.E_INVALID


def test_layered_versus_3d_embedding(fr3d):
    """The two forms share the forward operator but regularise different
    problems (z embedded or exact); at the same alpha their estimates differ
    by the z-padding gap, which is reported, not bounded."""
    g = geom(32, 32, 16)
    d = instance(g, 45, 0.02)
    F = dev(d["F"], 64)
    c3 = fr3d.Context()
    c3.load_kernel(32, 32, 16, precision=64)
    cl = ctx_layered(fr3d, g, 64)
    z0 = torch.empty_like(F)
    o3, ol = torch.empty_like(F), torch.empty_like(F)
    c3.apply_operator(F, o3)
    cl.apply_operator(F, ol)
    assert rel_l2(host(ol), host(o3)) < 1e-12
    c3.set_data(F, d["delta"])
    cl.set_data(F, d["delta"])
    r3 = c3.solve_alpha(1e-4, z0)
    z1 = torch.empty_like(F)
    rl = cl.solve_alpha(1e-4, z1)
    gap = rel_l2(host(z1), host(z0))
    print(f"[layered vs 3D] alpha 1e-4: zeta gap {gap:.3e}, residuals {rl['residual']:.6e} / {r3['residual']:.6e}")
    assert np.isfinite(gap) and gap > 0
    # both fit the data on Y to the same order at this alpha
    assert 1 / 1.5 <= rl["residual"] / r3["residual"] <= 1.5


def _pf_case(fr3d, g, seed, delta_rel, precision, **kw):
    d = instance(g, seed, delta_rel)
    c = ctx_layered(fr3d, g, precision)
    F = dev(d["F"], precision)
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    kxn = g.pshape[2] // 2 + 1
    al = torch.zeros((kxn, g.pshape[1]), dtype=torch.float64, device="cuda")
    fl = torch.zeros((kxn, g.pshape[1]), dtype=torch.int32, device="cuda")
    rep = c.solve_per_frequency(z, al, fl, **kw)
    ref = layered.solve_per_frequency(g, layered.lateral_kernel_spectrum(g), d["F"], d["delta"], **kw)
    # library [kx][ky] for kx <= Px/2 against the oracle's [ky][kx]
    return c, d, z, rep, ref, host(al), fl.cpu().numpy(), ref["alphas"][:, :kxn].T, ref["flags"][:, :kxn].T


@pytest.mark.parametrize("shape,seed,delta_rel", [((16, 16, 12), 45, 0.01), ((12, 8, 7), 46, 0.05),
                                                  ((24, 12, 9), 47, 0.02)])
def test_per_frequency_alphas_fp64_match_oracle(fr3d, shape, seed, delta_rel):
    # Algorithm 1 step 2 per lateral frequency: the same plain rule on every
    # system; every decision, alpha and flag agrees, and the estimate within
    # the SVD-route bar of the smallest alpha chosen
    g = geom(*shape)
    c, d, z, rep, ref, al, fl, ral, rfl = _pf_case(fr3d, g, seed, delta_rel, 64)
    assert np.array_equal(fl, rfl)
    assert np.allclose(al, ral, rtol=1e-12, atol=0)
    assert len(set(rfl.ravel().tolist())) >= 2          # several outcomes among the systems
    bar = 1e-9 * max(1.0, c.get_smax() / ral.min() / 1e6)
    assert rel_l2(host(z), ref["zeta"]) < bar
    assert rep["residual"] == pytest.approx(ref["r_norm"], rel=bar)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=bar)
    assert rep["alpha"] == pytest.approx(10.0 ** np.log10(ref["alphas"]).mean(), rel=1e-12)
    want = 0
    for v in np.unique(ref["flags"]):
        want |= int(v)
    assert rep["flags"] == want and rep["n_evals"] == 1


@pytest.mark.parametrize("filt", [1, 2])
def test_per_frequency_filters_fp64_match_oracle(fr3d, filt):
    # the same rule with the iterated-Tikhonov (order 3) and TSVD filters
    g = geom(12, 12, 8)
    d = instance(g, 48, 0.02)
    c = ctx_layered(fr3d, g, 64)
    c.set_filter(filt, 3 if filt == 1 else 1)
    F = dev(d["F"], 64)
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    kxn = g.pshape[2] // 2 + 1
    al = torch.zeros((kxn, g.pshape[1]), dtype=torch.float64, device="cuda")
    fl = torch.zeros((kxn, g.pshape[1]), dtype=torch.int32, device="cuda")
    c.solve_per_frequency(z, al, fl)
    ref = layered.solve_per_frequency(g, layered.lateral_kernel_spectrum(g), d["F"], d["delta"], method=filt,
                                      order=3 if filt == 1 else 1)
    assert np.array_equal(fl.cpu().numpy(), ref["flags"][:, :kxn].T)
    assert np.allclose(host(al), ref["alphas"][:, :kxn].T, rtol=1e-12, atol=0)
    bar = 1e-9 * max(1.0, c.get_smax() / ref["alphas"].min() / 1e6)
    assert rel_l2(host(z), ref["zeta"]) < bar


def test_per_frequency_fp32_bisection_to_the_end(fr3d):
    # FP32: with tol = 0 every search bisects to the end, so a decision that
    # FP32 rounding flips (rho within rounding of zero) moves the final alpha
    # only by the last interval, and the alphas differ by the shift of each
    # system's root: a relative error u in its residual moves log10 alpha by
    # u / s, s = d ln||r|| / d log10 alpha at the root (computed here by
    # dense solves of the system).  The FP32 spectrum carries u <~ 1e-5 of
    # the per-frequency residual (the transform's rounding, ~1e-7 of ||F||,
    # against residuals ~delta = 2e-2 ||F||).  The estimate moves less
    # than 1e-4: large shifts belong to flat residuals, whose x barely moves.
    g = geom(16, 16, 12)
    kw = dict(tol=0.0, max_steps=40)
    c, d, z, rep, ref, al, fl, ral, rfl = _pf_case(fr3d, g, 49, 0.02, 32, **kw)
    ends = rfl != discrepancy.MAXITER
    assert np.array_equal(fl[ends], rfl[ends]) and np.all(fl[~ends] == discrepancy.MAXITER)
    assert np.allclose(al[ends], ral[ends], rtol=1e-14, atol=0)
    A = layered.system_matrices(g, layered.lateral_kernel_spectrum(g))
    fh = np.moveaxis(layered.lateral_spectrum(g, d["F"]), 0, 2)
    for kx, ky in zip(*np.nonzero(~ends)):
        Am, f = A[ky, kx], fh[ky, kx]

        def lnr(t):
            x = np.linalg.solve(Am.T @ Am + 10.0 ** t * np.eye(Am.shape[1]), Am.T @ f)
            return np.log(np.linalg.norm(Am @ x - f))
        t = np.log10(ral[kx, ky])
        slope = (lnr(t + 1e-4) - lnr(t - 1e-4)) / 2e-4
        assert abs(np.log10(al[kx, ky]) - t) <= 1e-5 / slope + 1e-10, (kx, ky, slope)
    assert rel_l2(host(z), ref["zeta"]) < 1e-4


def test_per_frequency_single_alpha_equals_global_and_errors(fr3d):
    # a range of width ~0 pins every system to one alpha: the global estimate
    g = geom(12, 12, 8)
    d = instance(g, 50, 0.02)
    c = ctx_layered(fr3d, g, 64)
    F = dev(d["F"], 64)
    c.set_data(F, d["delta"])
    z1, z2 = torch.empty_like(F), torch.empty_like(F)
    c.solve_per_frequency(z1, log10_alpha_lo=-3.0, log10_alpha_hi=-3.0 + 1e-12, tol=0.0, max_steps=0)
    c.solve_alpha(1e-3, z2)
    assert rel_l2(host(z1), host(z2)) < 1e-11
    for kw in ({"candidates": 4}, {"h_op": 0.1}, {"mu": 0.1}):
        with pytest.raises(fr3d.Fr3dError) as ei:
            c.solve_per_frequency(z1, **kw)
        assert ei.value.status == fr3d.E_INVALID
    c3 = fr3d.Context()
    c3.load_kernel(12, 12, 8, precision=64)
    c3.set_data(F, d["delta"])
    with pytest.raises(fr3d.Fr3dError) as ei:
        c3.solve_per_frequency(z1)
    assert ei.value.status == fr3d.E_STATE


@pytest.mark.parametrize("precision", [64, 32])
def test_singular_values_against_oracle(fr3d, precision):
    # Fig. 6's quantity: the singular values of every distinct system, from
    # the one-sided Jacobi SVD on the device, against LAPACK on the oracle's
    # assembled systems (absolute error ~eps ||A||)
    g = geom(16, 12, 9)
    c = ctx_layered(fr3d, g, precision)
    sv = host(c.get_singular_values())
    A = layered.system_matrices(g, layered.lateral_kernel_spectrum(g))
    S = np.linalg.svd(A, compute_uv=False)                     # [Py][Px][M], descending
    kxn, pyh = g.pshape[2] // 2 + 1, g.pshape[1] // 2 + 1
    ref = np.transpose(S[:pyh, :kxn], (1, 0, 2))
    assert sv.shape == ref.shape
    assert np.abs(sv - ref).max() <= 1e-12 * ref.max()
    assert np.all(np.diff(sv, axis=2) <= 0)
    with pytest.raises(fr3d.Fr3dError) as ei:
        c3 = fr3d.Context()
        c3.load_kernel(8, 8, 8, precision=64)
        c3.get_singular_values()
    assert ei.value.status == fr3d.E_STATE
