"""GPU checks of the solves that write their report to device memory
(fr3d_solve_alpha_dev, fr3d_solve_discrepancy_dev), through the C-ABI.

* The enqueued search takes the same evaluations as the synchronous call:
  zeta bit for bit, the same flags and evaluation counts, the same norms
  (to the rounding of the device's pow and sqrt), for the plain rule, the
  seeded secant search, the K-candidate search and a fixed alpha, FP32 and
  FP64; in FP64 the alpha and zeta also match the oracle's rule.
* Captured with set_data into a HIP graph (torch.cuda.graph on the context's
  stream), the solve replays on new data in the captured buffer: every
  replay, with eager solves and synchronisations between replays, equals the
  eager synchronous solve of that data.
"""
import ctypes

import numpy as np
import pytest

from oracle import discrepancy, mlp, tikhonov
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


def rep_buffer(fr3d):
    return torch.zeros(ctypes.sizeof(fr3d.Report), dtype=torch.uint8, device="cuda")


def bias_predictor(c, bias):
    # a network whose output is its last bias: the seed is that log10 alpha
    p = mlp.init_params(13)
    for k in ("W1", "W2", "w3"):
        p[k] = p[k] * 0.0
    p["b3"][:] = bias
    flat = np.concatenate([p[name].ravel() for name, _ in mlp.PARAM_SHAPES]).astype(np.float32)
    nm = np.zeros(132, np.float32)
    nm[65:130] = 1.0
    nm[131] = 1.0
    c.predictor_set(flat, nm)


SEARCHES = {
    "bisection": {},
    "secant": dict(use_predictor=1, seed_slope=0.3, max_steps=8),
    "kary4": dict(candidates=4, max_steps=6),
    "walk": dict(use_predictor=1, max_steps=8),
}


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("search", sorted(SEARCHES))
def test_dev_report_equals_synchronous(fr3d, precision, search):
    g = geom(16, 16, 16)
    d = instance(g, 83, 0.02)
    dt = torch.float64 if precision == 64 else torch.float32
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=precision)
    bias_predictor(c, -3.0)
    F = torch.tensor(d["F"], dtype=dt, device="cuda")
    opts = dict(tol=1e-6, **SEARCHES[search])
    c.set_data(F, d["delta"])
    z_sync = torch.empty_like(F)
    ref = c.solve_discrepancy(z_sync, **opts)
    c.set_data(F, d["delta"])
    z_dev = torch.full_like(F, float("nan"))
    rb = rep_buffer(fr3d)
    c.solve_discrepancy_dev(z_dev, rb, **opts)
    torch.cuda.synchronize()
    rep = fr3d.Report.from_device(rb)
    print(search, precision, ref["n_evals"], ref["flags"], rep["n_evals"], rep["flags"], flush=True)
    assert rep["flags"] == ref["flags"] and not rep["flags"] & fr3d.UNFINISHED
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-14)
    # the device's pow and sqrt against the host's: to the last bit or two
    for k in ("residual", "zeta_norm", "target"):
        assert rep[k] == pytest.approx(ref[k], rel=4e-16), k
    for k in ("delta", "residual_full_box", "n_clamped"):
        assert rep[k] == ref[k], k
    assert torch.equal(z_dev, z_sync)
    if precision == 64 and search == "bisection":
        khat = np.fft.fftn(sample_kernel(g))

        def ev(a):
            o = tikhonov.solve_spectral(g, khat, d["F"], a)
            return o["r_norm"], o["zeta_norm"]
        orc = discrepancy.bisection(ev, d["delta"], tol=1e-6)
        assert rep["flags"] == orc["flags"] and rep["n_evals"] == orc["n_evals"]
        assert rep["alpha"] == pytest.approx(orc["alpha"], rel=1e-12)
        o = tikhonov.solve_spectral(g, khat, d["F"], orc["alpha"])
        assert rel_l2(z_dev.cpu().numpy(), o["zeta"]) < 1e-11


@pytest.mark.parametrize("precision", [32, 64])
def test_dev_fixed_alpha_and_errors(fr3d, precision):
    g = geom(16, 16, 16)
    d = instance(g, 84, 0.02)
    dt = torch.float64 if precision == 64 else torch.float32
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=precision)
    F = torch.tensor(d["F"], dtype=dt, device="cuda")
    rb = rep_buffer(fr3d)
    z = torch.empty_like(F)
    with pytest.raises(fr3d.Fr3dError) as ei:  # no data yet
        c.solve_alpha_dev(1e-3, z, rb)
    assert ei.value.status == fr3d.E_STATE
    c.set_data(F, d["delta"])
    z_sync = torch.empty_like(F)
    ref = c.solve_alpha(1e-3, z_sync)
    c.solve_alpha_dev(1e-3, z, rb)
    torch.cuda.synchronize()
    rep = fr3d.Report.from_device(rb)
    assert rep["n_evals"] == 1 and rep["flags"] == ref["flags"]
    assert rep["residual"] == pytest.approx(ref["residual"], rel=4e-16)
    assert rep["zeta_norm"] == pytest.approx(ref["zeta_norm"], rel=4e-16)
    assert rep["alpha"] == pytest.approx(1e-3, rel=1e-14)
    assert torch.equal(z, z_sync)
    lib = fr3d.lib()
    for a in (0.0, -1.0, float("nan")):
        assert lib.fr3d_solve_alpha_dev(c._ctx, a, ctypes.c_void_p(z.data_ptr()),
                                        ctypes.c_void_p(rb.data_ptr())) == fr3d.E_INVALID
    assert lib.fr3d_solve_alpha_dev(c._ctx, 1e-3, ctypes.c_void_p(z.data_ptr()), None) == fr3d.E_INVALID
    o = fr3d.default_opts(tol=-1.0)
    assert lib.fr3d_solve_discrepancy_dev(c._ctx, ctypes.byref(o), ctypes.c_void_p(z.data_ptr()),
                                          ctypes.c_void_p(rb.data_ptr())) == fr3d.E_INVALID
    c.set_timing(True)
    with pytest.raises(fr3d.Fr3dError) as ei:
        c.solve_discrepancy_dev(z, rb)
    assert ei.value.status == fr3d.E_STATE
    c.set_timing(False)


def test_dev_search_captured_in_graph_replays(fr3d):
    # set_data + the learned secant search captured once; each replay solves
    # the data then in the captured buffer
    n = 32
    g = geom(n, n, n)
    c = fr3d.Context()
    c.load_kernel(n, n, n, precision=32)
    bias_predictor(c, -4.0)
    opts = dict(use_predictor=1, seed_slope=0.05, max_steps=6, tol=1e-3)
    datas = [instance(g, 90 + i, 0.02 + 0.01 * i) for i in range(3)]
    delta = datas[0]["delta"]  # the captured delta is used by every replay
    F = torch.tensor(datas[0]["F"], dtype=torch.float32, device="cuda")
    z = torch.empty_like(F)
    rb = rep_buffer(fr3d)
    s = torch.cuda.Stream()
    c.set_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        c.set_data(F, delta)
        c.solve_discrepancy_dev(z, rb, **opts)
    torch.cuda.synchronize()
    c.set_stream(torch.cuda.current_stream())
    z_ref = torch.empty_like(F)
    for rnd in range(2):
        for i, dd in enumerate(datas):
            F.copy_(torch.tensor(dd["F"], dtype=torch.float32))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            rep = fr3d.Report.from_device(rb)
            # eager reference on the same context between replays
            c.set_data(F, delta)
            ref = c.solve_discrepancy(z_ref, **opts)
            print("replay", rnd, i, rep["n_evals"], rep["flags"], ref["n_evals"], ref["flags"], flush=True)
            assert rep["flags"] == ref["flags"] and rep["n_evals"] == ref["n_evals"]
            assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-14)
            assert rep["residual"] == pytest.approx(ref["residual"], rel=4e-16)
            assert torch.equal(z, z_ref)
