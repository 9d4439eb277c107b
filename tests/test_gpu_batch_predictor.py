"""GPU checks of the batch scheduler and the alpha predictor, through the C-ABI.

* Batch: every item's zeta and report equal the single-solve results bit for bit
  (the lanes run the same kernels on their own streams).
* Predictor: BF16-MFMA/FP32 forward and gradients against the BF16-emulating
  FP64 oracle on identical weights and inputs (<= 1e-3 relative L2 per
  tensor); Adam against its formula; checkpoint round trip; the seeded search
  takes the oracle rule's decisions (FP64 path).
"""
import math

import numpy as np
import pytest

from oracle import discrepancy, mlp, tikhonov
from oracle.geometry import sample_kernel

from gpu_helpers import geom, instance, oracle_features, rel_l2

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


def flat_params(p):
    return np.concatenate([p[name].ravel() for name, _ in mlp.PARAM_SHAPES]).astype(np.float32)


def unflat(v):
    out, o = {}, 0
    for name, shape in mlp.PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def identity_norm():
    nm = np.zeros(132, np.float32)
    nm[65:130] = 1.0
    nm[131] = 1.0
    return nm


@pytest.mark.parametrize("precision", [32, 64])
def test_batch_equals_single(fr3d, precision):
    g = geom(16, 16, 16)
    dt = torch.float64 if precision == 64 else torch.float32
    items = [instance(g, 60 + i, (0.01, 0.03, 0.05)[i % 3]) for i in range(5)]
    Fs = [torch.tensor(d["F"], dtype=dt, device="cuda") for d in items]
    deltas = [d["delta"] for d in items]
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=precision)
    single = []
    for F, dl in zip(Fs, deltas):
        z = torch.empty_like(F)
        c.set_data(F, dl)
        single.append((c.solve_discrepancy(z), z))
    c.set_lanes(3)
    zs = [torch.empty_like(F) for F in Fs]
    V = torch.empty_like(Fs[0])
    c.source_potential(V)
    cs = [torch.empty_like(F) for F in Fs]
    reps = c.solve_batch(Fs, deltas, zs, V0=V, c0=1.0, c_list=cs)
    torch.cuda.synchronize()
    for (rep1, z1), rep2, z2, cc in zip(single, reps, zs, cs):
        assert np.array_equal(host(z1), host(z2))
        for k in ("alpha", "residual", "zeta_norm", "n_evals", "flags"):
            assert rep1[k] == rep2[k]
        n_cl = c.recover_c(z2, V, 1.0, torch.empty_like(z2))
        assert rep2["n_clamped"] == n_cl


def test_batch_empty_and_errors(fr3d):
    g = geom(8, 8, 8)
    c = fr3d.Context()
    c.load_kernel(8, 8, 8, precision=32)
    assert c.solve_batch([], [], []) == []
    F = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(fr3d.Fr3dError):
        c.solve_batch([F], [-1.0], [torch.empty_like(F)])
    with pytest.raises(fr3d.Fr3dError):
        c.set_lanes(0)


def test_predictor_forward_matches_oracle(fr3d):
    p = mlp.init_params(5)
    flat = flat_params(p)
    p32 = unflat(flat)
    rg = np.random.default_rng(7)
    X = rg.standard_normal((200, 65)).astype(np.float32)
    c = fr3d.Context()
    c.predictor_set(flat, identity_norm())
    y = torch.empty(200, dtype=torch.float32, device="cuda")
    c.predictor_forward(torch.tensor(X, device="cuda"), y)
    yo, _ = mlp.forward(p32, X.astype(np.float64), bf16=True)
    print(f"[predictor] forward rel_l2 {rel_l2(host(y), yo):.3e}", flush=True)
    assert rel_l2(host(y), yo) < 1e-3
    # normalisation and de-normalisation are applied around the network
    nm = identity_norm()
    nm[:65] = 0.5
    nm[65:130] = 2.0
    nm[130], nm[131] = -4.0, 1.5
    c.predictor_set(flat, nm)
    c.predictor_forward(torch.tensor(X, device="cuda"), y)
    yo2, _ = mlp.forward(p32, (X.astype(np.float64) - 0.5) / 2.0, bf16=True)
    assert rel_l2(host(y), -4.0 + 1.5 * yo2) < 1e-3


def test_seed_matches_oracle_network(fr3d):
    # the single-row kernel that seeds a search computes the same network:
    # with the whole range open and any ratio accepted, the search returns
    # 10^(network output on the data's features), features and network
    # from the oracle
    p = mlp.init_params(5)
    flat = flat_params(p)
    p32 = unflat(flat)
    g = geom(24, 16, 12)
    d = instance(g, 72, 0.03)
    c = fr3d.Context()
    c.load_kernel(24, 16, 12, precision=64)
    nm = identity_norm()
    nm[130], nm[131] = -4.0, 1.5
    c.predictor_set(flat, nm)
    F = torch.tensor(d["F"], dtype=torch.float64, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    wide = dict(accept_lo=0.0, accept_hi=1e300, log10_alpha_lo=-60.0, log10_alpha_hi=60.0)
    rep = c.solve_discrepancy(z, use_predictor=1, **wide)
    assert rep["n_evals"] == 1 and rep["flags"] == 0
    x, _, near = oracle_features(g, d["F"], d["delta"])
    assert near == 0
    x = np.asarray(x, dtype=np.float64)
    yo, _ = mlp.forward(p32, x[None, :], bf16=True)
    assert math.log10(rep["alpha"]) == pytest.approx(-4.0 + 1.5 * float(yo[0]), abs=2e-3)
    # a calibration adds coef[0] + sum_k coef[1+k] x_k to the seed
    coef = np.random.default_rng(9).uniform(-0.05, 0.05, 66)
    c.predictor_set_calibration(coef)
    rep = c.solve_discrepancy(z, use_predictor=1, **wide)
    want = -4.0 + 1.5 * float(yo[0]) + coef[0] + float(coef[1:] @ x)
    assert math.log10(rep["alpha"]) == pytest.approx(want, abs=2e-3)
    for bad in ([0.0] * 65, [float("nan")] * 66):
        with pytest.raises(fr3d.Fr3dError) as ei:
            c.predictor_set_calibration(bad)
        assert ei.value.status == fr3d.E_INVALID
    c.predictor_set(flat, nm)  # a new network drops the calibration
    rep = c.solve_discrepancy(z, use_predictor=1, **wide)
    assert math.log10(rep["alpha"]) == pytest.approx(-4.0 + 1.5 * float(yo[0]), abs=2e-3)


def test_predictor_gradients_match_oracle(fr3d):
    p = mlp.init_params(9)
    flat = flat_params(p)
    p32 = unflat(flat)
    rg = np.random.default_rng(8)
    B = 256
    X = rg.standard_normal((B, 65)).astype(np.float32)
    t = rg.standard_normal(B).astype(np.float32)
    c = fr3d.Context()
    c.predictor_set(flat, identity_norm())
    grad = torch.empty(fr3d.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    c.predictor_train_step(torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"), 0.0, loss, grad)
    yo, cache = mlp.forward(p32, X.astype(np.float64), bf16=True)
    go = mlp.backward(p32, cache, t.astype(np.float64), bf16=True)
    gg = unflat(host(grad))
    for name, _ in mlp.PARAM_SHAPES:
        print(f"[predictor] gradient {name} rel_l2 {rel_l2(gg[name], go[name]):.3e}", flush=True)
    for name, _ in mlp.PARAM_SHAPES:
        assert rel_l2(gg[name], go[name]) < 1e-3, name
    assert float(host(loss)[0]) == pytest.approx(mlp.loss(yo, t), rel=1e-3)
    # lr = 0 leaves the parameters alone
    p_after, _ = c.predictor_get()
    assert np.array_equal(p_after, flat)


def test_predictor_adam_step(fr3d):
    flat = flat_params(mlp.init_params(11))
    rg = np.random.default_rng(9)
    X = torch.tensor(rg.standard_normal((64, 65)).astype(np.float32), device="cuda")
    t = torch.tensor(rg.standard_normal(64).astype(np.float32), device="cuda")
    c = fr3d.Context()
    c.predictor_set(flat, identity_norm())
    grad = torch.empty(fr3d.N_PARAMS, dtype=torch.float32, device="cuda")
    c.predictor_train_step(X, t, 1e-3, None, grad)
    p1, _ = c.predictor_get()
    g = host(grad)
    # first Adam step from zero moments: p - lr g / (|g| + eps)  (bias corrected)
    expect = flat.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.abs(p1 - expect).max() < 2e-6
    # the loss decreases over a few steps on a fixed batch
    losses = []
    lt = torch.empty(1, dtype=torch.float32, device="cuda")
    for _ in range(30):
        c.predictor_train_step(X, t, 1e-3, lt, None)
        losses.append(float(host(lt)[0]))
    assert losses[-1] < losses[0]


def test_predictor_checkpoint(fr3d, tmp_path):
    flat = flat_params(mlp.init_params(12))
    nm = identity_norm()
    nm[130] = -3.0
    c = fr3d.Context()
    c.predictor_set(flat, nm)
    path = str(tmp_path / "pred.bin")
    c.predictor_save(path)
    c2 = fr3d.Context()
    c2.predictor_load(path)
    p2, n2 = c2.predictor_get()
    assert np.array_equal(p2, flat) and np.array_equal(n2, nm)
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0xFF
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(fr3d.Fr3dError) as ei:
        c2.predictor_load(bad)
    assert ei.value.status == fr3d.E_INVALID


@pytest.mark.parametrize("bias,slope,tol,shift,snap,ratio", [
    (-3.0, 0.05, 1e-3, 0.0, 0.0, 0.0), (-6.5, 0.5, 1e-6, 0.0, 0.0, 0.0), (0.7, 0.2, 1e-3, 0.0, 0.0, 0.0),
    (-20.0, 0.03, 1e-3, 0.0, 0.0, 0.0), (-1.0, 2.0, 1e-9, 0.0, 0.0, 0.0), (-3.0, 0.3, 1e-6, -0.75, 0.0, 0.0),
    (-7.95, 0.3, 1e-6, 0.0, 0.1, 0.0), (-7.5, 0.3, 1e-6, 0.0, 0.4, 0.0), (-7.5, 0.3, 1e-6, 0.0, 0.6, 0.0),
    (-3.0, 5.0, 1e-9, 0.0, 0.0, 0.25), (-6.5, 0.05, 1e-9, 0.0, 0.0, 0.3), (-1.0, 0.5, 1e-9, 0.0, 0.0, 1.0),
    (-7.95, 0.3, 1e-6, 0.0, 0.1, 0.25), (0.7, 0.2, 1e-6, 0.0, 0.0, 0.25)])
def test_seeded_secant_matches_rule_fp64(fr3d, bias, slope, tol, shift, snap, ratio):
    # the secant refinement after the seed takes the oracle rule's decisions
    # (FP64, same evaluations), including the range ends and MAXITER; with a
    # slope ratio the first step's slope comes from the whole-box residual
    # at the seed
    g = geom(16, 16, 16)
    d = instance(g, 71, 0.02)
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=64)
    p = mlp.init_params(13)
    for k in ("W1", "W2", "w3"):
        p[k] = p[k] * 0.0
    p["b3"][:] = bias
    c.predictor_set(flat_params(p), identity_norm())
    F = torch.tensor(d["F"], dtype=torch.float64, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    kw = dict(tol=tol, accept_lo=1.0, accept_hi=1.0, max_steps=6)
    if shift:
        c.predictor_set_calibration([shift] + [0.0] * 65)
    rep = c.solve_discrepancy(z, use_predictor=1, seed_slope=slope, seed_snap_lo=snap, seed_slope_ratio=ratio, **kw)
    khat = np.fft.fftn(sample_kernel(g))

    def ev(a):
        o = tikhonov.solve_spectral(g, khat, d["F"], a)
        return o["r_norm"], o["zeta_norm"]
    # a calibration with only an intercept shifts the network's output before
    # the clip to the range
    ref = discrepancy.seeded_secant(ev, d["delta"], bias + shift, tol=tol, acc_lo=1.0, acc_hi=1.0, max_steps=6,
                                    slope=slope, snap=snap, slope_ratio=ratio,
                                    slope_at=lambda t: tikhonov.full_box_slope(g, khat, d["F"], 10.0 ** t))
    print("secant", bias, slope, ratio, "evals", rep["n_evals"], ref["n_evals"], flush=True)
    # the first point: the seed, or the lower range end for a seed within the margin
    assert ref["trace"][0][0] == (-8.0 if bias + shift < -8.0 + snap else min(max(bias + shift, -8.0), 0.0))
    assert rep["flags"] == ref["flags"]
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)
    o = tikhonov.solve_spectral(g, khat, d["F"], ref["alpha"])
    assert rel_l2(host(z), o["zeta"]) < 1e-11


@pytest.mark.parametrize("bias,snap", [(-3.0, 0.0), (-6.5, 0.0), (0.7, 0.0), (-20.0, 0.0), (-7.9, 0.2)])
def test_seeded_search_matches_rule_fp64(fr3d, bias, snap):
    # The network's output is steered by its last bias; the device search from
    # that seed takes the oracle rule's decisions (FP64, same evaluations).
    g = geom(16, 16, 16)
    d = instance(g, 70, 0.02)
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=64)
    p = mlp.init_params(13)
    for k in ("W1", "W2", "w3"):
        p[k] = p[k] * 0.0
    p["b3"][:] = bias
    c.predictor_set(flat_params(p), identity_norm())
    F = torch.tensor(d["F"], dtype=torch.float64, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    rep = c.solve_discrepancy(z, use_predictor=1, seed_snap_lo=snap)
    khat = np.fft.fftn(sample_kernel(g))

    def ev(a):
        o = tikhonov.solve_spectral(g, khat, d["F"], a)
        return o["r_norm"], o["zeta_norm"]
    ref = discrepancy.seeded(ev, d["delta"], bias, snap=snap)
    assert rep["flags"] == ref["flags"]
    assert rep["n_evals"] == ref["n_evals"]
    assert rep["alpha"] == pytest.approx(ref["alpha"], rel=1e-12)


@pytest.mark.parametrize("bias,ratio", [(-3.0, 0.25), (-6.5, 0.3), (-1.0, 1.0)])
def test_seeded_secant_slope_ratio_fp32(fr3d, bias, ratio):
    # FP32 transforms: the whole-box slope comes from the FP32 filter's
    # residual factors, so the steps need not match the FP64 rule point for
    # point; the answer must meet the rule (r/delta inside the window by the
    # oracle's FP64 residual at the device's alpha) and zeta must agree with
    # the oracle there
    g = geom(16, 16, 16)
    d = instance(g, 72, 0.02)
    c = fr3d.Context()
    c.load_kernel(16, 16, 16, precision=32)
    p = mlp.init_params(14)
    for k in ("W1", "W2", "w3"):
        p[k] = p[k] * 0.0
    p["b3"][:] = bias
    c.predictor_set(flat_params(p), identity_norm())
    F = torch.tensor(d["F"], dtype=torch.float32, device="cuda")
    c.set_data(F, d["delta"])
    z = torch.empty_like(F)
    tol = 1e-4
    rep = c.solve_discrepancy(z, use_predictor=1, seed_slope=5.0, seed_slope_ratio=ratio, tol=tol,
                              accept_lo=1.0, accept_hi=1.0, max_steps=20)
    print("fp32 secant", bias, ratio, "evals", rep["n_evals"], "flags", rep["flags"], flush=True)
    assert rep["flags"] & 7 == 0
    khat = np.fft.fftn(sample_kernel(g))
    o = tikhonov.solve_spectral(g, khat, d["F"], rep["alpha"])
    assert abs(o["r_norm"] / d["delta"] - 1.0) <= 2 * tol
    assert rel_l2(host(z), o["zeta"]) < 1e-5
