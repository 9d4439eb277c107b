"""Oracle parity of the exact kernel instances the measurements time.

* The headline workload (128^3 grids padded to 256^3, FP32) with the tile
  variants the autotuner picked for it (`Context.apply_tuning`: the entry
  tuned for batched solves, which the benchmark applies, and the single-lane
  entry): data spectrum, estimate at a fixed alpha and at the search's alpha,
  element by element against the FP64 oracle.
* Transform length 192 (n = 96, radix plan 16 x 4 x 3) on every axis, cubic
  and anisotropic, FP32 and FP64, default and tuned tiles; the alternative
  radix plans of lengths 192, 384 and 512 on every axis.
* The uneven-size batched workload: every instance the benchmark solves
  (shapes from {64, 96, 128, 192} per axis, so lengths 128, 192, 256 and 384),
  under the group solver with 16 candidates per step, each item's estimate
  against the oracle at the device's alpha.

Bars: spectra 2e-6 of their largest entry (FP32) / 1e-13 (FP64); estimates
1e-5 relative L2 (FP32) / 1e-11 (FP64); norms 1e-4 / 1e-10 relative.
"""
import json
import os

import numpy as np
import pytest

from oracle import synth, tikhonov
from oracle.geometry import sample_kernel
from oracle.operator import pad

from gpu_helpers import geom, half_spectrum, instance, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def fr3d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_01216_amd import fr3d as m
    return m


def dev(a, precision):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if precision == 64 else torch.float32,
                        device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def check_spectrum(c, g, Fh, precision):
    ref = half_spectrum(np.fft.fftn(pad(g, Fh)), g)
    got = host(c.get_data_spectrum())
    got = got[..., 0] + 1j * got[..., 1]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < (1e-13 if precision == 64 else 2e-6), err
    return err


def check_estimate(c, g, khat, Fh, alpha, zeta, rep, precision):
    o = tikhonov.solve_spectral(g, khat, Fh, alpha)
    err = rel_l2(host(zeta), o["zeta"])
    tol = 1e-11 if precision == 64 else 1e-5
    assert err < tol, err
    ntol = 1e-10 if precision == 64 else 1e-4
    assert rep["residual"] == pytest.approx(o["r_norm"], rel=ntol)
    assert rep["zeta_norm"] == pytest.approx(o["zeta_norm"], rel=ntol)
    return err, o


@pytest.mark.parametrize("batched", [True, False], ids=["batch-tiles", "single-lane-tiles"])
@pytest.mark.parametrize("index", [0, 1])
def test_headline_workload_with_bench_tiles(fr3d, index, batched):
    from paper_1703_01216_amd import inputs
    say(f"[bench-config] 128^3 -> 256^3 instance {index}, tuned tiles (batched {batched})")
    inst = inputs.workload_instance(2, index)
    g = geom(128, 128, 128)
    d = synth.make_data(g, inst["xi"], inst["noise"], inst["delta_rel"])
    c = fr3d.Context()
    c.load_kernel(128, 128, 128, precision=32)
    applied = c.apply_tuning(batched=batched)
    with open(fr3d.TUNING_PATH) as fh:
        cache = json.load(fh)
    # the bench applies the batch entry (its headline runs 8 lanes at once)
    want = cache.get("256x256x256/fp32/batch") if batched else None
    assert applied == (want or cache["256x256x256/fp32"])
    Fd = dev(d["F"], 32)
    Fh = host(Fd)
    c.set_data(Fd, d["delta"])
    es = check_spectrum(c, g, Fh, 32)
    khat = np.fft.fftn(sample_kernel(g))
    zeta = torch.empty_like(Fd)
    rep = c.solve_alpha(1e-4, zeta)
    e1, _ = check_estimate(c, g, khat, Fh, 1e-4, zeta, rep, 32)
    rep = c.solve_discrepancy(zeta)
    e2, o = check_estimate(c, g, khat, Fh, rep["alpha"], zeta, rep, 32)
    say(f"[bench-config] tiles {applied}: spectrum {es:.2e}, zeta(1e-4) {e1:.2e}, zeta(search alpha "
        f"{rep['alpha']:.4e}, flags {rep['flags']}, {rep['n_evals']} evals) {e2:.2e}")
    if rep["flags"] == 0:
        assert abs(o["r_norm"] / d["delta"] - 1) <= 1e-3 + 1e-5


LEN192 = [(96, 96, 96), (96, 24, 48), (16, 96, 32), (48, 32, 96)]


@pytest.mark.parametrize("tiles", ["default", "tuned"])
@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("shape", LEN192, ids=lambda s: "x".join(map(str, s)))
def test_length_192(fr3d, shape, precision, tiles):
    nx, ny, nz = shape
    say(f"[len192] shape {shape} precision {precision} tiles {tiles}")
    g = geom(nx, ny, nz)
    d = instance(g, 700 + nx + 3 * ny + 7 * nz, 0.02, recipe="inclusions")
    c = fr3d.Context()
    c.load_kernel(nx, ny, nz, precision=precision)
    if tiles == "tuned":
        applied = c.apply_tuning()
        if not applied:  # no cache entry for this precision: the non-default variants
            for p, sh in enumerate((2, 1, 1, 2, 1, 1)):
                c.set_tile(p, sh)
    Fd = dev(d["F"], precision)
    Fh = host(Fd)
    c.set_data(Fd, d["delta"])
    check_spectrum(c, g, Fh, precision)
    khat = np.fft.fftn(sample_kernel(g))
    zeta = torch.empty_like(Fd)
    rep = c.solve_alpha(1e-3, zeta)
    check_estimate(c, g, khat, Fh, 1e-3, zeta, rep, precision)
    rep = c.solve_discrepancy(zeta)
    check_estimate(c, g, khat, Fh, rep["alpha"], zeta, rep, precision)


PLAN_SHAPES = [(96, 12, 16), (16, 96, 24), (24, 16, 96), (192, 8, 12), (8, 192, 12), (12, 8, 192),
               (256, 8, 12), (8, 256, 12), (12, 8, 256)]


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("shape", PLAN_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_radix_plan_variants(fr3d, shape, variant):
    # the alternative radix plans of lengths 192, 384 and 512 (FP32) on each
    # axis, with every tile shift of each pass drawn at random: spectrum and
    # estimate against the oracle
    nx, ny, nz = shape
    say(f"[plans] shape {shape} variant {variant}")
    g = geom(nx, ny, nz)
    d = instance(g, 900 + nx + 5 * ny + 11 * nz, 0.02, recipe="inclusions")
    c = fr3d.Context()
    c.load_kernel(nx, ny, nz, precision=32)
    rg = np.random.default_rng(nx * 7 + ny * 3 + nz + variant)
    for p in range(6):
        c.set_tile(p, int(rg.integers(0, 3 if p in (0, 1, 3, 4) else 2)) + 4 * variant)
    Fd = dev(d["F"], 32)
    Fh = host(Fd)
    c.set_data(Fd, d["delta"])
    check_spectrum(c, g, Fh, 32)
    khat = np.fft.fftn(sample_kernel(g))
    zeta = torch.empty_like(Fd)
    rep = c.solve_alpha(1e-3, zeta)
    check_estimate(c, g, khat, Fh, 1e-3, zeta, rep, 32)


@pytest.mark.parametrize("index", range(8))
def test_batched_workload_items_against_oracle(fr3d, index):
    # instance `index` of the uneven-size workload, built as the benchmark
    # builds it (library operator and noise on the device), under its four
    # source sets q; the group solver with 16 candidates per step; the item
    # with q = index mod 4 against the oracle at the device's alpha, the
    # others within the rule
    from paper_1703_01216_amd import inputs
    r = inputs.workload_params(3, index)
    shape = r["shape"]
    nz, ny, nx = shape
    say(f"[workload3-items] instance {index} shape {shape}")
    ctxs, Fs, deltas = [], [], []
    for q in r["q"]:
        c = fr3d.Context()
        c.load_kernel(nx, ny, nz, q=q, precision=32)
        c.apply_tuning(batched=True)  # as the bench's batched workload
        V = torch.empty(shape, dtype=torch.float32, device="cuda")
        c.source_potential(V)
        xi = inputs.xi_torch(shape, r["inclusions"])
        F = torch.empty_like(xi)
        c.apply_operator(xi * V, F)
        deltas.append(c.add_noise(F, inputs.noise_torch(shape, r["seed"]), r["delta_rel"]))
        ctxs.append(c)
        Fs.append(F)
    zs = [torch.empty_like(F) for F in Fs]
    reps = fr3d.solve_group(ctxs, Fs, deltas, zs, candidates=16)
    torch.cuda.synchronize()
    for q, rep, dl in zip(r["q"], reps, deltas):
        say(f"[workload3-items] q={q}: alpha {rep['alpha']:.4e} r/delta {rep['residual'] / dl:.6f} "
            f"flags {rep['flags']} evals {rep['n_evals']}")
        if rep["flags"] == 0:
            assert abs(rep["residual"] / dl - 1) <= 1e-3
    k = index % 4
    q = r["q"][k]
    g = geom(nx, ny, nz, q=q)
    khat = np.fft.fftn(sample_kernel(g))
    o = tikhonov.solve_spectral(g, khat, host(Fs[k]), reps[k]["alpha"])
    err = rel_l2(host(zs[k]), o["zeta"])
    say(f"[workload3-items] q={q} against the oracle: rel_l2 {err:.2e}")
    assert err < 1e-5
    assert reps[k]["residual"] == pytest.approx(o["r_norm"], rel=1e-5)
    assert reps[k]["zeta_norm"] == pytest.approx(o["zeta_norm"], rel=1e-5)
    if reps[k]["flags"] == 0:
        assert abs(o["r_norm"] / deltas[k] - 1) <= 1e-3 + 1e-5
    for c in ctxs:
        c.close()
