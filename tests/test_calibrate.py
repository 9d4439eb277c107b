"""Host-side fits of the seed calibration (calibrate.fit): the coefficients
for the raw features reproduce the fitted standardised model, constant
features get no weight, and an exact linear relation and power law are
recovered (ridge -> 0)."""
import numpy as np
import pytest

from paper_1703_01216_amd import calibrate


def test_raw_coefficients_reproduce_the_fit():
    rg = np.random.default_rng(3)
    X = rg.standard_normal((80, 65)) * rg.uniform(0.1, 3.0, 65) + rg.uniform(-5, 5, 65)
    X[:, 10] = 2.5                                     # a constant feature
    X[:, 64] = rg.uniform(-2.3, -1.3, 80)             # the noise feature
    true = rg.uniform(-0.05, 0.05, 66)
    true[11] = 0.0
    dt = true[0] + X @ true[1:]
    s = 0.004 * 10.0 ** (-0.5 * X[:, 64])
    out = calibrate.fit(X, dt, np.log10(s), ridge=1e-9)
    c = np.array(out["coef"])
    assert c[11] == 0.0
    assert np.allclose(c[0] + X @ c[1:], dt, atol=1e-7)
    assert out["shift_residual_decades"] < 1e-7
    assert out["seed_slope"] == pytest.approx(0.004, rel=1e-9)
    assert out["seed_slope_x"] == pytest.approx(-0.5, abs=1e-9)
    assert out["seed_snap_lo"] == calibrate.SNAP_SIGMAS * out["shift_residual_decades"]
    # with ridge the raw coefficients still give the standardised model's predictions
    out = calibrate.fit(X, dt + 0.01 * rg.standard_normal(80), np.log10(s), ridge=1.0)
    c = np.array(out["coef"])
    pred_raw = c[0] + X @ c[1:]
    assert np.isfinite(pred_raw).all() and len(c) == 66
    assert np.std(pred_raw - dt) < 0.05
