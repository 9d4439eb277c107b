"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed
form, a textbook identity, a direct sum, a dense solve, or a value the
paper's model example fixes.  None of these tests touches the GPU.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import dft, discrepancy, features, layered, mlp, recovery, synth, tikhonov
from oracle.geometry import Geom, kernel_dz, kernel_fn, kernel_inv, sample_kernel, sources, v0
from oracle.operator import circulant_apply, forward_circulant, forward_direct, offset_table, pad
from paper_1703_01216_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- DFT (definition)

@pytest.mark.parametrize("p", [2, 3, 4, 6, 8, 12, 16])
def test_dft_matrix_on_pure_tones(p):
    # The DFT of exp(+2 pi i m j / P) is P at k = m and 0 elsewhere (orthogonality).
    j = np.arange(p)
    for m in range(p):
        x = np.exp(2j * np.pi * m * j / p)
        X = dft.dft_matrix(p) @ x
        ref = np.zeros(p, complex)
        ref[m] = p
        assert np.max(np.abs(X - ref)) < 1e-12 * p


def test_dft_delta_and_constant():
    p = 12
    d = np.zeros(p)
    d[0] = 1.0
    assert np.allclose(dft.dft_matrix(p) @ d, np.ones(p), atol=1e-15)
    assert np.allclose(dft.dft_matrix(p) @ np.ones(p), np.eye(p)[0] * p, atol=1e-12)


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8), (3, 6, 2)])
def test_dft3_full_separable_numpy_agree(shape):
    x = inputs.rng(1).standard_normal(shape) + 1j * inputs.rng(2).standard_normal(shape)
    full = dft.dft3_full(x)
    sep = dft.dft3(x)
    ref = np.fft.fftn(x)
    scale = np.abs(full).max()
    assert np.max(np.abs(full - sep)) < 1e-13 * scale
    assert np.max(np.abs(full - ref)) < 1e-13 * scale
    back = dft.dft3_full(full, inverse=True)
    assert np.max(np.abs(back - x)) < 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 24, 8), (6, 18, 32)])
def test_numpy_fft_against_separable_sums(shape):
    # numpy.fft serves the oracle only after this check against the sums (radices 2 and 3).
    x = inputs.rng(3).standard_normal(shape)
    sep = dft.dft3(x)
    ref = np.fft.fftn(x)
    assert np.max(np.abs(sep - ref)) < 1e-13 * np.abs(ref).max()
    inv = dft.dft3(ref, inverse=True)
    assert np.max(np.abs(inv - x)) < 1e-13 * np.abs(x).max()


def test_parseval():
    # Plancherel (Sec. 4, Lemma 1), discrete form: sum |x|^2 = P^-3 sum |X|^2.
    x = inputs.rng(4).standard_normal((8, 12, 6))
    X = dft.dft3(x)
    assert abs(np.sum(x * x) - np.sum(np.abs(X) ** 2) / x.size) < 1e-12 * np.sum(x * x)


# ---------------------------------------------------------------- kernel (Sec. 3, Eq. (8))

def test_kernel_closed_values():
    # On the axis K(0,0,z) = -1/z^2; K is odd in z; even in x and y.
    for z in (0.5, 1.0, 3.0, 40.0):
        assert kernel_dz(0.0, 0.0, z) == pytest.approx(-1.0 / z ** 2, rel=1e-15)
        assert kernel_inv(0.0, 0.0, z) == pytest.approx(1.0 / z, rel=1e-15)
    # 3-4-12 triangle: |x| = 13, K = -12 / 13^3.
    assert kernel_dz(3.0, 4.0, 12.0) == pytest.approx(-12.0 / 2197.0, rel=1e-15)
    assert kernel_dz(-3.0, 4.0, 12.0) == kernel_dz(3.0, -4.0, 12.0) == kernel_dz(3.0, 4.0, 12.0)
    assert kernel_dz(3.0, 4.0, -12.0) == -kernel_dz(3.0, 4.0, 12.0)


def test_kernel_is_z_derivative_of_inverse_distance():
    # K = d/dz (1/|x|) (Sec. 2, Eq. (6) kernel) -- central difference check.
    x, y, z, e = 1.3, -0.7, 5.1, 1e-5
    fd = (kernel_inv(x, y, z + e) - kernel_inv(x, y, z - e)) / (2 * e)
    assert kernel_dz(x, y, z) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("n,nz,D,h", [(8, 4, 6, 1.0), (6, 5, 7.5, 0.5)])
def test_sampled_table_values_and_symmetry(n, nz, D, h):
    g = Geom(n, n + 2, nz, h=h, D=D)
    k = sample_kernel(g)
    pz, py, px = g.pshape
    # slot a = n (P = 2n) is zero on every axis
    assert np.all(k[nz, :, :] == 0) and np.all(k[:, n + 2, :] == 0) and np.all(k[:, :, n] == 0)
    # value at (a, b, c) = (2, P-3, P-1): offsets (2, -3, -1)
    zz = (D - 1) * h
    ref = h ** 3 * (-zz) / ((2 * h) ** 2 + (3 * h) ** 2 + zz ** 2) ** 1.5
    assert k[pz - 1, py - 3, 2] == pytest.approx(ref, rel=1e-14)
    # even in the lateral offsets: k[c, b, a] = k[c, P-b, P-a]
    assert np.array_equal(k[:, :, 1:], k[:, :, 1:][:, :, ::-1])
    assert np.array_equal(k[:, 1:, :], k[:, 1:, :][:, ::-1, :])


@pytest.mark.parametrize("n,nz,D", [(16, 4, 8), (32, 4, 10)])
def test_lateral_sum_is_minus_solid_angle(n, nz, D):
    # The lateral integral of K at height z over [-a,a]x[-b,b] is minus the solid
    # angle of that rectangle seen from height z, 4 atan(ab / (z sqrt(a^2+b^2+z^2))).
    # The table's lateral midpoint sum covers a = b = (n - 1/2) h.
    g = Geom(n, n, nz, D=D)
    k = sample_kernel(g)
    for c in range(g.pshape[0]):
        if c == nz:
            continue
        z = g.d + (c if c < nz else c - g.pshape[0])
        a = n - 0.5
        om = 4 * math.atan(a * a / (z * math.sqrt(2 * a * a + z * z)))
        assert k[c].sum() == pytest.approx(-om, rel=1e-3)


def test_lateral_transform_closed_form():
    # 2D Fourier transform in (x,y) of K (Sec. 3, step to Eq. (9)) with kernel
    # e^{-i w.x}: K~(w, z) = -2 pi exp(-|w| z) for z > 0.  Truncation to the
    # lateral box of half-width L costs O(z/L).
    g = Geom(64, 64, 2, D=3)
    k = sample_kernel(g)
    P = g.pshape
    k2 = np.fft.fft2(k, axes=(1, 2))
    for c in (0, 1, 3):
        z = g.d + (c if c < g.nz else c - P[0])
        for (my, mx) in ((0, 1), (1, 1), (0, 4), (3, 4), (5, 12)):
            w = 2 * math.pi * math.hypot(mx / P[2], my / P[1])
            ref = -2 * math.pi * math.exp(-w * z)
            assert abs(k2[c, my, mx] - ref) < 1e-2 * abs(ref)


def test_kernel_spectrum_symmetry():
    # k even in x, y and real: s = |k^|^2 is even in every frequency; k^(kx,ky,-kz) = conj k^.
    g = Geom(6, 8, 4)
    khat, s, smax = tikhonov.kernel_spectrum(sample_kernel(g))
    rz = (-np.arange(g.pshape[0])) % g.pshape[0]
    ry = (-np.arange(g.pshape[1])) % g.pshape[1]
    rx = (-np.arange(g.pshape[2])) % g.pshape[2]
    assert np.allclose(khat, khat[:, ry, :], atol=1e-13 * np.sqrt(smax))
    assert np.allclose(khat, khat[:, :, rx], atol=1e-13 * np.sqrt(smax))
    assert np.allclose(khat[rz, :, :], khat.conj(), atol=1e-13 * np.sqrt(smax))
    assert smax == s.max()


# ---------------------------------------------------------------- forward operator (Eq. (8))

@pytest.mark.parametrize("shape,D,kind", [((6, 6, 6), None, 0), ((4, 5, 7), 6.5, 0), ((5, 5, 4), None, 1)])
def test_forward_direct_equals_circulant(shape, D, kind):
    # Convolution theorem on the zero-padded box vs the direct quadrature sum,
    # which evaluates K at cell-centre differences with no table and no wrap.
    nz, ny, nx = shape
    g = Geom(nx, ny, nz, D=D, kind=kind)
    zeta = inputs.rng(5).standard_normal(shape)
    a = forward_direct(g, zeta)
    b = forward_circulant(g, zeta)
    assert np.max(np.abs(a - b)) < 1e-13 * np.abs(a).max()


def test_anisotropic_cells_brute_force():
    # Thin layers (Sec. 6: vertical cells finer than lateral ones): the sum
    # over explicit cell centres ((i+.5)h, (j+.5)h, (k+.5)hz) of R and
    # ((i+.5)h, (j+.5)h, (D+k+.5)hz) of Y with weight h^2 hz, written out
    # point by point, equals the table-based direct sum and the circulant form.
    g = Geom(3, 2, 3, h=0.5, hz=0.125, D=9.0)
    zeta = inputs.rng(6).standard_normal(g.shape)
    K = kernel_fn(0)
    out = np.zeros(g.shape)
    for kz in range(3):
        for jy in range(2):
            for ix in range(3):
                y = np.array([(ix + .5) * 0.5, (jy + .5) * 0.5, (9.0 + kz + .5) * 0.125])
                acc = 0.0
                for kz2 in range(3):
                    for jy2 in range(2):
                        for ix2 in range(3):
                            r = np.array([(ix2 + .5) * 0.5, (jy2 + .5) * 0.5, (kz2 + .5) * 0.125])
                            d = y - r
                            acc += 0.5 * 0.5 * 0.125 * K(d[0], d[1], d[2]) * zeta[kz2, jy2, ix2]
                out[kz, jy, ix] = acc
    assert np.allclose(forward_direct(g, zeta), out, rtol=1e-13, atol=0)
    assert np.allclose(forward_circulant(g, zeta), out, rtol=1e-12, atol=1e-14 * np.abs(out).max())
    kt = layered.lateral_kernel_spectrum(g)
    assert np.allclose(layered.forward_layered(g, kt, zeta), out, rtol=1e-12, atol=1e-14 * np.abs(out).max())
    # the sources sit at nz + G/4 and nz + 3G/4 vertical cells
    src = sources(g)
    assert np.allclose(np.unique(src[:, 2]), [(3 + 1.5) * 0.125, (3 + 4.5) * 0.125])


@pytest.mark.slow
def test_forward_direct_equals_circulant_n32():
    g = Geom(32, 32, 32)
    inst = inputs.workload_instance(1, 0)
    zeta = inst["xi"] * v0(g)
    a = forward_direct(g, zeta)
    b = forward_circulant(g, zeta)
    assert np.linalg.norm(a - b) < 1e-13 * np.linalg.norm(a)


def test_offset_table_matches_wrapped_table():
    g = Geom(5, 4, 3, D=4.25)
    T = offset_table(g)
    k = sample_kernel(g)
    for dz in range(-2, 3):
        for dy in range(-3, 4):
            for dx in range(-4, 5):
                assert T[dz + 2, dy + 3, dx + 4] == k[dz % 6, dy % 8, dx % 10]


def test_circulant_direct_vs_fft():
    rg = inputs.rng(6)
    k = rg.standard_normal((4, 6, 4))
    u = rg.standard_normal((4, 6, 4))
    a = circulant_apply(k, u)
    b = np.fft.ifftn(np.fft.fftn(k) * np.fft.fftn(u)).real
    assert np.max(np.abs(a - b)) < 1e-13 * np.abs(a).max()


# ---------------------------------------------------------------- Tikhonov (Sec. 3-4)

@pytest.mark.parametrize("shape,alpha", [((4, 4, 4), 1e-3), ((3, 4, 6), 1e-5), ((6, 6, 6), 1e-2)])
def test_dense_normal_equations_equal_spectral(shape, alpha):
    # relative scale: alpha_abs = alpha max|k^|^2
    nz, ny, nx = shape
    g = Geom(nx, ny, nz)
    k = sample_kernel(g)
    khat, s, smax = tikhonov.kernel_spectrum(k)
    F = inputs.rng(7).standard_normal(shape)
    sp = tikhonov.solve_spectral(g, khat, F, alpha, relative=True)
    de = tikhonov.dense_tikhonov(g, k, F, alpha * smax)
    assert np.linalg.norm(sp["zeta"] - de["zeta"]) < 1e-10 * np.linalg.norm(de["zeta"])
    assert np.linalg.norm(sp["r"] - de["r"]) < 1e-10 * np.linalg.norm(de["r"])
    assert sp["r_full"] == pytest.approx(np.linalg.norm(de["r_full"]), rel=1e-10)
    assert sp["imag_max"] < 1e-12 * np.abs(sp["zeta"]).max()


@pytest.mark.parametrize("shape,alpha", [((3, 4, 4), 1e-3), ((3, 4, 6), 1e-5), ((4, 4, 4), 3e-2)])
def test_full_box_slope_is_the_derivative_of_dense_solves(shape, alpha):
    # the Parseval form of d ln ||r_box|| / d log10 alpha against a central
    # difference of the whole-box residual of the assembled normal equations
    nz, ny, nx = shape
    g = Geom(nx, ny, nz)
    k = sample_kernel(g)
    khat, s, smax = tikhonov.kernel_spectrum(k)
    F = inputs.rng(8).standard_normal(shape)
    h = 1e-4
    lr = [math.log(np.linalg.norm(tikhonov.dense_tikhonov(g, k, F, alpha * smax * 10.0 ** (j * h))["r_full"]))
          for j in (-1, 1)]
    fd = (lr[1] - lr[0]) / (2 * h)
    assert fd > 0
    assert tikhonov.full_box_slope(g, khat, F, alpha, relative=True) == pytest.approx(fd, rel=1e-6)


def test_full_box_slope_closed_forms():
    # identity kernel: e = a / (1 + a) everywhere, slope ln10 / (1 + a)
    g = Geom(4, 4, 4)
    k = np.zeros(g.pshape)
    k[0, 0, 0] = 1.0
    khat = np.fft.fftn(k)
    F = inputs.rng(12).standard_normal(g.shape)
    for a in (1e-6, 0.3, 7.0):
        assert tikhonov.full_box_slope(g, khat, F, a) == pytest.approx(math.log(10.0) / (1.0 + a), rel=1e-13)
    # a kernel without zero modes: r_box -> a k^-2 f^ as a -> 0 (slope ln 10),
    # and r_box -> f^ (slope 0) as a grows
    g = Geom(4, 4, 3)
    khat = np.fft.fftn(sample_kernel(g))
    F = inputs.rng(9).standard_normal(g.shape)
    assert tikhonov.full_box_slope(g, khat, F, 1e-14, relative=True) == pytest.approx(math.log(10.0), rel=1e-6)
    assert 0 < tikhonov.full_box_slope(g, khat, F, 1e8, relative=True) < 1e-6


@pytest.mark.parametrize("order", [1, 2, 5])
@pytest.mark.parametrize("shape,alpha", [((4, 4, 4), 1e-2), ((3, 4, 6), 1e-4)])
def test_iterated_tikhonov_equals_repeated_normal_equations(shape, alpha, order):
    # Sec. 5: iterated Tikhonov, by its definition (order solves of the
    # normal equations, each regularised toward the previous iterate).
    nz, ny, nx = shape
    g = Geom(nx, ny, nz)
    k = sample_kernel(g)
    khat = np.fft.fftn(k)
    F = inputs.rng(17).standard_normal(shape)
    sp = tikhonov.solve_spectral(g, khat, F, alpha, method=tikhonov.ITERATED, order=order)
    de = tikhonov.dense_iterated(g, k, F, alpha, order)
    assert np.linalg.norm(sp["zeta"] - de["zeta"]) < 1e-9 * np.linalg.norm(de["zeta"])
    assert np.linalg.norm(sp["r"] - de["r"]) < 1e-9 * np.linalg.norm(de["r"])
    if order == 1:
        t = tikhonov.solve_spectral(g, khat, F, alpha)
        assert np.allclose(sp["zeta"], t["zeta"], rtol=0, atol=1e-13 * np.abs(t["zeta"]).max())
    # more iterations fit the data more closely
    if order > 1:
        prev = tikhonov.solve_spectral(g, khat, F, alpha, method=tikhonov.ITERATED, order=order - 1)
        assert sp["r_full"] < prev["r_full"]


@pytest.mark.parametrize("shape", [(4, 4, 4), (3, 4, 6)])
def test_spectral_tsvd_equals_dense_svd(shape):
    # Sec. 5: truncated SVD; the singular values of the circulant matrix are |k^|.
    nz, ny, nx = shape
    g = Geom(nx, ny, nz)
    k = sample_kernel(g)
    khat = np.fft.fftn(k)
    s = np.sort(np.abs(khat).ravel() ** 2)
    F = inputs.rng(18).standard_normal(shape)
    C = tikhonov.circulant_matrix(k)
    sv = np.linalg.svd(C, compute_uv=False)
    assert np.allclose(np.sort(sv ** 2), s, rtol=1e-10, atol=1e-12 * s[-1])
    for frac in (0.05, 0.3, 0.7):
        # a cut half-way between two distinct values of s
        i = int(frac * len(s))
        while s[i + 1] - s[i] < 1e-6 * s[-1]:
            i += 1
        cut = 0.5 * (s[i] + s[i + 1])
        sp = tikhonov.solve_spectral(g, khat, F, cut, method=tikhonov.TSVD)
        de = tikhonov.dense_tsvd(g, k, F, cut)
        assert np.linalg.norm(sp["zeta"] - de["zeta"]) < 1e-9 * np.linalg.norm(de["zeta"])
        assert np.linalg.norm(sp["r"] - de["r"]) < 1e-9 * max(np.linalg.norm(de["r"]), 1e-30)


@pytest.mark.parametrize("alpha", [1e-10, 1e-7, 1e-4])
def test_near_exact_recovery_of_band_limited_zeta(alpha):
    # Circulant model, full-box data f = C zeta with zeta^ supported where
    # s >= 1e-3 s_max: the estimate's error spectrum is exactly
    # -a/(s+a) zeta^, so ||err|| / ||zeta|| <= alpha / (1e-3 + alpha).
    g = Geom(8, 8, 8)
    k = sample_kernel(g)
    khat, s, smax = tikhonov.kernel_spectrum(k)
    z = inputs.rng(8).standard_normal(g.pshape)
    zh = np.fft.fftn(z) * (s >= 1e-3 * smax)
    zeta = np.fft.ifftn(zh).real
    f = np.fft.ifftn(khat * np.fft.fftn(zeta)).real
    est, _ = tikhonov.solve_box(khat, f, alpha, relative=True)
    err = np.linalg.norm(est.real - zeta) / np.linalg.norm(zeta)
    assert err <= alpha / (1e-3 + alpha) * (1 + 1e-6) + 1e-13


def test_theorem1_error_decreases_with_noise():
    # Circulant model: with alpha chosen by the discrepancy principle the error
    # decreases as delta decreases (Theorem 1, qualitative).
    g = Geom(8, 8, 8)
    k = sample_kernel(g)
    khat, s, smax = tikhonov.kernel_spectrum(k)
    zeta = np.fft.ifftn(np.fft.fftn(inputs.rng(9).standard_normal(g.pshape)) * (s >= 1e-4 * smax)).real
    f0 = np.fft.ifftn(khat * np.fft.fftn(zeta)).real
    e = inputs.rng(10).standard_normal(g.pshape)
    errs = []
    for rel in (1e-1, 1e-2, 1e-3, 1e-4):
        ee = e * rel * np.linalg.norm(f0) / np.linalg.norm(e)
        f = f0 + ee
        delta = np.linalg.norm(ee)

        def ev(a):
            u, r = tikhonov.solve_box(khat, f, a, relative=True)
            return np.linalg.norm(r.real), np.linalg.norm(u.real)
        res = discrepancy.bisection(ev, delta, lo=-14)
        u, _ = tikhonov.solve_box(khat, f, res["alpha"], relative=True)
        errs.append(np.linalg.norm(u.real - zeta) / np.linalg.norm(zeta))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


def test_alpha_units_h_invariant():
    # In L2 units the functional h^3 (||C u - f||^2 + alpha ||u||^2) has the
    # same minimiser for every h once the table carries the weight h^3; the
    # dense solve confirms the absolute scale used by default.
    g = Geom(4, 4, 4, h=0.5, D=5)
    k = sample_kernel(g)
    khat, s, smax = tikhonov.kernel_spectrum(k)
    F = inputs.rng(17).standard_normal(g.shape)
    sp = tikhonov.solve_spectral(g, khat, F, 3e-6)
    de = tikhonov.dense_tikhonov(g, k, F, 3e-6)
    assert np.linalg.norm(sp["zeta"] - de["zeta"]) < 1e-9 * np.linalg.norm(de["zeta"])


def test_full_box_residual_and_norm_monotone():
    g = Geom(6, 6, 6)
    khat, s, smax = tikhonov.kernel_spectrum(sample_kernel(g))
    F = inputs.rng(11).standard_normal(g.shape)
    ts = np.linspace(-8, 0, 33)
    rf = [tikhonov.solve_spectral(g, khat, F, 10 ** t, relative=True)["r_full"] for t in ts]
    zn = []
    for t in ts:
        u, _ = tikhonov.solve_box(khat, pad(g, F), 10 ** t, relative=True)
        zn.append(np.linalg.norm(u.real))
    assert all(rf[i + 1] > rf[i] for i in range(len(rf) - 1))
    assert all(zn[i + 1] < zn[i] for i in range(len(zn) - 1))


# ---------------------------------------------------------------- discrepancy rule

def _identity_problem(delta_frac, n=4):
    # k = delta_0: k^ = 1, s = 1 (both alpha scales agree); zeta = F/(1+alpha),
    # r = -alpha F/(1+alpha), so ||r|| = delta at alpha* = delta / (||F|| - delta).
    g = Geom(n, n, n)
    k = np.zeros(g.pshape)
    k[0, 0, 0] = 1.0
    khat = np.fft.fftn(k)
    F = inputs.rng(12).standard_normal(g.shape)
    Fn = np.linalg.norm(F)
    delta = delta_frac * Fn

    def ev(a):
        out = tikhonov.solve_spectral(g, khat, F, a)
        out2 = tikhonov.solve_spectral(g, khat, F, a, relative=True)
        assert out["r_norm"] == out2["r_norm"]
        return out["r_norm"], out["zeta_norm"]
    return ev, delta, Fn


@pytest.mark.parametrize("frac", [0.01, 0.05, 0.3])
def test_bisection_reaches_closed_form_root(frac):
    ev, delta, Fn = _identity_problem(frac)
    a_star = delta / (Fn - delta)
    res = discrepancy.bisection(ev, delta, tol=1e-6)
    assert res["flags"] == 0
    assert res["alpha"] == pytest.approx(a_star, rel=1e-5)
    assert res["n_evals"] == len(res["trace"]) and res["n_evals"] >= 3
    # the first two points are the range ends, hi first
    assert res["trace"][0][0] == 0.0 and res["trace"][1][0] == -8.0


def test_bisection_flags():
    ev, delta, Fn = _identity_problem(0.6)
    # at alpha = 1 the identity residual is ||F||/2 < delta: no root below hi
    res = discrepancy.bisection(ev, delta)
    assert res["flags"] == discrepancy.NOROOT_HIGH and res["n_evals"] == 1 and res["alpha"] == 1.0
    ev, delta, Fn = _identity_problem(1e-12)
    res = discrepancy.bisection(ev, delta)
    assert res["flags"] == discrepancy.NOROOT_LOW and res["n_evals"] == 2 and res["alpha"] == 1e-8
    ev, delta, Fn = _identity_problem(0.05)
    res = discrepancy.bisection(ev, delta, tol=0.0, max_steps=5)
    assert res["flags"] == discrepancy.MAXITER
    assert res["trace"][-1][0] == res["t"]


def test_range_ends_accepted_within_tolerance():
    # An evaluated range end inside the tolerance is an answer, not a failure.
    ev, delta, Fn = _identity_problem(0.5)   # r(1) = ||F||/2 = delta exactly
    res = discrepancy.bisection(ev, delta, tol=1e-9)
    assert res["flags"] == 0 and res["n_evals"] == 1 and res["alpha"] == 1.0
    ev, delta, Fn = _identity_problem(0.05)
    a_lo = 1e-8
    r_lo = a_lo / (1 + a_lo) * Fn
    res = discrepancy.bisection(ev, r_lo * 1.0004, tol=1e-3)
    assert res["flags"] == 0 and res["n_evals"] == 2 and res["alpha"] == 1e-8


def test_seeded_search():
    ev, delta, Fn = _identity_problem(0.03)
    t_star = math.log10(delta / (Fn - delta))
    res = discrepancy.seeded(ev, delta, t_star + 0.01)
    assert res["flags"] == 0 and res["n_evals"] == 1
    for off in (-3.3, 2.7, 0.4, -0.2):
        res = discrepancy.seeded(ev, delta, t_star + off, tol=1e-6, acc_lo=1.0, acc_hi=1.0)
        assert res["flags"] == discrepancy.PRED_FALLBACK
        assert res["alpha"] == pytest.approx(10 ** t_star, rel=1e-5)
        # regula falsi converges in far fewer points than bisection would need
        assert res["n_evals"] < 20
    # the walk doubles its step from the seed: 0.25, 0.5, 1, 2 decades
    res = discrepancy.seeded(ev, delta, t_star - 3.3, tol=1e-6, acc_lo=1.0, acc_hi=1.0)
    ts = [t for t, *_ in res["trace"][:5]]
    assert [round(t - ts[0], 9) for t in ts] == [0.0, 0.25, 0.75, 1.75, 3.75]
    # no sign change up to the range end
    ev2, delta2, Fn2 = _identity_problem(0.6)
    res = discrepancy.seeded(ev2, delta2, -3.0)
    assert res["flags"] == discrepancy.PRED_FALLBACK | discrepancy.NOROOT_HIGH and res["alpha"] == 1.0


def _loglinear(t_star, s):
    # residual with ln(r/delta) = s (log10 alpha - t_star) exactly
    return lambda a: (math.exp(s * (math.log10(a) - t_star)), 1.0)


def test_seeded_secant_steps():
    # Newton with the true slope lands on the root; with twice the slope it
    # stops halfway and the secant through the two points (exact for a
    # straight line) lands on it next
    for s_true, s_assumed, n in ((0.05, 0.05, 2), (0.05, 0.1, 3), (0.7, 0.35, 3)):
        res = discrepancy.seeded_secant(_loglinear(-3.2, s_true), 1.0, -2.1, tol=1e-9, acc_lo=1.0, acc_hi=1.0,
                                        slope=s_assumed)
        assert res["flags"] == discrepancy.PRED_FALLBACK and res["n_evals"] == n
        assert res["t"] == pytest.approx(-3.2, abs=1e-9)
        ts = [t for t, *_ in res["trace"]]
        assert ts[1] == pytest.approx(-2.1 - s_true * (-2.1 + 3.2) / s_assumed, abs=1e-12)
    # the identity kernel's closed-form root from seeds on both sides
    ev, delta, Fn = _identity_problem(0.03)
    t_star = math.log10(delta / (Fn - delta))
    for off in (-3.3, 2.7, 0.4, -0.2):
        res = discrepancy.seeded_secant(ev, delta, t_star + off, tol=1e-9, acc_lo=1.0, acc_hi=1.0, slope=0.5)
        assert res["flags"] == discrepancy.PRED_FALLBACK
        assert res["alpha"] == pytest.approx(10 ** t_star, rel=1e-7)
        assert res["n_evals"] < 15
    # a seed inside the window is accepted at once
    res = discrepancy.seeded_secant(ev, delta, t_star + 1e-4, slope=0.5)
    assert res["flags"] == 0 and res["n_evals"] == 1


def test_seeded_secant_slope_from_the_whole_box():
    # with the ratio times the whole-box slope equal to the true slope of the
    # straight line, the first step lands on the root whatever slope is
    # assumed; a whole-box slope that is not positive keeps the assumed one
    tight = dict(tol=1e-9, acc_lo=1.0, acc_hi=1.0)
    seen = []

    def at(t):
        seen.append(t)
        return 0.2 / 0.25
    res = discrepancy.seeded_secant(_loglinear(-3.2, 0.2), 1.0, -2.1, slope=5.0, slope_at=at, slope_ratio=0.25,
                                    **tight)
    assert res["n_evals"] == 2 and res["t"] == pytest.approx(-3.2, abs=1e-12) and seen == [-2.1]
    base = discrepancy.seeded_secant(_loglinear(-3.2, 0.2), 1.0, -2.1, slope=5.0, **tight)
    assert base["n_evals"] > 2
    for at2, ratio in ((lambda t: -1.0, 0.25), (lambda t: 0.0, 0.25), (at, 0.0)):
        res = discrepancy.seeded_secant(_loglinear(-3.2, 0.2), 1.0, -2.1, slope=5.0, slope_at=at2,
                                        slope_ratio=ratio, **tight)
        assert res["trace"] == base["trace"]
    # a seed accepted at once asks for no slope
    seen.clear()
    res = discrepancy.seeded_secant(_loglinear(-3.2, 0.2), 1.0, -3.2, slope=5.0, slope_at=at, slope_ratio=0.25,
                                    **tight)
    assert res["n_evals"] == 1 and seen == []


def test_seeded_secant_range_ends_and_step_limit():
    # the root lies below lo: the first step clips to lo, rho(lo) > 0
    tight = dict(tol=1e-3, acc_lo=1.0, acc_hi=1.0)
    res = discrepancy.seeded_secant(_loglinear(-9.0, 0.1), 1.0, -5.0, slope=0.1, **tight)
    assert res["flags"] == discrepancy.PRED_FALLBACK | discrepancy.NOROOT_LOW
    assert res["alpha"] == 1e-8 and res["n_evals"] == 2
    # above hi
    res = discrepancy.seeded_secant(_loglinear(0.5, 0.1), 1.0, -1.0, slope=0.1, **tight)
    assert res["flags"] == discrepancy.PRED_FALLBACK | discrepancy.NOROOT_HIGH
    assert res["alpha"] == 1.0 and res["n_evals"] == 2
    # a tenfold slope overestimate and one step: MAXITER at the upper end,
    # which is the last point (no extra evaluation)
    res = discrepancy.seeded_secant(_loglinear(-3.0, 0.5), 1.0, -2.0, tol=1e-6, acc_lo=1.0, acc_hi=1.0,
                                    slope=5.0, max_steps=1)
    assert res["flags"] == discrepancy.PRED_FALLBACK | discrepancy.MAXITER
    assert res["t"] == pytest.approx(-2.1) and res["n_evals"] == 2
    # the bracket safeguard: an extrapolation past a known end becomes the
    # regula falsi point, so every point after the bracket stays inside it
    res = discrepancy.seeded_secant(_loglinear(-3.0, 0.5), 1.0, -1.0, tol=1e-9, acc_lo=1.0, acc_hi=1.0,
                                    slope=0.05)
    ts = [t for t, *_ in res["trace"]]
    assert ts[1] == -8.0 and all(-8.0 < t < -1.0 for t in ts[2:])
    assert res["t"] == pytest.approx(-3.0, abs=1e-9)


def test_seed_near_lower_end_starts_there():
    tight = dict(tol=1e-9, acc_lo=1.0, acc_hi=1.0)
    # root below the range, seed 0.05 decades above lo: with a 0.1-decade
    # margin the first point is lo, whose residual is above the target, so
    # the search ends there after one evaluation (two without the margin)
    for snap, n in ((0.1, 1), (0.0, 2), (0.04, 2)):
        res = discrepancy.seeded_secant(_loglinear(-8.3, 0.05), 1.0, -7.95, slope=0.05, snap=snap, **tight)
        assert res["flags"] == discrepancy.PRED_FALLBACK | discrepancy.NOROOT_LOW
        assert res["alpha"] == 1e-8 and res["n_evals"] == n
        assert res["trace"][0][0] == (-8.0 if snap > 0.05 else -7.95)
    # root inside the margin: from lo, Newton with the true slope of the
    # straight line lands on the root
    res = discrepancy.seeded_secant(_loglinear(-7.97, 0.05), 1.0, -7.95, slope=0.05, snap=0.1, **tight)
    assert res["flags"] == discrepancy.PRED_FALLBACK and res["n_evals"] == 2
    assert res["t"] == pytest.approx(-7.97, abs=1e-9)
    # the walk search starts at the same point; a seed above the margin is
    # kept as it is
    res = discrepancy.seeded(_loglinear(-8.3, 0.05), 1.0, -7.95, snap=0.1, **tight)
    assert res["flags"] & discrepancy.NOROOT_LOW and res["n_evals"] == 1
    res = discrepancy.seeded_secant(_loglinear(-3.0, 0.05), 1.0, -7.85, slope=0.05, snap=0.1, **tight)
    assert res["trace"][0][0] == -7.85


def test_seeded_matches_bisection_answer_quality():
    # same acceptance band: both searches end inside it
    ev, delta, Fn = _identity_problem(0.02)
    for t0 in (-6.0, -1.0, -2.2):
        r1 = discrepancy.seeded(ev, delta, t0, tol=1e-3, acc_lo=0.999, acc_hi=1.001)
        r2 = discrepancy.bisection(ev, delta, tol=1e-3)
        for res in (r1, r2):
            rr, _ = ev(res["alpha"])
            assert abs(rr / delta - 1) <= 1e-3


@pytest.mark.parametrize("K", [2, 5, 16])
@pytest.mark.parametrize("frac", [0.01, 0.05, 0.3])
def test_kary_reaches_closed_form_root(K, frac):
    ev, delta, Fn = _identity_problem(frac)
    a_star = delta / (Fn - delta)
    t_star = math.log10(a_star)
    res = discrepancy.kary(ev, delta, K=K, tol=1e-6)
    assert res["flags"] == 0
    assert res["alpha"] == pytest.approx(a_star, rel=1e-5)
    assert res["n_evals"] == K * res["steps"] + 1 == len(res["trace"])
    ts = [t for t, *_ in res["trace"]]
    # step 1: K points from lo to hi inclusive
    assert ts[0] == -8.0 and ts[K - 1] == 0.0
    assert np.allclose(np.diff(ts[:K]), 8.0 / (K - 1))
    # every later step: K equally spaced interior points of a bracket around t*
    # whose width shrinks by K + 1 per step
    width = 8.0 / (K - 1)
    for s in range(1, res["steps"]):
        pts = ts[s * K:(s + 1) * K]
        h = width / (K + 1)
        a = pts[0] - h
        assert np.allclose(np.diff(pts), h) and a - 1e-12 <= t_star <= a + width + 1e-12
        width = h
    # the answer is evaluated last, on its own
    assert ts[-1] == res["t"]


def test_kary_flags_and_best_candidate():
    ev, delta, Fn = _identity_problem(0.6)
    res = discrepancy.kary(ev, delta, K=16)
    assert res["flags"] == discrepancy.NOROOT_HIGH and res["alpha"] == 1.0 and res["n_evals"] == 17
    ev, delta, Fn = _identity_problem(1e-12)
    res = discrepancy.kary(ev, delta, K=16)
    assert res["flags"] == discrepancy.NOROOT_LOW and res["alpha"] == 1e-8 and res["n_evals"] == 17
    ev, delta, Fn = _identity_problem(0.05)
    t_star = math.log10(delta / (Fn - delta))
    res = discrepancy.kary(ev, delta, K=4, tol=0.0, max_steps=3)
    assert res["flags"] == discrepancy.MAXITER and res["n_evals"] == 13
    # b is the bracket's upper end: rho(b) >= 0 and b - a = 8/3/5/5 around t*
    assert res["t"] >= t_star and res["t"] - 8.0 / 3 / 25 <= t_star + 1e-12

    # several candidates inside the tolerance: the one closest to the target wins
    g = {3: 5e-4, 5: -2e-4, 9: 3e-4}

    def ev2(alpha):
        t = math.log10(alpha)
        j = round((t + 8.0) * 15 / 8.0)
        return 1.0 + g.get(j, (0.5 if j > 5 else -0.5)), 0.0
    res = discrepancy.kary(ev2, 1.0, K=16, tol=1e-3)
    assert res["flags"] == 0 and res["t"] == -8.0 + 5 * 8.0 / 15 and res["n_evals"] == 17


# ---------------------------------------------------------------- recovery and V0 (Sec. 2, Sec. 6)

def test_model_example_v0_closed_form():
    # Sec. 6 model example: ten sources (0,0,z0), (+-8,0,z0), (0,+-8,z0), z0 = 3, 5;
    # g = exp(-t) so A0 = 1, A2 = 2.  At (0,0,1.5):
    # V0 = -(1/4pi)(1/1.5 + 4/sqrt(64+1.5^2) + 1/3.5 + 4/sqrt(64+3.5^2)).
    with open(os.path.join(GOLDEN, "model_example.json")) as fh:
        ex = json.load(fh)
    assert ex["A0"] == pytest.approx(math.gamma(1)) and ex["A2"] == pytest.approx(math.gamma(3))
    x = np.array([0.0, 0.0, 1.5])
    v = sum(1.0 / np.linalg.norm(x - np.array(s)) for s in ex["sources"])
    ref = -(1 / (4 * math.pi)) * (1 / 1.5 + 4 / math.sqrt(64 + 2.25) + 1 / 3.5 + 4 / math.sqrt(64 + 12.25))
    assert -ex["A0"] / (4 * math.pi) * v == pytest.approx(ref, rel=1e-15)


def _model_example_cells():
    # Sec. 6 geometry on a grid where (0, 0, 1.5) is a cell centre: R = [-10, 10]^2 x [1, 2]
    # on 5 x 5 x 3 cells (h = 4, hz = 1/3), Y five layer thicknesses above R (D = 15).
    # The oracle's coordinates start at R's corner, so the model example's are the
    # oracle's shifted by (-10, -10, +1).
    mg = inputs.model_geometry(5, 3)
    g = Geom(mg["nx"], mg["ny"], mg["nz"], h=mg["h"], D=mg["D"], hz=mg["hz"])
    return g, np.array([-10.0, -10.0, 1.0])


def test_sources_are_the_model_example_cross():
    # Sec. 6: sources at (0,0,z0), (+-8,0,z0), (0,+-8,z0) for z0 = 3 and 5.  A lateral
    # offset of 0.4 (n - 1) cells, a height off by a cell or a swapped axis fails here.
    g, shift = _model_example_cells()
    with open(os.path.join(GOLDEN, "model_example.json")) as fh:
        ex = json.load(fh)
    got = sources(g) + shift
    ref = np.array(ex["sources"], dtype=np.float64)
    key = lambda a: sorted(map(tuple, np.round(a, 12)))  # noqa: E731
    assert key(got) == key(ref)
    assert np.max(np.abs(got - ref)) < 1e-12  # same order: centre, -x, +x, -y, +y per height


def test_v0_at_model_example_point_closed_form():
    # V0 = -(A0/4pi) sum_l 1/|x - x_l| (Sec. 2) with A0 = 1 (g = e^-t, Sec. 6) at the
    # cell centre (0, 0, 1.5): distances 1.5 and 3.5 to the centres of the two
    # heights and sqrt(64 + 1.5^2), sqrt(64 + 3.5^2) to the four lateral points.
    g, shift = _model_example_cells()
    zc = (np.arange(g.nz) + 0.5) * g.hv + shift[2]
    xc = (np.arange(g.nx) + 0.5) * g.h + shift[0]
    k, i = int(np.argmin(np.abs(zc - 1.5))), int(np.argmin(np.abs(xc)))
    assert abs(zc[k] - 1.5) < 1e-14 and abs(xc[i]) < 1e-14
    ref = -(1 / (4 * math.pi)) * (1 / 1.5 + 4 / math.sqrt(64 + 1.5 ** 2) + 1 / 3.5 + 4 / math.sqrt(64 + 3.5 ** 2))
    V = v0(g)
    assert abs(V[k, i, i] - ref) < 1e-14 * abs(ref)
    # linear in A0
    assert abs(v0(g, A0=2.5)[k, i, i] - 2.5 * ref) < 1e-14 * abs(ref)


def test_v0_negative_and_harmonic_in_R():
    # V0 = -(A0/4pi) sum 1/|x - x_l| < 0 (Sec. 2) and harmonic away from the sources.
    g = Geom(12, 12, 8)
    V = v0(g)
    assert np.all(V < 0)
    lap = (V[2:, 1:-1, 1:-1] + V[:-2, 1:-1, 1:-1] + V[1:-1, 2:, 1:-1] + V[1:-1, :-2, 1:-1]
           + V[1:-1, 1:-1, 2:] + V[1:-1, 1:-1, :-2] - 6 * V[1:-1, 1:-1, 1:-1])
    assert np.abs(lap).max() < 0.05 * np.abs(V).max()
    s = sources(g)
    assert s.shape == (10, 3) and np.all((s[:, 2] > g.nz) & (s[:, 2] < g.d))


def test_recovery_formula():
    V0 = np.full((2, 2, 2), -0.5)
    c0 = 0.5
    xi_true = np.array([0.0, 1 / c0 ** 2 - 0.25, 1 / c0 ** 2 - 1 / 9, 1 / c0 ** 2 + 1.0, 1 / c0 ** 2,
                        -1.0, 0.1, 2.0]).reshape(2, 2, 2)
    xi, c, ncl = recovery.recover(xi_true * V0, V0, c0)
    assert np.allclose(xi, xi_true, rtol=0, atol=1e-15)
    assert c.ravel()[0] == pytest.approx(c0) and c.ravel()[1] == pytest.approx(2.0) \
        and c.ravel()[2] == pytest.approx(3.0)
    assert ncl == 2 and c.ravel()[3] == pytest.approx(1 / math.sqrt(1e-6 / c0 ** 2))


# ---------------------------------------------------------------- synthesis

def test_synth_noise_level_exact():
    g = Geom(8, 8, 8)
    inst = inputs.workload_instance(1, 3, n=8)
    d = synth.make_data(g, inst["xi"], inst["noise"], 0.03)
    assert np.linalg.norm(d["F"] - d["AF"]) == pytest.approx(0.03 * np.linalg.norm(d["AF"]), rel=1e-12)
    assert d["delta"] == pytest.approx(0.03 * np.linalg.norm(d["AF"]), rel=1e-12)


# ---------------------------------------------------------------- features

def test_level_index_rule():
    # level = floor(4 log10(s / s_max)) + 64 clipped to [0, 63], by comparison
    # with the thresholds s_max 10^((j - 64)/4)
    smax = 3.7
    r = inputs.rng(21)
    s = smax * 10.0 ** r.uniform(-18.0, 0.0, size=4000)
    b = features.level_index(s, smax)
    ref = np.clip(np.floor(4.0 * np.log10(s / smax)) + 64, 0, 63).astype(np.int64)
    thr = features.thresholds(smax)
    near = np.min(np.abs(s[:, None] / thr[None, :] - 1.0), axis=1) < 1e-9
    assert np.array_equal(b[~near], ref[~near]) and (~near).sum() > 3900
    # exact thresholds open their level; s_max and above go to 63, zero to 0
    assert list(features.level_index(thr, smax)) == list(range(1, 64))
    assert list(features.level_index(np.nextafter(thr, 0.0), smax)) == list(range(0, 63))
    assert features.level_index(np.array([smax, 2 * smax, 0.0, 1e-300]), smax).tolist() == [63, 63, 0, 0]
    assert len(thr) == 63 and np.all(np.diff(thr) > 0)
    assert thr[-1] == pytest.approx(smax * 10 ** -0.25, rel=1e-15) and thr[0] == pytest.approx(smax * 10 ** -15.75, rel=1e-15)
    # only s / s_max matters
    assert np.array_equal(features.level_index(7.0 * s, 7.0 * smax), b)


def test_level_energy_parseval():
    g = Geom(8, 6, 4)
    F = inputs.rng(13).standard_normal(g.shape)
    fh = np.fft.fftn(pad(g, F))
    khat = np.fft.fftn(sample_kernel(g))
    s = (khat * khat.conj()).real
    E = features.level_energy(fh, s, s.max())
    assert E.sum() == pytest.approx(np.prod(g.pshape) * np.sum(F * F), rel=1e-12)
    # the sampled kernel spreads its spectrum over many levels
    assert (features.level_index(s, s.max()) == 63).any() and len(np.unique(features.level_index(s, s.max()))) > 10


def test_features_values_on_a_hand_built_spectrum():
    # 8^3 spectrum with |f^|^2 = 4 at k = 0 where s = s_max = 1 (level 63),
    # 9 at k = (0,0,1) and at (0,0,7) where s = 0.0125 (log10 -1.90 -> level
    # 56), 1 at the corner (4,4,4) where s = 2e-16 (log10 -15.70 -> level 1);
    # s = 1e-20 elsewhere (level 0, no energy).  Mean level energy
    # (4 + 18 + 1)/64; empty levels give log10(1e-30) = -30;
    # x_64 = log10(delta/||F||).
    fh = np.zeros((8, 8, 8), complex)
    fh[0, 0, 0] = 2.0
    fh[0, 0, 1] = 3.0
    fh[0, 0, 7] = 3.0j
    fh[4, 4, 4] = -1.0
    s = np.full((8, 8, 8), 1e-20)
    s[0, 0, 0] = 1.0
    s[0, 0, 1] = s[0, 0, 7] = 0.0125
    s[4, 4, 4] = 2e-16
    x, E = features.features(fh, 0.5, 20.0, s)
    ref = np.full(65, -30.0)
    ref[63] = math.log10(4 * 64 / 23)
    ref[56] = math.log10(18 * 64 / 23)
    ref[1] = math.log10(64 / 23)
    ref[64] = math.log10(0.025)
    assert np.max(np.abs(x - ref)) < 1e-13
    assert E[63] == 4 and E[56] == 18 and E[1] == 1 and E.sum() == 23
    # the identity kernel (s = 1 everywhere): all energy in the top level
    x1, E1 = features.features(fh, 0.5, 20.0, np.ones((8, 8, 8)))
    assert E1[63] == 23 and E1[:63].sum() == 0 and x1[63] == pytest.approx(math.log10(64))


# ---------------------------------------------------------------- MLP reference

def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 1 + 2 ** -8 + 2 ** -20])
    out = mlp.bf16_round(vals)
    assert list(out) == [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 1 + 2 ** -7]


def test_gelu_known_values():
    # GELU(x) = x Phi(x); Phi(1) = 0.8413447460685429 (standard normal CDF).
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert mlp.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(np.array(-1.0)) == pytest.approx(-0.15865525393145707, rel=1e-14)


def test_mlp_gradients_against_central_differences():
    p = mlp.init_params(3)
    X = inputs.rng(14).standard_normal((6, mlp.D_IN))
    t = inputs.rng(15).standard_normal(6)
    y, cache = mlp.forward(p, X, bf16=False)
    g = mlp.backward(p, cache, t, bf16=False)
    rg = inputs.rng(16)
    eps = 1e-6
    for name, _ in mlp.PARAM_SHAPES:
        idxs = [tuple(rg.integers(0, s) for s in p[name].shape) for _ in range(6)]
        for idx in idxs:
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += eps
            pm[name][idx] -= eps
            fd = (mlp.loss(mlp.forward(pp, X, False)[0], t) - mlp.loss(mlp.forward(pm, X, False)[0], t)) / (2 * eps)
            assert g[name][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_first_step():
    # After one step from zero moments the bias-corrected update is lr * g / (|g| + eps).
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 0.0])}
    opt = mlp.Adam(p, lr=1e-3)
    out = opt.step({"w": p["w"].copy()}, g)
    assert np.allclose(out["w"], p["w"] - 1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=0, atol=1e-15)


def test_mlp_param_count():
    p = mlp.init_params(0)
    assert sum(v.size for v in p.values()) == 25089


# ---------------------------------------------------------------- Algorithm 1 with per-frequency z-systems (Sec. 5)



@pytest.mark.parametrize("shape,kind", [((4, 3, 5), 0), ((3, 4, 4), 1), ((6, 6, 2), 0)])
def test_layered_forward_equals_direct_quadrature(shape, kind):
    # Eq. (14)'s systems, assembled from the lateral transform of the kernel,
    # reproduce the direct quadrature sum of Eq. (8) exactly (no wrap in z).
    nz, ny, nx = shape
    g = Geom(nx, ny, nz, kind=kind)
    kt = layered.lateral_kernel_spectrum(g)
    assert np.abs(kt.imag).max() < 1e-12 * np.abs(kt).max()   # K even in x and y
    z = inputs.rng(21).standard_normal(shape)
    assert np.allclose(layered.forward_layered(g, kt, z), forward_direct(g, z), rtol=0,
                       atol=1e-12 * np.abs(forward_direct(g, z)).max())


@pytest.mark.parametrize("method", [tikhonov.TIKHONOV, tikhonov.TSVD])
@pytest.mark.parametrize("shape", [(2, 2, 3), (3, 2, 2)])
def test_layered_solve_equals_assembled_operator(shape, method):
    # The per-frequency regularisation is the regularisation of the whole
    # (laterally embedded, z-exact) operator: normal equations / SVD of the
    # explicit matrix give the same estimate and residual.
    nz, ny, nx = shape
    g = Geom(nx, ny, nz)
    kt = layered.lateral_kernel_spectrum(g)
    F = inputs.rng(22).standard_normal(shape)
    S = np.linalg.svd(layered.assembled_operator(g), compute_uv=False)
    lam = np.unique(np.round(S * S, 12))
    alpha = 1e-3 if method == tikhonov.TIKHONOV else 0.5 * (lam[len(lam) // 2] + lam[len(lam) // 2 + 1])
    sp = layered.solve_layered(g, kt, F, alpha, method)
    de = layered.dense_layered(g, F, alpha, method)
    assert np.linalg.norm(sp["zeta"] - de["zeta"]) < 1e-9 * np.linalg.norm(de["zeta"])
    assert np.linalg.norm(sp["r"] - de["r"]) < 1e-9 * np.linalg.norm(de["r"])
    assert sp["imag_max"] < 1e-10 * np.abs(sp["zeta"]).max()
    # singular values of the assembled operator = those of all per-frequency systems
    Sf = np.sort(sp["singular_values"].ravel())
    assert np.allclose(np.sort(S)[-len(Sf):], Sf, rtol=1e-9, atol=1e-12 * S.max())


def test_layered_filters_and_monotone_residual():
    g = Geom(8, 8, 6)
    kt = layered.lateral_kernel_spectrum(g)
    F = inputs.rng(23).standard_normal(g.shape)
    prev = -1.0
    for a in (1e-6, 1e-4, 1e-2, 1.0):
        o = layered.solve_layered(g, kt, F, a)
        assert o["r_norm"] > prev
        prev = o["r_norm"]
    # iterated Tikhonov of order 1 = Tikhonov; higher order fits more closely
    o1 = layered.solve_layered(g, kt, F, 1e-3)
    i1 = layered.solve_layered(g, kt, F, 1e-3, tikhonov.ITERATED, 1)
    i3 = layered.solve_layered(g, kt, F, 1e-3, tikhonov.ITERATED, 3)
    assert np.allclose(o1["zeta"], i1["zeta"], rtol=0, atol=1e-12 * np.abs(o1["zeta"]).max())
    assert i3["r_norm"] < o1["r_norm"]


# ---------------------------------------------------------------- exact restricted-operator Tikhonov (Sec. 3-4)

from oracle import exact  # noqa: E402


@pytest.mark.parametrize("shape,kind", [((3, 4, 5), 0), ((4, 3, 3), 1)])
def test_exact_adjoint(shape, kind):
    # <A z, r>_Y = <z, A^T r>_R, and the spectral adjoint equals the direct sum
    nz, ny, nx = shape
    g = Geom(nx, ny, nz, kind=kind, hz=0.75)
    khat = np.fft.fftn(sample_kernel(g))
    z = inputs.rng(31).standard_normal(shape)
    r = inputs.rng(32).standard_normal(shape)
    at = exact.adjoint(g, khat, r)
    assert np.allclose(at, exact.adjoint_direct(g, r), rtol=0, atol=1e-12 * np.abs(at).max())
    lhs = float(np.sum(forward_direct(g, z) * r))
    rhs = float(np.sum(z * exact.adjoint_direct(g, r)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("alpha", [1e-1, 1e-3])
def test_exact_cg_equals_dense_normal_equations(alpha):
    g = Geom(4, 3, 3)
    F = inputs.rng(33).standard_normal(g.shape)
    de = exact.dense_exact(g, F, alpha)
    cg = exact.cg_exact(g, F, alpha, tol=1e-13)
    assert np.linalg.norm(cg["zeta"] - de["zeta"]) < 1e-9 * np.linalg.norm(de["zeta"])
    assert cg["r_norm"] == pytest.approx(de["r_norm"], rel=1e-9)
    # it minimises the exact functional: the embedded estimate restricted to R,
    # a feasible point, scores no better
    emb = tikhonov.solve_spectral(g, np.fft.fftn(sample_kernel(g)), F, alpha)["zeta"]

    def obj(z):
        return float(np.sum((forward_direct(g, z) - F) ** 2) + alpha * np.sum(z * z))
    assert obj(de["zeta"]) <= obj(emb) * (1 + 1e-12)
    assert obj(de["zeta"]) <= obj(de["zeta"] + 1e-3 * inputs.rng(34).standard_normal(g.shape))


def test_per_frequency_alphas_meet_their_discrepancy():
    # Algorithm 1 step 2 per frequency: every system's alpha is re-checked by an
    # independent dense normal-equation solve of that system (no SVD): inside
    # the tolerance, or on the flagged side of the target at the range end.
    g = Geom(4, 4, 5)
    kt = layered.lateral_kernel_spectrum(g)
    d = synth.make_data(g, inputs.xi_blobs(g.shape, 3, count=2, sigma=(1.0, 1.5)), inputs.noise(g.shape, 3), 0.05)
    F, delta = d["F"], d["delta"]
    out = layered.solve_per_frequency(g, kt, F, delta, tol=1e-6)
    A = layered.system_matrices(g, kt)
    fh = np.moveaxis(layered.lateral_spectrum(g, F), 0, 2)
    seen = set()
    for iy in range(A.shape[0]):
        for ix in range(A.shape[1]):
            a, fl = out["alphas"][iy, ix], out["flags"][iy, ix]
            Am, f = A[iy, ix], fh[iy, ix]
            x = np.linalg.solve(Am.T @ Am + a * np.eye(Am.shape[1]), Am.T @ f)
            r = np.linalg.norm(Am @ x - f)
            seen.add(int(fl))
            if fl == 0:
                assert abs(r / delta - 1) <= 1e-6 * (1 + 1e-6)
            elif fl == discrepancy.NOROOT_HIGH:
                assert a == 1.0 and r < delta
            elif fl == discrepancy.NOROOT_LOW:
                assert a == pytest.approx(1e-8) and r > delta
    assert 0 in seen and len(seen) >= 2          # the case mix the data produce
    assert out["imag_max"] < 1e-10 * np.abs(out["zeta"]).max()
    # with one alpha everywhere the per-frequency form reduces to the global one
    glob = layered.solve_layered(g, kt, F, 1e-3)
    same = layered.solve_per_frequency(g, kt, F, 0.0, lo=-3.0, hi=-3.0 + 1e-12, tol=0.0, max_steps=0)
    assert np.abs(same["alphas"] - 1e-3).max() < 1e-14
    assert np.linalg.norm(same["zeta"] - glob["zeta"]) < 1e-12 * np.linalg.norm(glob["zeta"])
