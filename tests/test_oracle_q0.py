"""Pins of the oracle's q0, PW92 correlation and saturation function (paper appendix) against
closed forms, textbook identities and finite differences."""
import math

import numpy as np
import pytest

from oracle import vdwdf


def test_printed_constants():
    # appendix: A, alpha1, beta1..4, Z_ab (DF1, DF2), a = 5, 12 terms
    assert vdwdf.PW92_A == 0.031091
    assert vdwdf.PW92_ALPHA1 == 0.2137
    assert vdwdf.PW92_BETA == (7.5957, 3.5876, 1.6382, 0.49294)
    assert vdwdf.ZAB["DF1"] == -0.8491 and vdwdf.ZAB["DF2"] == -1.887
    assert vdwdf.SATURATION_A == 5.0 and vdwdf.SATURATION_TERMS == 12


def test_pw92_high_density_slope_is_gell_mann_brueckner():
    # eps_c -> A ln r_s + const for r_s -> 0; A equals the exact coefficient (1 - ln 2)/pi^2
    rs = np.array([1e-8, 1e-7])
    eps, _ = vdwdf.pw92_correlation(rs)
    slope = (eps[1] - eps[0]) / math.log(10.0)
    assert slope == pytest.approx((1.0 - math.log(2.0)) / math.pi ** 2, rel=2e-4)
    # and the constant term is -2A ln(2 A beta1) (leading order of log(1 + 1/Q), Q ~ 2A beta1 sqrt(rs))
    c = eps[0] - vdwdf.PW92_A * math.log(rs[0])
    A, b1 = vdwdf.PW92_A, vdwdf.PW92_BETA[0]
    assert c == pytest.approx(2.0 * A * math.log(2.0 * A * b1), rel=1e-3)


def test_pw92_low_density_tail():
    # r_s -> inf: Q ~ 2A beta4 r_s^2 so eps_c r_s -> -alpha1/beta4
    rs = 1e14
    eps, _ = vdwdf.pw92_correlation(rs)
    assert eps * rs == pytest.approx(-vdwdf.PW92_ALPHA1 / vdwdf.PW92_BETA[3], rel=1e-5)
    assert np.all(vdwdf.pw92_correlation(np.geomspace(1e-3, 1e3, 50))[0] < 0)


def test_pw92_derivative_finite_difference():
    rs = np.geomspace(0.01, 200.0, 37)
    h = 1e-6 * rs
    _, d = vdwdf.pw92_correlation(rs)
    fd = (vdwdf.pw92_correlation(rs + h)[0] - vdwdf.pw92_correlation(rs - h)[0]) / (2 * h)
    np.testing.assert_allclose(d, fd, rtol=1e-7)


def test_q0_uniform_gas_is_ratio_of_lda_energies():
    # appendix: q0 = (eps_xc^0 / eps_x^LDA) k_F; for sigma = 0 eps_xc^0 = eps_x^LDA + eps_c^LDA with
    # eps_x^LDA = -3 k_F/(4 pi), and r_s k_F = (9 pi / 4)^{1/3} (textbook identities)
    n = np.geomspace(1e-6, 10.0, 23)
    kF = (3.0 * math.pi ** 2 * n) ** (1.0 / 3.0)
    rs = (9.0 * math.pi / 4.0) ** (1.0 / 3.0) / kF
    eps_c, _ = vdwdf.pw92_correlation(rs)
    eps_x = -3.0 * kF / (4.0 * math.pi)
    expect = (eps_x + eps_c) / eps_x * kF
    x, _, _ = vdwdf.q0_unsaturated(n, np.zeros_like(n), vdwdf.ZAB["DF1"])
    np.testing.assert_allclose(x, expect, rtol=1e-13)


def test_q0_gradient_term_sign_and_flavours():
    n = np.array([1e-3, 0.01, 0.1, 1.0])
    s = np.array([1e-6, 1e-3, 0.05, 2.0])
    x0, _, _ = vdwdf.q0_unsaturated(n, 0 * s, -0.8491)
    x1, _, _ = vdwdf.q0_unsaturated(n, s, -0.8491)
    x2, _, _ = vdwdf.q0_unsaturated(n, s, -1.887)
    kF = (3.0 * math.pi ** 2 * n) ** (1.0 / 3.0)
    np.testing.assert_allclose(x1 - x0, 0.8491 / 36.0 * s / (kF * n * n), rtol=1e-9)
    np.testing.assert_allclose((x2 - x0) / (x1 - x0), 1.887 / 0.8491, rtol=1e-9)
    assert np.all(x1 > x0)   # Z_ab < 0: gradients raise q0


@pytest.mark.parametrize("flavour", ["DF1", "DF2"])
def test_q0_partials_finite_difference(flavour):
    rng = np.random.default_rng(3)
    n = 10.0 ** rng.uniform(-3, 0, 40)
    s = n ** (8.0 / 3.0) * 10.0 ** rng.uniform(-2, 1, 40)
    zab = vdwdf.ZAB[flavour]
    _, dn, ds = vdwdf.q0_unsaturated(n, s, zab)
    hn, hs = 1e-6 * n, 1e-2 * s   # x is linear in sigma
    fdn = (vdwdf.q0_unsaturated(n + hn, s, zab)[0] - vdwdf.q0_unsaturated(n - hn, s, zab)[0]) / (2 * hn)
    fds = (vdwdf.q0_unsaturated(n, s + hs, zab)[0] - vdwdf.q0_unsaturated(n, s - hs, zab)[0]) / (2 * hs)
    np.testing.assert_allclose(dn, fdn, rtol=1e-7)
    np.testing.assert_allclose(ds, fds, rtol=1e-7)


def test_saturation_against_series_identity():
    # sum_{m>=1} t^m/m = -ln(1-t), so with 12 terms h_a(x) = a [1 - (1-t) exp(sum_{m>12} t^m/m)]
    a = 5.0
    t = np.linspace(0.05, 0.95, 31)
    tail = sum(t ** m / m for m in range(13, 4000))
    expect = a * (1.0 - (1.0 - t) * np.exp(tail))
    h, _ = vdwdf.saturation(a * t)
    np.testing.assert_allclose(h, expect, rtol=1e-13, atol=1e-14)
    # to first order in the tail R: h - x = -a (1-t) R, R = sum_{m>12} t^m/m
    tt = np.array([0.3, 0.4])
    R = sum(tt ** m / m for m in range(13, 4000))
    h, _ = vdwdf.saturation(a * tt)
    np.testing.assert_allclose(h - a * tt, -a * (1 - tt) * R, rtol=1e-6)


def test_saturation_shape_and_derivative():
    a = 5.0
    x = np.linspace(0.0, 30.0, 3001)
    h, hp = vdwdf.saturation(x)
    assert np.all(np.diff(h) >= 0) and np.all(h <= a) and h[-1] == a
    assert np.all(h[1:] < x[1:] + 1e-15)
    xs = np.linspace(0.1, 9.9, 60)
    fd = (vdwdf.saturation(xs + 1e-6)[0] - vdwdf.saturation(xs - 1e-6)[0]) / 2e-6
    np.testing.assert_allclose(vdwdf.saturation(xs)[1], fd, rtol=1e-6, atol=1e-9)
    # exact underflow for t >= 2: h = a, h' = 0, no NaN even for huge arguments
    h, hp = vdwdf.saturation(np.array([10.0, 1e10, 1e300]))
    assert np.all(h == a) and np.all(hp == 0.0)


def test_q0_vacuum_clamp_and_saturation_paths():
    q = np.array([1e-5, 0.1, 5.0])
    n = np.array([0.0, -1.0, 1e-31, 1e-24, 1e-3, 50.0, 1.0])
    s = np.array([0.0, 0.0, 0.0, 0.0, 1e-6, 0.0, 1e6])
    q0, dn, ds, vac = vdwdf.q0_and_derivatives(n, s, q, -0.8491)
    assert list(vac) == [True, True, True, False, False, False, False]
    assert q0[3] == 1e-5 and dn[3] == 0 and ds[3] == 0          # below the mesh: clamped
    assert q0[6] == 5.0 and dn[6] == 0 and ds[6] == 0           # saturated
    assert np.all(np.isfinite(q0)) and np.all(np.isfinite(dn)) and np.all(np.isfinite(ds))
