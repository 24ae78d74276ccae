"""Pins of the oracle's helper splines (Sec. 2), FFT conventions (Sec. 3) and |G| geometry."""
import itertools
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import vdwdf
from paper_1703_06999_amd import inputs

Q = inputs.log_qmesh()


def test_qmesh_shape():
    assert Q.shape == (20,) and Q[0] == pytest.approx(1e-5) and Q[-1] == pytest.approx(5.0)
    assert np.all(np.diff(Q) > 0)


def test_spline_kronecker_at_knots():
    c = vdwdf.spline_coefficients(Q)
    p, _ = vdwdf.spline_values(Q, c, Q)          # p[a][b] = p_a(q_b)
    np.testing.assert_allclose(p, np.eye(20), atol=1e-13)


def test_spline_matches_library_natural_spline():
    c = vdwdf.spline_coefficients(Q)
    q = np.random.default_rng(0).uniform(Q[0], Q[-1], 500)
    p, dp = vdwdf.spline_values(Q, c, q)
    for a in range(20):
        cs = CubicSpline(Q, np.eye(20)[a], bc_type="natural")
        np.testing.assert_allclose(p[a], cs(q), atol=1e-13)
        np.testing.assert_allclose(dp[a], cs(q, 1), atol=1e-11 * max(1, np.max(np.abs(dp[a]))))


def test_spline_partition_of_unity_and_linear_reproduction():
    c = vdwdf.spline_coefficients(Q)
    q = np.linspace(Q[0], Q[-1], 2001)
    p, dp = vdwdf.spline_values(Q, c, q)
    np.testing.assert_allclose(p.sum(axis=0), 1.0, atol=1e-13)
    np.testing.assert_allclose((Q[:, None] * p).sum(axis=0), q, atol=1e-13)
    np.testing.assert_allclose(dp.sum(axis=0), 0.0, atol=1e-10)


def test_spline_continuity_and_natural_ends():
    c = vdwdf.spline_coefficients(Q)
    h = np.diff(Q)
    a0, a1, a2, a3 = c
    # value, slope and curvature at the right end of interval b equal those at the left of b+1
    for b in range(18):
        d = h[b]
        np.testing.assert_allclose(a0[:, b] + a1[:, b] * d + a2[:, b] * d ** 2 + a3[:, b] * d ** 3,
                                   a0[:, b + 1], atol=1e-12)
        np.testing.assert_allclose(a1[:, b] + 2 * a2[:, b] * d + 3 * a3[:, b] * d ** 2, a1[:, b + 1],
                                   atol=1e-9 * np.max(np.abs(a1[:, b + 1])))
        np.testing.assert_allclose(2 * a2[:, b] + 6 * a3[:, b] * d, 2 * a2[:, b + 1],
                                   atol=1e-9 * np.max(np.abs(a2[:, b + 1])) + 1e-9)
    assert np.all(a2[:, 0] == 0.0)
    np.testing.assert_allclose(2 * a2[:, 18] + 6 * a3[:, 18] * h[18], 0.0, atol=1e-12)


def test_spline_derivative_finite_difference():
    c = vdwdf.spline_coefficients(Q)
    q = np.random.default_rng(1).uniform(0.01, 4.9, 200)
    _, dp = vdwdf.spline_values(Q, c, q)
    hh = 1e-7
    fd = (vdwdf.spline_values(Q, c, q + hh)[0] - vdwdf.spline_values(Q, c, q - hh)[0]) / (2 * hh)
    np.testing.assert_allclose(dp, fd, atol=2e-6 * np.max(np.abs(dp)))


def naive_dft(f):
    n1, n2, n3 = f.shape
    out = np.zeros(f.shape, dtype=complex)
    for m in itertools.product(range(n1), range(n2), range(n3)):
        s = 0j
        for j in itertools.product(range(n1), range(n2), range(n3)):
            s += f[j] * np.exp(-2j * np.pi * (j[0] * m[0] / n1 + j[1] * m[1] / n2 + j[2] * m[2] / n3))
        out[m] = s
    return out


@pytest.mark.parametrize("shape", [(1, 2, 2), (2, 2, 2), (3, 3, 3), (4, 6, 5)])
def test_fft_against_naive_dft(shape):
    f = np.random.default_rng(4).normal(size=shape)
    np.testing.assert_allclose(vdwdf.forward_fft(f), naive_dft(f), atol=1e-12 * f.size)
    np.testing.assert_allclose(vdwdf.inverse_fft(vdwdf.forward_fft(f)), f, atol=1e-14)


def test_fft_closed_forms():
    shape = (8, 9, 10)
    d = np.zeros(shape)
    d[0, 0, 0] = 1.0
    np.testing.assert_allclose(vdwdf.forward_fft(d), np.ones(shape), atol=1e-15)
    j = np.indices(shape)
    m = (2, 7, 3)
    pw = np.cos(2 * np.pi * (j[0] * m[0] / 8 + j[1] * m[1] / 9 + j[2] * m[2] / 10))
    fk = vdwdf.forward_fft(pw)
    expect = np.zeros(shape, dtype=complex)
    expect[m] = expect[(8 - m[0]) % 8, (9 - m[1]) % 9, (10 - m[2]) % 10] = pw.size / 2
    np.testing.assert_allclose(fk, expect, atol=1e-10)


def test_gvector_norms_orthogonal_and_even():
    cell = np.diag([3.0, 4.5, 5.0])
    grid = (4, 5, 6)
    kn = vdwdf.gvector_norms(grid, cell)
    for m in itertools.product(*(range(g) for g in grid)):
        mb = [mi if mi <= g // 2 else mi - g for mi, g in zip(m, grid)]
        expect = math.sqrt(sum((2 * math.pi * mb[i] / cell[i, i]) ** 2 for i in range(3)))
        assert kn[m] == pytest.approx(expect, rel=1e-14, abs=1e-14)


def test_gvector_norms_sheared_cell_even_in_g():
    cell = np.array([[4.0, 0.0, 0.0], [1.3, 3.5, 0.0], [0.4, -0.7, 5.0]])
    grid = (4, 6, 5)
    kn = vdwdf.gvector_norms(grid, cell)
    B = 2 * np.pi * np.linalg.inv(cell).T
    for m in itertools.product(*(range(g) for g in grid)):
        neg = tuple((-mi) % g for mi, g in zip(m, grid))
        assert kn[m] == pytest.approx(kn[neg], rel=1e-14)
        nyq = [g % 2 == 0 and mi == g // 2 for mi, g in zip(m, grid)]
        if not any(nyq):
            mb = np.array([mi if mi <= g // 2 else mi - g for mi, g in zip(m, grid)], dtype=float)
            assert kn[m] == pytest.approx(np.linalg.norm(mb @ B), rel=1e-13, abs=1e-14)
        else:
            # mean of |G|^2 over the two aliases +N/2 and -N/2 of the Nyquist components
            mb = np.array([mi if mi < g / 2 else mi - g for mi, g in zip(m, grid)], dtype=float)
            alt = mb.copy()
            for i in range(3):
                if nyq[i]:
                    alt[i] = -mb[i]
            g2 = 0.5 * (np.sum((mb @ B) ** 2) + np.sum((alt @ B) ** 2))
            assert kn[m] == pytest.approx(math.sqrt(g2), rel=1e-13)
