"""Pins of the oracle's semilocal LDA correlation (eq. 1's E_c^LDA, PW92 of the appendix):
the uniform-gas closed form, the functional derivative by finite differences, the high- and
low-density limits of v_c, and the vacuum rule."""
import math

import numpy as np
import pytest

from oracle import vdwdf

A = vdwdf.PW92_A


def triclinic_cell():
    return np.array([[7.0, 0.0, 0.0], [1.5, 6.0, 0.0], [-0.7, 0.9, 8.0]])


def test_uniform_gas_energy_is_volume_times_n_eps():
    # E = Omega n eps_c(r_s) with the textbook Wigner-Seitz radius r_s = (3/(4 pi n))^(1/3)
    cell = triclinic_cell()
    omega = abs(np.linalg.det(cell))
    for n0 in (1e-5, 3e-3, 0.2, 7.0):
        rs = (3.0 / (4.0 * math.pi * n0)) ** (1.0 / 3.0)
        eps, _ = vdwdf.pw92_correlation(rs)
        E, v = vdwdf.lda_correlation(np.full((3, 4, 5), n0), cell)
        assert E == pytest.approx(omega * n0 * float(eps), rel=1e-13)
        assert np.ptp(v) == 0.0


def test_potential_is_the_derivative_of_the_energy():
    # dE/dn_j = v_j Omega/N at every point (Richardson-extrapolated central differences).  The
    # differences are taken with the other points in vacuum, where they add nothing (pinned
    # below), so that the change of E is not lost against the rest of the sum.
    rng = np.random.default_rng(3)
    cell = triclinic_cell()
    n = np.exp(rng.uniform(np.log(1e-6), np.log(10.0), size=(3, 4, 5)))
    E, v = vdwdf.lda_correlation(n, cell)
    dV = abs(np.linalg.det(cell)) / n.size
    for j in range(n.size):
        h = 1e-3 * n.flat[j]

        def d(step):
            a, b = np.zeros_like(n), np.zeros_like(n)
            a.flat[j] = n.flat[j] + step
            b.flat[j] = n.flat[j] - step
            return (vdwdf.lda_correlation(a, cell)[0] - vdwdf.lda_correlation(b, cell)[0]) / (2 * step)
        fd = (4.0 * d(h / 2) - d(h)) / 3.0
        assert fd == pytest.approx(v.flat[j] * dV, rel=1e-9), j
    # and the energy is the sum of the points' parts
    parts = sum(vdwdf.lda_correlation(np.where(np.arange(n.size).reshape(n.shape) == j, n, 0.0), cell)[0]
                for j in range(n.size))
    assert E == pytest.approx(parts, rel=1e-13)


def test_high_density_limit_of_v_minus_eps():
    # eps_c -> A ln r_s + c (Gell-Mann--Brueckner), so v - eps = -(r_s/3) d eps/d r_s -> -A/3,
    # with A the exact coefficient (1 - ln 2)/pi^2
    n = np.array([3.0 / (4.0 * math.pi * 1e-8 ** 3)])
    _, v = vdwdf.lda_correlation(n, np.eye(3))
    rs = 1e-8
    eps, _ = vdwdf.pw92_correlation(rs)
    assert v[0] - float(eps) == pytest.approx(-(1.0 - math.log(2.0)) / (3.0 * math.pi ** 2), rel=5e-4)
    assert v[0] - float(eps) == pytest.approx(-A / 3.0, rel=1e-3)


def test_low_density_limit_of_v_over_eps():
    # eps_c ~ -(alpha1/beta4)/r_s for r_s -> inf, i.e. n eps_c ~ n^(4/3): v = (4/3) eps
    rs = 1e8
    n = np.array([3.0 / (4.0 * math.pi * rs ** 3)])
    _, v = vdwdf.lda_correlation(n, np.eye(3))
    eps, _ = vdwdf.pw92_correlation(rs)
    assert v[0] / float(eps) == pytest.approx(4.0 / 3.0, rel=1e-3)
    assert float(eps) * rs == pytest.approx(-vdwdf.PW92_ALPHA1 / vdwdf.PW92_BETA[3], rel=1e-3)


def test_vacuum_points_add_nothing():
    cell = np.eye(3) * 2.0
    n = np.array([0.0, 1e-31, 1e-29, 0.5]).reshape(1, 2, 2)
    E, v = vdwdf.lda_correlation(n, cell)
    assert v.flat[0] == 0.0 and v.flat[1] == 0.0 and v.flat[2] < 0.0
    E2, _ = vdwdf.lda_correlation(np.array([0.0, 0.0, 1e-29, 0.5]).reshape(1, 2, 2), cell)
    assert E == E2
