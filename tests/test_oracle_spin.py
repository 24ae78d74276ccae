"""Pins of the oracle's spin-polarised variant (Sec. 7 announces it; the paper prints no spin q0,
so the reading of the oracle's header is pinned here through what fixes it from outside):

* the spin interpolation f(zeta): its end values and f''(0) = 8 / (9 (2^{4/3} - 2)) by finite
  differences (pins the printed constant and f together);
* the spin-resolved PW92 fits: the zeta = 0 row is the appendix's form, and the high-density
  coefficients of the fully polarised gas and of the spin stiffness are the exact ones,
  (1 - ln 2)/(2 pi^2) and 1/(6 pi^2) (a mistyped A or a dropped sign fails them);
* the exchange part of q0: the fully polarised uniform gas gives 2^{1/3} k_F (exchange spin
  scaling, closed form);
* the reduction to the spin-paired functional at n_up = n_dn = n/2, sigma_uu = sigma_dd = sigma/4:
  the same q0, the same energy, dE/dn_s = dE/dn and dE/dsigma_ss = 2 dE/dsigma, on a grid with
  vacuum, saturation and the below-mesh clamp;
* the partial derivatives of q0 and of the energy by central finite differences on polarised
  inputs (this pins the chain rule of every channel, of zeta and of r_s);
* the exchange of the two spins."""
import math

import numpy as np
import pytest

from oracle import vdwdf
from paper_1703_06999_amd import inputs

KT = inputs.synthetic_kernel_table(nk=512, kmax=30.0)
ZAB = vdwdf.ZAB["DF1"]


def test_spin_interpolation_ends_and_curvature():
    f, _ = vdwdf.spin_interpolation(np.array([0.0, 1.0, -1.0]))
    assert f[0] == 0.0
    assert f[1] == pytest.approx(1.0, abs=1e-15) and f[2] == pytest.approx(1.0, abs=1e-15)
    h = 1e-4
    fp, _ = vdwdf.spin_interpolation(np.array([h, -h]))
    curvature = (fp[0] + fp[1]) / h ** 2
    assert curvature == pytest.approx(8.0 / (9.0 * (2.0 ** (4.0 / 3.0) - 2.0)), rel=1e-6)
    assert curvature == pytest.approx(vdwdf.PW92_FZZ0, rel=1e-6)
    z = np.linspace(-0.9, 0.9, 7)
    fz, dfz = vdwdf.spin_interpolation(z)
    fd = (vdwdf.spin_interpolation(z + 1e-6)[0] - vdwdf.spin_interpolation(z - 1e-6)[0]) / 2e-6
    assert np.allclose(dfz, fd, rtol=1e-8, atol=1e-8)   # the differences round to ~1e-10


def test_pw92_form_reproduces_the_appendix_set():
    rs = np.geomspace(1e-3, 1e3, 13)
    e, de = vdwdf.pw92_correlation(rs)
    g, dg = vdwdf.pw92_G(rs, vdwdf.PW92_A, vdwdf.PW92_ALPHA1, vdwdf.PW92_BETA)
    assert np.array_equal(e, g) and np.array_equal(de, dg)


def test_spin_correlation_limits_and_symmetry():
    rs = np.geomspace(1e-2, 1e2, 9)
    e0, _ = vdwdf.pw92_correlation(rs)
    eps, _, _ = vdwdf.pw92_spin_correlation(rs, 0.0)
    assert np.array_equal(eps, e0)
    e1, _ = vdwdf.pw92_G(rs, *vdwdf.PW92_FERRO)
    for z in (1.0, -1.0):
        assert np.allclose(vdwdf.pw92_spin_correlation(rs, z)[0], e1, rtol=1e-14, atol=0)
    for z in (0.3, 0.77):
        assert np.array_equal(vdwdf.pw92_spin_correlation(rs, z)[0], vdwdf.pw92_spin_correlation(rs, -z)[0])
    # polarising a gas raises its correlation energy per particle (less negative)
    assert np.all(vdwdf.pw92_spin_correlation(rs, 0.5)[0] > e0)
    assert np.all(e1 > e0)


def test_high_density_coefficients_are_the_exact_ones():
    # eps_c(r_s, 1) -> A_1 ln r_s with A_1 = (1 - ln 2)/(2 pi^2); alpha_c(r_s) -> -ln(r_s)/(6 pi^2)
    r1, r2 = 1e-9, 1e-8
    e1 = vdwdf.pw92_G(np.array([r1, r2]), *vdwdf.PW92_FERRO)[0]
    assert (e1[1] - e1[0]) / math.log(r2 / r1) == pytest.approx((1.0 - math.log(2.0)) / (2.0 * math.pi ** 2),
                                                                 rel=2e-3)
    ma = vdwdf.pw92_G(np.array([r1, r2]), *vdwdf.PW92_MINUS_ALPHA)[0]
    alpha = -ma
    assert (alpha[1] - alpha[0]) / math.log(r2 / r1) == pytest.approx(-1.0 / (6.0 * math.pi ** 2), rel=2e-3)


def test_spin_correlation_partials_by_finite_differences():
    rs = np.array([0.05, 0.7, 3.0, 40.0])
    for z in (-0.8, -0.2, 0.0, 0.35, 0.9):
        _, drs, dz = vdwdf.pw92_spin_correlation(rs, z)
        h = 1e-6 * rs
        fd_rs = (vdwdf.pw92_spin_correlation(rs + h, z)[0] - vdwdf.pw92_spin_correlation(rs - h, z)[0]) / (2 * h)
        assert np.allclose(drs, fd_rs, rtol=1e-7)
        hz = 1e-6
        fd_z = (vdwdf.pw92_spin_correlation(rs, z + hz)[0] - vdwdf.pw92_spin_correlation(rs, z - hz)[0]) / (2 * hz)
        assert np.allclose(dz, fd_z, rtol=1e-6, atol=1e-12)


def test_fully_polarised_uniform_gas_exchange_is_spin_scaled():
    # one spin, no gradient: the exchange part is k_F(2 n_up) = 2^{1/3} k_F(n)
    n = np.array([1e-4, 0.01, 0.3, 5.0])
    x, *_ = vdwdf.q0_spin_unsaturated(n, np.zeros_like(n), np.zeros_like(n), np.zeros_like(n), ZAB)
    kF = np.cbrt(3.0 * math.pi ** 2 * n)
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    e1, _ = vdwdf.pw92_G(rs, *vdwdf.PW92_FERRO)
    assert np.allclose(x, 2.0 ** (1.0 / 3.0) * kF - (4.0 * math.pi / 3.0) * e1, rtol=1e-14)


def test_q0_reduces_to_the_spin_paired_form():
    rng = np.random.default_rng(11)
    n = np.exp(rng.uniform(np.log(1e-6), np.log(10.0), 50))
    sigma = rng.uniform(0.0, 2.0, 50) * n ** (8.0 / 3.0)
    x, dnu, dnd, dsu, dsd = vdwdf.q0_spin_unsaturated(n / 2, n / 2, sigma / 4, sigma / 4, ZAB)
    xu, dxdn, dxds = vdwdf.q0_unsaturated(n, sigma, ZAB)
    assert np.allclose(x, xu, rtol=1e-13)
    assert np.allclose(dnu, dxdn, rtol=1e-11) and np.allclose(dnd, dxdn, rtol=1e-11)
    assert np.allclose(dsu, 2 * dxds, rtol=1e-13) and np.allclose(dsd, 2 * dxds, rtol=1e-13)


def test_q0_partials_by_finite_differences():
    rng = np.random.default_rng(5)
    nu = np.exp(rng.uniform(np.log(1e-4), np.log(3.0), 20))
    nd = nu * rng.uniform(0.0, 1.5, 20)
    su = rng.uniform(0.0, 1.0, 20) * nu ** (8.0 / 3.0)
    sd = rng.uniform(0.0, 1.0, 20) * nd ** (8.0 / 3.0)
    args = [nu, nd, su, sd]
    _, *partials = vdwdf.q0_spin_unsaturated(*args, ZAB)
    for i in range(4):
        h = 1e-6 * np.maximum(args[i], 1e-12)
        up = [a + h if k == i else a for k, a in enumerate(args)]
        dn = [a - h if k == i else a for k, a in enumerate(args)]
        fd = (vdwdf.q0_spin_unsaturated(*up, ZAB)[0] - vdwdf.q0_spin_unsaturated(*dn, ZAB)[0]) / (2 * h)
        assert np.allclose(partials[i], fd, rtol=2e-6, atol=1e-9 * np.max(np.abs(fd))), i


def paired_grid(seed):
    # blobs, a vacuum corner and a saturated tail on a small triclinic cell
    grid = (10, 9, 8)
    cell = np.array([[7.0, 0.0, 0.0], [0.8, 6.5, 0.0], [-0.4, 0.6, 6.0]])
    rng = np.random.default_rng(seed)
    n = np.exp(rng.uniform(np.log(1e-5), np.log(2.0), grid))
    n[:3, :3, :3] = 0.0
    n[0, 0, 3] = 1e-31
    sigma = rng.uniform(0.0, 3.0, grid) * np.maximum(n, 0.0) ** (8.0 / 3.0)
    sigma[5, 5, 5] = 1e6    # saturates
    return grid, cell, n, sigma


def test_energy_reduces_to_the_spin_paired_functional():
    _, cell, n, sigma = paired_grid(2)
    E, dedn, deds = vdwdf.energy_and_partials(n, sigma, cell, KT)
    Es, dnu, dnd, dsu, dsd = vdwdf.energy_and_partials_spin(n / 2, n / 2, sigma / 4, sigma / 4, cell, KT)
    assert Es == pytest.approx(E, rel=1e-13)
    scale = np.max(np.abs(dedn))
    assert np.max(np.abs(dnu - dedn)) <= 1e-11 * scale and np.max(np.abs(dnd - dedn)) <= 1e-11 * scale
    s2 = np.max(np.abs(deds))
    assert np.max(np.abs(dsu - 2 * deds)) <= 1e-12 * s2 and np.max(np.abs(dsd - 2 * deds)) <= 1e-12 * s2
    # vacuum points carry zeros
    assert np.all(dnu[:3, :3, :3] == 0.0) and np.all(dsu[:3, :3, :3] == 0.0)


def polarised_inputs(seed, grid=(8, 7, 6)):
    rng = np.random.default_rng(seed)
    cell = np.array([[6.0, 0.0, 0.0], [0.5, 6.5, 0.0], [0.3, -0.4, 5.5]])
    nu = np.exp(rng.uniform(np.log(1e-3), np.log(1.0), grid))
    nd = nu * rng.uniform(0.0, 1.0, grid)
    nd[0, 0, :] = 0.0                                   # fully polarised points
    su = rng.uniform(0.0, 0.5, grid) * nu ** (8.0 / 3.0)
    sd = rng.uniform(0.0, 0.5, grid) * nd ** (8.0 / 3.0)
    return cell, [nu, nd, su, sd]


def test_energy_partials_by_finite_differences():
    cell, args = polarised_inputs(8)
    E, *parts = vdwdf.energy_and_partials_spin(*args, cell, KT)
    dV = abs(np.linalg.det(cell)) / args[0].size
    rng = np.random.default_rng(9)
    for i in range(4):
        for j in rng.choice(args[0].size, 3, replace=False):
            if args[i].flat[j] == 0.0:
                continue
            # a step of 1e-3 of the value: smaller ones lose the change of E to its rounding
            # (sigma ~ 1e-7 moves E by ~1e-13 of itself at 1e-4)
            h = 1e-3 * args[i].flat[j]

            def d(step):
                up = [a.copy() for a in args]
                dn = [a.copy() for a in args]
                up[i].flat[j] += step
                dn[i].flat[j] -= step
                return (vdwdf.energy_and_partials_spin(*up, cell, KT)[0]
                        - vdwdf.energy_and_partials_spin(*dn, cell, KT)[0]) / (2 * step)
            fd = (4.0 * d(h / 2) - d(h)) / 3.0
            assert fd == pytest.approx(parts[i].flat[j] * dV, rel=2e-5), (i, j)


def test_exchanging_the_spins_exchanges_the_outputs():
    cell, (nu, nd, su, sd) = polarised_inputs(4)
    E, a, b, c, d = vdwdf.energy_and_partials_spin(nu, nd, su, sd, cell, KT)
    E2, a2, b2, c2, d2 = vdwdf.energy_and_partials_spin(nd, nu, sd, su, cell, KT)
    assert E2 == pytest.approx(E, rel=1e-14)
    for x, y in ((a, b2), (b, a2), (c, d2), (d, c2)):
        assert np.max(np.abs(x - y)) <= 1e-13 * np.max(np.abs(x))


def test_potentials_at_equal_spins_are_the_spin_paired_potential():
    _, cell, n, _ = paired_grid(3)
    n = n + 1e-3
    g = vdwdf.spectral_gradient(n, cell)
    E, v, _, _ = vdwdf.potential(n, cell, KT, grad=g)
    Es, vu, vd = vdwdf.potential_spin(n / 2, n / 2, g / 2, g / 2, cell, KT)
    assert Es == pytest.approx(E, rel=1e-13)
    scale = np.max(np.abs(v))
    assert np.max(np.abs(vu - v)) <= 1e-11 * scale and np.max(np.abs(vd - v)) <= 1e-11 * scale


def test_potentials_are_the_derivatives_of_the_energy():
    # with the spectral gradients of n_up and n_dn, E is a function of the two densities alone and
    # dE/dn_s(r_j) = v_s(r_j) Omega/N (Richardson central differences)
    cell, (nu, nd, _, _) = polarised_inputs(12)
    nd = nd + 1e-3          # keep both spins present, so the spectral gradients stay smooth in n
    dV = abs(np.linalg.det(cell)) / nu.size

    def energy(a, b):
        return vdwdf.potential_spin(a, b, vdwdf.spectral_gradient(a, cell), vdwdf.spectral_gradient(b, cell),
                                    cell, KT)[0]
    _, vu, vd = vdwdf.potential_spin(nu, nd, vdwdf.spectral_gradient(nu, cell), vdwdf.spectral_gradient(nd, cell),
                                     cell, KT)
    rng = np.random.default_rng(13)
    for s, v in ((0, vu), (1, vd)):
        for j in rng.choice(nu.size, 3, replace=False):
            base = (nu, nd)[s]
            h = 1e-3 * base.flat[j]

            def d(step):
                up, dn = base.copy(), base.copy()
                up.flat[j] += step
                dn.flat[j] -= step
                if s == 0:
                    return (energy(up, nd) - energy(dn, nd)) / (2 * step)
                return (energy(nu, up) - energy(nu, dn)) / (2 * step)
            fd = (4.0 * d(h / 2) - d(h)) / 3.0
            assert fd == pytest.approx(v.flat[j] * dV, rel=2e-5), (s, j)
