"""Spin-polarised entry (vdwxc_calculate_spin*, the variant Sec. 7 announces) against the FP64
oracle's spin functional, element by element, on seeded polarised densities: two different blob
sets for the two spins, a slab where the minority spin is exactly zero (fully polarised points), a
vacuum slab where both are zero, and the analytic |grad n_s|^2.

Tolerances as for the spin-paired partials (the conversions around the pipeline are FP64 in both
precisions): FP64 E <= 1e-10 relative, each of the four fields <= 1e-10 of its max-norm; FP32_MIXED
E <= 1e-5, dE/dn_s <= 1e-4 and dE/dsigma_ss <= 1e-3 of their max-norms.  Also: at n_up = n_dn the
spin entry reproduces the spin-paired entry of the same handle (the conversion's own rounding only:
E <= 1e-13, fields <= 1e-11 of their max-norms), and the argument checks."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import vdwdf
from paper_1703_06999_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KT = inputs.synthetic_kernel_table()

TOL = {"fp64": dict(e=1e-10, n=1e-10, s=1e-10), "fp32": dict(e=1e-5, n=1e-4, s=1e-3)}
NAMES = ("dedn_up", "dedn_dn", "dedsigma_uu", "dedsigma_dd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_06999_amd import vdwxc
    vdwxc.lib()
    return torch.device("cuda:0")


def polarised(grid, length, seed):
    """(n_up, n_dn, sigma_uu, sigma_dd) as float64 CPU tensors."""
    nu, gu = inputs.small_slater(grid, length, 4, seed, floor=2e-4)
    nd, gd = inputs.small_slater(grid, length, 3, seed + 50, floor=1e-4)
    nd, gd = 0.7 * nd, 0.7 * gd
    nd[:, :, : max(1, grid[2] // 6)] = 0.0          # fully polarised slab
    gd[:, :, :, : max(1, grid[2] // 6)] = 0.0
    nu[: max(1, grid[0] // 5)] = 0.0                 # vacuum slab (both spins zero there)
    nd[: max(1, grid[0] // 5)] = 0.0
    gu[:, : max(1, grid[0] // 5)] = 0.0
    gd[:, : max(1, grid[0] // 5)] = 0.0
    return nu, nd, torch.sum(gu * gu, dim=0), torch.sum(gd * gd, dim=0)


CASES = [((20, 18, 16), 9.0, 1), ((21, 15, 14), 8.5, 2), ((8, 12, 512), 44.0, 3)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("grid,length,seed", CASES, ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v))
def test_spin_matches_oracle(dev, precision, grid, length, seed):
    from paper_1703_06999_amd import vdwxc
    say(f"[spin parity] grid {grid} L {length} seed {seed} {precision}")
    args = polarised(grid, length, seed)
    cell = inputs.cubic_cell(length)
    ref = vdwdf.energy_and_partials_spin(*(a.numpy() for a in args), cell, KT)
    f = vdwxc.Functional(grid, cell, flavour="DF1", precision=precision, table=KT)
    try:
        E, *fields = f.spin(*(a.to(dev) for a in args))
    finally:
        f.close()
    tol = TOL[precision]
    de = abs(E - ref[0]) / abs(ref[0])
    say(f"    E {E:.15e} oracle {ref[0]:.15e} rel {de:.2e}")
    assert de <= tol["e"]
    for name, got, want, t in zip(NAMES, fields, ref[1:], (tol["n"], tol["n"], tol["s"], tol["s"])):
        got = got.cpu().numpy()
        err = float(np.max(np.abs(got - want))) / float(np.max(np.abs(want)))
        say(f"    {name}: max-norm rel {err:.2e}")
        assert err <= t, (name, err)
    # vacuum points carry zeros, fully polarised points no minority-sigma derivative
    v = slice(0, max(1, grid[0] // 5))
    for got in fields:
        assert float(torch.max(torch.abs(got[v]))) == 0.0
    assert float(torch.max(torch.abs(fields[3][:, :, : max(1, grid[2] // 6)]))) == 0.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_spin_at_equal_spins_is_the_spin_paired_entry(dev, precision):
    from paper_1703_06999_amd import vdwxc
    grid, length = (24, 20, 512), 46.0
    n, g = inputs.small_slater(grid, length, 5, 7, floor=1e-4, device="cuda")
    sigma = torch.sum(g * g, dim=0)
    f = vdwxc.Functional(grid, inputs.cubic_cell(length), flavour="DF1", precision=precision, table=KT)
    try:
        E, dedn, deds = f.calculate(n, sigma)
        Es, dnu, dnd, dsu, dsd = f.spin(0.5 * n, 0.5 * n, 0.25 * sigma, 0.25 * sigma)
    finally:
        f.close()
    de = abs(Es - E) / abs(E)
    say(f"[equal spins {precision}] E rel {de:.2e}")
    assert de <= 1e-13
    for got, want, name in ((dnu, dedn, "dedn_up"), (dnd, dedn, "dedn_dn"), (dsu, 2 * deds, "dedsigma_uu"),
                            (dsd, 2 * deds, "dedsigma_dd")):
        err = float(torch.max(torch.abs(got - want)) / torch.max(torch.abs(want)))
        say(f"    {name}: max-norm rel {err:.2e}")
        assert err <= 1e-11, (name, err)


def test_spin_argument_checks(dev):
    from paper_1703_06999_amd import vdwxc
    grid = (8, 8, 8)
    f = vdwxc.Functional(grid, inputs.cubic_cell(6.0), precision="fp64", table=KT)
    try:
        nu = torch.full(grid, 0.1, dtype=torch.float64, device=dev)
        nd = torch.full(grid, 0.05, dtype=torch.float64, device=dev)
        s = torch.full(grid, 0.01, dtype=torch.float64, device=dev)
        outs = [torch.empty_like(nu) for _ in range(4)]
        e = torch.zeros(1, dtype=torch.float64, device=dev)
        with pytest.raises(vdwxc.VdwxcError, match="overlap the inputs"):
            f.spin_async(nu, nd, s, s, [outs[0], outs[1], outs[2], nu], e)
        with pytest.raises(vdwxc.VdwxcError, match="overlap each other"):
            f.spin_async(nu, nd, s, s, [outs[0], outs[0], outs[2], outs[3]], e)
        L = vdwxc.lib()
        ptr = [ctypes.c_void_p(t.data_ptr()) for t in (nu, nd, s, s)] + [ctypes.c_void_p(t.data_ptr()) for t in outs]
        ptr[1] = ctypes.c_void_p(0)
        assert L.vdwxc_calculate_spin_async(f._h, *ptr, ctypes.c_void_p(e.data_ptr())) == vdwxc.EINVAL
        bad = nd.clone()
        bad[3, 3, 3] = float("nan")
        with pytest.raises(vdwxc.VdwxcError, match="NaN"):
            f.spin(nu, bad, s, s)
        # the handle still works afterwards
        E, *_ = f.spin(nu, nd, s, s)
        assert np.isfinite(E)
    finally:
        f.close()


def polarised_with_gradients(grid, length, seed):
    """(n_up, n_dn, grad_up, grad_dn) as float64 CPU tensors (the densities of `polarised`)."""
    nu, gu = inputs.small_slater(grid, length, 4, seed, floor=2e-4)
    nd, gd = inputs.small_slater(grid, length, 3, seed + 50, floor=1e-4)
    nd, gd = 0.7 * nd, 0.7 * gd
    nd[:, :, : max(1, grid[2] // 6)] = 0.0
    gd[:, :, :, : max(1, grid[2] // 6)] = 0.0
    return nu, nd, gu, gd


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("grid,length,seed", [CASES[0], CASES[2]],
                         ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v))
def test_spin_potential_matches_oracle(dev, precision, grid, length, seed):
    """v_up, v_dn against the oracle's spin potentials: FP64 E <= 1e-10 relative and each v <= 1e-10
    of its max-norm; FP32_MIXED E <= 1e-5 and v <= 1e-4 of its max-norm (n >= 1e-6 everywhere here)."""
    from paper_1703_06999_amd import vdwxc
    say(f"[spin potential] grid {grid} L {length} seed {seed} {precision}")
    nu, nd, gu, gd = polarised_with_gradients(grid, length, seed)
    cell = inputs.cubic_cell(length)
    E_ref, vu_ref, vd_ref = vdwdf.potential_spin(nu.numpy(), nd.numpy(), gu.numpy(), gd.numpy(), cell, KT)
    f = vdwxc.Functional(grid, cell, flavour="DF1", precision=precision, table=KT)
    try:
        E, vu, vd = f.spin_potential(nu.to(dev), nd.to(dev), gu.to(dev), gd.to(dev))
    finally:
        f.close()
    tol = TOL[precision]
    de = abs(E - E_ref) / abs(E_ref)
    say(f"    E {E:.15e} oracle {E_ref:.15e} rel {de:.2e}")
    assert de <= tol["e"]
    for name, got, want in (("v_up", vu, vu_ref), ("v_dn", vd, vd_ref)):
        err = float(np.max(np.abs(got.cpu().numpy() - want))) / float(np.max(np.abs(want)))
        say(f"    {name}: max-norm rel {err:.2e}")
        assert err <= tol["n"], (name, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_spin_potential_at_equal_spins_is_the_potential(dev, precision):
    from paper_1703_06999_amd import vdwxc
    grid, length = (24, 20, 512), 46.0
    n, g = inputs.small_slater(grid, length, 5, 9, floor=1e-4, device="cuda")
    f = vdwxc.Functional(grid, inputs.cubic_cell(length), flavour="DF1", precision=precision, table=KT)
    try:
        E, v = f.potential(n, g)
        Es, vu, vd = f.spin_potential(0.5 * n, 0.5 * n, 0.5 * g, 0.5 * g)
    finally:
        f.close()
    de = abs(Es - E) / abs(E)
    bound = 1e-10 if precision == "fp64" else 1e-5
    say(f"[equal spins, potential {precision}] E rel {de:.2e}")
    assert de <= 1e-13
    for name, got in (("v_up", vu), ("v_dn", vd)):
        err = float(torch.max(torch.abs(got - v)) / torch.max(torch.abs(v)))
        say(f"    {name}: max-norm rel {err:.2e}")
        assert err <= bound, (name, err)


def test_spin_potential_argument_checks(dev):
    from paper_1703_06999_amd import vdwxc
    grid = (8, 8, 8)
    f = vdwxc.Functional(grid, inputs.cubic_cell(6.0), precision="fp64", table=KT)
    try:
        nu = torch.full(grid, 0.1, dtype=torch.float64, device=dev)
        nd = torch.full(grid, 0.05, dtype=torch.float64, device=dev)
        g = torch.zeros((3,) + grid, dtype=torch.float64, device=dev)
        vu, vd = torch.empty_like(nu), torch.empty_like(nu)
        e = torch.zeros(1, dtype=torch.float64, device=dev)
        with pytest.raises(vdwxc.VdwxcError, match="overlap the inputs"):
            f.spin_potential_async(nu, nd, g, g, vu, g[1], e)
        with pytest.raises(vdwxc.VdwxcError, match="overlap each other"):
            f.spin_potential_async(nu, nd, g, g, vu, vu, e)
        L = vdwxc.lib()
        args = [ctypes.c_void_p(t.data_ptr()) for t in (nu, nd, g, g, vu, vd, e)]
        args[3] = ctypes.c_void_p(0)
        assert L.vdwxc_calculate_spin_potential_async(f._h, *args) == vdwxc.EINVAL
        assert "gradients" in L.vdwxc_last_error(f._h).decode()
        # a uniform polarised gas: no gradient, so v_s = dE/dn_s, and the call still works
        E, vu, vd = f.spin_potential(nu, nd, g, g)
        assert np.isfinite(E) and float(torch.std(vu)) <= 1e-12 * float(torch.max(torch.abs(vu)))
    finally:
        f.close()
