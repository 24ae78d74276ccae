"""The LDA correlation pass (vdwxc_calculate_lda_async: eq. 1's E_c^LDA and v_c^LDA, PW92 of the
appendix) against the oracle's lda_correlation, on ragged grids with vacuum points, on a
512-point slab of the nanoparticle workload (several grid-stride steps per thread), and its
FP64-in-both-precisions, NaN and repeatability rules.

Tolerances: v within 1e-13 relative at every point (a pointwise formula of cbrt, sqrt, log1p and
divisions, each within a few ulp on both sides, with no cancellation: v = eps - (r_s/3) deps and
deps > 0 > eps); E within 1e-12 relative (same-sign terms summed in different orders: at most
about 100 rounding steps of 1.1e-16 on the GPU side, log2 N on numpy's pairwise side)."""
import sys

import numpy as np
import pytest

from oracle import vdwdf
from paper_1703_06999_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KT = inputs.synthetic_kernel_table()


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


def compare(f, n, cell):
    E, v = f.lda(n)
    E_ref, v_ref = vdwdf.lda_correlation(n.cpu().numpy(), cell)
    v = v.cpu().numpy()
    err = np.abs(v - v_ref)
    assert np.all(err <= 1e-13 * np.abs(v_ref)), float(np.max(err / np.maximum(np.abs(v_ref), 1e-300)))
    assert np.array_equal(v == 0.0, v_ref == 0.0)
    assert abs(E - E_ref) <= 1e-12 * abs(E_ref), (E, E_ref)
    return E, v


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("grid,L,seed", [((40, 36, 50), 12.0, 1), ((1, 2, 2), 2.0, 6), ((5, 7, 3), 3.0, 7),
                                         ((64, 64, 64), 20.0, 3)])
def test_lda_ragged_grids(dev, precision, grid, L, seed):
    from paper_1703_06999_amd import vdwxc
    say(f"[lda] {grid} {precision}")
    n, _ = inputs.small_slater(grid, L, 4, seed=seed, floor=0.0)
    n = n.clone()
    n.view(-1)[::7] = 0.0                      # vacuum points
    n.view(-1)[3::11] = 1e-31
    cell = inputs.cubic_cell(L)
    f = vdwxc.Functional(grid, cell, precision=precision, table=KT)
    compare(f, n.to(dev), cell)
    f.close()


def test_lda_slab_of_the_nanoparticle(dev):
    from paper_1703_06999_amd import vdwxc
    w = inputs.workload("nanoparticle_slab", grid=(64, 512, 512))
    say(f"[lda] {w.name} {w.grid}")
    n, _ = w.density(device="cuda")
    f = vdwxc.Functional(w.grid, w.cell, precision="fp64", table=KT)
    compare(f, n, w.cell)
    f.close()


def test_lda_rules(dev):
    from paper_1703_06999_amd import vdwxc
    grid, L = (24, 18, 30), 7.0
    n, _ = inputs.small_slater(grid, L, 4, seed=11, floor=1e-4)
    n = n.to(dev)
    cell = inputs.cubic_cell(L)
    f64 = vdwxc.Functional(grid, cell, precision="fp64", table=KT)
    f32 = vdwxc.Functional(grid, cell, precision="fp32", table=KT)
    E1, v1 = f64.lda(n)
    E2, v2 = f64.lda(n)
    E3, v3 = f32.lda(n)
    # fixed-order sum: repeated calls are bitwise equal; the pass is FP64 in both precisions
    assert E1 == E2 == E3
    assert torch.equal(v1, v2) and torch.equal(v1, v3)
    # a NaN density: NaN at its point and in the energy, the other points unchanged
    bad = n.clone()
    bad.view(-1)[100] = float("nan")
    Eb, vb = f64.lda(bad)
    assert np.isnan(Eb)
    assert torch.isnan(vb.view(-1)[100])
    keep = torch.ones(n.numel(), dtype=torch.bool, device=dev)
    keep[100] = False
    assert torch.equal(vb.view(-1)[keep], v1.view(-1)[keep])
    # v must not be the density array
    with pytest.raises(vdwxc.VdwxcError):
        f64.lda(n, v=n)
    # the pass shows up in the per-stage timing
    f64.enable_timing(True)
    f64.lda(n)
    st = f64.read_timing()
    f64.enable_timing(False)
    assert "lda" in st and st["lda"][1] == 1
    f64.close()
    f32.close()
