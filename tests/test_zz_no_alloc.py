"""The allocation-free entry point vdwxc_calculate_potential_noalloc (work buffers in the library's
static array) against vdwxc_calculate_potential_async (the handle's own work buffers), called
through the C ABI: the same kernels, so the energy and the potential must be bitwise equal.  Two
calls in a row on different handles, the second with a smaller grid (the array keeps the first
call's contents), in both precisions, with the analytic and the spectral gradient; a grid whose
work memory exceeds the array is refused before any device work."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1703_06999_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KT = inputs.synthetic_kernel_table()
STATIC_BYTES = 128 << 20


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


def _both(grid, L, seed, precision, spectral):
    """(E, v) from the allocation-free entry and from the asynchronous one, same inputs."""
    from paper_1703_06999_amd import vdwxc
    n, g = inputs.small_slater(grid, L, 5, seed=seed, floor=1e-4, device="cuda")
    grad = None if spectral else g
    f = vdwxc.Functional(grid, inputs.cubic_cell(L), precision=precision, table=KT)
    assert vdwxc.workspace_bytes(grid, precision) <= STATIC_BYTES
    v0 = torch.full_like(n, float("nan"))
    e0 = torch.full((1,), float("nan"), dtype=torch.float64, device=n.device)
    v1 = torch.full_like(n, float("nan"))
    e1 = torch.full((1,), float("nan"), dtype=torch.float64, device=n.device)
    f.potential_noalloc(n, grad, v1, e1)
    f.potential_async(n, grad, v0, e0)
    torch.cuda.synchronize()
    f.close()
    return float(e1.item()), v1, float(e0.item()), v0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("spectral", [False, True])
def test_noalloc_matches_async_two_calls(dev, precision, spectral):
    say(f"[noalloc] {precision} spectral={spectral}")
    # first call: 64^3 (the largest cube whose work memory fits the array in FP64), then a smaller,
    # ragged grid on another handle
    for grid, L, seed in (((64, 64, 64), 12.0, 1), ((30, 21, 16), 7.0, 2)):
        E1, v1, E0, v0 = _both(grid, L, seed, precision, spectral)
        say(f"    {grid}: E static {E1:.15e} E own buffers {E0:.15e}")
        assert np.isfinite(E1) and E1 == E0
        assert torch.equal(v1, v0), float(torch.max(torch.abs(v1 - v0)))


def test_noalloc_refuses_grids_beyond_the_static_array(dev):
    from paper_1703_06999_amd import vdwxc
    say("[noalloc] too large")
    grid = (96, 96, 96)
    assert vdwxc.workspace_bytes(grid, "fp32") > STATIC_BYTES
    f = vdwxc.Functional(grid, inputs.cubic_cell(18.0), precision="fp32", table=KT)
    n = torch.full(grid, 0.01, dtype=torch.float64, device=dev)
    v = torch.empty_like(n)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    with pytest.raises(vdwxc.VdwxcError) as ei:
        f.potential_noalloc(n, None, v, e)
    assert ei.value.status == vdwxc.EINVAL and "static work memory" in str(ei.value)
    f.close()
