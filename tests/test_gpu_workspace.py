"""Handles without their own work memory (vdwxc_init_table_ex with VDWXC_INIT_NO_WORKSPACE) and
caller-owned work memory (vdwxc_set_workspace): the calls refuse to run without work memory,
reject a buffer that is too small or misaligned, and give bitwise the results of a handle with its
own memory, also after moving between buffers and back."""
import sys

import pytest

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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_external_workspace_matches_own(dev, precision):
    from paper_1703_06999_amd import vdwxc
    grid, L = (24, 18, 30), 7.0
    say(f"[workspace] {grid} {precision}")
    n, g = inputs.small_slater(grid, L, 4, seed=21, floor=1e-4)
    n, g = n.to(dev), g.to(dev)
    cell = inputs.cubic_cell(L)
    own = vdwxc.Functional(grid, cell, precision=precision, table=KT)
    E0, v0 = own.potential(n, g)
    El0, vl0 = own.lda(n)
    bare = vdwxc.Functional(grid, cell, precision=precision, table=KT, own_workspace=False)
    with pytest.raises(vdwxc.VdwxcError) as ei:
        bare.potential(n, g)
    assert ei.value.status == vdwxc.ESTATE
    need = vdwxc.workspace_bytes(grid, precision, KT.nq)
    with pytest.raises(vdwxc.VdwxcError):
        bare.set_workspace(torch.empty(need - 256, dtype=torch.uint8, device=dev))
    big = torch.empty(need + 4096, dtype=torch.uint8, device=dev)
    with pytest.raises(vdwxc.VdwxcError):
        bare.set_workspace(big[8:])                     # not 256-byte aligned
    bare.set_workspace(big)
    E1, v1 = bare.potential(n, g)
    assert E1 == E0 and torch.equal(v1, v0)
    El1, vl1 = bare.lda(n)
    assert El1 == El0 and torch.equal(vl1, vl0)
    # a second buffer, then the handle with its own memory moved to the first and back
    other = torch.empty(need, dtype=torch.uint8, device=dev)
    bare.set_workspace(other)
    E2, v2 = bare.potential(n, g)
    assert E2 == E0 and torch.equal(v2, v0)
    own.set_workspace(big)
    E3, v3 = own.potential(n, g)
    own.set_workspace(None)
    E4, v4 = own.potential(n, g)
    assert E3 == E4 == E0 and torch.equal(v3, v0) and torch.equal(v4, v0)
    # NULL returns a handle without memory to refusing calls
    bare.set_workspace(None)
    with pytest.raises(vdwxc.VdwxcError):
        bare.potential(n, g)
    # a NaN input is still reported through the attached memory's flags
    bare.set_workspace(other)
    bad = n.clone()
    bad.view(-1)[5] = float("nan")
    with pytest.raises(vdwxc.VdwxcError):
        bare.potential(bad, g)
    E5, v5 = bare.potential(n, g)
    assert E5 == E0 and torch.equal(v5, v0)
    own.close()
    bare.close()
