"""E_c^nl as a differentiable torch function with a hand-written backward.

The forward runs the library's potential entry with the spectral gradient of n (so the energy is a
function of n alone).  The backward needs no extra FFTs: v = delta E / delta n comes out of the
forward (paper Sec. 2), and for the discrete energy dE/dn_j = (Omega/N) v_j exactly, because the
spectral derivative is real and antisymmetric.

    f = Functional(grid, cell, precision="fp64", table=kt)
    n.requires_grad_(True)
    E = vdwxc_energy(n, f)      # 0-dim float64 tensor on the GPU
    E.backward()                # n.grad = dV * v
"""
from __future__ import annotations

import torch


class VdwxcEnergy(torch.autograd.Function):
    """forward(n, functional) -> E (0-dim); backward: grad_E * v * dV."""

    @staticmethod
    def forward(ctx, n, functional):
        n_in = n.detach()
        if not n_in.is_contiguous():
            n_in = n_in.contiguous()
        v = torch.empty_like(n_in)
        e = torch.empty(1, dtype=torch.float64, device=n_in.device)
        functional.potential_async(n_in, None, v, e)
        ctx.save_for_backward(v)
        ctx.dV = functional.dV
        return e[0]

    @staticmethod
    def backward(ctx, grad_e):
        (v,) = ctx.saved_tensors
        return grad_e * ctx.dV * v, None


def vdwxc_energy(n, functional):
    return VdwxcEnergy.apply(n, functional)
