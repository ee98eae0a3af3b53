"""torch.autograd glue over the library's checkpointed rollout and adjoint.

rollout(lattice, force, tau, T, K) runs T steps from the lattice's current
state with the per-point body force `force` [3, N] and relaxation time `tau`,
and returns u(T) [3, N]. Its backward calls the library's reverse sweep
(lbm_adjoint) and returns dL/dforce and dL/dtau. The forward and reverse
arithmetic all run in the HIP kernels; this module only moves tensors.
"""
from __future__ import annotations

import torch

from .lattice import Lattice


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, force, tau, lattice: Lattice, T: int, K: int, s0):
        lattice.set_populations(s0)
        lattice.set_tau(float(tau.detach().cpu()))
        lattice.set_force(force.detach())
        lattice.forward_checkpointed(T, K)
        _, u = lattice.macros()
        ctx.lattice = lattice
        ctx.tau_dtype = tau.dtype
        ctx.tau_device = tau.device
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lat: Lattice = ctx.lattice
        gF, gtau = lat.adjoint(grad_u.contiguous())
        gt = torch.tensor(gtau, dtype=ctx.tau_dtype, device=ctx.tau_device)
        return gF, gt, None, None, None, None


def rollout(lattice: Lattice, force: torch.Tensor, tau: torch.Tensor, T: int, K: int,
            s0: torch.Tensor | None = None) -> torch.Tensor:
    """u(T) of a T-step rollout; differentiable in `force` and `tau`.

    s0: initial populations [19, N] (default: the lattice's current state).
    Needs F32 storage and the AB pattern.
    """
    if s0 is None:
        s0 = lattice.populations()
    return _Rollout.apply(force, tau, lattice, int(T), int(K), s0)
