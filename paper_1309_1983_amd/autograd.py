"""torch.autograd glue over the library's checkpointed rollout and adjoint.

rollout(lattice, force, tau, T, K) runs T steps from the lattice's current
state with the per-point body force `force` (3*N values, component slowest:
[3, N] or [3, nz, ny, nx]) and relaxation time `tau`,
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
        ctx.force_shape = force.shape
        ctx.force_dtype = force.dtype
        ctx.tau_dtype = tau.dtype
        ctx.tau_device = tau.device
        return u

    @staticmethod
    def backward(ctx, grad_u):
        lat: Lattice = ctx.lattice
        gF, gtau = lat.adjoint(grad_u.contiguous())
        gt = torch.tensor(gtau, dtype=ctx.tau_dtype, device=ctx.tau_device)
        return gF.reshape(ctx.force_shape).to(ctx.force_dtype), gt, None, None, None, None


def rollout(lattice: Lattice, force: torch.Tensor, tau: torch.Tensor, T: int, K: int,
            s0: torch.Tensor | None = None) -> torch.Tensor:
    """u(T) of a T-step rollout; differentiable in `force` and `tau`.

    s0: initial populations [19, N] (default: the lattice's current state).
    Needs F32 storage and the AB pattern.
    """
    if force.numel() != 3 * lattice.N:
        raise ValueError(f"force must be a per-point field of 3*N = {3 * lattice.N} values (component "
                         f"slowest, e.g. [3, N]); got shape {tuple(force.shape)}. A uniform force is a "
                         f"field with equal values; its gradient is the sum of the field's.")
    if s0 is None:
        s0 = lattice.populations()
    return _Rollout.apply(force, tau, lattice, int(T), int(K), s0)
