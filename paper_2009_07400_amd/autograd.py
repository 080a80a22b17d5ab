"""torch.autograd interface to the trajectory gradients of the HIP library.

``lj_md(eps, sigma, x0, system, v0, n_steps)`` returns the positions after
n_steps velocity-Verlet steps of every box of ``system`` and differentiates
them with respect to the per-box LJ parameters and the initial positions:
the forward records checkpoints at every neighbor rebuild
(tmd_adjoint_forward), the backward runs the hand-written adjoint kernels
(tmd_adjoint_backward).  Lists and cutoff indicators are those of the forward
run, so the gradient is that of the discrete map almost everywhere.
"""

from __future__ import annotations

import torch

from .system import System


class LJMDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, sigma, x0, system: System, v0, n_steps: int):
        system.set_lj_params(eps.detach().double().cpu().tolist(), sigma.detach().double().cpu().tolist())
        system.set_state(x0.detach(), v0.detach() if torch.is_tensor(v0) else v0, step=0)
        system.adjoint_forward(int(n_steps))
        xT, _, _ = system.get_state()
        system.sync()
        ctx.system = system
        ctx.shapes = (eps.shape, eps.dtype, eps.device, sigma.shape, sigma.dtype, sigma.device, x0.dtype,
                      x0.device)
        return xT.contiguous().to(dtype=x0.dtype, device=x0.device)

    @staticmethod
    def backward(ctx, grad_xT):
        es, ed, edev, ss, sd, sdev, xd, xdev = ctx.shapes
        gx, _, ge, gs = ctx.system.adjoint_backward(grad_xT.detach())
        ctx.system.sync()
        return (ge.reshape(es).to(ed).to(edev), gs.reshape(ss).to(sd).to(sdev), gx.contiguous().to(xd).to(xdev),
                None, None, None)


def lj_md(eps: torch.Tensor, sigma: torch.Tensor, x0: torch.Tensor, system: System, v0, n_steps: int):
    """Positions [N, 3] after n_steps; differentiable in eps [n_boxes],
    sigma [n_boxes] and x0 [N, 3] (boxes concatenated)."""
    return LJMDFunction.apply(eps, sigma, x0, system, v0, n_steps)
