"""torch.autograd over the local sweeps.

``LocalSweep`` is the map from the packed controls x of every subdomain to
their packed local trajectories: the restricted model of each subdomain over
its own time interval (eq. restricted) with the frozen halo ring of the last
exchange, run by dd4dvar_forward_integrate.  Its backward is the library's
hand-written adjoint sweep (dd4dvar_adjoint_integrate): the transpose of the
discrete tangent-linear model applied in reverse time, with the incoming
trajectory gradient as forcing at every level.  Its forward-mode derivative
(``torch.autograd.forward_ad``) is the library's tangent-linear sweep
(dd4dvar_tangent_linear, the TLM of Alg. 6).  Autograd never traces the
time loop; any torch function of the trajectories (a misfit, a projection)
can be differentiated back to x, in reverse or forward mode.

``LocalCost`` is the regularized local functional of every subdomain
(eq. eq:cost:parallel1: background, observation and overlap terms) as a
differentiable map x -> J[nsub]; forward and adjoint run fused in
dd4dvar_local_cost_grad, and the backward scales each subdomain's gradient by
the incoming weight of its J.

Both keep the device trajectory that the adjoint linearizes around inside the
library context.  When another call has replaced it before backward runs,
backward integrates the saved controls again first (recomputation instead of
storing a second trajectory).  The local model also depends on the frozen
halo rings of the last exchange: when an exchange or a solve has replaced
them between forward and backward, the forward's trajectory can no longer be
recomputed, and backward (or the forward-mode derivative) raises instead of
returning the derivative of another function.
"""
from __future__ import annotations

import torch


def _controls_index(dd):
    """Subdomain of every packed control entry (int64, on the device)."""
    idx = getattr(dd, "_ctrl_sub", None)
    if idx is None:
        sizes = [3 * int(i[1]) * int(i[3]) for i in dd.info]
        idx = torch.repeat_interleave(torch.arange(dd.nsub, device=dd.device),
                                      torch.tensor(sizes, device=dd.device))
        dd._ctrl_sub = idx
    return idx


class LocalSweep(torch.autograd.Function):
    """x (packed FP64 controls) -> packed FP64 local trajectories."""

    @staticmethod
    def forward(fctx, x, dd):
        x = x.detach().contiguous()
        traj = dd.forward(x)
        fctx.dd = dd
        fctx.gen = dd.traj_generation
        fctx.ring_gen = dd.ring_generation
        fctx.save_for_backward(x)
        fctx.save_for_forward(x)
        return traj

    @staticmethod
    def _check_rings(fctx):
        if fctx.dd.ring_generation != fctx.ring_gen:
            raise RuntimeError("the frozen halo rings were replaced (exchange or solve) after "
                               "LocalSweep.forward: its derivative is no longer available")

    @staticmethod
    def jvp(fctx, x_t, dd_t):
        dd = fctx.dd
        (x,) = fctx.saved_tensors
        LocalSweep._check_rings(fctx)
        if dd.traj_generation != fctx.gen:
            dd.forward(x, with_traj=False)
            fctx.gen = dd.traj_generation
        return dd.tangent_linear(x_t.to(torch.float64).contiguous())

    @staticmethod
    def backward(fctx, g):
        dd = fctx.dd
        (x,) = fctx.saved_tensors
        LocalSweep._check_rings(fctx)
        if dd.traj_generation != fctx.gen:
            dd.forward(x, with_traj=False)
        return dd.adjoint(g.to(torch.float64).contiguous()), None


class LocalCost(torch.autograd.Function):
    """x (packed FP64 controls) -> J[nsub], the local functionals."""

    @staticmethod
    def forward(fctx, x, dd):
        J, grad = dd.cost_grad(x.detach().contiguous())
        fctx.dd = dd
        fctx.save_for_backward(grad)
        return J

    @staticmethod
    def backward(fctx, gJ):
        (grad,) = fctx.saved_tensors
        return grad * gJ.to(torch.float64)[_controls_index(fctx.dd)], None


def local_sweep(dd, x):
    return LocalSweep.apply(x, dd)


def local_cost(dd, x):
    return LocalCost.apply(x, dd)
