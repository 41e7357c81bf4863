"""torch.autograd over the local sweeps: the backward of LocalSweep is the
library's adjoint sweep, checked against the oracle's adjoint and against
centred finite differences; LocalCost's backward is the fused gradient.

Tolerances: FP64 1e-12 against the oracle adjoint (same bar as the adjoint
parity tests), FP32 1e-4; finite differences 1e-6 (FP64, step 1e-4 of the
background spread, centred: truncation ~1e-8, rounding ~1e-10)."""
import numpy as np
import pytest

import synth
from conftest import custom_problem, problem
from oracle import dd, ddmaps, local, model

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4}


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _setup(which, prec, seed=0):
    import torch
    from paper_2205_06649_amd.context import Context
    # "tz": the Turkel-Zwas variant (offsets 2, 2; frozen pads) on the c1 decomposition
    p = (custom_problem(dict(synth.CONFIGS["c1"], index=140, tz=(2, 2, 0.5))) if which == "tz"
         else problem(which))
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    ctx = Context(p, prec)
    rng = np.random.default_rng(seed)
    xs = [trajs[b.sub][0] + 0.3 * p.sigma_b[:, None, None] * rng.standard_normal(trajs[b.sub][0].shape)
          for b in maps.boxes]
    x = ctx.pack_ctrl(xs)
    return p, maps, rings, ctx, xs, x, torch


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["c1", "small", "tz"])
def test_local_sweep_backward_is_the_adjoint(which, prec):
    from paper_2205_06649_amd.autograd import local_sweep
    p, maps, rings, ctx, xs, x, torch = _setup(which, prec)
    rng = np.random.default_rng(3)
    w = [rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes]
    W = ctx.pack_traj(w)
    xr = x.clone().requires_grad_(True)
    traj = local_sweep(ctx, xr)
    (traj * W).sum().backward()
    grads = ctx.unpack_ctrl(xr.grad)
    g = model.Grid.of(p)
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        lt = local.forward(geo, xs[b.sub], rings[b.sub])
        ref = local.adjoint(geo, lt, rings[b.sub], w[b.sub])
        assert _rel(grads[b.sub], ref) <= TOL[prec], b.sub


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["c1", "small", "tz"])
def test_local_sweep_forward_mode_is_the_tlm(which, prec):
    """Forward-mode AD of LocalSweep (a dual tensor through the sweep) is the
    tangent-linear model: against the oracle's TLM per box, and consistent
    with the reverse mode (<M' dx, y> = <dx, M'^T y>)."""
    import torch.autograd.forward_ad as fwAD
    from paper_2205_06649_amd.autograd import local_sweep
    p, maps, rings, ctx, xs, x, torch = _setup(which, prec, seed=4)
    rng = np.random.default_rng(5)
    dxs = [p.sigma_b[:, None, None] * rng.standard_normal(xx.shape) for xx in xs]
    dx = ctx.pack_ctrl(dxs)
    with fwAD.dual_level():
        out = local_sweep(ctx, fwAD.make_dual(x, dx))
        tangent = fwAD.unpack_dual(out).tangent
    dt = ctx.unpack_traj(tangent)
    g = model.Grid.of(p)
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        lt = local.forward(geo, xs[b.sub], rings[b.sub])
        ref = local.tlm(geo, lt, rings[b.sub], dxs[b.sub])
        assert _rel(dt[b.sub], ref) <= TOL[prec], b.sub
    w = [rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes]
    W = ctx.pack_traj(w)
    xr = x.clone().requires_grad_(True)
    (local_sweep(ctx, xr) * W).sum().backward()
    lhs = float((tangent * W).sum())
    rhs = float((xr.grad * dx).sum())
    assert abs(lhs - rhs) <= (1e-12 if prec == "fp64" else 1e-5) * abs(lhs)


def test_local_sweep_nonlinear_loss_finite_differences():
    """A nonlinear torch loss of the trajectories: <grad, d> from autograd
    against centred differences of the loss."""
    from paper_2205_06649_amd.autograd import local_sweep
    p, maps, rings, ctx, xs, x, torch = _setup("c1", "fp64", seed=4)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    probe = torch.randn(ctx.traj_len, generator=gen, dtype=torch.float64, device="cuda")
    yref = ctx.forward(x) + 0.1 * probe.abs()

    def loss(xx):
        return 0.5 * ((local_sweep(ctx, xx) - yref) ** 2 * probe.abs()).sum()

    xr = x.clone().requires_grad_(True)
    loss(xr).backward()
    sb = torch.tensor(p.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    d = scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")
    an = float(torch.dot(xr.grad, d))
    eps = 1e-4
    with torch.no_grad():
        fd = (float(loss(x + eps * d)) - float(loss(x - eps * d))) / (2 * eps)
    assert abs(fd - an) / abs(an) < 1e-6, (fd, an)


def test_local_sweep_recomputes_a_replaced_trajectory():
    """Backward after another integration replaced the stored trajectory
    recomputes the linearization point from the saved controls."""
    from paper_2205_06649_amd.autograd import local_sweep
    p, maps, rings, ctx, xs, x, torch = _setup("small", "fp64", seed=5)
    W = torch.randn(ctx.traj_len, dtype=torch.float64, device="cuda")
    x1 = x.clone().requires_grad_(True)
    (local_sweep(ctx, x1) * W).sum().backward()
    x2 = x.clone().requires_grad_(True)
    t2 = local_sweep(ctx, x2)
    ctx.cost_grad(ctx.background_controls())          # replaces the trajectory
    (t2 * W).sum().backward()
    assert torch.equal(x1.grad, x2.grad)


def test_local_sweep_refuses_replaced_rings():
    """An exchange (or a solve) between forward and backward replaces the
    frozen halo rings the local model depends on, so the forward's trajectory
    cannot be recomputed: backward and the forward-mode derivative raise
    instead of returning the derivative about another trajectory."""
    import torch.autograd.forward_ad as fwAD
    from paper_2205_06649_amd.autograd import local_sweep
    p, maps, rings, ctx, xs, x, torch = _setup("small", "fp64", seed=7)
    W = torch.randn(ctx.traj_len, dtype=torch.float64, device="cuda")
    xr = x.clone().requires_grad_(True)
    t = local_sweep(ctx, xr)
    ctx.exchange(x + 1e-3 * W[:ctx.ctrl_len].abs())
    with pytest.raises(RuntimeError, match="halo rings"):
        (t * W).sum().backward()
    xr2 = x.clone().requires_grad_(True)
    t2 = local_sweep(ctx, xr2)
    ctx.solve(max_iter=2, max_outer=1)
    with pytest.raises(RuntimeError, match="halo rings"):
        (t2 * W).sum().backward()
    with fwAD.dual_level():
        xd = fwAD.make_dual(x, torch.ones_like(x))
        yd = local_sweep(ctx, xd)
        fwAD.unpack_dual(yd).tangent          # same rings: fine
    # with the rings unchanged since forward, a replaced trajectory is
    # recomputed (the exchange and the solve above left the current rings)
    xr3 = x.clone().requires_grad_(True)
    t3 = local_sweep(ctx, xr3)
    ctx.cost_grad(ctx.background_controls())
    (t3 * W).sum().backward()
    assert torch.isfinite(xr3.grad).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_local_cost_backward_is_the_fused_gradient(prec):
    from paper_2205_06649_amd.autograd import local_cost
    p, maps, rings, ctx, xs, x, torch = _setup("c1", prec, seed=6)
    w = torch.linspace(0.5, 2.0, ctx.nsub, dtype=torch.float64, device="cuda")
    xr = x.clone().requires_grad_(True)
    J = local_cost(ctx, xr)
    (J * w).sum().backward()
    J2, g2 = ctx.cost_grad(x)
    assert torch.equal(J.detach(), J2)
    parts = ctx.unpack_ctrl(xr.grad)
    ref = ctx.unpack_ctrl(g2)
    wh = w.cpu().numpy()
    for s in range(ctx.nsub):
        assert np.array_equal(parts[s], wh[s] * ref[s])
