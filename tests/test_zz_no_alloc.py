"""The no-allocation evaluation (dd4dvar_local_cost_grad_noalloc) through the
C ABI against dd4dvar_local_cost_grad: the same J and gradients bit for bit,
on two calls in a row on one GPU, the second with a smaller decomposition
(fewer tile partials in the shared static scratch), in FP32 persistent and
FP64 step-kernel plans."""
import numpy as np
import pytest

from conftest import problem

pytestmark = pytest.mark.gpu


def _eval_both(ctx, x):
    import torch
    from paper_2205_06649_amd import _lib as L
    J1 = torch.full((ctx.nsub,), float("nan"), dtype=torch.float64, device=ctx.device)
    g1 = torch.zeros(ctx.ctrl_len, dtype=torch.float64, device=ctx.device)
    J2, g2 = torch.full_like(J1, float("nan")), torch.zeros_like(g1)
    L.dd4dvar_local_cost_grad(ctx.handle, x.data_ptr(), J1.data_ptr(), g1.data_ptr(), ctx._stream())
    L.dd4dvar_local_cost_grad_noalloc(ctx.handle, x.data_ptr(), J2.data_ptr(), g2.data_ptr(),
                                      ctx._stream())
    ctx.synchronize()
    return (J1.cpu().numpy(), g1.cpu().numpy()), (J2.cpu().numpy(), g2.cpu().numpy())


def _controls(ctx, p, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    xb = ctx.background_controls()
    sb = torch.tensor(p.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    return xb + 0.3 * scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64,
                                          device="cuda")


@pytest.mark.parametrize("first,second", [(("c1", "fp32", 4), ("small", "fp64", 0)),
                                          (("c1", "fp32", 2), ("tiny2", "fp32", 0))])
def test_noalloc_equals_local_cost_grad(first, second):
    from paper_2205_06649_amd.context import Context
    ntiles = []
    for k, (which, prec, mode) in enumerate((first, second)):
        p = problem(which)
        ctx = Context(p, prec)
        ctx.set_exec_mode(mode)
        ntiles.append(sum(-(-int(i[1]) * int(i[3]) // 256) for i in ctx.info))
        x = _controls(ctx, p, 40 + k)
        (J1, g1), (J2, g2) = _eval_both(ctx, x)
        assert np.all(np.isfinite(J1)) and np.all(np.isfinite(g1))
        assert np.array_equal(J1, J2) and np.array_equal(g1, g2), (which, prec, mode)
        # and again after the other entry point ran: the scratch is rewritten
        (J3, g3), (J4, g4) = _eval_both(ctx, x)
        assert np.array_equal(J1, J4) and np.array_equal(g1, g4)
        ctx.close()
    assert ntiles[1] < ntiles[0], ntiles
