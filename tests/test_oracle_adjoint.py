"""Pins for the oracle's float64 gradient of the image loss (the adjoint of
the emission-absorption march).

Checked against central finite differences of the loss (float64), and the
closed form of dI/drho0 for a uniform medium (trilinear weights sum to one,
so the voxel gradients of one ray sum to the derivative of the uniform
closed form).
"""
import math

import numpy as np

from paper_2605_30294_amd import workloads as W

C32 = float(np.float32(0.025))


def test_gradient_matches_central_differences(orc):
    n = 16
    vol = W.blob_volume(n, 31).astype(np.float64)
    tgt_vol = W.blob_volume(n, 32)
    views = W.random_views(2, n, 24, 24, seed=33)
    grid = (2, 2, 2)
    target = orc.ea_render(tgt_vol, grid, views, c=C32)["image"]
    L, g, _ = orc.ea_loss_grad(vol, grid, views, target, c=C32)
    rng = np.random.default_rng(0)
    flat = vol.reshape(-1)
    picks = rng.choice(flat.size, 24, replace=False)
    for v in picks:
        eps = 1e-4 * max(1.0, abs(flat[v]))
        vp, vm = flat.copy(), flat.copy()
        vp[v] += eps
        vm[v] -= eps
        Lp, _, _ = orc.ea_loss_grad(vp.reshape(vol.shape), grid, views, target, c=C32, want_grad=False)
        Lm, _, _ = orc.ea_loss_grad(vm.reshape(vol.shape), grid, views, target, c=C32, want_grad=False)
        fd = (Lp - Lm) / (2 * eps)
        gv = g.reshape(-1)[v]
        assert abs(gv - fd) <= 1e-6 * abs(fd) + 1e-10, (v, gv, fd)


def test_uniform_medium_gradient_sum(orc):
    n, rho0 = 12, 0.8
    vol = W.uniform_volume(n, rho0)
    views = W.plusz_view(n, 6, 6)
    img = orc.ea_render(vol, (1, 1, 1), views, c=C32)["image"]
    target = img - 0.5                                   # dL/dI = 2 (I - I*) = 1 for every ray
    L, g, _ = orc.ea_loss_grad(vol, (1, 1, 1), views, target, c=C32)
    K = 2 * n
    r0 = float(np.float32(rho0))
    s = C32 * r0
    dI = -math.expm1(-K * s) + r0 * K * C32 * math.exp(-K * s)
    assert g.sum() == __import__("pytest").approx(36 * dI, rel=1e-12)
    assert L == __import__("pytest").approx(36 * 0.25, rel=1e-12)


def test_gradcheck_float64_small_volume(orc):
    """torch.autograd.gradcheck of the oracle's render and its adjoint as a
    float64 autograd function: 8^3 volume, 2x2x2 domains, two views. The
    adjoint gives vector-Jacobian products through the loss gradient: with
    target I* = I - g/2, dL/dI = 2 (I - I*) = g."""
    import torch

    n, grid = 8, (2, 2, 2)
    views = W.random_views(2, n, 6, 6, seed=41)

    class OracleRender(torch.autograd.Function):
        @staticmethod
        def forward(ctx, vol):
            img = orc.ea_render(vol.detach().numpy(), grid, views, c=C32)["image"]
            ctx.save_for_backward(vol)
            ctx.img = img
            return torch.from_numpy(img)

        @staticmethod
        def backward(ctx, g):
            (vol,) = ctx.saved_tensors
            target = ctx.img - 0.5 * g.detach().numpy()
            _, grad, _ = orc.ea_loss_grad(vol.detach().numpy(), grid, views, target, c=C32)
            return torch.from_numpy(grad)

    vol = torch.from_numpy(W.blob_volume(n, 40).astype(np.float64)).requires_grad_(True)
    assert torch.autograd.gradcheck(OracleRender.apply, (vol,), eps=1e-6, atol=1e-8, rtol=1e-6)
