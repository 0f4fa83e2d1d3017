"""GPU adjoint (reverse-replay) of the emission-absorption march.

The float32 GPU gradient of L = sum (I - I*)^2 is checked against the
oracle's float64 analytic gradient (relative L2 <= 1e-4 over all voxels),
against float64 central finite differences at seeded voxels, and the
backward rays must visit the forward's domains in exactly reversed order.
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, device
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu

C32 = float(np.float32(0.025))
REL_L2 = 1e-4


def _gpu_loss_grad(vol_np, tgt_np, grid, views, ray_mask=None, bwd_tile_items=0):
    dev = device()
    vol = torch.from_numpy(vol_np).to(dev).requires_grad_(True)
    with torch.no_grad():
        target = rafi.ea_render(torch.from_numpy(tgt_np).to(dev), grid, views, c=C32)["image"]
    img = rafi.ea_render_differentiable(vol, grid, views, c=C32, bwd_tile_items=bwd_tile_items)
    r = img - target
    if ray_mask is not None:
        r = r * torch.from_numpy(ray_mask.astype(np.float32)).to(dev)
    loss = (r * r).sum()
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), vol.grad.detach().cpu().numpy().astype(np.float64), target.cpu().numpy().astype(np.float64)


def _rays_near(views, ids, voxel, n, radius=2.5):
    """Rays of `ids` passing within `radius` voxels of voxel `voxel`'s centre
    (a conservative geometric filter; only those rays' losses depend on it)."""
    i, j, k = voxel % n, (voxel // n) % n, voxel // (n * n)
    c = np.array([i + 0.5, j + 0.5, k + 0.5])
    w, h = int(views[0]["width"]), int(views[0]["height"])
    vi = ids // (w * h)
    local = ids % (w * h)
    px, py = local % w, local // w
    o0 = views["org0"][vi].astype(np.float64)
    du = views["du"][vi].astype(np.float64)
    dv = views["dv"][vi].astype(np.float64)
    dr = views["dir"][vi].astype(np.float64)
    org = o0 + px[:, None] * du + py[:, None] * dv
    rel = c[None, :] - org
    along = np.sum(rel * dr, axis=1)
    perp = rel - along[:, None] * dr
    return ids[np.linalg.norm(perp, axis=1) <= radius]


def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# bwd_tile_items 0: one workgroup per CU over slices of the queue; 512: one per 512-ray tile
@pytest.mark.parametrize("bwd_tile", [0, 512])
@pytest.mark.parametrize("n,grid,nv,w", [(32, (2, 2, 2), 3, 32), (32, (4, 4, 4), 2, 40), (48, (3, 1, 2), 2, 24),
                                         (48, (1, 1, 1), 2, 30)])   # last: brick too big for LDS (global path)
def test_gradient_matches_float64_oracle(orc, n, grid, nv, w, bwd_tile):
    vol = W.blob_volume(n, 61)
    tgt = W.blob_volume(n, 62)
    views = W.random_views(nv, n, w, w, seed=63)
    announce(f"adjoint n={n} grid={grid} bwd_tile={bwd_tile}")
    L, g, target = _gpu_loss_grad(vol, tgt, grid, views, bwd_tile_items=bwd_tile)
    L64, g64, _ = orc.ea_loss_grad(vol, grid, views, target, c=C32)
    assert abs(L - L64) <= 1e-4 * abs(L64)
    assert _rel_l2(g, g64) <= REL_L2, _rel_l2(g, g64)
    # finite differences of the float64 loss at seeded voxels
    flat = vol.astype(np.float64).reshape(-1)
    for v in W.fd_voxels(n, 12, seed=64):
        eps = 1e-4 * max(1.0, abs(flat[v]))
        vp, vm = flat.copy(), flat.copy()
        vp[v] += eps
        vm[v] -= eps
        Lp, _, _ = orc.ea_loss_grad(vp.reshape(vol.shape), grid, views, target, c=C32, want_grad=False)
        Lm, _, _ = orc.ea_loss_grad(vm.reshape(vol.shape), grid, views, target, c=C32, want_grad=False)
        fd = (Lp - Lm) / (2 * eps)
        gv = g.reshape(-1)[v]
        assert abs(gv - fd) <= 1e-3 * abs(fd) + 1e-6 * np.abs(g).max(), (v, gv, fd)


def test_backward_replays_reversed_visits():
    dev = device()
    n, grid = 64, (4, 4, 4)
    vol = torch.from_numpy(W.blob_volume(n, 71)).to(dev)
    views = W.random_views(3, n, 48, 48, seed=72)
    n_rays = 3 * 48 * 48
    stride = 12
    vdev = rafi.views_to_device(views, dev)
    image = torch.empty(n_rays, dtype=torch.float32, device=dev)
    tau = torch.empty_like(image)
    klast = torch.empty(n_rays, dtype=torch.int32, device=dev)
    flog = torch.full((n_rays, stride), -1, dtype=torch.int32, device=dev)
    fcnt = torch.zeros(n_rays, dtype=torch.int32, device=dev)
    blog = torch.full((n_rays, stride), -1, dtype=torch.int32, device=dev)
    bcnt = torch.zeros(n_rays, dtype=torch.int32, device=dev)
    ctx = rafi.Context(64, rafi.EA_ITEM_BYTES, n_rays)
    fjob = rafi.ea_job(vol, grid, vdev, 3, 48, 48, image, tau, klast, c=C32, visit_log=flog, visit_count=fcnt)
    rounds_f = rafi.ea_render_job(ctx, fjob)
    bjob = rafi.ea_job(vol, grid, vdev, 3, 48, 48, image, tau, klast, c=C32, visit_log=blog, visit_count=bcnt)
    grad = torch.zeros_like(vol)
    rounds_b = rafi.ea_backward_job(ctx, bjob, torch.ones_like(image), grad)
    torch.cuda.synchronize()
    assert rounds_f == rounds_b
    fl, bl = flog.cpu().numpy(), blog.cpu().numpy()
    fc, bc = fcnt.cpu().numpy(), bcnt.cpu().numpy()
    assert np.array_equal(fc, bc) and fc.max() <= stride
    for r in range(n_rays):
        k = fc[r]
        assert np.array_equal(bl[r, :k], fl[r, :k][::-1])
    ctx.close()


def test_uniform_medium_gradient_sum():
    dev = device()
    n, rho0 = 16, 0.8
    vol = torch.full((n, n, n), rho0, dtype=torch.float32, device=dev, requires_grad=True)
    views = W.plusz_view(n, 8, 8)
    img = rafi.ea_render_differentiable(vol, (2, 2, 2), views, c=C32)
    img.sum().backward()                                          # dL/dI = 1 for every ray
    K, r0 = 2 * n, float(np.float32(rho0))
    s = C32 * r0
    dI = -np.expm1(-K * s) + r0 * K * C32 * np.exp(-K * s)
    assert float(vol.grad.sum()) == pytest.approx(64 * dI, rel=1e-4)


def test_repeated_views_gradient_scales():
    """One view repeated 32 times: coinciding rays add to the same LDS words
    of the gradient region at nearly the same moments, so the flush's
    compare-and-swaps lose races and retry. Every add must still land once:
    the gradient is 32 times the single view's, up to float32 rounding."""
    dev = device()
    n = 32
    vol_np = W.blob_volume(n, 71)
    one = W.random_views(1, n, 32, 32, seed=72)
    rep = np.concatenate([one] * 32)
    announce("adjoint repeated views x32")

    def grad_of(views):
        vol = torch.from_numpy(vol_np).to(dev).requires_grad_(True)
        img = rafi.ea_render_differentiable(vol, (2, 2, 2), views, c=C32)
        img.sum().backward()                                      # dL/dI = 1 for every ray
        torch.cuda.synchronize()
        return vol.grad.detach().cpu().numpy().astype(np.float64)

    g1 = grad_of(one)
    g32 = grad_of(rep)
    assert np.abs(g1).max() > 0
    assert _rel_l2(g32, 32.0 * g1) <= 1e-5, _rel_l2(g32, 32.0 * g1)


def test_adjoint_scale_sampled(orc):
    """128^3 in 4x4x4 bricks, 64 views x 256^2 rays, target from a second volume.
    The whole forward and backward run on the GPU; the float64 oracle checks
    the gradient of the loss restricted to one view's rays (65536 rays), and
    finite differences of that loss at 32 seeded voxels."""
    dev = device()
    n, grid = 128, (4, 4, 4)
    vol = W.blob_volume(n, W.SEED_ADJ_VOLUME)
    tgt = W.blob_volume(n, W.SEED_ADJ_TARGET)
    views = W.random_views(64, n, 256, 256)
    announce("adjoint 128^3 x 64 views")
    L_all, g_all, target = _gpu_loss_grad(vol, tgt, grid, views)
    assert np.isfinite(g_all).all() and np.abs(g_all).max() > 0
    per = 256 * 256
    mask = np.zeros(64 * per, dtype=bool)
    mask[5 * per:6 * per] = True                                  # view 5
    L, g, _ = _gpu_loss_grad(vol, tgt, grid, views, ray_mask=mask)
    ids = np.nonzero(mask)[0]
    L64, g64, _ = orc.ea_loss_grad(vol, grid, views, target, c=C32, ray_ids=ids)
    assert _rel_l2(g, g64) <= REL_L2, _rel_l2(g, g64)
    flat = vol.astype(np.float64).reshape(-1)
    hit = np.nonzero(np.abs(g64.reshape(-1)) > 1e-3 * np.abs(g64).max())[0]
    rng = np.random.default_rng(W.SEED_ADJ_FD)
    for v in rng.choice(hit, 32, replace=False):
        eps = 1e-4 * max(1.0, abs(flat[v]))
        vp, vm = flat.copy(), flat.copy()
        vp[v] += eps
        vm[v] -= eps
        near = _rays_near(views, ids, v, n)
        assert len(near) > 0
        Lp, _, _ = orc.ea_loss_grad(vp.reshape(vol.shape), grid, views, target, c=C32, ray_ids=near, want_grad=False)
        Lm, _, _ = orc.ea_loss_grad(vm.reshape(vol.shape), grid, views, target, c=C32, ray_ids=near, want_grad=False)
        fd = (Lp - Lm) / (2 * eps)
        gv = g.reshape(-1)[v]
        assert abs(gv - fd) <= 1e-3 * abs(fd) + 1e-6 * np.abs(g).max(), (v, gv, fd)


def test_gradient_of_a_permuted_volume(orc):
    """A non-contiguous volume (a permuted view of the leaf tensor): the render
    works on a contiguous copy that must outlive the forward; the gradient
    reaches the leaf through the permutation and matches the float64 oracle.
    Allocations between forward and backward would reuse a freed copy."""
    dev = device()
    n, grid = 32, (2, 2, 2)
    vol_np = W.blob_volume(n, 65)
    tgt_np = W.blob_volume(n, 66)
    views = W.random_views(2, n, 32, 32, seed=67)
    announce("adjoint of a permuted volume")
    leaf = torch.from_numpy(np.ascontiguousarray(vol_np.transpose(2, 1, 0))).to(dev).requires_grad_(True)
    vol = leaf.permute(2, 1, 0)                      # equals vol_np, not contiguous
    assert not vol.is_contiguous()
    with torch.no_grad():
        target = rafi.ea_render(torch.from_numpy(tgt_np).to(dev), grid, views, c=C32)["image"]
    img = rafi.ea_render_differentiable(vol, grid, views, c=C32)
    junk = [torch.full((n, n, n), 7.0, device=dev) for _ in range(4)]   # takes freed blocks, if any
    loss = ((img - target) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    del junk
    g = leaf.grad.permute(2, 1, 0).cpu().numpy().astype(np.float64)
    L64, g64, _ = orc.ea_loss_grad(vol_np, grid, views, target.cpu().numpy().astype(np.float64), c=C32)
    assert abs(float(loss.detach()) - L64) <= 1e-4 * abs(L64)
    assert _rel_l2(g, g64) <= REL_L2, _rel_l2(g, g64)
