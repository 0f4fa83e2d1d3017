"""GPU parity of the emission-absorption march-and-forward path.

Routing (per-round counts, the ray ids in every domain queue in order, the
sample index where each ray finishes) must match the oracle bit for bit;
float32 integrals and optical depths within 1e-5 relative of the oracle's
float64 values.
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, device, rel_close
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu

C32 = float(np.float32(0.025))
RTOL = 1e-5
# float32 cannot hold per-sample terms below its normal range (2^-126 ~ 1.2e-38);
# a ray sums at most a few hundred of them, so 1e-35 absolute covers underflow
# and is far below any value that carries information.
ATOL = 1e-35


def _stepwise(vol_t, grid, views, dt=0.5, c=C32, tile_items=None, emit_mode=rafi.SLOTS_ORDERED):
    """Run the rounds one at a time, snapshotting every queue.  Tiles of 512
    items or more select the LDS-staged march kernel when the brick fits."""
    dev = vol_t.device
    nv, w, h = len(views), int(views[0]["width"]), int(views[0]["height"])
    n_rays = nv * w * h
    ctx = rafi.Context(int(np.prod(grid)), rafi.EA_ITEM_BYTES, n_rays, debug=True)
    vdev = rafi.views_to_device(views, dev)
    image = torch.full((n_rays,), -1.0, dtype=torch.float32, device=dev)
    tau = torch.zeros(n_rays, dtype=torch.float32, device=dev)
    klast = torch.zeros(n_rays, dtype=torch.int32, device=dev)
    job = rafi.ea_job(vol_t, grid, vdev, nv, w, h, image, tau, klast, dt, c, emit_mode=emit_mode)
    rafi.ea_raygen(ctx, job)
    if tile_items:
        ctx.set_tile_items(tile_items)
    counts, queues = [], []
    while True:
        cnt, total, rc = ctx.round()
        q, offs = ctx.copy_queue()
        counts.append(cnt)
        queues.append(q.cpu().numpy().view(np.int32).reshape(-1, 4)[:, 0].copy())
        if total == 0:
            break
        if emit_mode == rafi.SLOTS_APPEND:
            ctx.open(total, rafi.SLOTS_APPEND)
        rafi.ea_march(ctx, job)
    torch.cuda.synchronize()
    st = ctx.stats()
    ctx.close()
    return dict(image=image.cpu().numpy(), tau=tau.cpu().numpy(), klast=klast.cpu().numpy(),
                counts=np.array(counts), queue=np.concatenate(queues), stats=st)


def _compare(g, o):
    assert g["counts"].shape == o["round_counts"].shape
    assert np.array_equal(g["counts"], o["round_counts"])
    assert np.array_equal(g["queue"], o["queue"])
    assert np.array_equal(g["klast"], o["klast"])
    ok, i, r = rel_close(g["image"], o["image"], RTOL, ATOL)
    assert ok, f"image ray {i}: gpu {g['image'][i]!r} oracle {o['image'][i]!r} ({r:.3g} x tol)"
    ok, i, r = rel_close(g["tau"], o["tau"], RTOL, ATOL)
    assert ok, f"tau ray {i}: gpu {g['tau'][i]!r} oracle {o['tau'][i]!r}"
    assert g["stats"]["bad_dest"] == 0 and g["stats"]["dropped"] == 0


@pytest.mark.parametrize("tile_items", [None, 2048])
def test_cfg0_plusz_64cube(orc, tile_items):
    """64^3 blobs, 2x2x2 domains, 128x128 rays along +z."""
    dev = device()
    vol = W.blob_volume(64, W.SEED_CFG0_VOLUME)
    views = W.plusz_view(64, 128, 128)
    announce(f"ea cfg0 tile_items={tile_items}")
    g = _stepwise(torch.from_numpy(vol).to(dev), (2, 2, 2), views, tile_items=tile_items)
    o = orc.ea_render(vol, (2, 2, 2), views, c=C32, queue_cap=1 << 20)
    assert len(g["counts"]) == 3
    _compare(g, o)


@pytest.mark.parametrize("rho", [0.0, 0.4, 2.4, 2.6, 40.0])
def test_uniform_medium_closed_form(rho):
    """A uniform medium of density rho, 2x2x2 bricks, 32^3, a +z view: every
    ray takes m = 64 samples of sigma = c rho, so I = rho (1 - exp(-m
    sigma)) and tau = m sigma exactly (float64 here, no oracle). The
    densities put sigma on both sides of 1/16, where the march's emission
    weight changes from its series to the library expm1, and 40 gives
    sigma = 1 per sample."""
    dev = device()
    n = 32
    announce(f"ea uniform medium rho={rho}")
    vol = torch.full((n, n, n), rho, dtype=torch.float32, device=dev)
    views = W.plusz_view(n, 16, 16)
    m = int(views[0]["n_samples"])
    r = rafi.ea_render(vol, (2, 2, 2), views, c=C32, want_tau=True)
    torch.cuda.synchronize()
    image = r["image"].cpu().numpy()
    tau = r["tau"].cpu().numpy()
    r["ctx"].close()
    sigma = C32 * float(np.float32(rho))
    I_ref = float(np.float32(rho)) * -np.expm1(-m * sigma)
    ok, i, rr = rel_close(image, np.full_like(image, I_ref, dtype=np.float64), RTOL, ATOL)
    assert ok, f"image ray {i}: gpu {image[i]!r} closed form {I_ref!r} ({rr:.3g} x tol)"
    ok, i, rr = rel_close(tau, np.full_like(tau, m * sigma, dtype=np.float64), RTOL, ATOL)
    assert ok, f"tau ray {i}: gpu {tau[i]!r} closed form {m * sigma!r}"


@pytest.mark.parametrize("n,w", [(1290, 86), (1292, 76)])
def test_large_volume_cell_index(n, w):
    """Volumes of at most 1290^3 voxels take the march's 32-bit cell index,
    larger ones the 64-bit one (here 1292^3, 8.6 GB, where i + n j + n^2 k
    passes 2^31). A density linear in x and z, which trilinear
    interpolation reproduces to float32 rounding, 2x2x2 bricks, a +z view
    whose rays sit at exactly representable x (pixel spacing n / w = 15 or
    17 voxels). Reference: the emission-absorption sum over each ray's
    samples of the analytic density, in float64 (no oracle)."""
    dev = device()
    a, bx, bz = 0.02, 1.0e-5, 2.0e-5
    announce(f"ea large volume n={n}")
    xx = torch.arange(n, device=dev, dtype=torch.float32).view(1, 1, n)
    zz = torch.arange(n, device=dev, dtype=torch.float32).view(n, 1, 1)
    vol = (a + bz * zz + bx * xx).expand(n, n, n).contiguous()       # [z, y, x]
    del xx, zz
    views = W.plusz_view(n, w, w)
    ns = int(views[0]["n_samples"])
    try:
        r = rafi.ea_render(vol, (2, 2, 2), views, c=C32, want_tau=True)
        torch.cuda.synchronize()
        image = r["image"].cpu().numpy().reshape(w, w)
        tau = r["tau"].cpu().numpy().reshape(w, w)
        klast = r["klast"].cpu().numpy()
        r["ctx"].close()
    finally:
        del vol
        torch.cuda.empty_cache()
    assert np.all(klast == ns)
    sx = n / w
    x = 0.5 * sx + sx * np.arange(w)                                   # every ray of a column shares x
    z = (np.arange(ns) + 0.5) * 0.5
    u_z = np.clip(z - 0.5, 0.0, n - 1)
    rho = a + bx * (x[:, None] - 0.5) + bz * u_z[None, :]              # [x, sample]
    sigma = C32 * rho
    t_before = np.cumsum(sigma, axis=1) - sigma
    I_ref = np.sum(np.exp(-t_before) * -np.expm1(-sigma) * rho, axis=1)
    tau_ref = np.sum(sigma, axis=1)
    # image rows are y, columns x: compare every ray with its column's reference
    ok, i, rr = rel_close(image, np.broadcast_to(I_ref[None, :], (w, w)), RTOL, ATOL)
    assert ok, f"image ray {i}: ({rr:.3g} x tol)"
    ok, i, rr = rel_close(tau, np.broadcast_to(tau_ref[None, :], (w, w)), RTOL, ATOL)
    assert ok, f"tau ray {i}: ({rr:.3g} x tol)"


@pytest.mark.parametrize("n,grid,nv,w,h,seed", [
    (32, (4, 4, 4), 3, 20, 20, 1), (32, (2, 1, 4), 2, 33, 17, 2), (48, (3, 2, 1), 2, 40, 40, 3),
    (16, (1, 1, 1), 1, 7, 9, 4), (64, (4, 2, 2), 4, 64, 64, 5),
])
@pytest.mark.parametrize("tile_items", [None, 512])
def test_rotated_views(orc, n, grid, nv, w, h, seed, tile_items):
    dev = device()
    vol = W.blob_volume(n, 100 + seed)
    views = W.random_views(nv, n, w, h, seed=200 + seed)
    announce(f"ea rotated n={n} grid={grid} tile_items={tile_items}")
    g = _stepwise(torch.from_numpy(vol).to(dev), grid, views, tile_items=tile_items)
    o = orc.ea_render(vol, grid, views, c=C32, queue_cap=1 << 22)
    _compare(g, o)


def _segments(queue, counts):
    """Split a concatenation of per-round, per-domain queues into its segments."""
    ends = np.cumsum(counts.reshape(-1).astype(np.int64))
    return np.split(queue, ends[:-1])


@pytest.mark.parametrize("n,grid,nv,w,seed", [(64, (4, 4, 4), 2, 48, 11), (48, (3, 2, 1), 3, 30, 12)])
def test_append_emission(orc, n, grid, nv, w, seed):
    """Forwarding through the paper's append queue (rafi_emit): every round's
    per-domain queue holds the oracle's rays as a multiset, and images,
    optical depths and end samples equal the slot-ordered run bit for bit."""
    dev = device()
    vol = W.blob_volume(n, 300 + seed)
    views = W.random_views(nv, n, w, w, seed=400 + seed)
    announce(f"ea append n={n} grid={grid}")
    t = torch.from_numpy(vol).to(dev)
    a = _stepwise(t, grid, views, emit_mode=rafi.SLOTS_APPEND)
    g = _stepwise(t, grid, views)
    o = orc.ea_render(vol, grid, views, c=C32, queue_cap=1 << 22)
    assert np.array_equal(a["counts"], o["round_counts"])
    for sa, so in zip(_segments(a["queue"], a["counts"]), _segments(o["queue"], o["round_counts"])):
        assert np.array_equal(np.sort(sa), np.sort(so))
    for key in ("image", "tau", "klast"):
        assert np.array_equal(a[key].view(np.uint32), g[key].view(np.uint32)), key
    assert a["stats"]["bad_dest"] == 0 and a["stats"]["dropped"] == 0
    r = rafi.ea_render(t, grid, views, c=C32, want_tau=True, emit_mode=rafi.SLOTS_APPEND)
    torch.cuda.synchronize()
    assert np.array_equal(r["image"].cpu().numpy().view(np.uint32), g["image"].view(np.uint32))


def test_append_overflow_is_counted():
    """Append emits beyond the opened slots are dropped, counted and reported."""
    dev = device()
    n, grid = 64, (2, 2, 2)
    vol = torch.from_numpy(W.blob_volume(n, W.SEED_CFG0_VOLUME)).to(dev)
    views = W.plusz_view(n, 128, 128)
    n_rays = 128 * 128
    ctx = rafi.Context(8, rafi.EA_ITEM_BYTES, n_rays)
    vdev = rafi.views_to_device(views, dev)
    image = torch.zeros(n_rays, dtype=torch.float32, device=dev)
    job = rafi.ea_job(vol, grid, vdev, 1, 128, 128, image, emit_mode=rafi.SLOTS_APPEND)
    rafi.ea_raygen(ctx, job)
    _, total, _ = ctx.round(counts=False)
    assert total == n_rays                      # every +z ray enters a z-low brick
    ctx.open(1000, rafi.SLOTS_APPEND)            # room for 1000 of the 16384 forwards
    rafi.ea_march(ctx, job)
    _, total, rc = ctx.round(counts=False, allow=(0, rafi.ERR_OVERFLOW))
    assert rc == rafi.ERR_OVERFLOW and total == 1000
    assert ctx.stats()["dropped"] == n_rays - 1000
    ctx.close()


def test_render_entry_point_and_determinism(orc):
    dev = device()
    vol = W.blob_volume(64, 7)
    views = W.random_views(2, 64, 96, 96, seed=8)
    t = torch.from_numpy(vol).to(dev)
    a = rafi.ea_render(t, (4, 4, 4), views, c=C32, want_tau=True)
    b = rafi.ea_render(t, (4, 4, 4), views, c=C32, want_tau=True)
    torch.cuda.synchronize()
    assert torch.equal(a["image"], b["image"]) and a["rounds"] == b["rounds"]
    o = orc.ea_render(vol, (4, 4, 4), views, c=C32)
    assert a["rounds"] == o["rounds"]
    ok, i, r = rel_close(a["image"].cpu().numpy(), o["image"], RTOL, ATOL)
    assert ok, (i, r)


def test_adjoint_scale_forward_sampled(orc):
    """128^3, 4x4x4 bricks, 64 views of 256x256: all rays on the GPU, a seeded
    sample of rays through the oracle one by one."""
    dev = device()
    vol = W.blob_volume(128, W.SEED_ADJ_VOLUME)
    views = W.random_views(64, 128, 256, 256)
    announce("ea 128^3 x 64 views forward")
    r = rafi.ea_render(torch.from_numpy(vol).to(dev), (4, 4, 4), views, c=C32, want_tau=True)
    torch.cuda.synchronize()
    img = r["image"].cpu().numpy()
    rng = np.random.default_rng(1)
    ids = np.sort(rng.choice(img.size, 20000, replace=False))
    o = orc.ea_brute(vol, (4, 4, 4), views, c=C32, ray_ids=ids)
    ok, i, rr = rel_close(img[ids], o["image"], RTOL, ATOL)
    assert ok, (ids[i], img[ids[i]], o["image"][i], rr)
    assert 3 <= r["rounds"] <= 12


def test_adjoint_scale_forward_exact(orc):
    """128^3, 4x4x4 bricks, 64 views of 256x256 (4.2M rays): every round's
    per-domain counts and queue (ray ids in order), and every ray's last
    sample index, equal the oracle's bit for bit; every integral and optical
    depth within 1e-5 relative (oracle threaded for speed: its results do
    not depend on the thread count)."""
    dev = device()
    vol = W.blob_volume(128, W.SEED_ADJ_VOLUME)
    views = W.random_views(64, 128, 256, 256)
    announce("ea 128^3 x 64 views forward, exact")
    g = _stepwise(torch.from_numpy(vol).to(dev), (4, 4, 4), views)
    r = rafi.ea_render(torch.from_numpy(vol).to(dev), (4, 4, 4), views, c=C32, want_tau=True)
    torch.cuda.synchronize()
    assert np.array_equal(r["image"].cpu().numpy(), g["image"]) and r["rounds"] == len(g["counts"])
    assert np.array_equal(r["klast"].cpu().numpy(), g["klast"])
    orc.set_threads(orc.default_threads())
    try:
        o = orc.ea_render(vol, (4, 4, 4), views, c=C32, queue_cap=1 << 24)
    finally:
        orc.set_threads(1)
    _compare(g, o)
