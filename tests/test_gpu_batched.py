"""GPU batched form: many uneven scenes per launch.

Every scene's image must be bit-identical to rendering that scene alone with
the plain path (same per-ray arithmetic, different scheduling), for every
tuning (graph replay or direct launches, tile sizes, workgroup sizes), and
within 1e-5 of the float64 oracle."""
import numpy as np
import pytest
import torch

from gpu_util import announce, device, rel_close
from paper_2605_30294_amd import autotune, rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu

C32 = float(np.float32(0.025))
RTOL, ATOL = 1e-5, 1e-35


def _plain_images(vols, scenes):
    imgs, rounds = [], []
    for n, grid, view, off in scenes:
        v = vols[off:off + n ** 3].reshape(n, n, n)
        r = rafi.ea_render(v, grid, np.array([view]), c=C32)
        imgs.append(r["image"])
        rounds.append(r["rounds"])
        r["ctx"].close()
    return torch.cat(imgs), max(rounds)


def _small_batch(dev):
    specs = W.draw_scenes(12, seed=77, n_range=(8, 48), rays_side_range=(5, 40))
    views = []
    for i, sp in enumerate(specs):
        if i % 3 == 2:   # some scenes get a rotated view
            views.append(W.random_views(1, sp.n, sp.rays_side, sp.rays_side + 3, seed=300 + i)[0])
        else:
            views.append(W.plusz_view(sp.n, sp.rays_side, sp.rays_side)[0])
    vols, scenes = rafi.build_batch_inputs(specs, dev, views=views)
    return specs, vols, scenes


@pytest.mark.parametrize("tuning", [
    dict(),
    dict(use_graph=False, rounds_per_sync=1),
    dict(split_tile=1024, march_block=64, march_grid=7, rounds_per_sync=2),
    dict(split_tile=8192, march_block=512, march_grid=3000, use_graph=True, rounds_per_sync=16),
])
def test_batched_equals_plain_and_oracle(orc, tuning):
    dev = device()
    specs, vols, scenes = _small_batch(dev)
    announce(f"batched small {tuning}")
    b = rafi.Batch(scenes, c=C32)
    if tuning:
        b.set_tuning(**{**dict(split_tile=4096, march_block=256, march_grid=2048, use_graph=True,
                               rounds_per_sync=4), **tuning})
    image = torch.full((b.n_rays,), -7.0, dtype=torch.float32, device=dev)
    rounds = b.render(vols, image)
    plain, plain_rounds = _plain_images(vols, scenes)
    torch.cuda.synchronize()
    assert rounds == plain_rounds
    assert torch.equal(image, plain)
    img = image.cpu().numpy()
    vh = vols.cpu().numpy()
    base = 0
    for n, grid, view, off in scenes:
        m = int(view["width"]) * int(view["height"])
        o = orc.ea_render(vh[off:off + n ** 3].reshape(n, n, n), grid, np.array([view]), c=C32)
        ok, i, r = rel_close(img[base:base + m], o["image"], RTOL, ATOL)
        assert ok, (n, grid, i, r)
        base += m
    b.close()


def test_batched_repeat_and_graph_replay():
    """Several renders in a row through one captured graph give the same image."""
    dev = device()
    specs, vols, scenes = _small_batch(dev)
    b = rafi.Batch(scenes, c=C32)
    first = torch.empty(b.n_rays, dtype=torch.float32, device=dev)
    b.render(vols, first)
    for _ in range(3):
        again = torch.zeros_like(first)
        b.render(vols, again)
        torch.cuda.synchronize()
        assert torch.equal(first, again)
    b.close()


def test_batched_256_scenes(orc, tmp_path, monkeypatch):
    """256 uneven scenes (edges 32-256, 1-64 domains, 1K-1M rays): autotuned
    batched render equals the per-scene plain renders bit for bit; the oracle
    checks a seeded sample of rays of eight scenes."""
    dev = device()
    monkeypatch.setenv("RAFI_TUNE_CACHE", str(tmp_path / "tune.json"))
    specs = W.draw_scenes(256)
    announce("batched 256 scenes")
    vols, scenes = rafi.build_batch_inputs(specs, dev)
    b = rafi.Batch(scenes, c=C32)
    image = torch.empty(b.n_rays, dtype=torch.float32, device=dev)
    best, ms, _ = autotune.tune_batch(b, vols, image, space={"split_tile": [4096], "march_block": [256],
                                                              "march_grid": [2048, 4096], "use_graph": [1],
                                                              "rounds_per_sync": [8]}, reps=1)
    b.render(vols, image)
    plain, _ = _plain_images(vols, scenes)
    torch.cuda.synchronize()
    assert torch.equal(image, plain)
    img = image.cpu().numpy()
    rng = np.random.default_rng(11)
    for s in rng.choice(len(scenes), 8, replace=False):
        n, grid, view, off = scenes[s]
        m = int(view["width"]) * int(view["height"])
        base = int(b.scenes[s].ray_base)
        ids = np.sort(rng.choice(m, min(m, 2000), replace=False))
        vol = vols[off:off + n ** 3].reshape(n, n, n).cpu().numpy()
        o = orc.ea_brute(vol, grid, np.array([view]), c=C32, ray_ids=ids)
        ok, i, r = rel_close(img[base + ids], o["image"], RTOL, ATOL)
        assert ok, (s, i, r)
    b.close()
