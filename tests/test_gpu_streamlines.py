"""GPU parity of the RK4 streamline march-and-forward path.

Endpoints, step counts, finish reasons, per-round counts and the particle
ids in every domain queue must equal the oracle's bit for bit (the whole
path is float32 with the same operations)."""
import numpy as np
import pytest
import torch

from gpu_util import announce, device
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stepwise(field, grid, seeds, h=0.25, max_steps=2000, steps_per_visit=0, refill_lanes=0, packed=True,
              quad_items=rafi.SL_QUAD_ITEMS):
    dev = device()
    N = len(seeds)
    f4 = torch.from_numpy(np.ascontiguousarray(field)).to(dev)
    if packed:
        f4 = rafi.sl_pack(f4)
    ctx = rafi.Context(int(np.prod(grid)), rafi.SL_ITEM_BYTES, N, debug=True)
    ep = torch.zeros((N, 3), dtype=torch.float32, device=dev)
    st = torch.zeros(N, dtype=torch.int32, device=dev)
    why = torch.zeros(N, dtype=torch.int32, device=dev)
    job = rafi.sl_job(f4, grid, ep, st, why, h, max_steps, steps_per_visit, refill_lanes=refill_lanes,
                      quad_items=quad_items)
    rafi.sl_seed(ctx, job, torch.from_numpy(seeds).to(dev))
    counts, queues = [], []
    while True:
        cnt, total, rc = ctx.round()
        q, _ = ctx.copy_queue()
        counts.append(cnt)
        queues.append(q.cpu().numpy().view(np.int32).reshape(-1, 4)[:, 3].copy())
        if total == 0:
            break
        rafi.sl_advance(ctx, job)
    torch.cuda.synchronize()
    stats = ctx.stats()
    ctx.close()
    return dict(endpoint=ep.cpu().numpy(), steps=st.cpu().numpy(), reason=why.cpu().numpy(),
                counts=np.array(counts), queue=np.concatenate(queues), stats=stats)


def _compare(g, o):
    assert np.array_equal(g["endpoint"].view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(g["steps"], o["steps"])
    assert np.array_equal(g["reason"], o["reason"])
    assert np.array_equal(g["counts"], o["round_counts"])
    assert np.array_equal(g["queue"], o["queue"])
    assert g["stats"]["bad_dest"] == 0 and g["stats"]["dropped"] == 0


# refill_lanes 0: one thread per particle (quad 0), or four lanes per particle in
# launches over at most `quad` particles; 1..64: persistent waves that take new
# particles whenever that many lanes are idle (1 and 64 are the extremes)
@pytest.mark.parametrize("refill,quad", [(0, 0), (0, rafi.SL_QUAD_ITEMS), (0, 2048),
                                               (1, 0), (16, 0), (64, 0)])
@pytest.mark.parametrize("n,grid,N,max_steps", [(64, (4, 4, 4), 4096, 2000), (64, (2, 1, 4), 3001, 500),
                                                (32, (1, 1, 1), 100, 300), (96, (3, 4, 2), 2000, 800)])
def test_abc_matches_oracle(orc, n, grid, N, max_steps, refill, quad):
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n, seed=N + n)
    announce(f"sl abc n={n} grid={grid} N={N} refill={refill} quad={quad}")
    g = _stepwise(field, grid, seeds, max_steps=max_steps, refill_lanes=refill, quad_items=quad)
    o = orc.streamlines(field, grid, seeds, max_steps=max_steps, queue_cap=1 << 24)
    _compare(g, o)


@pytest.mark.parametrize("refill", [0, 8])
@pytest.mark.parametrize("cap", [1, 7, 64])
def test_steps_per_visit_cap(orc, cap, refill):
    """At most `cap` steps per domain visit (cap 1 = the paper's one update per
    round): per-round queues follow the capped schedule, results do not move."""
    field = W.abc_field(32)
    seeds = W.streamline_seeds(256, 32, seed=5)
    announce(f"sl steps_per_visit={cap} refill={refill}")
    g = _stepwise(field, (2, 2, 2), seeds, max_steps=120, steps_per_visit=cap, refill_lanes=refill)
    o = orc.streamlines(field, (2, 2, 2), seeds, max_steps=120, steps_per_visit=cap, max_rounds=1000,
                        queue_cap=1 << 22)
    _compare(g, o)
    u = orc.streamlines(field, (2, 2, 2), seeds, max_steps=120)
    assert np.array_equal(g["endpoint"], u["endpoint"]) and np.array_equal(g["steps"], u["steps"])


@pytest.mark.parametrize("refill,quad", [(0, 0), (0, rafi.SL_QUAD_ITEMS), (16, 0)])
def test_unpadded_field_layout(orc, refill, quad):
    """The n^3 x 3 field read as is (12-byte voxels) gives the same routing and
    results as the padded layout."""
    n, grid, N = 64, (4, 2, 2), 3000
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n, seed=77)
    announce(f"sl unpadded field refill={refill} quad={quad}")
    g = _stepwise(field, grid, seeds, max_steps=900, refill_lanes=refill, packed=False,
                  quad_items=quad)
    o = orc.streamlines(field, grid, seeds, max_steps=900, queue_cap=1 << 24)
    _compare(g, o)


def test_constant_field_exact(orc):
    n = 256
    field = W.constant_field(n, (0.5, 0.0, 0.0))
    rng = np.random.default_rng(0)
    x0 = rng.integers(1024, 250 * 1024, 500) / 1024.0
    seeds = np.stack([x0, rng.uniform(0, n, 500), rng.uniform(0, n, 500)], 1).astype(np.float32)
    announce("sl constant field")
    g = _stepwise(field, (4, 4, 4), seeds, max_steps=100000)
    steps = np.ceil((256.0 - x0) / 0.125).astype(np.int64)
    assert np.array_equal(g["steps"], steps)
    assert np.array_equal(g["endpoint"][:, 0].astype(np.float64), x0 + 0.125 * steps)


@pytest.mark.parametrize("quad", [0, rafi.SL_QUAD_ITEMS])
def test_zero_field_stagnates(orc, quad):
    """A zero field: every particle stops after one step, where it started
    (the one-lane kernel's visit estimate then divides by zero speeds, and
    seeds on brick faces give 0/0; neither may change a result)."""
    n, grid = 32, (4, 2, 1)
    field = W.constant_field(n, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(3)
    seeds = rng.uniform(0, n, (700, 3)).astype(np.float32)
    seeds[:100, 0] = 8.0 * rng.integers(0, 4, 100)      # on x brick faces
    seeds[100:200, 1] = 16.0 * rng.integers(0, 2, 100)  # on y brick faces
    announce(f"sl zero field quad={quad}")
    g = _stepwise(field, grid, seeds, max_steps=50, quad_items=quad)
    o = orc.streamlines(field, grid, seeds, max_steps=50, queue_cap=1 << 20)
    _compare(g, o)
    assert np.all(g["steps"] == 1) and np.all(g["reason"] == 1)
    assert np.array_equal(g["endpoint"].view(np.uint32), seeds.view(np.uint32))


def test_full_cfg1_sampled(orc):
    """256^3 ABC, 4x4x4 bricks, 1M seeds, RK4 h = 0.25, <= 2000 steps: the whole
    job on the GPU, a seeded sample of 4096 particles through the oracle."""
    dev = device()
    n, N = 256, 1 << 20
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n)
    announce("sl cfg1 full")
    f4 = rafi.sl_pack(torch.from_numpy(field).to(dev))
    r = rafi.sl_trace(f4, (4, 4, 4), torch.from_numpy(seeds).to(dev))
    r2 = rafi.sl_trace(f4, (4, 4, 4), torch.from_numpy(seeds).to(dev), steps_per_visit=64)
    torch.cuda.synchronize()
    ep, st, why = r["endpoint"].cpu().numpy(), r["steps"].cpu().numpy(), r["reason"].cpu().numpy()
    # the capped schedule gives the same particles bit for bit; its cross-brick
    # forwards equal the uncapped run's forwards minus the seeding round
    assert torch.equal(r["endpoint"], r2["endpoint"]) and torch.equal(r["steps"], r2["steps"])
    assert int(r2["counters"][0]) == r["forwarded"] - N == int(r["counters"][0])
    assert int(r["counters"][1]) == 0 and r2["forwarded"] == N + int(r2["counters"].sum())
    r3 = rafi.sl_trace(f4, (4, 4, 4), torch.from_numpy(seeds).to(dev), steps_per_visit=32, tail_items=30000)
    assert torch.equal(r["endpoint"], r3["endpoint"]) and torch.equal(r["steps"], r3["steps"])
    assert int(r3["counters"][0]) == int(r["counters"][0])
    # persistent waves with lane refill: same particles, same forward counts;
    # run twice so the second launch sees the work counter reset by the first
    for _ in range(2):
        r4 = rafi.sl_trace(f4, (4, 4, 4), torch.from_numpy(seeds).to(dev), steps_per_visit=128, refill_lanes=16)
        assert torch.equal(r["endpoint"], r4["endpoint"]) and torch.equal(r["steps"], r4["steps"])
        assert torch.equal(r["reason"], r4["reason"])
        assert int(r4["counters"][0]) == int(r["counters"][0])
        assert r4["forwarded"] == N + int(r4["counters"].sum())
    # one lane per particle in every launch: same particles
    r6 = rafi.sl_trace(f4, (4, 4, 4), torch.from_numpy(seeds).to(dev), quad_items=0)
    assert torch.equal(r["endpoint"], r6["endpoint"]) and torch.equal(r["steps"], r6["steps"])
    assert torch.equal(r["reason"], r6["reason"]) and r6["forwarded"] == r["forwarded"]
    # the unpadded field layout: same particles
    r5 = rafi.sl_trace(torch.from_numpy(field).to(dev), (4, 4, 4), torch.from_numpy(seeds).to(dev),
                       steps_per_visit=128)
    assert torch.equal(r["endpoint"], r5["endpoint"]) and torch.equal(r["steps"], r5["steps"])
    assert torch.equal(r["reason"], r5["reason"])
    ids = np.sort(np.random.default_rng(2).choice(N, 4096, replace=False))
    o = orc.streamlines_brute(field, (4, 4, 4), seeds[ids])
    assert np.array_equal(ep[ids].view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(st[ids], o["steps"])
    assert np.array_equal(why[ids], o["reason"])
    # properties over all particles
    assert np.all((why >= 1) & (why <= 3)) and np.all((st >= 1) & (st <= 2000))
    assert np.all(st[why == 3] == 2000)
    out = np.any((ep < 0) | (ep >= n), axis=1)
    assert np.array_equal(out, why == 2)


def test_full_cfg1_exact(orc):
    """256^3 ABC, 4x4x4 bricks, all 1M seeds, RK4 h = 0.25, <= 2000 steps, under
    the benchmark's schedule (rafi.SL_STEPS_PER_VISIT steps per visit, lane
    quads for launches over at most 98304 particles, unpadded field). The pipelined job's endpoints,
    step counts and reasons, and the stepwise run's per-round counts and
    queues, equal the oracle's bit for bit (oracle threaded for speed: its
    results do not depend on the thread count)."""
    dev = device()
    n, N, grid = 256, 1 << 20, (4, 4, 4)
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n)
    announce("sl cfg1 full, exact")
    r = rafi.sl_trace(torch.from_numpy(field).to(dev), grid, torch.from_numpy(seeds).to(dev),
                      steps_per_visit=rafi.SL_STEPS_PER_VISIT)
    torch.cuda.synchronize()
    ep, st, why = r["endpoint"].cpu().numpy(), r["steps"].cpu().numpy(), r["reason"].cpu().numpy()
    r["ctx"].close()
    g = _stepwise(field, grid, seeds, steps_per_visit=rafi.SL_STEPS_PER_VISIT, packed=False)
    assert np.array_equal(g["endpoint"].view(np.uint32), ep.view(np.uint32))
    orc.set_threads(orc.default_threads())
    try:
        o = orc.streamlines(field, grid, seeds, steps_per_visit=rafi.SL_STEPS_PER_VISIT, queue_cap=1 << 23)
    finally:
        orc.set_threads(1)
    assert g["counts"].shape[0] == r["rounds"] == o["rounds"]
    _compare(g, o)
    assert np.array_equal(ep.view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(st, o["steps"]) and np.array_equal(why, o["reason"])


@pytest.mark.parametrize("n,packed", [(564, False), (512, True)])
def test_large_field_global_loads(orc, n, packed):
    """Fields of more than 2^31 - 1 bytes (564^3 x 12 B, 512^3 x 16 B) are
    read with 64-bit addresses, smaller ones through a buffer resource: the
    one-lane kernel (quad_items 0) must match the oracle on both sides."""
    dev = device()
    field_d = W.abc_field(n, device=dev)
    f = rafi.sl_pack(field_d) if packed else field_d
    assert f.numel() * 4 > 2**31 - 1
    seeds = W.streamline_seeds(256, n, seed=11)
    announce(f"sl large field n={n} packed={packed}")
    r = rafi.sl_trace(f, (4, 4, 4), torch.from_numpy(seeds).to(dev), steps_per_visit=rafi.SL_STEPS_PER_VISIT,
                      quad_items=0)
    torch.cuda.synchronize()
    ep, st, why = r["endpoint"].cpu().numpy(), r["steps"].cpu().numpy(), r["reason"].cpu().numpy()
    r["ctx"].close()
    field = field_d.cpu().numpy()
    del f, field_d, r
    torch.cuda.empty_cache()
    o = orc.streamlines_brute(field, (4, 4, 4), seeds)
    assert np.array_equal(ep.view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(st, o["steps"])
    assert np.array_equal(why, o["reason"])


@pytest.mark.parametrize("quad", [0, rafi.SL_QUAD_ITEMS])
@pytest.mark.parametrize("n", [8, 2])
def test_edge_seeds_tiny_fields(orc, n, quad):
    """Seeds on brick faces, just below them and below n, at -0.0 and
    outside the volume, in 8^3 and 2^3 fields of 2x2x2 bricks (1-voxel bricks
    at n = 2): routing, counts and results equal the oracle's with one lane
    or a lane quad per particle."""
    b = n // 2
    below = lambda v: float(np.nextafter(np.float32(v), np.float32(0)))
    vals = [0.0, -0.0, float(b), below(b), below(n), 0.3 * n]
    grid_pts = np.array([(x, y, z) for x in vals for y in vals for z in vals], dtype=np.float32)
    outside = np.array([[-0.5, 1.0, 1.0], [n, 0.5, 0.5], [0.5, n + 0.25, 0.5], [0.5, 0.5, -1e-7],
                        [below(n), below(n), n], [-0.0, -0.0, -1.0], [1e9, 0, 0], [0, -1e9, 0], [0, 0, n]],
                       dtype=np.float32)
    seeds = np.concatenate([grid_pts, outside])
    field = W.abc_field(n)
    announce(f"sl edge seeds n={n} quad={quad}")
    g = _stepwise(field, (2, 2, 2), seeds, max_steps=300, quad_items=quad)
    o = orc.streamlines(field, (2, 2, 2), seeds, max_steps=300, queue_cap=1 << 22)
    _compare(g, o)


def test_streamline_autotune(orc, tmp_path, monkeypatch):
    """The schedule autotuner times whole traces over (steps_per_visit,
    tail_items, refill_lanes, quad_items), sets the job to the fastest, caches
    it; results under the chosen schedule equal the oracle's."""
    from paper_2605_30294_amd import autotune
    monkeypatch.setenv("RAFI_TUNE_CACHE", str(tmp_path / "tune.json"))
    dev = device()
    n, grid, N = 64, (4, 4, 4), 4096
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n, seed=21)
    announce("sl autotune")
    f4 = rafi.sl_pack(torch.from_numpy(field).to(dev))
    ctx = rafi.Context(64, rafi.SL_ITEM_BYTES, N)
    ep = torch.zeros((N, 3), dtype=torch.float32, device=dev)
    st = torch.zeros(N, dtype=torch.int32, device=dev)
    why = torch.zeros(N, dtype=torch.int32, device=dev)
    job = rafi.sl_job(f4, grid, ep, st, why, 0.25, 600)
    space = [(32, 0, 0, 0), (32, 0, 0, 4096), (16, 0, 8, 0), (64, 1024, 0, 2048)]
    d_seeds = torch.from_numpy(seeds).to(dev)
    best, ms, results = autotune.tune_streamlines(ctx, job, d_seeds, space=space)
    assert tuple(best) in space and len(results) == len(space) and ms > 0
    assert (job.steps_per_visit, job.tail_items, job.refill_lanes, job.quad_items) == tuple(best)
    again, _, cached = autotune.tune_streamlines(ctx, job, d_seeds, space=space)
    assert tuple(again) == tuple(best) and cached == []
    rafi.sl_trace_job(ctx, job, d_seeds)
    torch.cuda.synchronize()
    o = orc.streamlines_brute(field, grid, seeds, max_steps=600)
    assert np.array_equal(ep.cpu().numpy().view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(st.cpu().numpy(), o["steps"])
    assert np.array_equal(why.cpu().numpy(), o["reason"])
    ctx.close()


@pytest.mark.parametrize("quad", [0, rafi.SL_QUAD_ITEMS])
@pytest.mark.parametrize("N", [0, 1, 65])
def test_empty_and_few_seeds(orc, N, quad):
    """No seeds: one forward step with nothing in it, no launch. One seed and
    a ragged 65 (a partial quad workgroup and wave): the oracle's results."""
    dev = device()
    n = 32
    field = W.abc_field(n)
    seeds = W.streamline_seeds(max(N, 1), n, seed=9)[:N]
    announce(f"sl few seeds N={N} quad={quad}")
    f4 = rafi.sl_pack(torch.from_numpy(field).to(dev))
    r = rafi.sl_trace(f4, (2, 2, 2), torch.from_numpy(seeds).to(dev).reshape(N, 3), max_steps=400,
                      steps_per_visit=16, quad_items=quad)
    torch.cuda.synchronize()
    assert r["endpoint"].shape == (N, 3) and r["steps"].shape == (N,)
    if N == 0:
        assert r["forwarded"] == 0 and r["rounds"] == 1
        return
    o = orc.streamlines_brute(field, (2, 2, 2), seeds, max_steps=400)
    assert np.array_equal(r["endpoint"].cpu().numpy().view(np.uint32), o["endpoint"].view(np.uint32))
    assert np.array_equal(r["steps"].cpu().numpy(), o["steps"])
    assert np.array_equal(r["reason"].cpu().numpy(), o["reason"])
