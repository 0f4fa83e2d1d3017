"""Autotuner for the batched form: picks split tile, march workgroup size,
persistent grid and rounds between host checks by timing whole batched
renders of the actual workload, and caches the winner in a JSON file keyed
by device name and workload shape (RAFI_TUNE_CACHE, default
~/.cache/rafi_tune.json)."""
from __future__ import annotations

import itertools
import json
import os

import torch

DEFAULT_SPACE = {
    "split_tile": [2048, 4096, 8192],
    "march_block": [128, 256],
    "march_grid": [1024, 2048, 4096],
    "use_graph": [1],
    "rounds_per_sync": [8],
}


def cache_path() -> str:
    return os.environ.get("RAFI_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rafi_tune.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def batch_key(batch) -> str:
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{dev}|batch|scenes={len(batch.scenes)}|rays={batch.n_rays}|domains={batch.n_domains}"


def time_render(batch, volumes, image, reps=2) -> float:
    batch.render(volumes, image)  # warm-up (and graph capture)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        batch.render(volumes, image)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def tune_batch(batch, volumes, image, space=None, reps=2, use_cache=True):
    """Returns (best tuning dict, best ms, all results)."""
    path = cache_path()
    key = batch_key(batch)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        batch.set_tuning(**best)
        return best, cache[key]["ms"], []
    space = space or DEFAULT_SPACE
    names = list(space)
    results = []
    for combo in itertools.product(*(space[k] for k in names)):
        t = dict(zip(names, combo))
        batch.set_tuning(**t)
        results.append((time_render(batch, volumes, image, reps), t))
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    batch.set_tuning(**best)
    if use_cache:
        cache[key] = {"tuning": best, "ms": best_ms}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, best_ms, results


# (steps_per_visit, tail_items, refill_lanes, quad_items); the quad launches
# apply only with refill_lanes 0
STREAMLINE_SPACE = ([(c, t, r, 0) for c in (32, 64, 96, 128, 256, 512) for t in (0, 65536) for r in (8, 16, 32)]
                    + [(c, t, 0, q) for c in (32, 64, 96, 128, 256, 512) for t in (0, 65536)
                       for q in (0, 65536, 98304, 131072, 262144)])


def _set_schedule(job, tuning):
    job.steps_per_visit, job.tail_items, job.refill_lanes, job.quad_items = (int(v) for v in tuning)


def tune_streamlines(ctx, job, seeds, space=None, reps=1, use_cache=True):
    """Picks (steps_per_visit, tail_items, refill_lanes, quad_items) for a
    streamline job by timing whole traces; results do not depend on the choice.
    Returns (best, ms, results)."""
    from . import rafi

    path = cache_path()
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    key = (f"{dev}|streamlines|n={job.n}|grid={list(job.grid)}|seeds={seeds.shape[0]}|max_steps={job.max_steps}"
           f"|schedule=cap,tail,refill,quad")
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache and len(cache[key]["tuning"]) == 4:
        _set_schedule(job, cache[key]["tuning"])
        return tuple(cache[key]["tuning"]), cache[key]["ms"], []
    results = []
    for tuning in (space or STREAMLINE_SPACE):
        _set_schedule(job, tuning)
        rafi.sl_trace_job(ctx, job, seeds)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            rafi.sl_trace_job(ctx, job, seeds)
        t1.record()
        torch.cuda.synchronize()
        results.append((t0.elapsed_time(t1) / reps, tuple(tuning)))
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    _set_schedule(job, best)
    if use_cache:
        cache[key] = {"tuning": list(best), "ms": best_ms}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, best_ms, results
