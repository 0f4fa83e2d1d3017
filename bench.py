#!/usr/bin/env python3
"""Benchmark of the single-GPU work-forwarding hot path.

One "step" is one whole streamline job: 1M seeds in a 256^3 ABC velocity
field split into 4x4x4 domains, RK4 (h = 0.25 voxel, <= 2000 steps), every
particle forwarded at each brick exit until no particle is left -- seeding,
all forward steps (stable multi-split) and all domain-kernel launches, inputs
resident in HBM before the timed region starts.

Prints ONE JSON line. `value` is forwarded items per second over the whole
job: the forwards the workload itself requires (every seed delivered to its
first brick plus every brick-exit forward; a property of the workload, the
same for any schedule) divided by the job's GPU wall time. A particle that
has taken `--steps-per-visit` steps in one launch is also forwarded to its
own brick so that a round never waits on one long-lived particle; those
same-brick forwards are reported separately and not counted in `value`. Also reported: RK4 steps per second, the
roofline of the dominant kernels (the RK4 brick march: every domain launch,
one lane per particle in large launches, a lane quad per particle in small
ones) from HIP events taken
on the stream it runs on, the CPU oracle on a bounded sample, and extras: the
64M-item x 32-byte multi-split microbenchmark (uniform and Zipf over 1024
destinations) against the HBM roofline, and the 128^3 / 64-view
emission-absorption forward render.

    python bench.py [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "forwarded items/s + ray samples/s on 1 MI355X, % HBM peak; batched/adjoint vs plain"
HBM_PEAK_GBS = 8000.0
# float32 vector peak, published: 157.3 TFLOP/s = 256 CUs x 128 float32
# lanes per clock (packed pairs on 64 lanes) x 2 (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12
# The ceiling without packed math (this build emits no packed float32
# instructions): 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz = 78.6 TFLOP/s.
ALU_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# RK4 steps per brick visit of the streamline job (the library's measured best;
# the same value as rafi.SL_STEPS_PER_VISIT)
STEPS_PER_VISIT = 112
# Algorithmic float32 flops of one RK4 step (FMA = 2): per trilinear vec3
# sample 2 subs for the weights x 3 axes + 7 lerps (sub + fma) x 3 components
# = 69; four samples = 276; three stage offsets (3 fma) = 18; the weighted
# sum (2 fma + add) x 3 = 15; the update (3 fma) = 6.  Total 315.
RK4_FLOPS_PER_STEP = 315
# Algorithmic bytes per item of one forward step: read item + read dest +
# write item.
def split_bytes_per_item(item_bytes: int) -> int:
    return 2 * item_bytes + 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# HBM-side bytes per RK4 launch (mean over every domain launch of the job,
# both kernels): FETCH_SIZE + WRITE_SIZE per dispatch, scaled by a plain copy
# of known size (profiles/rk4_advance_256cube_1Mseeds.md), for the source
# file and schedule (steps_per_visit, tail_items, refill_lanes, quad_items)
# below; reported only while both still hold.
RK4_TRAFFIC = {"kernel": "advance_kernel<3, true> + advance_quad_kernel<3>", "bytes_per_launch": 408020608,
               "source": "paper_2605_30294_amd/csrc/streamline.hip", "source_sha256_16": "6a95fa3e013ff3be",
               "schedule": (112, 0, 0, 98304), "field_layout": "unpadded"}


def rk4_traffic(schedule, layout):
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), RK4_TRAFFIC["source"])
    h = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    if h != RK4_TRAFFIC["source_sha256_16"] or tuple(schedule) != RK4_TRAFFIC["schedule"] \
            or layout != RK4_TRAFFIC["field_layout"]:
        return None
    return RK4_TRAFFIC["bytes_per_launch"]


def streamline_job(args, dev):
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    n, grid, N, h, max_steps = 256, (4, 4, 4), 1 << 20, 0.25, 2000
    field = W.abc_field(n, device=dev)          # [n, n, n, 3]: the unpadded layout
    f4 = rafi.sl_pack(field)                    # [n, n, n, 4]: the padded layout
    layouts = {"padded": f4, "unpadded": field}
    seeds_np = W.streamline_seeds(N, n)
    seeds = torch.from_numpy(seeds_np).to(dev)
    ctx = rafi.Context(64, rafi.SL_ITEM_BYTES, N)
    endpoint = torch.empty((N, 3), dtype=torch.float32, device=dev)
    steps = torch.empty(N, dtype=torch.int32, device=dev)
    reason = torch.empty(N, dtype=torch.int32, device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    quad = rafi.SL_QUAD_ITEMS if args.quad_items is None else args.quad_items
    # the schedule sweep runs on the chosen layout (under "auto", the unpadded one)
    first = layouts["unpadded" if args.field_layout == "auto" else args.field_layout]
    job = rafi.sl_job(first, grid, endpoint, steps, reason, h, max_steps, args.steps_per_visit, counters,
                      args.tail_items, args.refill_lanes, quad)
    tuned = None
    if args.autotune or args.steps_per_visit < 0:      # sweep the schedule (results do not depend on it)
        from paper_2605_30294_amd import autotune
        tuned, _, sweep = autotune.tune_streamlines(ctx, job, seeds)
        log("streamline schedule sweep (ms, (steps_per_visit, tail_items, refill_lanes, quad_items)): "
            + ", ".join(f"{m:.2f} {t}" for m, t in sweep))
    # field layout: the same values with 16 or 12 bytes per voxel; keep the faster
    layout_ms = {}
    for name, f in (layouts.items() if args.field_layout == "auto" or args.autotune else ()):
        lj = rafi.sl_job(f, grid, endpoint, steps, reason, h, max_steps, job.steps_per_visit, counters,
                         job.tail_items, job.refill_lanes, job.quad_items)
        rafi.sl_trace_job(ctx, lj, seeds)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(2):
            rafi.sl_trace_job(ctx, lj, seeds)
        b.record()
        torch.cuda.synchronize()
        layout_ms[name] = a.elapsed_time(b) / 2
    layout = min(layout_ms, key=layout_ms.get) if layout_ms else args.field_layout
    log("streamline field layout (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in layout_ms.items())
        + f"; using {layout}")
    job = rafi.sl_job(layouts[layout], grid, endpoint, steps, reason, h, max_steps, job.steps_per_visit, counters,
                      job.tail_items, job.refill_lanes, job.quad_items)
    for _ in range(args.warmup):
        rafi.sl_trace_job(ctx, job, seeds)
    torch.cuda.synchronize()
    counters.zero_()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    fwd = rounds = 0
    for _ in range(args.steps):
        rounds, fwd = rafi.sl_trace_job(ctx, job, seeds)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    rk4_steps = int(steps.sum().item())
    cross = int(counters[0].item()) // args.steps
    self_fwd = int(counters[1].item()) // args.steps
    # per-kernel breakdown from one more job with event pairs around every launch
    # (outside the timed region: the events cost a few microseconds per round)
    ctx.set_profiling(True)
    rafi.sl_trace_job(ctx, job, seeds)
    prof = ctx.profile()
    ctx.set_profiling(False)
    log(f"streamlines: {ms:.3f} ms/job, rounds {rounds}, forward-step items {fwd} "
        f"(seeds {N}, cross-brick {cross}, same-brick {self_fwd}), rk4 steps {rk4_steps}")
    per_job = 1.0
    dom_ms = prof["domain_ms"] * per_job
    split_ms = prof["split_ms"] * per_job
    launches = prof["domain_calls"] * per_job
    avg_launch_ms = dom_ms / max(launches, 1)
    flops_per_launch = rk4_steps * RK4_FLOPS_PER_STEP / max(launches, 1)
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    schedule = (job.steps_per_visit, job.tail_items, job.refill_lanes, job.quad_items)
    fw = 3 if layout == "unpadded" else 4
    # the one-lane kernel reads fields of at most 2^31 - 1 bytes through a buffer resource
    one_lane = f"advance_kernel<{fw}, {'true' if n ** 3 * fw * 4 <= 2 ** 31 - 1 else 'false'}>"
    if job.refill_lanes:
        kernels = f"advance_persistent_kernel<{fw}>"
    elif job.quad_items:
        kernels = f"{one_lane} + advance_quad_kernel<{fw}> (launches over <= {job.quad_items} particles)"
    else:
        kernels = one_lane
    out = dict(ms=ms, rounds=rounds, forwarded=N + cross, step_items=fwd, self_fwd=self_fwd, rk4_steps=rk4_steps,
               schedule=schedule, field_layout=layout,
               domain_ms=dom_ms, split_ms=split_ms,
               launches=launches, avg_launch_ms=avg_launch_ms,
               roofline={"kernel": kernels + ", RK4 brick march: every domain launch", "bound": "alu",
                         "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                         "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                         "peak_unpacked": round(ALU_UNPACKED_TFLOPS, 1),
                         "frac_unpacked": round(achieved / ALU_UNPACKED_TFLOPS, 4),
                         "traffic": rk4_traffic(schedule, layout),
                         "traffic_unit": "bytes per launch (HBM side: FETCH_SIZE + WRITE_SIZE, calibrated)",
                         "per_launch_flops": flops_per_launch, "avg_launch_ms": round(avg_launch_ms, 4)})
    ctx.close()
    return out, seeds_np


def cpu_baseline(seeds_np, n_sample, n_single):
    """The C oracle (untuned) on the host: the first n_sample seeds of the job
    on all host cores (OpenMP over the items of each domain and round), and
    the first n_single seeds on one core. Forwarded items as in `value`: the
    oracle integrates until exit, so every forward after the seeding round
    crosses a brick boundary."""
    import numpy as np

    import oracle
    from paper_2605_30294_amd import workloads as W

    field = W.abc_field(256)
    host_cpus = len(os.sched_getaffinity(0))

    def run(n, threads):
        oracle.set_threads(threads)
        try:
            sample = np.ascontiguousarray(seeds_np[:n])
            t = time.perf_counter()
            r = oracle.streamlines(field, (4, 4, 4), sample, h=0.25, max_steps=2000)
            return time.perf_counter() - t, int(r["round_counts"].sum()), int(r["steps"].sum())
        finally:
            oracle.set_threads(1)

    threads = oracle.default_threads()
    dt, fwd, rk4 = run(n_sample, threads)
    log(f"cpu oracle: {n_sample} seeds on {threads} threads ({host_cpus} host CPUs) in {dt:.2f} s, "
        f"forwarded {fwd}")
    dt1, fwd1, rk41 = run(n_single, 1)
    log(f"cpu oracle: {n_single} seeds on 1 thread in {dt1:.2f} s, forwarded {fwd1}")
    sample = "all 1M seeds" if n_sample == len(seeds_np) else f"first {n_sample} of the 1M seeds"
    return {"value": fwd / dt, "unit": "forwarded items/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample}, same field/grid/RK4 settings, C oracle with OpenMP over the items of each "
                      f"domain and round on {threads} threads ({dt:.1f} s, {rk4} RK4 steps)",
            "host_cpus": host_cpus, "rk4_steps_per_s": rk4 / dt,
            "single_thread": {"value": fwd1 / dt1, "unit": "forwarded items/s", "cores": 1,
                              "sample": f"first {n_single} of the 1M seeds ({dt1:.1f} s)"}}


def split_microbench(dev, reps, S=32):
    """64M items of S bytes (32: an id and 7 float32 words; 44: the paper's
    ray size, the same with 10 words) over 1024 destinations, uniform and
    Zipf; every scatter shape, then the best one timed."""
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    N, D = 1 << 26, 1024
    items = torch.from_numpy(W.split_items(N, S // 4).view(np.int32)).to(dev)
    res = {}
    ctx = rafi.Context(D, S, N)

    def timed(reps_):
        ctx.round(counts=False)                      # warm-up; slots are left intact
        ctx.set_profiling(True)
        for _ in range(reps_):
            ctx.round(counts=False)
        p = ctx.profile()
        ctx.set_profiling(False)
        return p["split_ms"] / p["split_calls"], p["scatter_ms"] / p["scatter_calls"]

    for dist in ("uniform", "zipf"):
        dest = torch.from_numpy(W.split_dest(N, D, dist)).to(dev)
        ctx.begin(N)
        ctx.emit_bulk(items, dest)
        # workgroup shape of the scatter: every shape gives the same bytes
        shapes = {}
        for v in range(1, 18):
            rafi.split_set_variant(v)
            shapes[v] = timed(3)[0]
        best = min(shapes, key=shapes.get)
        rafi.split_set_variant(best)
        split_ms, scat_ms = timed(reps)
        rafi.split_set_variant(0)
        alg = split_bytes_per_item(S) * N
        res[dist] = {"split_ms": round(split_ms, 4), "scatter_ms": round(scat_ms, 4),
                     "items_per_s": N / (split_ms * 1e-3), "GBps": alg / (split_ms * 1e-3) / 1e9,
                     "frac_hbm": alg / (split_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "scatter_GBps": alg / (scat_ms * 1e-3) / 1e9, "shape": best,
                     "shape_ms": {k: round(v, 4) for k, v in shapes.items()}}
        log(f"split {dist} S={S}: {split_ms:.3f} ms ({res[dist]['GBps']:.0f} GB/s algorithmic), scatter {scat_ms:.3f} ms, "
            f"shapes {res[dist]['shape_ms']}")
        del dest
    ctx.close()
    del items
    torch.cuda.empty_cache()
    return res


def split_domain_sweep(dev, reps, domains=(16, 64, 256, 1024, 4096)):
    """The same 64M x 32-byte split over a range of destination counts
    (uniform), best scatter shape each: how the time depends on the number of
    output regions written at once."""
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    N, S = 1 << 26, 32
    items = torch.from_numpy(W.split_items(N).view(np.int32)).to(dev)
    out = {}
    for D in domains:
        dest = torch.from_numpy(W.split_dest(N, D, "uniform")).to(dev)
        ctx = rafi.Context(D, S, N)
        ctx.begin(N)
        ctx.emit_bulk(items, dest)
        best = None
        for v in (0, 1, 12, 13, 14, 15):
            try:
                rafi.split_set_variant(v)
                ctx.round(counts=False)
                ctx.set_profiling(True)
                for _ in range(reps):
                    ctx.round(counts=False)
                p = ctx.profile()
                ctx.set_profiling(False)
                ms = p["split_ms"] / p["split_calls"]
                if best is None or ms < best[0]:
                    best = (ms, v, p["scatter_ms"] / p["scatter_calls"])
            finally:
                rafi.split_set_variant(0)
        ctx.close()
        del dest
        out[D] = {"split_ms": round(best[0], 4), "scatter_ms": round(best[2], 4), "shape": best[1],
                  "GBps": split_bytes_per_item(S) * N / (best[0] * 1e-3) / 1e9}
        log(f"split D={D}: {best[0]:.3f} ms (scatter {best[2]:.3f}), {out[D]['GBps']:.0f} GB/s")
    return out


def ea_forward(dev, reps):
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    n, grid = 128, (4, 4, 4)
    vol = W.blob_volume(n, W.SEED_ADJ_VOLUME, device=dev)
    views = W.random_views(64, n, 256, 256)
    c = float(np.float32(0.025))
    r = rafi.ea_render(vol, grid, views, c=c, want_tau=True)
    ctx, job = r["ctx"], r["job"]
    torch.cuda.synchronize()
    kl, kf = r["klast"], r["kfirst"]
    samples = int((kl - kf).clamp(min=0).sum().item())
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        rounds = rafi.ea_render_job(ctx, job)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    ctx.set_profiling(True)                 # breakdown from one more render
    rafi.ea_render_job(ctx, job)
    p = ctx.profile()
    ctx.close()
    out = {"workload": "128^3 blobs, 4x4x4 domains, 64 views x 256^2 rays", "ms": round(ms, 4),
           "rounds": rounds, "samples": samples, "samples_per_s": samples / (ms * 1e-3),
           "march_ms": round(p["domain_ms"], 4), "split_ms": round(p["split_ms"], 4),
           "rays_forwarded_per_s": p["split_items"] / (ms * 1e-3)}
    log(f"ea forward: {ms:.3f} ms, {samples} samples, {out['samples_per_s']:.3g} samples/s")
    return out


def delta_tracking(dev, reps):
    """Delta-tracking path tracing: 128^3 blobs, 4x4x4 bricks, 16 views x 256^2
    paths (one per pixel), up to 4 scattering events each with a shadow ray."""
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    n, grid, B = 128, (4, 4, 4), 4
    vol = W.blob_volume(n, W.SEED_ADJ_VOLUME, device=dev)
    views = W.random_views(16, n, 256, 256)
    kappa = 0.5                      # about 0.3 scattering events per path in this volume
    smax = float(np.float32(kappa * float(vol.max().item())))
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    r = rafi.dt_render(vol, grid, views, kappa, smax, 0.8, (0.0, 0.6, 0.8), 1.0, B, 11)
    ctx, job = r["ctx"], r["job"]
    job.counters = rafi._dptr(counters)
    rafi.dt_render_job(ctx, job)
    torch.cuda.synchronize()
    counters.zero_()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        rounds = rafi.dt_render_job(ctx, job)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    points, hits = (int(v) // reps for v in counters.cpu().tolist())
    ctx.set_profiling(True)                 # breakdown from one more render
    rafi.dt_render_job(ctx, job)
    p = ctx.profile()
    reps = 1
    n_paths = 16 * 256 * 256
    ctx.close()
    out = {"workload": "128^3 blobs, 4x4x4 domains, 16 views x 256^2 paths, kappa 0.5, albedo 0.8, "
                       "<=4 scattering events + shadow rays",
           "ms": round(ms, 4), "rounds": rounds, "paths_per_s": n_paths / (ms * 1e-3),
           "tentative_points": points, "real_collisions": hits, "points_per_s": points / (ms * 1e-3),
           "trace_ms": round(p["domain_ms"] / reps, 4), "split_ms": round(p["split_ms"] / reps, 4),
           "forwarded_items_per_s": p["split_items"] / reps / (ms * 1e-3)}
    log(f"delta tracking: {ms:.3f} ms, {rounds} rounds, {points} tentative points, {hits} collisions, "
        f"{out['points_per_s']:.3g} points/s")
    return out


def nbody_exchange(dev, reps):
    """Multi-context, multi-phase forwarding: the N-body essential-tree
    exchange, 2^16 clustered particles in 64 Morton domains, cells of level
    4, theta 0.5, softening 1e-3, dt 1e-3. A step = migration round, key
    sort, hierarchy, two virtual-particle rounds and a request round, forces."""
    import time

    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    n, D = 1 << 16, 64
    nb = rafi.NBody(rafi.nb_to_device(W.nbody_particles(n), dev), D, cell_level=4, theta=0.5, eps=1e-3, dt=1e-3)
    nb.step(0.0)                      # accelerations at t = 0
    nb.step()
    torch.cuda.synchronize()
    items = interactions = 0
    t0 = time.perf_counter()
    for _ in range(reps):
        rc, sz = nb.step()
        items += int(rc.sum())
        npd = rc[0].astype(np.int64)
        interactions += int((npd * (npd - 1)).sum() + (npd * rc[3].astype(np.int64)).sum())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    nb.close()
    out = {"workload": "N-body essential-tree exchange: 2^16 clustered particles, 64 Morton domains, "
                       "level-4 cells, theta 0.5, three contexts (40/24/4-byte items)",
           "ms_per_step": round(ms, 4), "forwarded_items_per_step": items // reps,
           "forwarded_items_per_s": items / reps / (ms * 1e-3),
           "round_items": {"particles": int(rc[0].sum()), "virtual_1": int(rc[1].sum()),
                           "requests": int(rc[2].sum()), "virtual_2": int(rc[3].sum())},
           "interactions_per_step": interactions // reps,
           "interactions_per_s": interactions / reps / (ms * 1e-3)}
    log(f"nbody: {ms:.3f} ms/step, {out['forwarded_items_per_step']} forwarded items, "
        f"{out['interactions_per_step']} interactions ({out['interactions_per_s']:.3g}/s)")
    return out


def ea_adjoint(dev, reps):
    """128^3 / 64 bricks / 64 views x 256^2: forward render, then the
    reverse-replay backward of the L2 image loss against a second volume."""
    import numpy as np
    import torch

    from paper_2605_30294_amd import rafi
    from paper_2605_30294_amd import workloads as W

    n, grid = 128, (4, 4, 4)
    c = float(np.float32(0.025))
    vol = W.blob_volume(n, W.SEED_ADJ_VOLUME, device=dev)
    tgt = W.blob_volume(n, W.SEED_ADJ_TARGET, device=dev)
    views = W.random_views(64, n, 256, 256)
    target = rafi.ea_render(tgt, grid, views, c=c)["image"]
    r = rafi.ea_render(vol, grid, views, c=c, want_tau=True)
    ctx, job = r["ctx"], r["job"]
    grad_image = 2.0 * (r["image"] - target)
    grad = torch.zeros_like(vol)
    rafi.ea_backward_job(ctx, job, grad_image, grad)      # warm-up
    torch.cuda.synchronize()
    samples = int((r["klast"] - r["kfirst"]).clamp(min=0).sum().item())
    # rays per backward workgroup (each workgroup flushes its brick's gradient
    # once): the same gradient up to float32 summation order; keep the fastest
    sweep = {}
    for tile in (0, 4096, 8192, 16384):
        job.bwd_tile_items = tile
        rafi.ea_backward_job(ctx, job, grad_image, grad)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(2):
            grad.zero_()
            rafi.ea_backward_job(ctx, job, grad_image, grad)
        b.record()
        torch.cuda.synchronize()
        sweep[tile] = round(a.elapsed_time(b) / 2, 4)
    job.bwd_tile_items = min(sweep, key=sweep.get)
    log(f"adjoint backward tile sweep (ms): {sweep}")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        rafi.ea_render_job(ctx, job)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        grad.zero_()
        rafi.ea_backward_job(ctx, job, grad_image, grad)
    ev[3].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    bwd = ev[2].elapsed_time(ev[3]) / reps
    ctx.close()
    out = {"workload": "128^3, 4x4x4 bricks, 64 views x 256^2, L2 loss vs second volume",
           "forward_ms": round(fwd, 4), "backward_ms": round(bwd, 4), "backward_over_forward": round(bwd / fwd, 3),
           "samples": samples, "forward_samples_per_s": samples / (fwd * 1e-3),
           "backward_samples_per_s": samples / (bwd * 1e-3), "bwd_tile_items": job.bwd_tile_items,
           "bwd_tile_sweep_ms": sweep}
    log(f"adjoint: forward {fwd:.3f} ms, backward {bwd:.3f} ms ({bwd / fwd:.2f}x)")
    return out


def batched(dev, reps):
    """256 uneven scenes: one batched render (autotuned, graph-replayed rounds)
    against rendering the scenes one at a time with the plain path."""
    import numpy as np
    import torch

    from paper_2605_30294_amd import autotune, rafi
    from paper_2605_30294_amd import workloads as W

    c = float(np.float32(0.025))
    specs = W.draw_scenes(256)
    vols, scenes = rafi.build_batch_inputs(specs, dev)
    b = rafi.Batch(scenes, c=c)
    image = torch.empty(b.n_rays, dtype=torch.float32, device=dev)
    best, _, _ = autotune.tune_batch(b, vols, image, reps=1)
    ms_b = autotune.time_render(b, vols, image, reps=reps)
    # plain, one scene at a time (contexts and jobs prepared outside the timing)
    plain = []
    samples = 0
    for n, grid, view, off in scenes:
        v = vols[off:off + n ** 3].reshape(n, n, n)
        r = rafi.ea_render(v, grid, np.array([view]), c=c, want_tau=True)
        samples += int((r["klast"] - r["kfirst"]).clamp(min=0).sum().item())
        plain.append(r)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        for r in plain:
            rafi.ea_render_job(r["ctx"], r["job"])
    t1.record()
    torch.cuda.synchronize()
    ms_p = t0.elapsed_time(t1) / reps
    same = bool(torch.equal(image, torch.cat([r["image"] for r in plain])))
    for r in plain:
        r["ctx"].close()
    b.close()
    out = {"workload": "256 scenes: edges 32-256 log-uniform, 1-64 domains, 1K-1M rays (+z)",
           "rays": b.n_rays, "samples": samples, "batched_ms": round(ms_b, 3), "sequential_plain_ms": round(ms_p, 3),
           "speedup": round(ms_p / ms_b, 3), "batched_samples_per_s": samples / (ms_b * 1e-3),
           "tuning": best, "bit_identical_to_plain": same}
    log(f"batched: {ms_b:.2f} ms vs sequential plain {ms_p:.2f} ms ({ms_p / ms_b:.2f}x), identical={same}")
    return out


def plain_copy(dev, reps):
    """A device-to-device copy of exactly 2 GiB per launch: the reference for
    scaling the HBM traffic counters."""
    import torch

    nbytes = 2 << 30
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms, "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seeds", type=int, default=1 << 20,
                    help="seeds of the job the oracle runs on all host cores for cpu_baseline")
    ap.add_argument("--cpu-seeds-single", type=int, default=65536,
                    help="seeds the oracle runs on one core (cpu_baseline.single_thread)")
    ap.add_argument("--only", default=None,
                    choices=["streamlines", "split", "split-domains", "ea", "adjoint", "batched", "dt", "nbody",
                             "copy"],
                    help="run one leg alone (for profilers) and print its result")
    ap.add_argument("--tail-items", type=int, default=0,
                    help="launches with at most this many particles integrate uncapped")
    ap.add_argument("--refill-lanes", type=int, default=0,
                    help="persistent RK4 waves refill when this many lanes are idle (0: one thread per "
                         "particle); ignored when the schedule is autotuned")
    ap.add_argument("--quad-items", type=int, default=None,
                    help="launches over at most this many particles run four lanes per particle (default: "
                         "the library's SL_QUAD_ITEMS; 0: never); ignored when the schedule is autotuned")
    ap.add_argument("--field-layout", default="unpadded", choices=["auto", "padded", "unpadded"],
                    help="RK4 field with 16-byte (padded) or 12-byte voxels; auto keeps the faster")
    ap.add_argument("--autotune", action="store_true",
                    help="sweep (steps_per_visit, tail_items, refill_lanes, quad_items) and the field layout "
                         "before timing "
                         "instead of using the defaults below (the measured best on MI355X)")
    ap.add_argument("--steps-per-visit", type=int, default=STEPS_PER_VISIT,
                    help="RK4 steps a particle takes per domain visit before it is forwarded to its own "
                         "brick (0 = until it leaves, -1 = autotune with the tail threshold); results do "
                         "not depend on it")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: every domain of the forwarding path is resident on a "
              "single MI355X and the exchange is a device-local split (no multi-GPU exchange); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name}, {props.multi_processor_count} CUs, "
        f"LDS per workgroup {getattr(props, 'shared_memory_per_block', 'n/a')} B")

    if args.only is not None:
        if args.only == "streamlines":
            res = streamline_job(args, dev)[0]
        elif args.only == "split":
            res = {"32": split_microbench(dev, reps=args.steps), "44": split_microbench(dev, reps=args.steps, S=44)}
        elif args.only == "split-domains":
            res = split_domain_sweep(dev, reps=args.steps)
        elif args.only == "ea":
            res = ea_forward(dev, reps=args.steps)
        elif args.only == "adjoint":
            res = ea_adjoint(dev, reps=args.steps)
        elif args.only == "batched":
            res = batched(dev, reps=args.steps)
        elif args.only == "dt":
            res = delta_tracking(dev, reps=args.steps)
        elif args.only == "nbody":
            res = nbody_exchange(dev, reps=args.steps)
        else:
            res = plain_copy(dev, reps=args.steps)
        print(json.dumps({"only": args.only, "result": res}, default=str), flush=True)
        return

    sl, seeds_np = streamline_job(args, dev)
    extras = {}
    if not args.no_extras:
        extras["multisplit_64M_x32B_1024dest"] = split_microbench(dev, reps=20)
        extras["multisplit_64M_x44B_1024dest"] = split_microbench(dev, reps=20, S=44)
        extras["ea_forward"] = ea_forward(dev, reps=5)
        extras["adjoint_vs_forward"] = ea_adjoint(dev, reps=3)
        extras["batched_vs_plain"] = batched(dev, reps=2)
        extras["delta_tracking"] = delta_tracking(dev, reps=3)
        extras["nbody_exchange"] = nbody_exchange(dev, reps=3)
    cpu = None if args.no_cpu else cpu_baseline(seeds_np, args.cpu_seeds, args.cpu_seeds_single)

    value = sl["forwarded"] / (sl["ms"] * 1e-3)
    line = {
        "metric": METRIC, "value": value, "unit": "forwarded items/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sl["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "streamlines: 256^3 ABC field (A=1, B=sqrt(2/3), C=sqrt(1/3)), 4x4x4 domains, "
                               "1M uniform seeds, RK4 h=0.25 voxel, <=2000 steps, forwarded at every brick exit",
                   "seeds": 1 << 20, "domains": 64, "item_bytes": 16},
        "samples_per_s": sl["rk4_steps"] / (sl["ms"] * 1e-3),
        "samples_unit": "RK4 steps/s",
        "rounds": sl["rounds"], "forwarded_per_step": sl["forwarded"],
        "forward_step_items_per_step": sl["step_items"], "same_brick_forwards_per_step": sl["self_fwd"],
        "schedule": {"steps_per_visit": sl["schedule"][0], "tail_items": sl["schedule"][1],
                     "refill_lanes": sl["schedule"][2], "quad_items": sl["schedule"][3],
                     "field_layout": sl["field_layout"]},
        "time_split": {"domain_kernels_ms": round(sl["domain_ms"], 4), "forward_steps_ms": round(sl["split_ms"], 4)},
        "roofline": sl["roofline"],
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
