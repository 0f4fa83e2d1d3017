"""The round loops that enqueue each domain launch before the host has read
the forward step's total (rafi_ea_render, rafi_sl_trace, rafi_dt_render,
rafi_ea_backward), run on debug contexts: every output slot is pre-set to the
poison destination, so a slot that a launch over-counted or left unwritten
would be reported as a bad destination. Results equal the round-by-round
drivers' and the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import announce, device, rel_close
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu

C32 = float(np.float32(0.025))


@pytest.mark.parametrize("emit_mode", [rafi.SLOTS_ORDERED, rafi.SLOTS_APPEND])
def test_ea_render_debug(orc, emit_mode):
    dev = device()
    n, grid = 48, (3, 2, 2)
    vol = W.blob_volume(n, 501)
    views = W.random_views(3, n, 40, 40, seed=502)
    n_rays = 3 * 40 * 40
    announce(f"pipelined ea render emit_mode={emit_mode}")
    ctx = rafi.Context(12, rafi.EA_ITEM_BYTES, n_rays, debug=True)
    r = rafi.ea_render(torch.from_numpy(vol).to(dev), grid, views, c=C32, ctx=ctx, want_tau=True,
                       emit_mode=emit_mode)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["bad_dest"] == 0 and st["dropped"] == 0
    o = orc.ea_render(vol, grid, views, c=C32)
    assert r["rounds"] == o["rounds"]
    assert np.array_equal(r["klast"].cpu().numpy(), o["klast"])
    ok, i, rr = rel_close(r["image"].cpu().numpy(), o["image"], 1e-5, 1e-35)
    assert ok, (i, rr)
    ctx.close()


def test_sl_trace_debug(orc):
    dev = device()
    n, grid, N = 64, (4, 2, 2), 3000
    field = W.abc_field(n)
    seeds = W.streamline_seeds(N, n, seed=503)
    announce("pipelined sl trace")
    ctx = rafi.Context(16, rafi.SL_ITEM_BYTES, N, debug=True)
    for refill, cap in ((0, 0), (0, 16), (16, 16)):
        r = rafi.sl_trace(torch.from_numpy(field).to(dev), grid, torch.from_numpy(seeds).to(dev), max_steps=700,
                          ctx=ctx, steps_per_visit=cap, refill_lanes=refill)
        torch.cuda.synchronize()
        st = ctx.stats()
        assert st["bad_dest"] == 0 and st["dropped"] == 0
        o = orc.streamlines(field, grid, seeds, max_steps=700, steps_per_visit=cap, max_rounds=4000)
        assert r["rounds"] == o["rounds"]
        assert np.array_equal(r["endpoint"].cpu().numpy().view(np.uint32), o["endpoint"].view(np.uint32))
        assert np.array_equal(r["steps"].cpu().numpy(), o["steps"])
        assert r["forwarded"] == int(o["round_counts"].sum())
    ctx.close()


def test_dt_render_debug(orc):
    dev = device()
    n, grid, B = 32, (2, 2, 2), 3
    vol = W.blob_volume(n, 504)
    views = W.random_views(2, n, 24, 24, seed=505)
    kappa = 0.3
    smax = float(np.float32(kappa * float(vol.max())))
    announce("pipelined dt render")
    ctx = rafi.Context(8, rafi.DT_ITEM_BYTES, rafi.dt_capacity(2 * 24 * 24, B), debug=True)
    r = rafi.dt_render(torch.from_numpy(vol).to(dev), grid, views, kappa, smax, 0.8, (0.0, 0.6, 0.8), 1.0, B, 5,
                       ctx=ctx)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["bad_dest"] == 0 and st["dropped"] == 0
    o = orc.dt_render(vol, grid, views, kappa, smax, 0.8, (0.0, 0.6, 0.8), 1.0, B, 5)
    assert r["rounds"] == o["rounds"]
    ok, i, rr = rel_close(r["contrib"].cpu().numpy().ravel(), o["contrib"].ravel(), 1e-5, 1e-30)
    assert ok, (i, rr)
    ctx.close()


def test_max_rounds_reported():
    """A round limit below what the job needs ends the loop with
    RAFI_ERR_MAX_ROUNDS after exactly that many forward steps."""
    dev = device()
    n = 64
    vol = torch.from_numpy(W.blob_volume(n, W.SEED_CFG0_VOLUME)).to(dev)
    views = W.plusz_view(n, 64, 64)
    with pytest.raises(rafi.RafiError) as e:
        rafi.ea_render(vol, (2, 2, 2), views, c=C32, max_rounds=2)
    assert e.value.code == rafi.ERR_MAX_ROUNDS
    r = rafi.ea_render(vol, (2, 2, 2), views, c=C32, max_rounds=3)
    assert r["rounds"] == 3
