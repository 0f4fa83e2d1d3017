"""Pins for the delta-tracking oracle (volume path tracing over bricks).

Each check rests on something other than the oracle's own arithmetic: the
published known-answer vectors of Philox4x32-10, float64 logarithms, the
closed form of single scattering in a homogeneous slab, the exponential law
of free paths, and invariance of every path under a change of bricks (the
tentative collisions use one global majorant, so bricks only route)."""
import math

import numpy as np
import pytest

from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_philox_known_answers(orc):
    # known-answer vectors published with the Random123 library (Salmon et al., SC 2011)
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in cases:
        assert list(orc.philox4x32_10(ctr, key)) == want


def test_logf_against_float64(orc):
    k = np.unique(np.concatenate([np.arange(1, 4097), np.arange(1, 1 << 24, 4099), [1 << 24]]))
    x = (k.astype(np.float64) * 2.0 ** -24).astype(np.float32)     # every value 1 - u can take
    got = orc.dt_logf(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    nz = ref != 0
    assert np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])) < 4e-7
    assert got[x == 1.0][0] == 0.0
    assert np.all(np.diff(got) >= 0)                               # monotone


def _slab(orc, n, rho0, kappa, smax, B, seed, grid=(1, 1, 1), albedo=1.0, w=64):
    vol = W.uniform_volume(n, rho0)
    views = W.plusz_view(n, w, w)
    return orc.dt_render(vol, grid, views, kappa, smax, albedo, (0.0, 0.0, -1.0), 1.0, B, seed)


def test_single_scatter_closed_form(orc):
    """Rays along +z through a homogeneous cube of depth L, light behind the
    camera: the single-scattering radiance is albedo/(4 pi) (1 - exp(-2 sigma L))/2."""
    n, rho0, kappa = 16, 1.0, 0.1
    sig, L = kappa * rho0, float(n)
    vals = []
    for seed in range(6):                                         # 6 x 4096 independent paths
        r = _slab(orc, n, rho0, kappa, 2.5 * sig, 1, seed)
        vals.append(r["contrib"][:, 0])
    v = np.concatenate(vals)
    want = (1.0 / (4 * math.pi)) * (1 - math.exp(-2 * sig * L)) / 2
    se = v.std() / math.sqrt(len(v))
    assert abs(v.mean() - want) < 5 * se, (v.mean(), want, se)


def test_first_collision_probability(orc):
    """A path crosses depth L without a real collision with probability
    exp(-sigma L) (delta tracking samples the true free-path law)."""
    n, rho0, kappa = 16, 1.0, 0.08
    hits = []
    for seed in range(6):
        r = _slab(orc, n, rho0, kappa, 4 * kappa, 1, 100 + seed)
        hits.append(r["contrib"][:, 0] > 0)
    h = np.concatenate(hits)
    p_miss = math.exp(-kappa * rho0 * n)
    se = math.sqrt(p_miss * (1 - p_miss) / len(h))
    assert abs((1 - h.mean()) - p_miss) < 5 * se


def test_zero_albedo_and_empty_volume(orc):
    r = _slab(orc, 16, 1.0, 0.1, 0.2, 2, 7, albedo=0.0)
    assert np.all(r["contrib"] == 0.0)
    r = _slab(orc, 16, 0.0, 0.1, 0.2, 2, 7)
    assert np.all(r["contrib"] == 0.0)
    assert r["rounds"] == 2                                       # raygen, one visit each, then empty


@pytest.mark.parametrize("grid", [(2, 2, 2), (4, 2, 1), (1, 4, 4)])
def test_bricks_only_route(orc, grid):
    """Every path's contributions are the same bits whatever the bricks."""
    n = 32
    vol = W.blob_volume(n, 21)
    views = W.random_views(2, n, 24, 24, seed=22)
    smax = 0.06 * float(vol.max()) * 1.25
    args = (0.06, smax, 0.8, (0.6, 0.0, 0.8), 2.0, 3, 9)
    a = orc.dt_render(vol, (1, 1, 1), views, *args)
    b = orc.dt_render(vol, grid, views, *args)
    assert np.array_equal(a["contrib"].view(np.uint64), b["contrib"].view(np.uint64))
    assert b["rounds"] >= a["rounds"]


def test_round_invariants(orc):
    n, grid = 32, (2, 2, 2)
    vol = W.blob_volume(n, 23)
    views = W.random_views(1, n, 32, 32, seed=24)
    smax = 0.05 * float(vol.max()) * 1.1
    r = orc.dt_render(vol, grid, views, 0.05, smax, 0.9, (0.0, 0.6, 0.8), 1.0, 4, 3, queue_cap=1 << 20)
    q = r["queue"]
    assert r["queue_len"] == r["round_counts"].sum()
    kind, bounce, stream = q[:, 10], q[:, 9].astype(np.int64), q[:, 7]
    # streams: 2b for the path after b scattering events, 2b + 1 for the shadow ray of event b
    assert np.all(stream[kind == 0] == 2 * bounce[kind == 0])
    assert np.all(stream[kind == 1] == 2 * bounce[kind == 1] + 1)
    assert np.all(bounce < 4)
    # bounced directions are unit vectors, isotropic
    d = q[:, 3:6].copy().view(np.float32).astype(np.float64)
    bounced = (kind == 0) & (bounce > 0)
    assert bounced.sum() > 100
    assert np.allclose(np.linalg.norm(d[bounced], axis=1), 1.0, atol=1e-6)
    # every queued point lies in the domain it is queued for
    p = q[:, 0:3].copy().view(np.float32)
    doms = np.repeat(np.tile(np.arange(8), r["rounds"]), r["round_counts"].reshape(-1).astype(np.int64))
    b = (np.floor(p).astype(np.int64) // (n // 2))
    assert np.array_equal(b[:, 0] + 2 * (b[:, 1] + 2 * b[:, 2]), doms)
    # at most one shadow ray per scattering event: nothing written past max_bounce events
    assert np.all(np.isfinite(r["contrib"])) and np.all(r["contrib"] >= 0)


def _linear_volume_f32(n, a, b, c, d):
    # dyadic slopes and voxel centres: every voxel value is exact in float32
    x = np.arange(n, dtype=np.float64) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    v = a * X + b * Y + c * Z + d
    assert np.array_equal(v.astype(np.float32).astype(np.float64), v)
    return v.astype(np.float32)


def test_density_sampler_linear_data_strides_and_clamp(orc):
    """The delta-tracking medium's float32 trilinear sampler reproduces a
    linear density with distinct per-axis slopes (so a swapped stride or
    axis fails), within float32 rounding, inside the centre lattice and in
    the half-voxel clamp band at every face, where it takes the value at the
    clamped coordinate."""
    n = 12
    a, b, c, d = 0.75, -1.25, 2.5, 40.0
    vol = _linear_volume_f32(n, a, b, c, d)
    scale = abs(d) + (abs(a) + abs(b) + abs(c)) * n
    tol = 8 * np.finfo(np.float32).eps * scale
    rng = np.random.default_rng(5)
    pts = list(rng.uniform(0.5, n - 0.5, (300, 3)).astype(np.float32))
    band = []
    for ax in range(3):
        for lo in (True, False):
            for _ in range(20):
                q = rng.uniform(0.5, n - 0.5, 3).astype(np.float32)
                q[ax] = np.float32(rng.uniform(0.0, 0.5) if lo else rng.uniform(n - 0.5, n))
                band.append(q)
    band += [np.float32([0.0, 0.0, 0.0]), np.float32([n - 1e-3] * 3), np.float32([0.25, n - 0.25, 6.0]),
             np.float32([-2.0, 5.5, n + 3.0])]
    for q in pts + band:
        qc = np.clip(q.astype(np.float64), 0.5, n - 0.5)
        exact = a * qc[0] + b * qc[1] + c * qc[2] + d
        assert abs(float(orc.dt_density(vol, q)) - exact) <= tol, (q, exact)
    # voxel centres give the voxel values exactly
    for (i, j, k) in [(0, 0, 0), (3, 7, 11), (11, 11, 11), (5, 0, 9), (11, 0, 4)]:
        assert orc.dt_density(vol, (i + 0.5, j + 0.5, k + 0.5)) == vol[k, j, i]
    # a stride error would move the value by far more than the tolerance
    assert abs(b - c) * 1.0 > 100 * tol


def test_collision_probability_in_a_linear_medium(orc):
    """Non-uniform medium: density a + b x + c z (a ramp in x and z), +z rays.
    A path leaves the cube without a real collision with probability
    exp(-kappa * integral of the clamped density along its ray). Checked per
    band of pixel columns (x), so that swapping the sampler's axes or
    strides, which flattens or reverses the x dependence, fails."""
    n, w, kappa = 16, 64, 0.02
    a, b, c = 0.5, 0.25, 0.125
    x = np.arange(n, dtype=np.float64) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    vol = (a + b * X + c * Z).astype(np.float32)
    smax = kappa * float(vol.max()) * 1.5
    views = W.plusz_view(n, w, w)
    seeds = 8
    miss = np.zeros((w, w))                   # [py, px]
    for seed in range(seeds):
        r = orc.dt_render(vol, (2, 2, 2), views, kappa, smax, 1.0, (0.0, 0.0, -1.0), 1.0, 1, 200 + seed)
        miss += (r["contrib"][:, 0] == 0).reshape(w, w)
    px = (np.arange(w) + 0.5) * (n / w)
    xc = np.clip(px, 0.5, n - 0.5)
    zint = 0.5 * 0.5 + ((n - 0.5) ** 2 - 0.25) / 2 + 0.5 * (n - 0.5)   # integral of clamp(z) over [0, n]
    p_col = np.exp(-kappa * ((a + b * xc) * n + c * zint))
    bands = 4
    for k in range(bands):
        cols = slice(k * w // bands, (k + 1) * w // bands)
        trials = seeds * w * (w // bands)
        m = miss[:, cols].sum() / trials
        p = p_col[cols].mean()
        se = math.sqrt(p * (1 - p) / trials)
        assert abs(m - p) < 5 * se, (k, m, p, se)
    # the bands differ by far more than their standard errors
    assert p_col[: w // bands].mean() - p_col[-w // bands:].mean() > 40 * se
