"""Pins for the oracle's RK4 streamline tracer and its round loop (Sec. 5.4).

Checked against: exact motion in a constant field (dyadic seeds), the RK4
update polynomial for linear fields (x' = G x + b gives
x_{m+1} = x_m + h (I + hG/2 + (hG)^2/6 + (hG)^3/24)(G x_m + b), worked out in
float64 with numpy), stagnation and the step limit, the unpartitioned
brute-force trace, and the paper's one-step-per-round form.
"""
import numpy as np
import pytest

from paper_2605_30294_amd import workloads as W


def test_constant_field_exact_motion(orc):
    n = 256
    f = W.constant_field(n, (0.5, 0.0, 0.0))
    rng = np.random.default_rng(0)
    x0 = rng.integers(1024, 250 * 1024, 300) / 1024.0              # dyadic, >= 1
    seeds = np.stack([x0, rng.uniform(0, n, 300), rng.uniform(0, n, 300)], 1).astype(np.float32)
    r = orc.streamlines(f, (4, 4, 4), seeds, h=0.25, max_steps=100000, visit_stride=8)
    steps_exp = np.ceil((256.0 - x0) / 0.125).astype(np.int64)
    # the exiting step is the first with x >= 256
    assert np.array_equal(r["steps"], steps_exp)
    assert np.array_equal(r["endpoint"][:, 0].astype(np.float64), x0 + 0.125 * steps_exp)
    assert np.array_equal(r["endpoint"][:, 1:], seeds[:, 1:])
    assert np.all(r["reason"] == orc.SL_EXITED)
    # visits: bricks along x from the seed's brick to the last one, same (by, bz)
    by = (seeds[:, 1].astype(np.int64) // 64)
    bz = (seeds[:, 2].astype(np.int64) // 64)
    for i in range(300):
        bx0 = int(x0[i]) // 64
        exp = [bx + 4 * (by[i] + 4 * bz[i]) for bx in range(bx0, 4)]
        assert list(r["visits"][i][:len(exp)]) == exp
        assert np.all(r["visits"][i][len(exp):] == -1)


def _rk4_linear_reference(G, b, x0, h, m):
    """float64 RK4 for x' = G x + b, written as the update polynomial."""
    I3 = np.eye(3)
    Z = h * G
    Phi = I3 + Z / 2 + Z @ Z / 6 + Z @ Z @ Z / 24
    x = x0.astype(np.float64).copy()
    for _ in range(m):
        x = x + h * (Phi @ (G @ x + b))
    return x


@pytest.mark.parametrize("G,b", [
    (np.diag([0.4, 0.0, 0.0]), np.zeros(3)),                          # scalar growth, z = hG = 0.1
    (np.array([[0.05, -0.30, 0.02], [0.25, 0.03, -0.1], [0.0, 0.12, -0.04]]) * 0.1,
     np.array([0.3, -0.2, 0.5])),                                      # full 3x3 coupling
])
def test_linear_field_rk4_polynomial(orc, G, b):
    n = 64
    x = np.arange(n, dtype=np.float64) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.empty((n, n, n, 3), dtype=np.float32)
    for c in range(3):
        f[..., c] = b[c] + G[c, 0] * X + G[c, 1] * Y + G[c, 2] * Z
    seeds = np.array([[10.0, 20.0, 30.0], [12.5, 30.25, 25.0], [20.0, 32.0, 33.0],
                      [8.0, 28.0, 31.0]], dtype=np.float32)
    m = 10
    r = orc.streamlines(f, (2, 2, 2), seeds, h=0.25, max_steps=m)
    assert np.all(r["reason"] == orc.SL_MAXSTEPS) and np.all(r["steps"] == m)
    for i in range(len(seeds)):
        ref = _rk4_linear_reference(G, b, seeds[i].astype(np.float64), 0.25, m)
        assert np.all(ref > 1.0) and np.all(ref < n - 1.0)             # stayed where trilinear is exact
        assert np.allclose(r["endpoint"][i], ref, rtol=3e-6, atol=3e-6)
    # sensitivity: a third-order update (dropping the h^4 term) lands more
    # than ten tolerances away in the scalar-growth case
    if G[1, 1] == 0.0 and G[0, 1] == 0.0:
        z = 0.1
        wrong = 10.0 * (1 + z + z * z / 2 + z ** 3 / 6) ** m
        assert abs(r["endpoint"][0, 0] - wrong) > 10 * 3e-6 * wrong


def test_stagnation_and_step_limit(orc):
    n = 32
    seeds = W.streamline_seeds(100, n, seed=4)
    r = orc.streamlines(W.constant_field(n, (0, 0, 0)), (2, 2, 2), seeds)
    assert np.all(r["reason"] == orc.SL_STAGNANT) and np.all(r["steps"] == 1)
    assert np.array_equal(r["endpoint"], seeds)
    r = orc.streamlines(W.constant_field(n, (1e-3, 0, 0)), (2, 2, 2), seeds, max_steps=10)
    assert np.all(r["reason"] == orc.SL_MAXSTEPS) and np.all(r["steps"] == 10)


@pytest.mark.parametrize("grid", [(4, 4, 4), (2, 1, 4), (1, 1, 1)])
def test_partitioned_equals_unpartitioned_abc(orc, grid):
    n = 64
    f = W.abc_field(n)
    seeds = W.streamline_seeds(512, n, seed=21)
    r = orc.streamlines(f, grid, seeds, max_steps=400, visit_stride=40)
    b = orc.streamlines_brute(f, grid, seeds, max_steps=400, visit_stride=40)
    assert np.array_equal(r["endpoint"], b["endpoint"])
    assert np.array_equal(r["steps"], b["steps"])
    assert np.array_equal(r["reason"], b["reason"])
    assert np.array_equal(r["visits"], b["visits"])
    nvis = (r["visits"] >= 0).sum(axis=1)
    rc = r["round_counts"].sum(axis=1).astype(np.int64)
    for k in range(r["rounds"]):
        assert rc[k] == int((nvis > k).sum())


def test_one_step_per_round_equals_until_exit(orc):
    n = 32
    f = W.abc_field(n)
    seeds = W.streamline_seeds(64, n, seed=22)
    a = orc.streamlines(f, (2, 2, 2), seeds, max_steps=150)
    b = orc.streamlines(f, (2, 2, 2), seeds, max_steps=150, one_step=True, max_rounds=1000)
    assert np.array_equal(a["endpoint"], b["endpoint"])
    assert np.array_equal(a["steps"], b["steps"])
    assert np.array_equal(a["reason"], b["reason"])
    assert b["rounds"] == int(a["steps"].max()) + 1


def test_vector_sampler_linear_field_components_and_clamp(orc):
    """The RK4 sampler's float32 trilinear of a 3-component field reproduces a
    linear field whose components have distinct gradients, within float32
    rounding: inside the centre lattice and in the half-voxel clamp band at
    every face, where each component takes its value at the clamped
    coordinate (per axis: clamp q to [1/2, n - 1/2])."""
    n = 10
    G = np.array([[0.5, -0.25, 1.0], [-1.5, 0.75, 0.125], [2.0, 1.25, -0.5]])
    b = np.array([30.0, -20.0, 10.0])
    x = np.arange(n, dtype=np.float64) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.empty((n, n, n, 3), dtype=np.float64)
    for c in range(3):
        f[..., c] = b[c] + G[c, 0] * X + G[c, 1] * Y + G[c, 2] * Z
    assert np.array_equal(f.astype(np.float32).astype(np.float64), f)   # dyadic: exact in float32
    f = f.astype(np.float32)
    tol = 8 * np.finfo(np.float32).eps * (np.abs(b) + np.abs(G).sum(1) * n)
    rng = np.random.default_rng(6)
    pts = list(rng.uniform(0.5, n - 0.5, (300, 3)).astype(np.float32))
    for ax in range(3):
        for lo in (True, False):
            for _ in range(20):
                q = rng.uniform(0.5, n - 0.5, 3).astype(np.float32)
                q[ax] = np.float32(rng.uniform(0.0, 0.5) if lo else rng.uniform(n - 0.5, n))
                pts.append(q)
    pts += [np.float32([0.0, 0.0, 0.0]), np.float32([n - 1e-3] * 3), np.float32([0.49, 9.51, 0.01])]
    for q in pts:
        qc = np.clip(q.astype(np.float64), 0.5, n - 0.5)
        exact = b + G @ qc
        got = orc.tri_vec3(f, q).astype(np.float64)
        assert np.all(np.abs(got - exact) <= tol), (q, got, exact)
    # voxel centres give the voxel's three components exactly
    for (i, j, k) in [(0, 0, 0), (9, 9, 9), (2, 7, 4)]:
        assert np.array_equal(orc.tri_vec3(f, (i + 0.5, j + 0.5, k + 0.5)), f[k, j, i])
