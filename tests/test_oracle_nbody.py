"""Pins of the oracle's multi-context N-body step (O8: the essential-tree
exchange of Sec. 5.5) against facts that do not reuse its arithmetic: bit
interleaving, equal-count decomposition, stable grouping, conservation of
particles and of mass through the exchange, the geometry of the acceptance
test, and the direct gravitational sum in float64 where the exchange
reduces to it."""
import numpy as np
import pytest

import oracle as O
from paper_2605_30294_amd import workloads as W


def _unique_masses(p):
    # distinct masses identify particles (the item has no id field)
    n = len(p)
    p = p.copy()
    p["mass"] = ((np.arange(n) + 1.0) / (n * (n + 1) / 2.0)).astype(np.float32)
    return p


def _morton_ref(x, y, z):
    q = [min(max(int(np.float32(c) * np.float32(1024.0)), 0), 1023) for c in (x, y, z)]
    key = 0
    for b in range(10):
        for a in range(3):
            key |= ((q[a] >> b) & 1) << (3 * b + a)
    return key


def test_morton_is_bit_interleaving():
    rng = np.random.default_rng(0)
    pts = rng.random((500, 3)).astype(np.float32)
    edge = np.array([[0, 0, 0], [np.nextafter(np.float32(1), np.float32(0))] * 3, [0.5, 0.25, 0.125],
                     [1 / 1024, 2 / 1024, 1023 / 1024]], dtype=np.float32)
    for x, y, z in np.concatenate([pts, edge]):
        assert O.morton30(x, y, z) == _morton_ref(x, y, z)
    # x is the lowest bit of each triple
    assert O.morton30(1 / 1024, 0, 0) == 1 and O.morton30(0, 1 / 1024, 0) == 2 and O.morton30(0, 0, 1 / 1024) == 4


@pytest.mark.parametrize("n,D", [(4096, 8), (3000, 7), (5000, 64), (100, 1)])
def test_splitters_give_equal_counts(n, D):
    p = W.nbody_particles(n, seed=n + D)
    K = O.nb_splitters(p, D)
    keys = np.array([_morton_ref(*x) for x in p["pos"]], dtype=np.int64)
    assert K[0] == 0 and K[-1] == 1 << 30 and np.all(np.diff(K.astype(np.int64)) >= 0)
    owner = np.searchsorted(K[1:-1].astype(np.int64), keys, side="right")
    counts = np.bincount(owner, minlength=D)
    if len(np.unique(keys)) == n:   # distinct keys: quantile splitters split exactly
        expect = np.diff((np.arange(D + 1) * n) // D)
        assert np.array_equal(counts, expect)
    q, c = O.nb_seed(p, K)
    assert np.array_equal(c.astype(np.int64), counts)


def test_seed_is_a_stable_grouping_by_owner():
    p = _unique_masses(W.nbody_particles(2000, seed=3))
    K = O.nb_splitters(p, 8)
    q, c = O.nb_seed(p, K)
    keys = np.array([_morton_ref(*x) for x in p["pos"]], dtype=np.int64)
    owner = np.searchsorted(K[1:-1].astype(np.int64), keys, side="right")
    order = np.argsort(owner, kind="stable")
    assert np.array_equal(q.view(np.uint8), p[order].view(np.uint8))


def _by_mass(a):
    return a[np.argsort(a["mass"])]


@pytest.mark.parametrize("theta,level", [(0.5, 4), (0.8, 3), (0.3, 5)])
def test_step_invariants(theta, level):
    n, D = 4096, 8
    p = _unique_masses(W.nbody_particles(n, seed=11))
    K = O.nb_splitters(p, D)
    q, _ = O.nb_seed(p, K)
    r = O.nb_step(q, K, dt=2e-3, cell_level=level, theta=theta)
    out, rc = r["queue"], r["round_counts"]
    # every particle once, grouped by the domain owning its new key, key order within
    assert np.array_equal(np.sort(out["mass"]), np.sort(p["mass"]))
    keys = np.array([_morton_ref(*x) for x in out["pos"]], dtype=np.int64)
    owner = np.searchsorted(K[1:-1].astype(np.int64), keys, side="right")
    assert np.all(np.diff(owner) >= 0) and np.all(np.diff(keys) >= 0)
    assert np.array_equal(np.bincount(owner, minlength=D), rc[0].astype(np.int64))
    nonempty = int(np.count_nonzero(rc[0]))
    # round 1: every root to every other non-empty domain
    assert rc[1].sum() == nonempty * (nonempty - 1) == len(r["vp1"])
    # a root is either accepted (it stays, first in round 2) or answered
    acc = len(r["vp1"]) - len(r["rr"])
    assert rc[2].sum() == len(r["rr"]) and rc[3].sum() == len(r["vp2"]) >= acc
    # each domain's remote list carries every other domain's mass exactly once
    offs = np.concatenate([[0], np.cumsum(rc[3].astype(np.int64))])
    mass_dom = np.array([out["mass"][owner == d].astype(np.float64).sum() for d in range(D)])
    for d in range(D):
        lst = r["vp2"][offs[d]:offs[d + 1]]
        if rc[0][d] == 0:
            continue
        got = np.array([lst["mass"][lst["src"] == s].astype(np.float64).sum() for s in range(D)])
        want = mass_dom.copy()
        want[d] = 0.0
        assert np.allclose(got, want, rtol=1e-5, atol=0), d
        # answers are leaves (size 0) or cells/roots whose centre lies outside the receiver's box
        box_lo = out["pos"][owner == d].min(0)
        box_hi = out["pos"][owner == d].max(0)
        far = lst[lst["smax"] > 0]
        outside = np.any((far["pos"] < box_lo) | (far["pos"] > box_hi), axis=1)
        assert np.all(outside)
        # and satisfy size < theta * distance to the box (float64, up to rounding)
        gap = np.maximum(np.maximum(box_lo - far["pos"], far["pos"] - box_hi), 0.0).astype(np.float64)
        dist = np.sqrt((gap ** 2).sum(1))
        assert np.all(far["smax"] < theta * dist * (1 + 1e-5))
        # answered cells have the level's edge; roots the largest edge of their domain's box
        cells = far[far["smax"] != np.float32(2.0 ** -level)]
        for v in cells:
            s_box = out["pos"][owner == v["src"]]
            assert v["smax"] == np.float32((s_box.max(0) - s_box.min(0)).max())


def _direct(pos, mass, eps, absolute=False, block=1024):
    """float64 softened direct sum over all other particles, in row blocks
    (bounded temporaries); absolute=True sums |term| per component."""
    x = pos.astype(np.float64)
    m = mass.astype(np.float64)
    out = np.empty_like(x)
    for b0 in range(0, len(x), block):
        b1 = min(b0 + block, len(x))
        d = x[None, :, :] - x[b0:b1, None, :]
        r2 = (d ** 2).sum(-1) + eps * eps
        r2[np.arange(b1 - b0), np.arange(b0, b1)] = np.inf
        t = m[None, :, None] * d / r2[..., None] ** 1.5
        out[b0:b1] = (np.abs(t) if absolute else t).sum(1)
    return out


@pytest.mark.parametrize("n,D", [(1500, 6), (9000, 2)])
def test_theta_zero_is_the_direct_sum(n, D):
    """theta = 0 accepts nothing: every particle reaches every other domain as
    a leaf, so each force is the direct softened sum (float64 reference,
    summed here in another order): equal up to the float32 rounding of the
    stored acceleration."""
    eps = 1e-2
    p = _unique_masses(W.nbody_particles(n, seed=21))
    K = O.nb_splitters(p, D)
    q, _ = O.nb_seed(p, K)
    r = O.nb_step(q, K, dt=0.0, theta=0.0, eps=eps)
    out = r["queue"]
    assert len(r["rr"]) == len(r["vp1"]) and np.all(r["vp2"]["smax"] == 0)
    assert np.array_equal(_by_mass(out)["pos"].view(np.uint32), _by_mass(q)["pos"].view(np.uint32))  # dt = 0
    a = _direct(out["pos"], out["mass"], eps)
    err = np.linalg.norm(out["acc"].astype(np.float64) - a, axis=1)
    assert np.all(err <= 2e-7 * np.linalg.norm(a, axis=1) + 1e-12 * np.abs(a).max())
    # the terms' magnitudes: the same sums with |term| per component (the
    # oracle takes eps as a float32 parameter)
    e32 = float(np.float32(eps))
    mag = _direct(out["pos"], out["mass"], e32, absolute=True)
    assert np.allclose(r["acc_mag"], mag, rtol=1e-12, atol=0)
    # momentum: sum m a vanishes up to float32 rounding
    mom = (out["mass"][:, None].astype(np.float64) * out["acc"]).sum(0)
    assert np.all(np.abs(mom) <= 1e-5 * (np.abs(out["mass"][:, None] * out["acc"]).sum(0)))


def test_two_bodies_closed_form():
    """One particle per domain: each feels the other's softened pull exactly,
    m (x1 - x0) / (|x1 - x0|^2 + eps^2)^1.5, and the kick adds dt/2 of it."""
    p = np.zeros(2, dtype=W.NB_PARTICLE_DTYPE)
    p["pos"] = [[0.25, 0.25, 0.25], [0.75, 0.5, 0.25]]
    p["mass"] = [0.5, 0.25]
    K = O.nb_splitters(p, 2)
    q, c = O.nb_seed(p, K)
    assert list(c) == [1, 1]
    eps, dt = 0.05, 0.01
    r = O.nb_step(q, K, dt=dt, theta=0.0, eps=eps)
    out = _by_mass(r["queue"])
    for i, j in ((0, 1), (1, 0)):
        d = out["pos"][j].astype(np.float64) - out["pos"][i]
        a = out["mass"][j] * d / (d @ d + eps * eps) ** 1.5
        assert np.allclose(out["acc"][i], a, rtol=1.2e-7, atol=0)
        # velocity: the first half-kick used a = 0, the second dt/2 a
        assert np.allclose(out["vel"][i], 0.5 * dt * a, rtol=3e-7, atol=1e-12)


def test_drift_wraps_and_kicks():
    """Positions after a step: wrap(x + dt (v + dt/2 a_prev)), the leapfrog
    drift with the stored acceleration, in float64 within rounding."""
    n, D, dt = 1000, 4, 0.05
    p = _unique_masses(W.nbody_particles(n, seed=5, vel_sigma=0.5))
    K = O.nb_splitters(p, D)
    q, _ = O.nb_seed(p, K)
    q = O.nb_step(q, K, dt=0.0)["queue"]                 # accelerations at t = 0
    r = O.nb_step(q, K, dt=dt)
    a0, a1 = _by_mass(q), _by_mass(r["queue"])
    v = a0["vel"].astype(np.float64) + 0.5 * dt * a0["acc"]
    x = a0["pos"] + dt * v
    x = x - np.floor(x)
    diff = np.abs(a1["pos"] - x)
    diff = np.minimum(diff, 1.0 - diff)                  # across the periodic seam
    assert np.all(diff < 1e-6)
    assert np.any(np.abs(a0["pos"] + dt * v - x) > 0.5)  # some particles did wrap
