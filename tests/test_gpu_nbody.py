"""GPU parity of the multi-context, multi-phase forwarding step (the N-body
essential-tree exchange of Sec. 5.5) against the oracle.

Before every step the GPU's particle queue is re-seeded from the oracle's, so
both sides route the same state. Bit-exact: the Morton splitters, the queue
after each seed (and the drifted positions and masses after each step), the
per-domain counts of the four forward rounds, the first virtual-particle
queue, the refinement requests and the remote lists. The forces are float32
sums on the GPU (in an order of its own) against the oracle's float64 sums in
plain order: per component within 1e-5 of the sum of the terms' magnitudes
(measured worst about 2.3e-6), and velocities within that times dt/2 plus one
float32 ulp."""
import numpy as np
import pytest
import torch

from gpu_util import announce, device
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu

FORCE_RTOL = 1e-5   # of the sum of the force terms' magnitudes, per component


def _unique_masses(p):
    n = len(p)
    p = p.copy()
    p["mass"] = ((np.arange(n) + 1.0) / (n * (n + 1) / 2.0)).astype(np.float32)
    return p


def _same(a, b):
    return a.shape == b.shape and np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                                                 np.ascontiguousarray(b).view(np.uint8))


def _check_forces(got, want, acc_mag, dt):
    for f in ("pos", "mass"):
        assert np.array_equal(np.ascontiguousarray(got[f]).view(np.uint32),
                              np.ascontiguousarray(want[f]).view(np.uint32)), f
    tol = FORCE_RTOL * acc_mag
    err = np.abs(got["acc"].astype(np.float64) - want["acc"])
    assert np.all(err <= tol), float((err / tol).max())
    hdt = float(np.float32(0.5) * np.float32(dt))
    ulp = np.spacing(np.abs(want["vel"])).astype(np.float64)
    verr = np.abs(got["vel"].astype(np.float64) - want["vel"])
    assert np.all(verr <= hdt * tol + ulp), float((verr / (hdt * tol + ulp)).max())


def _run(orc, p, D, level, theta, eps, dts, debug=True):
    dev = device()
    K = orc.nb_splitters(p, D)
    nb = rafi.NBody(rafi.nb_to_device(p, dev), D, cell_level=level, theta=theta, eps=eps, debug=debug,
                    log_vp1=True)
    try:
        assert np.array_equal(nb.splitters.cpu().numpy().view(np.uint32), K)
        q, _ = orc.nb_seed(p, K, cell_level=level, theta=theta, eps=eps)
        assert _same(nb.particles(), q)
        for k, dt in enumerate(dts):
            if k:
                # the oracle's state becomes the GPU's: a stable re-grouping of a grouped queue
                nb.reseed(rafi.nb_to_device(q, dev))
                assert _same(nb.particles(), q)
            rc, sz = nb.step(dt)
            r = orc.nb_step(q, K, dt, cell_level=level, theta=theta, eps=eps, log_cap=1 << 24)
            q = r["queue"]
            assert np.array_equal(rc, r["round_counts"])
            assert list(sz) == [len(r["vp1"]), len(r["rr"]), len(r["vp2"])]
            vp1 = nb.vp1[: int(sz[0])].cpu().numpy().reshape(-1).view(rafi.NB_VIRTUAL_DTYPE)
            assert _same(vp1, r["vp1"])
            assert np.array_equal(nb.requests(), r["rr"])
            assert _same(nb.remote_lists(), r["vp2"])
            _check_forces(nb.particles(), q, r["acc_mag"], dt)
            for c in (nb.P, nb.V, nb.R):
                st = c.stats()
                assert st["bad_dest"] == 0 and st["dropped"] == 0
        return q
    finally:
        nb.close()


@pytest.mark.parametrize("n,D,level,theta,eps,dts", [
    (4096, 8, 4, 0.5, 1e-3, [0.0, 2e-3, 2e-3]),
    (3001, 7, 3, 0.8, 1e-2, [0.0, 5e-3]),
    (5000, 64, 5, 0.3, 1e-3, [0.0, 1e-3]),
    (2000, 16, 2, 0.0, 1e-3, [1e-3]),          # theta 0: every particle to every other domain
    (1000, 1, 4, 0.5, 1e-3, [0.0, 1e-3]),      # one domain: no exchange
    (777, 3, 10, 1.5, 1e-3, [1e-3, 1e-3]),     # finest cells
    (8192, 1, 4, 0.5, 1e-3, [1e-3]),           # one domain of 8192: the largest sorted in LDS
    (20000, 2, 4, 0.5, 1e-3, [0.0, 1e-3]),     # domains over 8192: the three digit passes
])
def test_nbody_matches_oracle(orc, n, D, level, theta, eps, dts):
    announce(f"nbody n={n} D={D} L={level} theta={theta}")
    p = _unique_masses(W.nbody_particles(n, seed=n + D))
    _run(orc, p, D, level, theta, eps, dts)


def test_nbody_migration_empties_domains(orc):
    """Few particles per domain and large velocities: domains empty out and
    fill up between steps; empty domains send and receive nothing."""
    announce("nbody migration")
    p = _unique_masses(W.nbody_particles(300, seed=9, vel_sigma=2.0))
    q = _run(orc, p, 64, 4, 0.5, 1e-3, [0.0, 0.05, 0.05])
    K = orc.nb_splitters(p, 64)
    keys = np.array([orc.morton30(*x) for x in q["pos"]], dtype=np.int64)
    owner = np.searchsorted(K[1:-1].astype(np.int64), keys, side="right")
    assert np.count_nonzero(np.bincount(owner, minlength=64)) < 64


def test_nbody_full_size(orc):
    """2^16 particles in 64 Morton domains, cells of level 4, theta 0.5:
    the benchmark's workload, one step, everything compared."""
    announce("nbody full size")
    p = W.nbody_particles(1 << 16)
    _run(orc, p, 64, 4, 0.5, 1e-3, [1e-3], debug=False)


def test_nbody_overflow_is_reported(orc):
    """Answers that do not fit the virtual-particle context: RAFI_ERR_OVERFLOW,
    and nothing of the second round is emitted."""
    dev = device()
    p = W.nbody_particles(2000, seed=4)
    nb = rafi.NBody(rafi.nb_to_device(p, dev), 8, theta=0.0, virtual_capacity=8 * 7 + 100)
    try:
        with pytest.raises(rafi.RafiError) as e:
            nb.step(0.0)
        assert e.value.code == rafi.ERR_OVERFLOW
    finally:
        nb.close()
