"""Seeded synthetic inputs for the forwarding hot path.

This module is shared by the HIP path, the tests and the benchmark. It holds
input synthesis only: volumes, vector fields, seed points, destination draws,
camera frames and scene draws. None of the forwarding method's arithmetic
(routing, sampling positions, integration, splitting) lives here.

Every array is produced from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed draw order, so the same seed gives the same bytes on every machine.
Large volumes can be built with torch on a device; the recipe uses only IEEE
multiplies and adds after a host-side ``exp`` of 1-D factors, so the device
result is bit-identical to the host result (checked by a test).

Layout conventions (all C order, x fastest):
  * scalar volume  ``vol[z, y, x]``            float32, voxel centres at i+0.5
  * vector field   ``field[z, y, x, c]``       float32, c = (vx, vy, vz)
  * seeds          ``seeds[i, c]``             float32 positions in voxels
  * view           ``VIEW_DTYPE`` record: org0, du, dv, dir (float32 xyz),
                   width, height, n_samples (int32)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# One orthographic view. Ray (px, py) starts at org0 + px*du + py*dv and walks
# along dir; sample k sits at parameter (k + 0.5) * dt. Both sides of the
# parity check evaluate those expressions themselves; this record only carries
# the camera frame.
VIEW_DTYPE = np.dtype([
    ("org0", "<f4", 3), ("du", "<f4", 3), ("dv", "<f4", 3), ("dir", "<f4", 3),
    ("width", "<i4"), ("height", "<i4"), ("n_samples", "<i4"), ("pad", "<i4"),
])
assert VIEW_DTYPE.itemsize == 64

# Default seeds per workload.
SEED_CFG0_VOLUME = 0
SEED_CFG1_SEEDS = 1
SEED_SPLIT_UNIFORM = 2
SEED_SPLIT_ZIPF = 3
SEED_SPLIT_PAYLOAD = 4
SEED_BATCH_SCENES = 5
SEED_ADJ_VOLUME = 6
SEED_ADJ_TARGET = 7
SEED_ADJ_VIEWS = 8
SEED_ADJ_FD = 9
SEED_NBODY = 10


# ---------------------------------------------------------------- volumes ---

@dataclass(frozen=True)
class Blob:
    centre: tuple
    sigma: float
    amp: float


def draw_blobs(n: int, seed: int, n_blobs: int = 8):
    """Blob parameters in draw order: centre ~ U[0,n)^3, sigma ~ U[4,10],
    amplitude ~ U[0.5,2], one blob after the other."""
    rng = np.random.default_rng(seed)
    blobs = []
    for _ in range(n_blobs):
        c = rng.uniform(0.0, n, 3)
        s = rng.uniform(4.0, 10.0)
        a = rng.uniform(0.5, 2.0)
        blobs.append(Blob(tuple(float(v) for v in c), float(s), float(a)))
    return blobs


def _blob_factors(n: int, blobs):
    """Per-blob 1-D Gaussian factors at voxel centres, float64, host side."""
    x = np.arange(n, dtype=np.float64) + 0.5
    out = []
    for b in blobs:
        inv = 1.0 / (2.0 * b.sigma * b.sigma)
        gx = np.exp(-((x - b.centre[0]) ** 2) * inv)
        gy = np.exp(-((x - b.centre[1]) ** 2) * inv)
        gz = np.exp(-((x - b.centre[2]) ** 2) * inv)
        out.append((b.amp, gx, gy, gz))
    return out


def blob_volume(n: int, seed: int, n_blobs: int = 8, device=None):
    """Sum of seeded isotropic Gaussian blobs at voxel centres, float32.

    rho(x) = sum_b A_b exp(-|x - c_b|^2 / (2 sigma_b^2)), evaluated in float64
    as the product of three 1-D factors, summed blob by blob, then rounded to
    float32. With ``device`` set, the outer products run in torch on that
    device (same operation order, so the same bytes) and a torch tensor is
    returned; otherwise a numpy array.
    """
    fac = _blob_factors(n, draw_blobs(n, seed, n_blobs))
    if device is None:
        acc = np.zeros((n, n, n), dtype=np.float64)
        for a, gx, gy, gz in fac:
            t = ((a * gz)[:, None, None] * gy[None, :, None]) * gx[None, None, :]
            acc = acc + t
        return acc.astype(np.float32)
    import torch
    acc = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for a, gx, gy, gz in fac:
        tz = torch.from_numpy(a * gz).to(device)
        ty = torch.from_numpy(gy).to(device)
        tx = torch.from_numpy(gx).to(device)
        t = (tz[:, None, None] * ty[None, :, None]) * tx[None, None, :]
        acc = acc + t
    return acc.to(torch.float32)


def uniform_volume(n: int, rho0: float) -> np.ndarray:
    return np.full((n, n, n), rho0, dtype=np.float32)


# ----------------------------------------------------------------- fields ---

ABC_A = 1.0
ABC_B = math.sqrt(2.0 / 3.0)
ABC_C = math.sqrt(1.0 / 3.0)


def abc_field(n: int, A: float = ABC_A, B: float = ABC_B, C: float = ABC_C, device=None):
    """Arnold-Beltrami-Childress velocity sampled at voxel centres.

    With x' = 2 pi x / n per axis (x at i + 0.5):
      v = (A sin z' + C cos y',  B sin x' + A cos z',  C sin y' + B cos x'),
    evaluated in float64 from 1-D tables, rounded to float32, stored
    field[z, y, x, c]. Velocities are in voxels per unit time.
    """
    x = (np.arange(n, dtype=np.float64) + 0.5) * (2.0 * math.pi / n)
    s, c = np.sin(x), np.cos(x)
    if device is None:
        f = np.empty((n, n, n, 3), dtype=np.float32)
        f[..., 0] = (A * s[:, None, None] + C * c[None, :, None]) + np.zeros((1, 1, n))
        f[..., 1] = (B * s[None, None, :] + A * c[:, None, None]) + np.zeros((1, n, 1))
        f[..., 2] = (C * s[None, :, None] + B * c[None, None, :]) + np.zeros((n, 1, 1))
        return f
    import torch
    ts, tc = torch.from_numpy(s).to(device), torch.from_numpy(c).to(device)
    f = torch.empty((n, n, n, 3), dtype=torch.float32, device=device)
    z64 = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    f[..., 0] = ((A * ts[:, None, None] + C * tc[None, :, None]) + z64).to(torch.float32)
    f[..., 1] = ((B * ts[None, None, :] + A * tc[:, None, None]) + z64).to(torch.float32)
    f[..., 2] = ((C * ts[None, :, None] + B * tc[None, None, :]) + z64).to(torch.float32)
    return f


def constant_field(n: int, v) -> np.ndarray:
    f = np.empty((n, n, n, 3), dtype=np.float32)
    f[...] = np.asarray(v, dtype=np.float32)
    return f


def linear_field(n: int, grad: np.ndarray, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """v_c(x) = offset_c + sum_a grad[c, a] * x_a at voxel centres (float64 -> float32)."""
    x = np.arange(n, dtype=np.float64) + 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.empty((n, n, n, 3), dtype=np.float32)
    for c in range(3):
        f[..., c] = offset[c] + grad[c][0] * X + grad[c][1] * Y + grad[c][2] * Z
    return f


def streamline_seeds(n_seeds: int, n: int, seed: int = SEED_CFG1_SEEDS) -> np.ndarray:
    """Uniform seeds in [0, n)^3: float32(U[0,1)^3 * n), clamped below n."""
    rng = np.random.default_rng(seed)
    p = (rng.random((n_seeds, 3)) * n).astype(np.float32)
    below = np.nextafter(np.float32(n), np.float32(0))
    np.minimum(p, below, out=p)
    return p


# ------------------------------------------------------ N-body particles ---

# One particle record as the N-body contexts carry it (40 bytes): position,
# velocity, acceleration (the item's force slot), mass.
NB_PARTICLE_DTYPE = np.dtype([("pos", "<f4", 3), ("vel", "<f4", 3), ("acc", "<f4", 3), ("mass", "<f4")])
assert NB_PARTICLE_DTYPE.itemsize == 40


def nbody_particles(n: int, seed: int = SEED_NBODY, n_clumps: int = 8, sigma: float = 0.06,
                    vel_sigma: float = 0.02) -> np.ndarray:
    """Clustered particles in the unit box: n_clumps Gaussian clumps (centres
    U[0,1)^3, spread sigma per axis), wrapped periodically into [0, 1),
    Gaussian velocities (vel_sigma per axis), zero acceleration, equal masses
    1/n. Draw order: centres, clump of each particle, offsets, velocities."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_clumps, 3))
    which = rng.integers(0, n_clumps, n)
    pos = centres[which] + rng.normal(0.0, sigma, (n, 3))
    pos = pos - np.floor(pos)
    vel = rng.normal(0.0, vel_sigma, (n, 3))
    out = np.zeros(n, dtype=NB_PARTICLE_DTYPE)
    p32 = pos.astype(np.float32)
    p32[p32 >= np.float32(1.0)] = np.float32(0.0)
    out["pos"] = p32
    out["vel"] = vel.astype(np.float32)
    out["mass"] = np.float32(1.0 / n)
    return out


# ------------------------------------------------------------ split draws ---

def zipf_cdf(n_domains: int, s: float = 1.1) -> np.ndarray:
    k = np.arange(1, n_domains + 1, dtype=np.float64)
    w = k ** (-s)
    cdf = np.cumsum(w)
    return cdf / cdf[-1]


def split_dest(n: int, n_domains: int, dist: str = "uniform", seed=None) -> np.ndarray:
    """Destination per slot: uniform over [0, D), or truncated Zipf(s=1.1)
    with P(dest = k-1) proportional to k^-1.1, k = 1..D."""
    if dist == "uniform":
        rng = np.random.default_rng(SEED_SPLIT_UNIFORM if seed is None else seed)
        return rng.integers(0, n_domains, n, dtype=np.int32)
    if dist == "zipf":
        rng = np.random.default_rng(SEED_SPLIT_ZIPF if seed is None else seed)
        u = rng.random(n)
        d = np.searchsorted(zipf_cdf(n_domains), u, side="right")
        return np.minimum(d, n_domains - 1).astype(np.int32)
    raise ValueError(dist)


def split_items(n: int, item_words: int = 8, seed: int = SEED_SPLIT_PAYLOAD) -> np.ndarray:
    """Work items as uint32 words: word 0 = int32 id = slot index, the other
    words float32 U[0,1) bit patterns. Shape (n, item_words)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, item_words), dtype=np.uint32)
    out[:, 0] = np.arange(n, dtype=np.uint32)
    if item_words > 1:
        out[:, 1:] = rng.random((n, item_words - 1), dtype=np.float32).view(np.uint32)
    return out


# ------------------------------------------------------------------ views ---

def view_record(org0, du, dv, direction, width, height, n_samples) -> np.ndarray:
    v = np.zeros((), dtype=VIEW_DTYPE)
    v["org0"] = np.asarray(org0, dtype=np.float64).astype(np.float32)
    v["du"] = np.asarray(du, dtype=np.float64).astype(np.float32)
    v["dv"] = np.asarray(dv, dtype=np.float64).astype(np.float32)
    v["dir"] = np.asarray(direction, dtype=np.float64).astype(np.float32)
    v["width"], v["height"], v["n_samples"] = width, height, n_samples
    return v


def plusz_view(n: int, width: int, height: int, dt: float = 0.5) -> np.ndarray:
    """Orthographic rays along +z covering the x-y face; pixel spacing n/width."""
    sx, sy = n / width, n / height
    ns = int(math.ceil(n / dt))
    return np.array([view_record((0.5 * sx, 0.5 * sy, 0.0), (sx, 0, 0), (0, sy, 0),
                                 (0, 0, 1), width, height, ns)])


def random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_views(n_views: int, n: int, width: int, height: int, seed: int = SEED_ADJ_VIEWS,
                 dt: float = 0.5) -> np.ndarray:
    """Orthographic views at seeded random rotations about the volume centre.

    Image extent W = n*sqrt(3) (the cube's diagonal) in both directions; rays
    start W/2 before the centre plane and carry ceil(W/dt) samples.
    """
    rng = np.random.default_rng(seed)
    W = n * math.sqrt(3.0)
    ns = int(math.ceil(W / dt))
    centre = np.full(3, n / 2.0)
    out = np.zeros(n_views, dtype=VIEW_DTYPE)
    for i in range(n_views):
        R = random_rotation(rng)
        su, sv = W / width, W / height
        org0 = centre + R @ np.array([(0.5 - width / 2.0) * su, (0.5 - height / 2.0) * sv, -W / 2.0])
        out[i] = view_record(org0, R @ np.array([su, 0, 0]), R @ np.array([0, sv, 0]),
                             R @ np.array([0, 0, 1.0]), width, height, ns)
    return out


# ----------------------------------------------------------------- scenes ---

@dataclass(frozen=True)
class SceneSpec:
    n: int
    grid: tuple
    rays_side: int
    volume_seed: int


def draw_scenes(n_scenes: int = 256, seed: int = SEED_BATCH_SCENES,
                n_range=(32, 256), rays_side_range=(32, 1024)):
    """Uneven scenes: edge n = 4*round(2^u/4), u ~ U[log2 lo, log2 hi]; domain
    grid g_a drawn from {1, 2, 4} per axis; rays s^2 with s = round(2^U) over
    the given side range; scene s's volume uses seed 1000 + s."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log2(n_range[0]), math.log2(n_range[1])
    rlo, rhi = math.log2(rays_side_range[0]), math.log2(rays_side_range[1])
    out = []
    for s in range(n_scenes):
        u = rng.uniform(lo, hi)
        n = int(4 * round(2.0 ** u / 4.0))
        g = tuple(int(x) for x in rng.choice([1, 2, 4], size=3))
        side = int(round(2.0 ** rng.uniform(rlo, rhi)))
        out.append(SceneSpec(n, g, side, 1000 + s))
    return out


def fd_voxels(n: int, count: int = 32, seed: int = SEED_ADJ_FD) -> np.ndarray:
    """Seeded voxel indices (linear, x fastest) for finite-difference checks,
    drawn from the interior (1 voxel away from the faces)."""
    rng = np.random.default_rng(seed)
    ijk = rng.integers(1, n - 1, size=(count, 3))
    return (ijk[:, 0] + n * (ijk[:, 1] + n * ijk[:, 2])).astype(np.int64)
