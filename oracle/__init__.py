"""CPU oracle for the work-forwarding hot path -- TEST INFRASTRUCTURE ONLY.

Thin numpy/ctypes front end of ``rafi_oracle.c``. Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
product library never does, and the two share no code. See the C file for
the definitions each function follows and the passages of the paper they
restate.

Parity status of every function is recorded in the C file's header notes and
in the tests under ``tests/test_oracle_*.py`` (each function is pinned by at
least one check that does not reuse the oracle's own arithmetic).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rafi_oracle.c")
_LIB = os.path.join(_HERE, "librafi_oracle.so")

DONE = -1
SL_LIVE, SL_STAGNANT, SL_EXITED, SL_MAXSTEPS = 0, 1, 2, 3


# RAFI_ORACLE_SANITIZE=1 builds a separate copy with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; load it with libasan preloaded).
_SANITIZE = os.environ.get("RAFI_ORACLE_SANITIZE") == "1"
if _SANITIZE:
    _LIB = os.path.join(_HERE, "librafi_oracle_asan.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]
        if _SANITIZE:
            cmd += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
        cmd += ["-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


def default_threads() -> int:
    """Threads for a timed oracle run: the CPUs this process may use, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def set_threads(n: int) -> None:
    """Run the per-item loops on n OpenMP threads (1: sequential, the
    default). Results are the same bits for every n."""
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


class EAParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("g", C.c_int32 * 3), ("dt", C.c_float), ("c", C.c_float)]


class SLParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("g", C.c_int32 * 3), ("h", C.c_float), ("max_steps", C.c_int32)]


class DTParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("g", C.c_int32 * 3), ("kappa", C.c_float), ("smax", C.c_float),
                ("albedo", C.c_float), ("light", C.c_float * 3), ("radiance", C.c_float),
                ("max_bounce", C.c_int32), ("seed", C.c_uint32)]


class NBParams(C.Structure):
    _fields_ = [("n_domains", C.c_int32), ("cell_level", C.c_int32), ("dt", C.c_float), ("theta", C.c_float),
                ("eps", C.c_float)]


# record layouts of the three N-body item types (see the C file, O8)
NB_PARTICLE = np.dtype([("pos", "<f4", 3), ("vel", "<f4", 3), ("acc", "<f4", 3), ("mass", "<f4")])
NB_VP = np.dtype([("pos", "<f4", 3), ("mass", "<f4"), ("smax", "<f4"), ("src", "<i4")])

_p = C.c_void_p


def _declare(L):
    L.oracle_morton30.argtypes = [C.c_float, C.c_float, C.c_float]
    L.oracle_morton30.restype = C.c_uint32
    L.oracle_nb_splitters.argtypes = [_p, C.c_int64, C.c_int32, _p]
    L.oracle_nb_splitters.restype = C.c_int
    L.oracle_nb_seed.argtypes = [C.POINTER(NBParams), _p, _p, C.c_int64, _p, _p]
    L.oracle_nb_seed.restype = C.c_int
    L.oracle_nb_step.argtypes = [C.POINTER(NBParams), _p, _p, C.c_int64, _p, _p, C.c_uint64, _p, C.c_uint64, _p,
                                 C.c_uint64, _p, _p]
    L.oracle_nb_step.restype = C.c_int
    L.oracle_philox4x32_10.argtypes = [_p, _p, _p]
    L.oracle_philox4x32_10.restype = None
    L.oracle_dt_logf.argtypes = [C.c_float]
    L.oracle_dt_logf.restype = C.c_float
    L.oracle_dt_render.argtypes = [_p, C.POINTER(DTParams), _p, C.c_int32, _p, _p, C.c_int32, _p, _p,
                                   C.c_uint64, _p]
    L.oracle_dt_render.restype = C.c_int
    L.oracle_multisplit.argtypes = [C.c_uint64, C.c_uint32, _p, _p, C.c_int32, _p, _p, _p, _p, _p]
    L.oracle_multisplit.restype = C.c_int
    L.oracle_set_threads.argtypes = [C.c_int32]
    L.oracle_set_threads.restype = None
    L.oracle_get_threads.argtypes = []
    L.oracle_get_threads.restype = C.c_int32
    L.oracle_trilinear.argtypes = [_p, C.c_int32, C.c_float, C.c_float, C.c_float]
    L.oracle_trilinear.restype = C.c_double
    L.oracle_tri_vec3.argtypes = [_p, C.c_int32, C.c_float, C.c_float, C.c_float, _p]
    L.oracle_tri_vec3.restype = None
    L.oracle_dt_density.argtypes = [_p, C.c_int32, C.c_float, C.c_float, C.c_float]
    L.oracle_dt_density.restype = C.c_float
    L.oracle_ea_render.argtypes = [_p, C.POINTER(EAParams), _p, C.c_int32, _p, _p, _p, C.c_int32,
                                   _p, _p, C.c_uint64, _p, _p, C.c_int32]
    L.oracle_ea_render.restype = C.c_int
    L.oracle_ea_brute.argtypes = [_p, C.POINTER(EAParams), _p, C.c_int32, _p, C.c_int64, _p, _p,
                                  _p, C.c_int32]
    L.oracle_ea_brute.restype = C.c_int
    L.oracle_ea_ray_samples.argtypes = [_p, C.POINTER(EAParams), _p, C.c_int32, C.c_int64, _p, C.c_int32]
    L.oracle_ea_ray_samples.restype = C.c_int32
    L.oracle_ea_loss_grad.argtypes = [_p, C.POINTER(EAParams), _p, C.c_int32, _p, _p, C.c_int64,
                                      _p, _p, _p]
    L.oracle_ea_loss_grad.restype = C.c_int
    L.oracle_streamlines.argtypes = [_p, C.POINTER(SLParams), _p, C.c_int64, C.c_int32, _p, _p, _p,
                                     C.c_int32, _p, _p, C.c_uint64, _p, _p, C.c_int32]
    L.oracle_streamlines.restype = C.c_int
    L.oracle_streamlines_brute.argtypes = [_p, C.POINTER(SLParams), _p, C.c_int64, _p, _p, _p, _p,
                                           C.c_int32]
    L.oracle_streamlines_brute.restype = C.c_int


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------ multisplit ---

def multisplit(items: np.ndarray, dest: np.ndarray, n_domains: int):
    """Stable split of ``items`` (shape (n, ...), any dtype, one row per slot)
    by ``dest``. Returns (out, counts, offsets, n_done, n_bad); ``out`` holds
    offsets[-1] rows."""
    items = np.ascontiguousarray(items)
    dest = np.ascontiguousarray(dest, dtype=np.int32)
    n = dest.shape[0]
    assert items.shape[0] == n
    row_bytes = items.itemsize * (int(np.prod(items.shape[1:])) if items.ndim > 1 else 1)
    out = np.empty_like(items)
    counts = np.zeros(n_domains, dtype=np.uint64)
    offsets = np.zeros(n_domains + 1, dtype=np.uint64)
    nd, nb = C.c_uint64(0), C.c_uint64(0)
    rc = lib().oracle_multisplit(n, row_bytes, _ptr(items), _ptr(dest), n_domains, _ptr(out),
                                 _ptr(counts), _ptr(offsets), C.byref(nd), C.byref(nb))
    if rc != 0:
        raise RuntimeError(f"oracle_multisplit failed: {rc}")
    return out[: int(offsets[-1])], counts, offsets, nd.value, nb.value


# ------------------------------------------------------------------- EA ---

def trilinear(volume: np.ndarray, q) -> float:
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    return lib().oracle_trilinear(_ptr(vol), vol.shape[0], float(q[0]), float(q[1]), float(q[2]))


def tri_vec3(field: np.ndarray, q) -> np.ndarray:
    """The RK4 sampler (O4): float32 trilinear of an [n, n, n, 3] field
    (x fastest, 3 components per voxel) at q, clamp-to-edge."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    out = np.zeros(3, dtype=np.float32)
    lib().oracle_tri_vec3(_ptr(f), f.shape[0], *(float(np.float32(c)) for c in q), _ptr(out))
    return out


def dt_density(volume: np.ndarray, q) -> np.ndarray:
    """The delta-tracking density sampler (O7): float32 trilinear of an
    [n, n, n] float32 volume (x fastest) at q, clamp-to-edge."""
    v = np.ascontiguousarray(volume, dtype=np.float32)
    return np.float32(lib().oracle_dt_density(_ptr(v), v.shape[0], *(float(np.float32(c)) for c in q)))


def _ea_params(n, grid, dt, c):
    return EAParams(int(n), (C.c_int32 * 3)(*[int(g) for g in grid]), float(dt), float(c))


def n_rays_of(views) -> int:
    return int(sum(int(v["width"]) * int(v["height"]) for v in views))


def ea_render(volume, grid, views, dt=0.5, c=0.025, max_rounds=256, queue_cap=0,
              visit_stride=0, want_rounds=True):
    """Partitioned round loop (O2 + O3). Returns a dict with image, tau, klast,
    rounds, round_counts [rounds, D], queue (ray ids per forward step,
    concatenated) and visits [n_rays, visit_stride]."""
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    n = vol.shape[0]
    views = np.ascontiguousarray(views)
    nr = n_rays_of(views)
    D = int(np.prod(grid))
    P = _ea_params(n, grid, dt, c)
    image = np.zeros(nr, dtype=np.float64)
    tau = np.zeros(nr, dtype=np.float64)
    klast = np.zeros(nr, dtype=np.int32)
    rc = np.zeros((max_rounds, D), dtype=np.uint64) if want_rounds else None
    q = np.zeros(max(queue_cap, 1), dtype=np.int64) if queue_cap else None
    qlen = C.c_uint64(0)
    vis = np.zeros((nr, visit_stride), dtype=np.int32) if visit_stride else None
    rounds = lib().oracle_ea_render(_ptr(vol), C.byref(P), _ptr(views), len(views), _ptr(image),
                                    _ptr(tau), _ptr(klast), max_rounds, _ptr(rc), _ptr(q),
                                    queue_cap, C.byref(qlen), _ptr(vis), visit_stride)
    if rounds < 0:
        raise RuntimeError(f"oracle_ea_render failed: {rounds}")
    out = dict(image=image, tau=tau, klast=klast, rounds=rounds, visits=vis)
    if rc is not None:
        out["round_counts"] = rc[:rounds]
    if q is not None:
        out["queue"] = q[: min(qlen.value, queue_cap)]
        out["queue_len"] = qlen.value
    return out


def ea_brute(volume, grid, views, dt=0.5, c=0.025, ray_ids=None, visit_stride=0):
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    views = np.ascontiguousarray(views)
    P = _ea_params(vol.shape[0], grid, dt, c)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, dtype=np.int64)
    m = n_rays_of(views) if ids is None else len(ids)
    image = np.zeros(m, dtype=np.float64)
    tau = np.zeros(m, dtype=np.float64)
    vis = np.zeros((m, visit_stride), dtype=np.int32) if visit_stride else None
    lib().oracle_ea_brute(_ptr(vol), C.byref(P), _ptr(views), len(views), _ptr(ids),
                          0 if ids is None else len(ids), _ptr(image), _ptr(tau), _ptr(vis),
                          visit_stride)
    return dict(image=image, tau=tau, visits=vis)


def ea_ray_samples(volume, grid, views, ray, dt=0.5, c=0.025):
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    views = np.ascontiguousarray(views)
    P = _ea_params(vol.shape[0], grid, dt, c)
    cap = int(max(v["n_samples"] for v in views))
    buf = np.zeros(cap, dtype=np.float64)
    m = lib().oracle_ea_ray_samples(_ptr(vol), C.byref(P), _ptr(views), len(views), int(ray),
                                    _ptr(buf), cap)
    return buf[:m]


def ea_loss_grad(volume, grid, views, target, dt=0.5, c=0.025, ray_ids=None, want_grad=True):
    """Loss sum (I - I*)^2 and its float64 gradient w.r.t. the voxels (O6)."""
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    views = np.ascontiguousarray(views)
    tgt = np.ascontiguousarray(target, dtype=np.float64)
    P = _ea_params(vol.shape[0], grid, dt, c)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, dtype=np.int64)
    m = n_rays_of(views) if ids is None else len(ids)
    image = np.zeros(m, dtype=np.float64)
    grad = np.zeros(vol.shape, dtype=np.float64) if want_grad else None
    loss = C.c_double(0.0)
    rc = lib().oracle_ea_loss_grad(_ptr(vol), C.byref(P), _ptr(views), len(views), _ptr(tgt),
                                   _ptr(ids), 0 if ids is None else len(ids), _ptr(image),
                                   _ptr(grad), C.byref(loss))
    if rc != 0:
        raise RuntimeError(f"oracle_ea_loss_grad failed: {rc}")
    return loss.value, grad, image


# ----------------------------------------------------------- streamlines ---

def _sl_params(n, grid, h, max_steps):
    return SLParams(int(n), (C.c_int32 * 3)(*[int(g) for g in grid]), float(h), int(max_steps))


def streamlines(field, grid, seeds, h=0.25, max_steps=2000, one_step=False, max_rounds=100000,
                queue_cap=0, visit_stride=0, want_rounds=True, steps_per_visit=0):
    """Partitioned round loop (O2 + O4). steps_per_visit caps the RK4 steps a
    particle takes per domain visit (0 = until it leaves; one_step means 1)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    n = f.shape[0]
    s = np.ascontiguousarray(seeds, dtype=np.float32)
    N = s.shape[0]
    D = int(np.prod(grid))
    P = _sl_params(n, grid, h, max_steps)
    ep = np.zeros((N, 3), dtype=np.float32)
    st = np.zeros(N, dtype=np.int32)
    why = np.zeros(N, dtype=np.int32)
    rc = np.zeros((max_rounds, D), dtype=np.uint64) if want_rounds else None
    q = np.zeros(max(queue_cap, 1), dtype=np.int32) if queue_cap else None
    qlen = C.c_uint64(0)
    vis = np.zeros((N, visit_stride), dtype=np.int32) if visit_stride else None
    cap = 1 if one_step else int(steps_per_visit)
    rounds = lib().oracle_streamlines(_ptr(f), C.byref(P), _ptr(s), N, cap, _ptr(ep),
                                      _ptr(st), _ptr(why), max_rounds, _ptr(rc), _ptr(q), queue_cap,
                                      C.byref(qlen), _ptr(vis), visit_stride)
    if rounds < 0:
        raise RuntimeError(f"oracle_streamlines failed: {rounds}")
    out = dict(endpoint=ep, steps=st, reason=why, rounds=rounds, visits=vis)
    if rc is not None:
        out["round_counts"] = rc[:rounds]
    if q is not None:
        out["queue"] = q[: min(qlen.value, queue_cap)]
        out["queue_len"] = qlen.value
    return out


def streamlines_brute(field, grid, seeds, h=0.25, max_steps=2000, visit_stride=0):
    f = np.ascontiguousarray(field, dtype=np.float32)
    s = np.ascontiguousarray(seeds, dtype=np.float32)
    N = s.shape[0]
    P = _sl_params(f.shape[0], grid, h, max_steps)
    ep = np.zeros((N, 3), dtype=np.float32)
    st = np.zeros(N, dtype=np.int32)
    why = np.zeros(N, dtype=np.int32)
    vis = np.zeros((N, visit_stride), dtype=np.int32) if visit_stride else None
    lib().oracle_streamlines_brute(_ptr(f), C.byref(P), _ptr(s), N, _ptr(ep), _ptr(st), _ptr(why),
                                   _ptr(vis), visit_stride)
    return dict(endpoint=ep, steps=st, reason=why, visits=vis)


# ------------------------------------------------------------ delta tracking

def philox4x32_10(ctr, key):
    """Philox4x32-10 block: counter (4 x uint32), key (2 x uint32) -> 4 x uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def dt_logf(x):
    """The float32 natural logarithm used for free-flight distances, x in (0, 1]."""
    L = lib()
    return np.array([L.oracle_dt_logf(float(v)) for v in np.asarray(x, dtype=np.float32).ravel()],
                    dtype=np.float32)


def dt_params(n, grid, kappa, smax, albedo, light, radiance, max_bounce, seed):
    return DTParams(int(n), (C.c_int32 * 3)(*[int(g) for g in grid]), float(kappa), float(smax), float(albedo),
                    (C.c_float * 3)(*[float(v) for v in light]), float(radiance), int(max_bounce),
                    int(seed) & 0xFFFFFFFF)


def dt_render(volume, grid, views, kappa, smax, albedo, light, radiance, max_bounce, seed,
              max_rounds=4096, queue_cap=0):
    """Delta-tracking round loop (O7). Returns dict(contrib [n_paths, max_bounce]
    float64, image (sum over scattering events, float64), rounds,
    round_counts [rounds, D], queue [len, 11] uint32 (p, d bits, path, stream,
    count, bounce, kind per queued item), weights [len] float64)."""
    vol = np.ascontiguousarray(volume, dtype=np.float32)
    n = vol.shape[0]
    views = np.ascontiguousarray(views)
    n_paths = n_rays_of(views)
    D = int(np.prod(grid))
    P = dt_params(n, grid, kappa, smax, albedo, light, radiance, max_bounce, seed)
    contrib = np.zeros((n_paths, max_bounce), dtype=np.float64)
    rc = np.zeros((max_rounds, D), dtype=np.uint64)
    q = np.zeros((max(queue_cap, 1), 11), dtype=np.uint32)
    wl = np.zeros(max(queue_cap, 1), dtype=np.float64)
    qlen = C.c_uint64(0)
    rounds = lib().oracle_dt_render(_ptr(vol), C.byref(P), _ptr(views), len(views), _ptr(contrib),
                                    _ptr(wl) if queue_cap else None, max_rounds, _ptr(rc),
                                    _ptr(q) if queue_cap else None, queue_cap, C.byref(qlen))
    if rounds < 0:
        raise RuntimeError(f"oracle_dt_render failed: {rounds}")
    out = dict(contrib=contrib, image=contrib.sum(axis=1), rounds=rounds, round_counts=rc[:rounds])
    if queue_cap:
        m = min(qlen.value, queue_cap)
        out["queue"] = q[:m]
        out["weights"] = wl[:m]
        out["queue_len"] = qlen.value
    return out


# ---------------------------------------------------------------- O8 ---

def morton30(x, y, z) -> int:
    return int(lib().oracle_morton30(float(x), float(y), float(z)))


def nb_splitters(particles, n_domains: int) -> np.ndarray:
    """Morton splitters K[0..D] of a particle set (O8)."""
    pos = np.ascontiguousarray(np.asarray(particles)["pos"], dtype=np.float32)
    K = np.zeros(n_domains + 1, dtype=np.uint32)
    rc = lib().oracle_nb_splitters(_ptr(pos), pos.shape[0], n_domains, _ptr(K))
    if rc != 0:
        raise RuntimeError(f"oracle_nb_splitters failed: {rc}")
    return K


def _nb_params(n_domains, cell_level, dt, theta, eps):
    return NBParams(int(n_domains), int(cell_level), float(dt), float(theta), float(eps))


def nb_seed(particles, K, cell_level=4, theta=0.5, eps=1e-3):
    """Round 0 of the particle context: the input in any order to the owning
    domains. Returns (queue, counts)."""
    src = np.ascontiguousarray(particles, dtype=NB_PARTICLE)
    D = len(K) - 1
    q = np.zeros_like(src)
    counts = np.zeros(D, dtype=np.uint64)
    P = _nb_params(D, cell_level, 0.0, theta, eps)
    K = np.ascontiguousarray(K, dtype=np.uint32)
    rc = lib().oracle_nb_seed(C.byref(P), _ptr(K), _ptr(src), src.shape[0], _ptr(q), _ptr(counts))
    if rc != 0:
        raise RuntimeError(f"oracle_nb_seed failed: {rc}")
    return q, counts


def nb_step(queue, K, dt, cell_level=4, theta=0.5, eps=1e-3, log_cap=1 << 22):
    """One step of O8 on a particle queue. Returns the new queue, the four
    rounds' per-domain counts (particle, virtual 1, request, virtual 2), the
    three exchange queues and, per particle of the new queue, the sum of its
    force terms' magnitudes per component (acc_mag, float64)."""
    q = np.array(queue, dtype=NB_PARTICLE, copy=True)
    D = len(K) - 1
    P = _nb_params(D, cell_level, dt, theta, eps)
    K = np.ascontiguousarray(K, dtype=np.uint32)
    rc_counts = np.zeros((4, D), dtype=np.uint64)
    cap1 = D * max(D - 1, 1)
    vp1 = np.zeros(cap1, dtype=NB_VP)
    rr = np.zeros(cap1, dtype=np.int32)
    vp2 = np.zeros(log_cap, dtype=NB_VP)
    lens = np.zeros(3, dtype=np.uint64)
    acc_mag = np.zeros((q.shape[0], 3), dtype=np.float64)
    rc = lib().oracle_nb_step(C.byref(P), _ptr(K), _ptr(q), q.shape[0], _ptr(rc_counts), _ptr(vp1), cap1,
                              _ptr(rr), cap1, _ptr(vp2), log_cap, _ptr(lens), _ptr(acc_mag))
    if rc != 0:
        raise RuntimeError(f"oracle_nb_step failed: {rc}")
    n1, nr, n2 = (int(x) for x in lens)
    if n2 > log_cap:
        raise RuntimeError("second virtual-particle queue longer than log_cap")
    return dict(queue=q, round_counts=rc_counts, vp1=vp1[:n1], rr=rr[:nr], vp2=vp2[:n2], acc_mag=acc_mag)
