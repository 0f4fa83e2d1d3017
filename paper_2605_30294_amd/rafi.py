"""Python binding of librafi.so (ctypes): argument marshalling only.

Every step of the forwarding path runs in the library's HIP kernels; this
module converts torch tensors and numpy records into the C structs and
pointers the C ABI (include/rafi.h) takes, calls it, and raises on error
codes. PyTorch supplies device memory and the current stream.

The library must have been built (``python -m paper_2605_30294_amd.build``);
there is no fallback: importing the binding without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librafi.so")

RAFI_OK = 0
RAFI_DONE = -1
RAFI_POISON = -2
ERR_ARG, ERR_OOM, ERR_HIP, ERR_OVERFLOW, ERR_BAD_DEST, ERR_MAX_ROUNDS, ERR_STATE, ERR_TOO_LARGE = range(-1, -9, -1)
SLOTS_ORDERED, SLOTS_APPEND = 0, 1
EA_ITEM_BYTES = 16
DT_ITEM_BYTES = 48
SL_ITEM_BYTES = 16


class RafiError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class DeviceView(C.Structure):
    _fields_ = [("in_items", C.c_void_p), ("in_offsets", C.c_void_p), ("in_tile_offsets", C.c_void_p),
                ("out_items", C.c_void_p), ("out_dest", C.c_void_p), ("dropped", C.c_void_p),
                ("n_in", C.c_uint64), ("n_slots", C.c_uint64), ("capacity", C.c_uint64),
                ("item_bytes", C.c_uint32), ("n_domains", C.c_int32), ("tile_items", C.c_uint32),
                ("n_tiles", C.c_uint32), ("append", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_uint64), ("forwarded", C.c_uint64), ("done", C.c_uint64),
                ("bad_dest", C.c_uint64), ("dropped", C.c_uint64), ("last_total", C.c_uint64)]


class Profile(C.Structure):
    _fields_ = [("split_ms", C.c_double), ("scatter_ms", C.c_double), ("domain_ms", C.c_double),
                ("split_calls", C.c_uint64), ("scatter_calls", C.c_uint64), ("domain_calls", C.c_uint64),
                ("split_slots", C.c_uint64), ("split_items", C.c_uint64)]


class EAJob(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("views", C.c_void_p), ("image", C.c_void_p), ("tau", C.c_void_p),
                ("klast", C.c_void_p), ("kfirst", C.c_void_p), ("visit_log", C.c_void_p),
                ("visit_count", C.c_void_p), ("n", C.c_int32), ("grid", C.c_int32 * 3),
                ("n_views", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("dt", C.c_float),
                ("c", C.c_float), ("visit_stride", C.c_int32), ("emit_mode", C.c_int32),
                ("bwd_tile_items", C.c_uint32)]


class SLJob(C.Structure):
    _fields_ = [("field4", C.c_void_p), ("endpoint", C.c_void_p), ("steps", C.c_void_p), ("reason", C.c_void_p),
                ("counters", C.c_void_p), ("n", C.c_int32), ("grid", C.c_int32 * 3), ("h", C.c_float),
                ("max_steps", C.c_int32), ("steps_per_visit", C.c_int32), ("tail_items", C.c_uint32),
                ("refill_lanes", C.c_int32), ("field_stride", C.c_int32), ("quad_items", C.c_uint32)]


class NBJob(C.Structure):
    _fields_ = [("n_domains", C.c_int32), ("cell_level", C.c_int32), ("dt", C.c_float), ("theta", C.c_float),
                ("eps", C.c_float), ("splitters", C.c_void_p), ("workspace", C.c_void_p), ("capacity", C.c_uint64),
                ("log_vp1", C.c_void_p), ("log_vp1_cap", C.c_uint64)]


class DTJob(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("views", C.c_void_p), ("contrib", C.c_void_p), ("image", C.c_void_p),
                ("n", C.c_int32), ("grid", C.c_int32 * 3), ("n_views", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("kappa", C.c_float), ("smax", C.c_float), ("albedo", C.c_float),
                ("light", C.c_float * 3), ("radiance", C.c_float), ("max_bounce", C.c_int32),
                ("seed", C.c_uint32), ("counters", C.c_void_p)]


class ViewRec(C.Structure):
    _fields_ = [("org0", C.c_float * 3), ("du", C.c_float * 3), ("dv", C.c_float * 3), ("dir", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32), ("n_samples", C.c_int32), ("pad", C.c_int32)]


class SceneRec(C.Structure):
    _fields_ = [("volume_offset", C.c_uint64), ("view", ViewRec), ("n", C.c_int32), ("grid", C.c_int32 * 3),
                ("ray_base", C.c_uint32), ("dom_base", C.c_int32)]


class BatchTuning(C.Structure):
    _fields_ = [("split_tile", C.c_uint32), ("march_block", C.c_uint32), ("march_grid", C.c_uint32),
                ("use_graph", C.c_int32), ("rounds_per_sync", C.c_int32)]


assert C.sizeof(ViewRec) == 64 and C.sizeof(SceneRec) == 96

_P = C.c_void_p
_U64P = C.POINTER(C.c_uint64)
_SIGS = {
    "rafi_create": ([C.c_int32, C.c_uint32, C.c_uint64, C.POINTER(C.c_void_p)], C.c_int),
    "rafi_destroy": ([_P], None),
    "rafi_resize": ([_P, C.c_uint64], C.c_int),
    "rafi_set_stream": ([_P, _P], C.c_int),
    "rafi_set_debug": ([_P, C.c_int32], C.c_int),
    "rafi_set_tile_items": ([_P, C.c_uint32], C.c_int),
    "rafi_view": ([_P, C.POINTER(DeviceView)], C.c_int),
    "rafi_begin": ([_P, C.c_uint64], C.c_int),
    "rafi_open": ([_P, C.c_uint64, C.c_int32], C.c_int),
    "rafi_round": ([_P, _P, _U64P], C.c_int),
    "rafi_emit_bulk": ([_P, _P, _P, C.c_uint64], C.c_int),
    "rafi_copy_queue": ([_P, _P, _P], C.c_int),
    "rafi_stats": ([_P, C.POINTER(Stats)], C.c_int),
    "rafi_set_profiling": ([_P, C.c_int32], C.c_int),
    "rafi_get_profile": ([_P, C.POINTER(Profile)], C.c_int),
    "rafi_strerror": ([C.c_int], C.c_char_p),
    "rafi_multisplit_workspace": ([C.c_uint64, C.c_int32, C.c_uint32, _U64P], C.c_int),
    "rafi_split_set_variant": ([C.c_int32], C.c_int),
    "rafi_multisplit": ([_P, _P, C.c_uint64, C.c_uint32, C.c_int32, _P, _P, _P, _P, C.c_uint64, _P], C.c_int),
    "rafi_multisplit_noalloc": ([_P, _P, C.c_uint64, C.c_uint32, C.c_int32, _P, _P, _P, _P], C.c_int),
    "rafi_ea_raygen": ([_P, C.POINTER(EAJob)], C.c_int),
    "rafi_ea_march": ([_P, C.POINTER(EAJob)], C.c_int),
    "rafi_ea_render": ([_P, C.POINTER(EAJob), C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "rafi_ea_backward": ([_P, C.POINTER(EAJob), _P, _P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "rafi_batch_create": ([C.POINTER(SceneRec), C.c_int32, C.c_float, C.c_float, C.POINTER(C.c_void_p)], C.c_int),
    "rafi_batch_destroy": ([_P], None),
    "rafi_batch_set_stream": ([_P, _P], C.c_int),
    "rafi_batch_set_tuning": ([_P, C.POINTER(BatchTuning)], C.c_int),
    "rafi_batch_info": ([_P, _U64P, C.POINTER(C.c_int32)], C.c_int),
    "rafi_batch_render": ([_P, _P, _P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "rafi_sl_pack": ([_P, C.c_int32, _P, _P], C.c_int),
    "rafi_sl_seed": ([_P, C.POINTER(SLJob), _P, C.c_uint64], C.c_int),
    "rafi_sl_advance": ([_P, C.POINTER(SLJob)], C.c_int),
    "rafi_sl_trace": ([_P, C.POINTER(SLJob), _P, C.c_uint64, C.c_int32, C.POINTER(C.c_int32), _U64P], C.c_int),
    "rafi_dt_capacity": ([C.c_uint64, C.c_int32, _U64P], C.c_int),
    "rafi_dt_raygen": ([_P, _P], C.c_int),
    "rafi_dt_trace": ([_P, _P], C.c_int),
    "rafi_dt_render": ([_P, _P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "rafi_nb_workspace": ([C.c_uint64, C.c_int32, C.POINTER(C.c_uint64)], C.c_int),
    "rafi_nb_splitters": ([_P, C.c_uint64, C.c_int32, _P, _P, _P], C.c_int),
    "rafi_nb_seed": ([_P, _P, _P, C.c_uint64], C.c_int),
    "rafi_nb_step": ([_P, _P, _P, _P, _P, _P], C.c_int),
}

_lib = None


def lib():
    """Load librafi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_30294_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().rafi_strerror(code).decode()


def _check(code: int, what: str, ok=(RAFI_OK,)):
    if code not in ok:
        raise RafiError(code, what)
    return code


def _dptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    p = t.data_ptr()
    if p == 0 and t.numel() == 0:
        # torch gives empty tensors no address; a view of a non-empty storage still has one
        p = t.untyped_storage().data_ptr() + t.storage_offset() * t.element_size()
    return C.c_void_p(p)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def views_to_device(views: np.ndarray, device) -> torch.Tensor:
    """Copy VIEW_DTYPE records to the device as raw bytes."""
    v = np.ascontiguousarray(views, dtype=W.VIEW_DTYPE)
    return torch.from_numpy(v.view(np.uint8).copy()).to(device)


# ------------------------------------------------------------- context ---

class Context:
    """One forwarding context (queues of `capacity` items of `item_bytes`)."""

    def __init__(self, n_domains: int, item_bytes: int, capacity: int, stream=None, debug=False):
        h = C.c_void_p()
        _check(lib().rafi_create(n_domains, item_bytes, capacity, C.byref(h)), "rafi_create")
        self._h = h
        self.n_domains, self.item_bytes, self.capacity = n_domains, item_bytes, capacity
        _check(lib().rafi_set_stream(self._h, _stream(stream)), "rafi_set_stream")
        if debug:
            _check(lib().rafi_set_debug(self._h, 1), "rafi_set_debug")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().rafi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        _check(lib().rafi_set_stream(self._h, _stream(stream)), "rafi_set_stream")

    def set_tile_items(self, t: int):
        _check(lib().rafi_set_tile_items(self._h, t), "rafi_set_tile_items")

    def view(self) -> DeviceView:
        v = DeviceView()
        _check(lib().rafi_view(self._h, C.byref(v)), "rafi_view")
        return v

    def begin(self, n_slots: int):
        _check(lib().rafi_begin(self._h, n_slots), "rafi_begin")

    def open(self, n_slots: int, mode: int = SLOTS_ORDERED):
        """Reopen this round's output slots (ordered or append), keeping the input queue."""
        _check(lib().rafi_open(self._h, n_slots, mode), "rafi_open")

    def emit_bulk(self, items: torch.Tensor, dest: torch.Tensor):
        _check(lib().rafi_emit_bulk(self._h, _dptr(items), _dptr(dest), dest.numel()), "rafi_emit_bulk")

    def round(self, counts: bool = True, allow=(RAFI_OK,)):
        """Forward step. Returns (counts array or None, total, return code)."""
        cnt = np.zeros(self.n_domains, dtype=np.uint64) if counts else None
        total = C.c_uint64(0)
        rc = lib().rafi_round(self._h, None if cnt is None else cnt.ctypes.data_as(C.c_void_p), C.byref(total))
        _check(rc, "rafi_round", ok=allow)
        return cnt, total.value, rc

    def copy_queue(self):
        """(items as uint8 tensor [n_in, item_bytes], offsets uint64 numpy [D+1])."""
        n_in = self.view().n_in
        dev = torch.device("cuda", torch.cuda.current_device())
        items = torch.empty((max(n_in, 1), self.item_bytes), dtype=torch.uint8, device=dev)
        offs = torch.empty(self.n_domains + 1, dtype=torch.int64, device=dev)
        _check(lib().rafi_copy_queue(self._h, _dptr(items), _dptr(offs)), "rafi_copy_queue")
        torch.cuda.synchronize()
        return items[:n_in], offs.cpu().numpy().astype(np.uint64)

    def set_profiling(self, on: bool):
        _check(lib().rafi_set_profiling(self._h, int(on)), "rafi_set_profiling")

    def profile(self) -> dict:
        p = Profile()
        _check(lib().rafi_get_profile(self._h, C.byref(p)), "rafi_get_profile")
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    def stats(self) -> dict:
        s = Stats()
        _check(lib().rafi_stats(self._h, C.byref(s)), "rafi_stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}


# ----------------------------------------------------------- multisplit ---

def split_set_variant(v: int):
    _check(lib().rafi_split_set_variant(v), "rafi_split_set_variant")


def multisplit_workspace(n: int, n_domains: int, item_bytes: int) -> int:
    b = C.c_uint64(0)
    _check(lib().rafi_multisplit_workspace(n, n_domains, item_bytes, C.byref(b)), "rafi_multisplit_workspace")
    return b.value


def multisplit(items: torch.Tensor, dest: torch.Tensor, n_domains: int, out=None, workspace=None,
               stream=None):
    """Stateless forward step on device tensors.

    items: [n, item_bytes // 4] 32-bit words (any 4-byte dtype); dest: int32 [n].
    Returns (out, offsets int64 tensor [D+1], summary int64 tensor [4]:
    total, done, bad, 0)."""
    n = dest.numel()
    S = items.element_size() * (items.shape[1] if items.dim() > 1 else 1)
    if out is None:
        out = torch.empty_like(items)
    offsets = torch.empty(n_domains + 1, dtype=torch.int64, device=dest.device)
    summary = torch.empty(4, dtype=torch.int64, device=dest.device)
    ws_bytes = multisplit_workspace(n, n_domains, S)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dest.device)
    _check(lib().rafi_multisplit(_dptr(items), _dptr(dest), n, S, n_domains, _dptr(out), _dptr(offsets),
                                 _dptr(summary), _dptr(workspace), workspace.numel(), _stream(stream)),
           "rafi_multisplit")
    return out, offsets, summary


def multisplit_noalloc(items: torch.Tensor, dest: torch.Tensor, n_domains: int, out: torch.Tensor,
                       offsets: torch.Tensor, summary: torch.Tensor, stream=None):
    """The stateless forward step with the library's fixed device scratch
    buffer as its workspace (rafi_multisplit_noalloc): the caller passes
    every output (out like items, offsets int64 [D+1], summary int64 [4])
    and nothing is allocated. Results as multisplit()."""
    n = dest.numel()
    S = items.element_size() * (items.shape[1] if items.dim() > 1 else 1)
    _check(lib().rafi_multisplit_noalloc(_dptr(items), _dptr(dest), n, S, n_domains, _dptr(out), _dptr(offsets),
                                         _dptr(summary), _stream(stream)), "rafi_multisplit_noalloc")
    return out, offsets, summary


# -------------------------------------------------------------- EA march ---

def ea_job(volume: torch.Tensor, grid, views_dev: torch.Tensor, n_views: int, width: int, height: int,
           image: torch.Tensor, tau=None, klast=None, dt=0.5, c=0.025, kfirst=None, visit_log=None,
           visit_count=None, emit_mode=SLOTS_ORDERED) -> EAJob:
    n = volume.shape[0] if volume.dim() == 3 else -1
    if volume.dim() != 3 or tuple(volume.shape) != (n, n, n) or volume.dtype != torch.float32:
        raise ValueError(f"volume must be a float32 [n, n, n] tensor, got {volume.dtype} {tuple(volume.shape)}")
    stride = 0 if visit_log is None else visit_log.shape[1]
    return EAJob(_dptr(volume), _dptr(views_dev), _dptr(image), _dptr(tau), _dptr(klast), _dptr(kfirst),
                 _dptr(visit_log), _dptr(visit_count), n, (C.c_int32 * 3)(*[int(g) for g in grid]), n_views,
                 width, height, float(dt), float(c), stride, int(emit_mode), 0)


def ea_raygen(ctx: Context, job: EAJob):
    _check(lib().rafi_ea_raygen(ctx.handle, C.byref(job)), "rafi_ea_raygen")


def ea_march(ctx: Context, job: EAJob):
    _check(lib().rafi_ea_march(ctx.handle, C.byref(job)), "rafi_ea_march")


def ea_render_job(ctx: Context, job: EAJob, max_rounds: int = 1024) -> int:
    r = C.c_int32(0)
    _check(lib().rafi_ea_render(ctx.handle, C.byref(job), max_rounds, C.byref(r)), "rafi_ea_render")
    return r.value


def ea_backward_job(ctx: Context, job: EAJob, grad_image: torch.Tensor, grad_volume: torch.Tensor,
                    max_rounds: int = 1024) -> int:
    """Accumulate dL/dV into grad_volume for dL/dI = grad_image (reverse replay)."""
    r = C.c_int32(0)
    _check(lib().rafi_ea_backward(ctx.handle, C.byref(job), _dptr(grad_image), _dptr(grad_volume), max_rounds,
                                  C.byref(r)), "rafi_ea_backward")
    return r.value


def ea_render(volume: torch.Tensor, grid, views: np.ndarray, dt=0.5, c=0.025, ctx: Context | None = None,
              max_rounds: int = 1024, want_tau=False, emit_mode=SLOTS_ORDERED):
    """Render all rays of `views` through `volume` (device float32 [n,n,n]).
    Returns dict(image, tau, klast, rounds)."""
    dev = volume.device
    nv = len(views)
    w, h = int(views[0]["width"]), int(views[0]["height"])
    n_rays = nv * w * h
    if ctx is None:
        ctx = Context(int(np.prod(grid)), EA_ITEM_BYTES, max(n_rays, 1))
    vdev = views_to_device(views, dev)
    image = torch.empty(n_rays, dtype=torch.float32, device=dev)
    tau = torch.empty(n_rays, dtype=torch.float32, device=dev) if want_tau else None
    klast = torch.empty(n_rays, dtype=torch.int32, device=dev) if want_tau else None
    kfirst = torch.empty(n_rays, dtype=torch.int32, device=dev) if want_tau else None
    job = ea_job(volume, grid, vdev, nv, w, h, image, tau, klast, dt, c, kfirst, emit_mode=emit_mode)
    rounds = ea_render_job(ctx, job, max_rounds)
    return dict(image=image, tau=tau, klast=klast, kfirst=kfirst, rounds=rounds, ctx=ctx, job=job,
                views_dev=vdev)


# ------------------------------------------------------------ streamlines ---

def sl_pack(field: torch.Tensor) -> torch.Tensor:
    n = field.shape[0]
    if field.dim() != 4 or tuple(field.shape) != (n, n, n, 3) or field.dtype != torch.float32:
        raise ValueError(f"field must be a float32 [n, n, n, 3] tensor, got {field.dtype} {tuple(field.shape)}")
    f4 = torch.empty((n, n, n, 4), dtype=torch.float32, device=field.device)
    _check(lib().rafi_sl_pack(_dptr(field), n, _dptr(f4), _stream()), "rafi_sl_pack")
    return f4


SL_QUAD_ITEMS = 98304  # launch size at and below which four lanes carry each particle
# RK4 steps per brick visit of the benchmark's 256^3 / 1M-seed job (its measured
# best; results do not depend on it)
SL_STEPS_PER_VISIT = 112


def sl_job(field4: torch.Tensor, grid, endpoint, steps, reason=None, h=0.25, max_steps=2000,
           steps_per_visit=0, counters=None, tail_items=0, refill_lanes=0,
           quad_items=SL_QUAD_ITEMS) -> SLJob:
    """field4: the packed [n, n, n, 4] field of sl_pack, or the [n, n, n, 3] field
    itself (read unpadded). counters: optional int64 device tensor [2]
    (cross-brick forwards, same-brick forwards). Schedule (results do not
    depend on it): steps_per_visit caps the RK4 steps per brick visit (0: none),
    uncapped in launches over at most tail_items particles; refill_lanes > 0
    runs persistent waves; launches over at most quad_items particles (with
    refill_lanes 0) run four lanes per particle (0: never)."""
    stride = int(field4.shape[-1])
    n = field4.shape[0]
    if field4.dim() != 4 or stride not in (3, 4) or tuple(field4.shape[:3]) != (n, n, n) \
            or field4.dtype != torch.float32 or not field4.is_contiguous():
        raise ValueError("field must be a contiguous float32 [n, n, n, 3] or [n, n, n, 4] tensor, got "
                         f"{field4.dtype} {tuple(field4.shape)}")
    return SLJob(_dptr(field4), _dptr(endpoint), _dptr(steps), _dptr(reason), _dptr(counters), field4.shape[0],
                 (C.c_int32 * 3)(*[int(g) for g in grid]), float(h), int(max_steps), int(steps_per_visit),
                 int(tail_items), int(refill_lanes), stride, int(quad_items))


def sl_seed(ctx: Context, job: SLJob, seeds: torch.Tensor):
    _check(lib().rafi_sl_seed(ctx.handle, C.byref(job), _dptr(seeds), seeds.shape[0]), "rafi_sl_seed")


def sl_advance(ctx: Context, job: SLJob):
    _check(lib().rafi_sl_advance(ctx.handle, C.byref(job)), "rafi_sl_advance")


def sl_trace_job(ctx: Context, job: SLJob, seeds: torch.Tensor, max_rounds: int = 100000):
    r = C.c_int32(0)
    fwd = C.c_uint64(0)
    _check(lib().rafi_sl_trace(ctx.handle, C.byref(job), _dptr(seeds), seeds.shape[0], max_rounds, C.byref(r),
                               C.byref(fwd)), "rafi_sl_trace")
    return r.value, fwd.value


def sl_trace(field4: torch.Tensor, grid, seeds: torch.Tensor, h=0.25, max_steps=2000, ctx: Context | None = None,
             max_rounds: int = 100000, steps_per_visit=0, tail_items=0, refill_lanes=0,
             quad_items=SL_QUAD_ITEMS):
    dev = field4.device
    N = seeds.shape[0]
    if ctx is None:
        ctx = Context(int(np.prod(grid)), SL_ITEM_BYTES, max(N, 1))
    # at least one row, so that the output pointers are valid also for no seeds
    endpoint = torch.empty((max(N, 1), 3), dtype=torch.float32, device=dev)[:N]
    steps = torch.empty(max(N, 1), dtype=torch.int32, device=dev)[:N]
    reason = torch.empty(max(N, 1), dtype=torch.int32, device=dev)[:N]
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    job = sl_job(field4, grid, endpoint, steps, reason, h, max_steps, steps_per_visit, counters, tail_items,
                 refill_lanes, quad_items)
    rounds, fwd = sl_trace_job(ctx, job, seeds, max_rounds)
    return dict(endpoint=endpoint, steps=steps, reason=reason, rounds=rounds, forwarded=fwd, ctx=ctx,
                counters=counters)


class EARender(torch.autograd.Function):
    """Emission-absorption render as a differentiable op of the volume.

    forward: the bricked march-and-forward render (tau and the last sample
    index are recorded per ray); backward: the reverse-replay adjoint kernel.
    Both run in the library; this class only moves tensors."""

    @staticmethod
    def forward(fctx, volume, grid, views, dt, c, rafi_ctx, bwd_tile_items=0):
        # the job holds the raw address of the contiguous volume: keep that
        # tensor (a copy when the input is a permuted or sliced view) alive
        # until the backward has read it
        vol = volume.detach().contiguous()
        out = ea_render(vol, grid, views, dt=dt, c=c, ctx=rafi_ctx, want_tau=True)
        out["job"].bwd_tile_items = int(bwd_tile_items)
        fctx.keep = (out["ctx"], out["job"], out["views_dev"], out["tau"], out["klast"], out["kfirst"],
                     out["image"], vol)
        fctx.save_for_backward(volume)   # autograd's check against in-place changes
        return out["image"]

    @staticmethod
    def backward(fctx, grad_image):
        fctx.saved_tensors
        rctx, job, _views, _tau, _klast, _kfirst, _image, vol = fctx.keep
        grad = torch.zeros_like(vol, memory_format=torch.contiguous_format)
        ea_backward_job(rctx, job, grad_image.contiguous().to(torch.float32), grad)
        return grad, None, None, None, None, None, None


def ea_render_differentiable(volume: torch.Tensor, grid, views: np.ndarray, dt=0.5, c=0.025,
                             rafi_ctx: Context | None = None, bwd_tile_items: int = 0) -> torch.Tensor:
    """bwd_tile_items: 0 lets the backward spread the queue evenly over one
    workgroup per CU; k > 0 gives each k-ray tile its own workgroup."""
    if rafi_ctx is None:
        n_rays = len(views) * int(views[0]["width"]) * int(views[0]["height"])
        rafi_ctx = Context(int(np.prod(grid)), EA_ITEM_BYTES, max(n_rays, 1))
    return EARender.apply(volume, tuple(grid), views, float(dt), float(c), rafi_ctx, int(bwd_tile_items))


# ---------------------------------------------------------------- batched ---

def view_rec(v) -> ViewRec:
    r = ViewRec()
    for k in ("org0", "du", "dv", "dir"):
        getattr(r, k)[:] = [float(x) for x in np.asarray(v[k], dtype=np.float32)]
    r.width, r.height, r.n_samples = int(v["width"]), int(v["height"]), int(v["n_samples"])
    return r


class Batch:
    """Many independent scenes rendered together (rafi_batch_*).

    scenes: list of (n, grid, view record, volume_offset in floats)."""

    def __init__(self, scenes, dt=0.5, c=0.025, stream=None):
        arr = (SceneRec * len(scenes))()
        for i, (n, grid, view, off) in enumerate(scenes):
            arr[i].volume_offset = int(off)
            arr[i].view = view_rec(view)
            arr[i].n = int(n)
            arr[i].grid[:] = [int(g) for g in grid]
        h = C.c_void_p()
        _check(lib().rafi_batch_create(arr, len(scenes), float(dt), float(c), C.byref(h)), "rafi_batch_create")
        self._h = h
        self.scenes = arr
        nr, nd = C.c_uint64(0), C.c_int32(0)
        _check(lib().rafi_batch_info(self._h, C.byref(nr), C.byref(nd)), "rafi_batch_info")
        self.n_rays, self.n_domains = nr.value, nd.value
        _check(lib().rafi_batch_set_stream(self._h, _stream(stream)), "rafi_batch_set_stream")

    def close(self):
        if self._h:
            lib().rafi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, split_tile=4096, march_block=256, march_grid=2048, use_graph=True, rounds_per_sync=4):
        t = BatchTuning(split_tile, march_block, march_grid, int(use_graph), rounds_per_sync)
        _check(lib().rafi_batch_set_tuning(self._h, C.byref(t)), "rafi_batch_set_tuning")

    def render(self, volumes: torch.Tensor, image: torch.Tensor, max_rounds: int = 1024) -> int:
        r = C.c_int32(0)
        _check(lib().rafi_batch_render(self._h, _dptr(volumes), _dptr(image), max_rounds, C.byref(r)),
               "rafi_batch_render")
        return r.value


def build_batch_inputs(specs, device, views=None):
    """Concatenated device volume buffer and Batch scene tuples for
    workloads.SceneSpec specs (blob volumes, +z views unless given)."""
    offs, vols, scenes = [], [], []
    off = 0
    for i, sp in enumerate(specs):
        v = W.blob_volume(sp.n, sp.volume_seed, device=device).reshape(-1)
        vols.append(v)
        view = W.plusz_view(sp.n, sp.rays_side, sp.rays_side)[0] if views is None else views[i]
        scenes.append((sp.n, sp.grid, view, off))
        off += v.numel()
    return torch.cat(vols), scenes


# ------------------------------------------------------- delta tracking ---

def dt_capacity(n_paths: int, max_bounce: int) -> int:
    cap = C.c_uint64(0)
    _check(lib().rafi_dt_capacity(n_paths, max_bounce, C.byref(cap)), "rafi_dt_capacity")
    return cap.value


def dt_job(volume: torch.Tensor, grid, views_dev: torch.Tensor, n_views: int, width: int, height: int,
           contrib: torch.Tensor, image=None, kappa=0.05, smax=None, albedo=0.8, light=(0.0, 0.0, -1.0),
           radiance=1.0, max_bounce=4, seed=0, counters=None) -> DTJob:
    """smax defaults to kappa * max(volume) (the smallest valid majorant).
    counters: optional int64 device tensor [2] (tentative points, real collisions)."""
    n = volume.shape[0]
    if smax is None:
        smax = float(kappa) * float(volume.max())
    return DTJob(_dptr(volume), _dptr(views_dev), _dptr(contrib), _dptr(image), n,
                 (C.c_int32 * 3)(*[int(g) for g in grid]), n_views, width, height, float(kappa), float(smax),
                 float(albedo), (C.c_float * 3)(*[float(v) for v in light]), float(radiance), int(max_bounce),
                 int(seed) & 0xFFFFFFFF, _dptr(counters))


def dt_raygen(ctx: Context, job: DTJob):
    _check(lib().rafi_dt_raygen(ctx.handle, C.byref(job)), "rafi_dt_raygen")


def dt_trace(ctx: Context, job: DTJob):
    _check(lib().rafi_dt_trace(ctx.handle, C.byref(job)), "rafi_dt_trace")


def dt_render_job(ctx: Context, job: DTJob, max_rounds: int = 100000) -> int:
    r = C.c_int32(0)
    _check(lib().rafi_dt_render(ctx.handle, C.byref(job), max_rounds, C.byref(r)), "rafi_dt_render")
    return r.value


def dt_render(volume: torch.Tensor, grid, views: np.ndarray, kappa=0.05, smax=None, albedo=0.8,
              light=(0.0, 0.0, -1.0), radiance=1.0, max_bounce=4, seed=0, ctx: Context | None = None,
              max_rounds: int = 100000):
    """Delta-tracking render of all paths of `views` (one path per pixel).
    Returns dict(image [n_paths], contrib [n_paths, max_bounce], rounds, ctx)."""
    dev = volume.device
    nv = len(views)
    w, h = int(views[0]["width"]), int(views[0]["height"])
    n_paths = nv * w * h
    if ctx is None:
        ctx = Context(int(np.prod(grid)), DT_ITEM_BYTES, dt_capacity(max(n_paths, 1), max_bounce))
    vdev = views_to_device(views, dev)
    contrib = torch.empty((n_paths, max_bounce), dtype=torch.float32, device=dev)
    image = torch.empty(n_paths, dtype=torch.float32, device=dev)
    job = dt_job(volume, grid, vdev, nv, w, h, contrib, image, kappa, smax, albedo, light, radiance, max_bounce,
                 seed)
    rounds = dt_render_job(ctx, job, max_rounds)
    return dict(image=image, contrib=contrib, rounds=rounds, ctx=ctx, job=job, views_dev=vdev)


# ------------------------------------------- multi-context N-body exchange ---
NB_PARTICLE_BYTES, NB_VIRTUAL_BYTES, NB_REQUEST_BYTES = 40, 24, 4
# record layouts, for reading queues back
NB_PARTICLE_DTYPE = W.NB_PARTICLE_DTYPE
NB_VIRTUAL_DTYPE = np.dtype([("pos", "<f4", 3), ("mass", "<f4"), ("smax", "<f4"), ("src", "<i4")])


def nb_workspace_bytes(n: int, n_domains: int) -> int:
    b = C.c_uint64(0)
    _check(lib().rafi_nb_workspace(n, n_domains, C.byref(b)), "rafi_nb_workspace")
    return b.value


def nb_to_device(particles: np.ndarray, device) -> torch.Tensor:
    """Particle records -> float32 device tensor [n, 10] (40-byte rows)."""
    a = np.ascontiguousarray(particles, dtype=W.NB_PARTICLE_DTYPE)
    return torch.from_numpy(a.view(np.float32).reshape(-1, 10).copy()).to(device)


def nb_from_bytes(items: torch.Tensor, dtype) -> np.ndarray:
    """A queue copied out as bytes -> numpy records."""
    return items.cpu().numpy().reshape(-1).view(dtype)


class NBody:
    """The three contexts, workspace and splitters of the essential-tree
    exchange (rafi_nb_step), for one particle set. Only allocation and
    argument marshalling happen here; every step runs in the library."""

    def __init__(self, particles: torch.Tensor, n_domains: int, cell_level: int = 4, theta: float = 0.5,
                 eps: float = 1e-3, dt: float = 1e-3, virtual_capacity: int | None = None, debug: bool = False,
                 log_vp1: bool = False):
        assert particles.dtype == torch.float32 and particles.dim() == 2 and particles.shape[1] == 10
        dev = particles.device
        n, D = particles.shape[0], n_domains
        self.n, self.D = n, D
        self.workspace = torch.empty(max(nb_workspace_bytes(n, D), 1), dtype=torch.uint8, device=dev)
        self.splitters = torch.empty(D + 1, dtype=torch.int32, device=dev)
        _check(lib().rafi_nb_splitters(_dptr(particles), n, D, _dptr(self.splitters), _dptr(self.workspace),
                                       _stream()), "rafi_nb_splitters")
        vcap = virtual_capacity if virtual_capacity is not None else D * max(D - 1, 1) + n * max(D - 1, 1)
        self.P = Context(D, NB_PARTICLE_BYTES, max(n, 1), debug=debug)
        self.V = Context(D, NB_VIRTUAL_BYTES, max(vcap, 1), debug=debug)
        self.R = Context(D, NB_REQUEST_BYTES, max(D * max(D - 1, 1), 1), debug=debug)
        self.vp1 = (torch.empty((D * max(D - 1, 1), NB_VIRTUAL_BYTES), dtype=torch.uint8, device=dev)
                    if log_vp1 else None)
        self.job = NBJob(D, cell_level, dt, theta, eps, self.splitters.data_ptr(), self.workspace.data_ptr(), n,
                         self.vp1.data_ptr() if log_vp1 else None, self.vp1.shape[0] if log_vp1 else 0)
        _check(lib().rafi_nb_seed(self.P.handle, C.byref(self.job), _dptr(particles), n), "rafi_nb_seed")

    def reseed(self, particles: torch.Tensor):
        """Round 0 again (rafi_nb_seed): the particle queue becomes these
        particles, in any order, grouped by their owning domains."""
        assert particles.dtype == torch.float32 and particles.dim() == 2 and particles.shape[1] == 10
        assert particles.shape[0] <= self.n
        self._seed_src = particles   # read by the seed kernel on the library's stream
        _check(lib().rafi_nb_seed(self.P.handle, C.byref(self.job), _dptr(particles), particles.shape[0]),
               "rafi_nb_seed")

    def step(self, dt: float | None = None):
        """One step; returns (round counts [4, D], queue sizes [3])."""
        if dt is not None:
            self.job.dt = dt
        rc = np.zeros((4, self.D), dtype=np.uint64)
        sz = np.zeros(3, dtype=np.uint64)
        _check(lib().rafi_nb_step(self.P.handle, self.V.handle, self.R.handle, C.byref(self.job),
                                  rc.ctypes.data_as(C.c_void_p), sz.ctypes.data_as(C.c_void_p)), "rafi_nb_step")
        return rc, sz

    def particles(self) -> np.ndarray:
        q, _ = self.P.copy_queue()
        return nb_from_bytes(q, W.NB_PARTICLE_DTYPE)

    def remote_lists(self) -> np.ndarray:
        q, _ = self.V.copy_queue()
        return nb_from_bytes(q, NB_VIRTUAL_DTYPE)

    def requests(self) -> np.ndarray:
        q, _ = self.R.copy_queue()
        return q.cpu().numpy().reshape(-1).view(np.int32)

    def close(self):
        for c in (self.P, self.V, self.R):
            c.close()


# Short names of the Python layer: the differentiable emission-absorption
# render (a torch.autograd.Function underneath) and the streamline trace.
render = ea_render_differentiable
trace_streamlines = sl_trace
