"""The C ABI library loads and exports every symbol its headers declare;
argument validation rejects bad calls before touching a device (no GPU use)."""
import ctypes as C
import os
import re

import pytest

from paper_2605_30294_amd import rafi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        if "__device__" in text:     # device-side inline header: nothing to export
            continue
        for m in re.finditer(r"^(?:int|void|const char \*)\s*\*?\s*(rafi_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = rafi.lib()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert names <= set(rafi._SIGS), sorted(names - set(rafi._SIGS))


def test_argument_validation_without_device():
    L = rafi.lib()
    h = C.c_void_p()
    assert L.rafi_create(0, 16, 100, C.byref(h)) == rafi.ERR_ARG
    assert L.rafi_create(8, 6, 100, C.byref(h)) == rafi.ERR_ARG          # not a multiple of 4
    assert L.rafi_create(8, 512, 100, C.byref(h)) == rafi.ERR_ARG        # too large
    assert L.rafi_create(8, 16, 0, C.byref(h)) == rafi.ERR_ARG
    assert L.rafi_create(8, 16, 1 << 32, C.byref(h)) == rafi.ERR_ARG
    assert L.rafi_create(10000, 16, 100, C.byref(h)) == rafi.ERR_ARG     # too many domains
    b = C.c_uint64(0)
    assert L.rafi_multisplit_workspace(1 << 20, 0, 32, C.byref(b)) == rafi.ERR_ARG
    assert L.rafi_multisplit_workspace(1 << 20, 1024, 32, C.byref(b)) == rafi.RAFI_OK and b.value > 0
    # misaligned pointers are rejected before any launch
    assert L.rafi_multisplit(C.c_void_p(8), C.c_void_p(16), 10, 16, 4, C.c_void_p(32), C.c_void_p(64),
                             C.c_void_p(128), C.c_void_p(256), 1 << 20, None) == rafi.ERR_ARG
    for code in range(0, -9, -1):
        assert rafi.strerror(code) != "unknown error"
    assert L.rafi_round(None, None, None) == rafi.ERR_ARG
    assert L.rafi_ea_render(None, None, 1, None) == rafi.ERR_ARG
    assert L.rafi_sl_trace(None, None, None, 0, 1, None, None) == rafi.ERR_ARG
    assert L.rafi_open(None, 10, rafi.SLOTS_APPEND) == rafi.ERR_ARG
    assert L.rafi_dt_raygen(None, None) == rafi.ERR_ARG
    assert L.rafi_dt_trace(None, None) == rafi.ERR_ARG
    assert L.rafi_dt_render(None, None, 10, None) == rafi.ERR_ARG
    assert L.rafi_nb_workspace(1000, 0, C.byref(b)) == rafi.ERR_ARG
    assert L.rafi_nb_workspace(1000, 2048, C.byref(b)) == rafi.ERR_ARG
    assert L.rafi_nb_workspace(1000, 64, C.byref(b)) == rafi.RAFI_OK and b.value > 1000 * 40
    assert L.rafi_nb_splitters(None, 10, 4, None, None, None) == rafi.ERR_ARG
    assert L.rafi_nb_seed(None, None, None, 0) == rafi.ERR_ARG
    assert L.rafi_nb_step(None, None, None, None, None, None) == rafi.ERR_ARG
    # the no-allocation split refuses problems beyond its fixed scratch buffer
    # (checked before any device call) and misaligned pointers
    assert L.rafi_multisplit_noalloc(C.c_void_p(256), C.c_void_p(512), 1 << 26, 32, 4096, C.c_void_p(1024),
                                     C.c_void_p(2048), C.c_void_p(4096), None) == rafi.ERR_TOO_LARGE
    assert L.rafi_multisplit_noalloc(C.c_void_p(8), C.c_void_p(16), 10, 16, 4, C.c_void_p(32), C.c_void_p(64),
                                     C.c_void_p(128), None) == rafi.ERR_ARG
    assert L.rafi_split_set_variant(18) == rafi.ERR_ARG
    assert L.rafi_split_set_variant(-1) == rafi.ERR_ARG


def test_dt_capacity_bound():
    """Capacity for delta tracking: 2 slots per visit x (the path + one shadow
    ray per scattering event) per path."""
    L = rafi.lib()
    cap = C.c_uint64(0)
    assert L.rafi_dt_capacity(1000, 4, C.byref(cap)) == rafi.RAFI_OK and cap.value == 2 * 1000 * 5
    assert L.rafi_dt_capacity(1000, 0, C.byref(cap)) == rafi.ERR_ARG
    assert L.rafi_dt_capacity(1 << 31, 1, C.byref(cap)) == rafi.ERR_ARG


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes struct of the binding has the field offsets and size that a
    C compiler gives the header's struct (compiled here with gcc)."""
    import subprocess
    structs = {"rafi_device_view": rafi.DeviceView, "rafi_ea_job": rafi.EAJob, "rafi_sl_job": rafi.SLJob,
               "rafi_dt_job": rafi.DTJob, "rafi_nb_job": rafi.NBJob, "rafi_ortho_view": rafi.ViewRec, "rafi_ea_scene": rafi.SceneRec,
               "rafi_batch_tuning": rafi.BatchTuning, "rafi_stats_t": rafi.Stats, "rafi_profile": rafi.Profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rafi.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_python_layer_names():
    """The Python layer's entry points: a context with round(), the
    differentiable render, the streamline trace and the stateless split."""
    assert callable(rafi.Context.round)
    assert rafi.render is rafi.ea_render_differentiable
    assert rafi.trace_streamlines is rafi.sl_trace
    assert callable(rafi.multisplit)
    assert issubclass(rafi.EARender, __import__("torch").autograd.Function)


def test_binding_rejects_bad_volume_and_field_shapes():
    """The job builders check shape and dtype before any pointer reaches the
    library: a non-cubic or non-float32 volume or field would make the
    kernels read n^3 voxels past the allocation."""
    import torch
    views = None
    img = torch.empty(4)
    for vol in (torch.zeros(4, 4, 2), torch.zeros(4, 4, 4, dtype=torch.float16), torch.zeros(4, 4),
                torch.zeros(4, 4, 4, dtype=torch.float64)):
        with pytest.raises(ValueError):
            rafi.ea_job(vol, (1, 1, 1), views, 1, 2, 2, img)
    ep, st = torch.empty(1, 3), torch.empty(1, dtype=torch.int32)
    for f in (torch.zeros(8, 8, 4, 3), torch.zeros(8, 8, 8, 2), torch.zeros(8, 8, 8, 3, dtype=torch.float16),
              torch.zeros(8, 8, 8)):
        with pytest.raises(ValueError):
            rafi.sl_job(f, (1, 1, 1), ep, st)
    for f in (torch.zeros(8, 8, 4, 3), torch.zeros(8, 8, 8, 3, dtype=torch.float64)):
        with pytest.raises(ValueError):
            rafi.sl_pack(f)
