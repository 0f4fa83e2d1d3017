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
    for code in range(0, -8, -1):
        assert rafi.strerror(code) != "unknown error"
    assert L.rafi_round(None, None, None) == rafi.ERR_ARG
    assert L.rafi_ea_render(None, None, 1, None) == rafi.ERR_ARG
    assert L.rafi_sl_trace(None, None, None, 0, 1, None, None) == rafi.ERR_ARG
