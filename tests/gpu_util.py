"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def rel_close(gpu, ref, rtol, atol=0.0):
    """Elementwise |gpu - ref| <= rtol * |ref| + atol; returns (ok, worst index, worst ratio)."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    err = np.abs(g - r)
    bound = rtol * np.abs(r) + atol
    ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1), np.where(err > 0, np.inf, 0))
    i = int(np.argmax(ratio)) if ratio.size else 0
    return bool(np.all(err <= bound)), i, float(ratio.flat[i]) if ratio.size else 0.0


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
