"""The oracle's threaded mode (OpenMP over the items of one domain and
round, for timing) gives the same bits as the sequential loops: every
result, per-round count and queue."""
import numpy as np
import pytest

from paper_2605_30294_amd import workloads as W


@pytest.fixture
def threads(orc):
    yield orc
    orc.set_threads(1)


def _same(a, b):
    for k, v in a.items():
        if isinstance(v, np.ndarray):
            assert v.dtype == b[k].dtype and np.array_equal(v.view(np.uint8), b[k].view(np.uint8)), k
        else:
            assert v == b[k], k


def _both(orc, fn):
    orc.set_threads(1)
    a = fn()
    orc.set_threads(4)
    assert orc.get_threads() == 4
    b = fn()
    orc.set_threads(1)
    return a, b


def test_streamlines_thread_count_independent(threads):
    orc = threads
    f = W.abc_field(48)
    seeds = W.streamline_seeds(3000, 48, seed=31)
    for spv in (0, 17):
        a, b = _both(orc, lambda: orc.streamlines(f, (4, 2, 3), seeds, max_steps=600, steps_per_visit=spv,
                                                  queue_cap=1 << 20, visit_stride=16))
        _same(a, b)
    a, b = _both(orc, lambda: orc.streamlines_brute(f, (4, 2, 3), seeds, max_steps=600, visit_stride=16))
    _same(a, b)


def test_ea_render_thread_count_independent(threads):
    orc = threads
    vol = W.blob_volume(40, 32)
    views = W.random_views(3, 40, 30, 30, seed=33)
    a, b = _both(orc, lambda: orc.ea_render(vol, (2, 4, 2), views, queue_cap=1 << 20))
    _same(a, b)
    a, b = _both(orc, lambda: orc.ea_brute(vol, (2, 4, 2), views, visit_stride=12))
    _same(a, b)


def test_dt_render_thread_count_independent(threads):
    orc = threads
    vol = W.blob_volume(32, 34)
    views = W.random_views(1, 32, 32, 32, seed=35)
    smax = 0.05 * float(vol.max()) * 1.1
    a, b = _both(orc, lambda: orc.dt_render(vol, (2, 2, 2), views, 0.05, smax, 0.9, (0.0, 0.6, 0.8), 1.0, 3, 5,
                                            queue_cap=1 << 20))
    _same(a, b)
