"""Host-side logic of bench.py and the schedule autotuner (no GPU)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_rk4_traffic_only_for_the_measured_source_and_schedule():
    """The counter-derived bytes per launch are reported only for the source
    file and schedule they were taken with; anything else gives None."""
    b = _bench()
    sched, layout = b.RK4_TRAFFIC["schedule"], b.RK4_TRAFFIC["field_layout"]
    assert b.rk4_traffic(sched, layout) == b.RK4_TRAFFIC["bytes_per_launch"]
    other = tuple(sched[:-1]) + (sched[-1] + 1,)
    assert b.rk4_traffic(other, layout) is None
    assert b.rk4_traffic(sched, "padded" if layout != "padded" else "unpadded") is None


def test_bench_default_schedule_matches_measured_counters():
    """The default command line runs the schedule the counters describe."""
    b = _bench()
    from paper_2605_30294_amd import rafi
    assert b.STEPS_PER_VISIT == rafi.SL_STEPS_PER_VISIT
    assert b.RK4_TRAFFIC["schedule"] == (rafi.SL_STEPS_PER_VISIT, 0, 0, rafi.SL_QUAD_ITEMS)


def test_streamline_tuning_space():
    """Schedules are (steps_per_visit, tail_items, refill_lanes, quad_items);
    quad launches are swept only without lane refill (they never combine)."""
    from paper_2605_30294_amd import autotune
    assert all(len(t) == 4 for t in autotune.STREAMLINE_SPACE)
    assert all(t[3] == 0 for t in autotune.STREAMLINE_SPACE if t[2] > 0)
    assert any(t[3] > 0 for t in autotune.STREAMLINE_SPACE)
