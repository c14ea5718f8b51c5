"""Host-side helpers of bench.py that need no GPU."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_changed_caps_keep_the_flow_feasible():
    """The re-solve leg's capacity changes touch the asked fraction of the
    slots with capacity, raise half by 1..40, and never cut a slot below the
    flow it carries (so the kept flow stays feasible and the solve resumes)."""
    sys.path.insert(0, ROOT)
    import bench
    rng = np.random.default_rng(5)
    cap = rng.integers(0, 60, size=20000).astype(np.int32)
    flow = np.where(rng.random(20000) < 0.5, rng.integers(-30, 30, size=20000), 0).astype(np.int32)
    flow = np.minimum(flow, cap)
    new = bench._changed_caps(cap, flow, 0.1, np.random.default_rng(7))
    changed = np.flatnonzero(new != cap)
    assert (cap[changed] > 0).all()
    assert changed.size <= int(0.1 * np.count_nonzero(cap > 0))
    up = new > cap
    assert ((new - cap)[up] <= 40).all() and up.sum() > 0
    assert (new >= np.maximum(flow, 0)).all() and (new >= 0).all()
    assert (new[~up] <= cap[~up]).all()


def test_stream_instances_are_generated_in_order():
    """The generator pool yields the stream's instances in index order, equal
    to generating them one by one (the batched, served and plain legs replay
    the same stream)."""
    sys.path.insert(0, ROOT)
    import bench
    from workloads import stream_instance
    got = list(bench._instances(6, 3e3, 2, ahead=3))
    assert [i for i, _ in got] == list(range(6))
    for i, g in got:
        ref = stream_instance(i, n_hi=3e3)
        assert g.n == ref.n and (g.head == ref.head).all() and (g.cap == ref.cap).all()


def test_schedule_cache_is_tuned_elsewhere_and_within_the_candidates():
    """Every workload in the committed schedule cache was tuned on another
    instance of its generator rule (a seed offset), never the benchmarked one,
    and its schedule is one of the autotuner's candidates (the full-size GPU
    tests check every candidate against the oracle's goldens)."""
    import json
    from paper_1507_01926_amd.autotune import SCHEDULE_CACHE, SCHEDULES
    with open(SCHEDULE_CACHE) as fh:
        cache = json.load(fh)
    assert {"c2", "c3"} <= set(cache)
    cands = {(rd, fd, lc) for rd, fd, lc in SCHEDULES}
    for name, entry in cache.items():
        assert "seed offset" in entry["tuned_on"] and "not the benchmarked instance" in entry["tuned_on"]
        k = entry["knobs"]
        assert (k["round_divisor"], k["freq_den"], k["level_charge"]) in cands, name
        assert entry["ms"] == min(c["ms"] for c in entry["candidates"])
