"""Batched solver (one persistent launch, one workgroup per instance) against
the oracle, through the C ABI.  Needs a GPU."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, random_graph, stream_instance
from tests._graphs import path_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


def _check_one(g, r, sched=None):
    B = oracle.sync_maxflow(g, schedule=sched or {})
    assert r["status"] == 0
    assert r["value"] == B["value"] and r["cut_capacity"] == B["value"]
    assert (r["sink_side"] == B["tstar"]).all()
    assert (r["flow"].astype(np.int64) == B["flow"]).all()
    assert r["rounds"] == B["rounds"] and r["rounds2"] == B["rounds2"]
    assert r["pushes"] == B["pushes"] and r["relabels"] == B["relabels"]
    assert r["global_relabels"] == B["global_relabels"]


def test_batch_mixed_instances(ctx):
    import paper_1507_01926_amd as mf
    graphs = [random_graph(4 + i % 25, 3 * (4 + i % 25), 500 + i) for i in range(40)]
    graphs += [make_config("c1"), make_config("c2", 32), make_config("c3", 16), make_config("c4a", 64),
               make_config("c4b", 32)]
    print(f"batch of {len(graphs)}", flush=True)
    res, ms = mf.batch_solve(ctx, graphs)
    for g, r in zip(graphs, res):
        _check_one(g, r)


@pytest.mark.parametrize("lanes", [4, 8, 16, 32])
def test_batch_lane_counts(ctx, lanes):
    import paper_1507_01926_amd as mf
    graphs = [make_config("c2", 32), make_config("c4b", 32), random_graph(20, 60, 7)]
    res, _ = mf.batch_solve(ctx, graphs, opts=[mf.options(lanes_per_vertex=lanes) for _ in graphs])
    for g, r in zip(graphs, res):
        assert r["lanes_per_vertex"] == lanes
        _check_one(g, r)


def test_batch_schedules_and_stream_instances(ctx):
    import paper_1507_01926_amd as mf
    graphs = [stream_instance(i, n_hi=2e4) for i in range(24)]
    opts, scheds = [], []
    for i, g in enumerate(graphs):
        rc = (12 * g.n + 2 * g.slots) // [0, 16, 128][i % 3] if i % 3 else 0
        lc = [0, 5000, 50000][(i // 3) % 3]
        simple = i % 4 == 3
        opts.append(mf.options(gr_round_charge=rc, gr_level_charge=lc, simple_rounds=simple))
        scheds.append(dict(round_charge=rc, level_charge=lc, simple=int(simple)))
    res, _ = mf.batch_solve(ctx, graphs, opts=opts)
    for g, r, sc in zip(graphs, res, scheds):
        _check_one(g, r, sc)


def test_batch_invalid_instance_does_not_stop_others(ctx):
    import paper_1507_01926_amd as mf
    good = path_graph([5, 3, 8])
    bad = path_graph([5, 3, 8]); bad.cap = bad.cap.copy(); bad.cap[0] = -2
    bad2 = path_graph([5, 3, 8]); bad2.rev = bad2.rev.copy(); bad2.rev[1] = 0
    res, _ = mf.batch_solve(ctx, [good, bad, good, bad2])
    assert res[0]["status"] == 0 and res[0]["value"] == 3
    assert res[2]["status"] == 0 and res[2]["value"] == 3
    assert res[1]["status"] == mf.MF_EINVAL and res[3]["status"] == mf.MF_EINVAL


def test_batch_equals_plain_solver(ctx):
    import paper_1507_01926_amd as mf
    graphs = [make_config("c3", 16), make_config("c4a", 64)]
    res, _ = mf.batch_solve(ctx, graphs)
    for g, r in zip(graphs, res):
        p = ctx.solve(g)
        assert p["value"] == r["value"] and (p["flow"] == r["flow"]).all()
        assert (p["sink_side"] == r["sink_side"]).all() and p["rounds"] == r["rounds"]


def test_schedule_autotuner_plain(ctx):
    """The autotuner's schedule search on one uploaded graph: every
    candidate is timed, and the schedule it picks gives the oracle's
    results run with that schedule."""
    from paper_1507_01926_amd.autotune import Autotuner, SCHEDULES, knobs_to_options
    g = make_config("c2", 16)
    dg = ctx.upload(g)
    try:
        entry = Autotuner(ctx, cache_path=None).tune_schedule(dg, g, reps=1)
        assert len(entry["candidates"]) == len(SCHEDULES)
        k = entry["knobs"]
        r = dg.solve(knobs_to_options(g, k))
        B = oracle.sync_maxflow(g, schedule=dict(round_charge=(12 * g.n + 2 * g.slots) // k["round_divisor"],
                                                 freq_num=1, freq_den=k["freq_den"],
                                                 level_charge=k["level_charge"]))
        assert r["value"] == B["value"] and r["cut_capacity"] == B["value"]
        assert r["rounds"] == B["rounds"] and r["global_relabels"] == B["global_relabels"]
    finally:
        dg.free()
