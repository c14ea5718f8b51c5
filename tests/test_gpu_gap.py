"""The gap rule (MF_GAP_RELABEL) on the GPU against oracle B's gap rule, bit
for bit (value, T*, per-slot flow, round, push, relabel and global-relabel
counts, and the labels each phase's gap rule lifted).  Needs a GPU."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, random_graph
from tests._graphs import graph_from_json

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


def _same(ctx, g, simple=False, lanes=0, tag=""):
    import paper_1507_01926_amd as mf
    r = ctx.solve(g, mf.options(gap=True, simple_rounds=simple, lanes_per_vertex=lanes))
    B = oracle.sync_maxflow(g, schedule=dict(gap=1, simple=int(simple)))
    assert r["value"] == B["value"], tag
    assert (r["sink_side"] == B["tstar"]).all(), tag
    assert (r["flow"].astype(np.int64) == B["flow"]).all(), tag
    for k in ("rounds", "rounds2", "pushes", "relabels", "global_relabels", "bfs_levels"):
        assert r[k] == B[k], (tag, k, r[k], B[k])
    assert r["gap_lifts"] == B["gap_lifts"] and r["gap_lifts2"] == B["gap_lifts2"], tag
    return r, B


def test_gap_hand_trace(ctx):
    gold = json.load(open(os.path.join(GOLDEN, "gap_rule_trace.json")))
    g = graph_from_json(gold["graph"])
    r, _ = _same(ctx, g, tag="hand trace")
    ref = gold["with_gap"]["phase1"]
    assert (r["rounds"], r["gap_lifts"], r["relabels"], r["pushes"]) == \
        (ref["rounds"], ref["gap_lifts"], ref["relabels"], ref["pushes"])
    assert r["flow"].tolist() == gold["phase2"]["flow"]


def test_gap_random_graphs(ctx):
    lifted = 0
    for seed in range(80):
        n = 4 + seed % 30
        g = random_graph(n, (2 + seed % 4) * n, seed)
        r, B = _same(ctx, g, simple=seed % 3 == 0, lanes=(1, 4, 16)[seed % 3], tag=f"seed {seed}")
        lifted += B["gap_lifts"] + B["gap_lifts2"]
    assert lifted > 0


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 32), ("c4b", 16)])
def test_gap_families(ctx, name, f):
    g = make_config(name, f)
    print(f"gap {name}/{f}", flush=True)
    sys.stdout.flush()
    _same(ctx, g, tag=name)


def test_gap_refused_where_unsupported(ctx):
    import paper_1507_01926_amd as mf
    g = make_config("c1")
    res, _ = mf.batch_solve(ctx, [g], opts=[mf.options(gap=True)])
    assert res[0]["status"] == mf.MF_EINVAL
    with pytest.raises(mf.MaxflowError):
        ctx.solve(g, mf.options(gap=True, persistent=True))
