"""Full-size parity: each benchmark workload at its full size, solved by the
HIP path in the launch configuration the benchmark times (the paper's
global-relabel rule plus a per-round charge of (12n+2m)/128), against the
expected results that the CPU oracle wrote into tests/golden/full_<name>.json
(value and sink side T* from sequential FIFO push-relabel; round, push,
relabel, global-relabel and BFS-level counts and the per-slot flow from the
synchronous rounds).  Needs a GPU."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAMES = [n for n in ("c1", "c2", "c3", "c4a", "c4b") if os.path.exists(os.path.join(GOLDEN, f"full_{n}.json"))]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", NAMES)
def test_full_size_workload(name):
    import paper_1507_01926_amd as mf
    gold = json.load(open(os.path.join(GOLDEN, f"full_{name}.json")))
    print(f"full-size {name}: generating", flush=True)
    g = make_config(name)
    assert (g.n, g.slots, g.m_arcs, g.s, g.t) == (gold["n"], gold["slots"], gold["arcs"], gold["s"], gold["t"])
    sc = gold["sync"]["schedule"]
    assert sc["round_charge"] == max(1, (12 * g.n + 2 * g.slots) // 128)
    ctx = mf.Context(0)
    try:
        print(f"full-size {name}: solving n={g.n} slots={g.slots}", flush=True)
        r = ctx.solve(g, mf.options(gr_round_charge=sc["round_charge"]))
    finally:
        ctx.close()
    sys.stdout.flush()
    assert r["value"] == gold["value"] and r["cut_capacity"] == gold["cut"]
    assert int(r["sink_side"].sum()) == gold["tstar_count"]
    assert _sha(r["sink_side"].astype(np.uint8)) == gold["tstar_sha256"]
    s = gold["sync"]
    assert (r["rounds"], r["rounds2"], r["global_relabels"], r["bfs_levels"]) == \
        (s["rounds"], s["rounds2"], s["global_relabels"], s["bfs_levels"])
    assert (r["pushes"], r["relabels"]) == (s["pushes"], s["relabels"])
    assert _sha(r["flow"].astype("<i4")) == s["flow_sha256"]
    # the flow is a maximum flow in its own right (conservation, capacities,
    # antisymmetry, no residual s-t path, cut of T* equals the value)
    code, val, cut = oracle.check_certificate(g, r["flow"].astype(np.int64), r["sink_side"])
    assert code == 0, oracle.CERT_CODES[code]
    assert val == cut == gold["value"]


_GRAPHS = {}


def _graph(name):
    if name not in _GRAPHS:
        _GRAPHS.clear()
        _GRAPHS[name] = make_config(name)
    return _GRAPHS[name]


def _schedule_cases():
    from paper_1507_01926_amd.autotune import SCHEDULES
    cases = []
    for name in NAMES:
        for sc in SCHEDULES[1:]:
            if name in ("c3", "c4a") and sc[2] == 0:
                continue                    # deep-search graphs: the level-charge schedule only
            cases.append((name, sc))
    return cases


@pytest.mark.parametrize("name,sched", _schedule_cases())
def test_full_size_other_schedules(name, sched):
    """The schedules the benchmark's autotuner chooses among change rounds and
    per-slot flow, never the value, the cut or the sink side."""
    import paper_1507_01926_amd as mf
    from paper_1507_01926_amd.autotune import knobs_to_options
    gold = json.load(open(os.path.join(GOLDEN, f"full_{name}.json")))
    g = _graph(name)
    rd, fd, lc = sched
    print(f"full-size {name}: schedule {sched}", flush=True)
    ctx = mf.Context(0)
    try:
        r = ctx.solve(g, knobs_to_options(g, dict(round_divisor=rd, freq_den=fd, level_charge=lc)))
    finally:
        ctx.close()
    sys.stdout.flush()
    assert r["value"] == gold["value"] and r["cut_capacity"] == gold["cut"]
    assert _sha(r["sink_side"].astype(np.uint8)) == gold["tstar_sha256"]
    code, val, cut = oracle.check_certificate(g, r["flow"].astype(np.int64), r["sink_side"])
    assert code == 0, oracle.CERT_CODES[code]
