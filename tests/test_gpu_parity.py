"""Parity of the HIP path with the oracle, through the C ABI.  Needs a GPU.

The GPU runs the synchronous rounds with each round a function of its start
state (pushes into a vertex become visible at the end of the round), so the
whole solve is deterministic: value, per-slot flow, sink side, round, push,
relabel and global-relabel counts must equal oracle B's bit for bit, for any
lane count.  Value, cut capacity and the sink side T* must also equal oracle
A's (sequential FIFO push-relabel), and the flow must pass the certificate.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, random_graph, from_pairs
from tests._graphs import path_graph, uniform_row_grid, planted_matching, graph_from_json

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(ctx, g, sched=None, lanes=0, check_a=True, **extra):
    import paper_1507_01926_amd as mf
    sched = dict(sched or {})
    gpu_sched = {("gr_" + k if not k.startswith("gr_") else k): v for k, v in sched.items() if k != "simple"}
    if sched.get("simple"):
        gpu_sched["simple_rounds"] = True
    opt = mf.options(lanes_per_vertex=lanes, **extra, **gpu_sched)
    osched = {k.replace("gr_", "").replace("freq_num", "freq_num"): v for k, v in sched.items()}
    r = ctx.solve(g, opt)
    B = oracle.sync_maxflow(g, schedule=osched)
    assert r["value"] == B["value"]
    assert r["cut_capacity"] == B["value"]
    assert (r["sink_side"] == B["tstar"]).all()
    assert (r["flow"].astype(np.int64) == B["flow"]).all()
    assert r["rounds"] == B["rounds"] and r["rounds2"] == B["rounds2"]
    assert r["pushes"] == B["pushes"] and r["relabels"] == B["relabels"]
    assert r["global_relabels"] == B["global_relabels"]
    assert r["bfs_levels"] == B["bfs_levels"]
    if check_a:
        A = oracle.fifo_maxflow(g, preflow_only=True)
        assert r["value"] == A["value"] and (r["sink_side"] == A["tstar"]).all()
    code, val, cut = oracle.check_certificate(g, r["flow"].astype(np.int64), r["sink_side"])
    assert code == 0, oracle.CERT_CODES[code]
    return r


@pytest.mark.parametrize("grid_path", [False, True])
def test_hand_traced_example(ctx, grid_path):
    """Small graphs run on one workgroup by default; grid_path forces the
    grid-wide kernels.  Both must reproduce the hand trace."""
    import paper_1507_01926_amd as mf
    gold = json.load(open(os.path.join(GOLDEN, "prsn_two_vertex_trace.json")))
    g = graph_from_json(gold["graph"])
    cap = np.array(gold["graph"]["cap"])
    for lanes in (1, 2, 4, 64):
        r1 = ctx.solve(g, mf.options(max_rounds=1, lanes_per_vertex=lanes, grid_path=grid_path),
                       allow_timeout=True)
        assert r1["status"] == mf.MF_ETIMEOUT
        assert (cap - r1["flow"]).tolist() == gold["after_round_1"]["res"]
        r = ctx.solve(g, mf.options(lanes_per_vertex=lanes, grid_path=grid_path))
        ph = gold["phase1"]
        assert r["value"] == ph["value"] and r["rounds"] == ph["rounds"]
        assert r["pushes"] == ph["pushes"] and r["relabels"] == ph["relabels"]
        assert r["global_relabels"] == ph["global_relabels"]
        assert r["sink_side"].tolist() == ph["tstar"] and r["cut_capacity"] == ph["cut"]
        assert r["rounds2"] == gold["phase2"]["rounds"]
        assert r["flow"].tolist() == gold["phase2"]["flow"]


@pytest.mark.parametrize("grid_path", [False, True])
@pytest.mark.parametrize("chunk", range(4))
def test_random_small_graphs(ctx, chunk, grid_path):
    for seed in range(chunk * 40, chunk * 40 + 40):
        n = 4 + seed % 30
        g = random_graph(n, (2 + seed % 5) * n, seed, cap_max=50)
        _note(f"random seed={seed} n={n} slots={g.slots} grid_path={grid_path}")
        _compare(ctx, g, lanes=[0, 1, 2, 8, 64][seed % 5], grid_path=grid_path)


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 32), ("c4b", 16),
                                    ("c2", 8), ("c4a", 16), ("c2", 64), ("c3", 32), ("c4b", 128)])
def test_families_scaled(ctx, name, f):
    g = make_config(name, f)
    _note(f"family {name}/{f} n={g.n} slots={g.slots}")
    _compare(ctx, g)
    if g.n <= 8192:
        _compare(ctx, g, grid_path=True, check_a=False)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_lane_count_does_not_change_results(ctx, lanes):
    g = make_config("c2", 16)
    _note(f"lanes={lanes}")
    _compare(ctx, g, lanes=lanes, check_a=False)


@pytest.mark.parametrize("sched", [dict(round_charge=5000), dict(freq_num=1, freq_den=1),
                                   dict(alpha=1, beta=0), dict(round_charge=100000, alpha=30),
                                   dict(level_charge=20000), dict(level_charge=200000, round_charge=5000)])
def test_schedules(ctx, sched):
    g = make_config("c3", 8)
    _note(f"schedule {sched}")
    _compare(ctx, g, sched=sched, check_a=False)


@pytest.mark.parametrize("name,f,lanes", [("c1", 1, 0), ("c2", 16, 0), ("c2", 64, 8), ("c3", 8, 0),
                                           ("c4a", 32, 0), ("c4b", 16, 0), ("c4b", 16, 32)])
def test_simple_rounds_match_oracle(ctx, name, f, lanes):
    """The simple synchronous variant of Sec. 3 (MF_SIMPLE_ROUNDS) against the
    oracle run with the same rounds: value, T*, per-slot flow and counts."""
    g = make_config(name, f)
    _note(f"simple rounds {name}/{f} lanes={lanes}")
    _compare(ctx, g, sched=dict(simple=1, round_charge=(12 * g.n + 2 * g.slots) // 128), lanes=lanes)
    if g.n <= 8192:
        _compare(ctx, g, sched=dict(simple=1), lanes=lanes, grid_path=True, check_a=False)
    _compare(ctx, g, sched=dict(simple=1), persistent=True, check_a=False)


@pytest.mark.parametrize("grid_path", [False, True])
def test_simple_rounds_random_small_graphs(ctx, grid_path):
    for seed in range(300, 340):
        n = 4 + seed % 30
        g = random_graph(n, (2 + seed % 5) * n, seed, cap_max=50)
        _note(f"simple rounds random seed={seed} n={n} grid_path={grid_path}")
        _compare(ctx, g, sched=dict(simple=1), lanes=[0, 1, 2, 8, 64][seed % 5], grid_path=grid_path)


@pytest.mark.parametrize("k", [1, 2, 7, 30])
def test_state_after_k_rounds(ctx, k):
    import paper_1507_01926_amd as mf
    g = make_config("c4a", 32)
    _note(f"max_rounds={k}")
    r = ctx.solve(g, mf.options(max_rounds=k), allow_timeout=True)
    B = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k)
    assert B["stopped"] and r["status"] == mf.MF_ETIMEOUT
    assert (g.cap.astype(np.int64) - r["flow"] == B["res"]).all()
    assert r["rounds"] == k


def test_edge_cases(ctx):
    import paper_1507_01926_amd as mf
    # only a direct s->t arc
    g = from_pairs(2, np.array([0]), np.array([1]), np.array([9]), np.array([0]), 0, 1, m_arcs=1)
    r = ctx.solve(g)
    assert r["value"] == 9 and r["flow"].tolist() == [9, -9] and r["sink_side"].tolist() == [0, 1]
    # no arcs at all
    g = from_pairs(3, np.array([], int), np.array([], int), np.array([], int), np.array([], int), 0, 2,
                   m_arcs=0)
    r = ctx.solve(g)
    assert r["value"] == 0 and r["sink_side"].tolist() == [0, 0, 1]
    # t unreachable
    g = from_pairs(5, np.array([0, 1]), np.array([1, 2]), np.array([5, 5]), np.zeros(2, int), 0, 4,
                   m_arcs=2)
    r = ctx.solve(g)
    assert r["value"] == 0 and r["flow"].tolist() == [0] * g.slots
    # all capacities zero
    g = uniform_row_grid(4, 4, 0, vert_cap=0, term_cap=0)
    r = ctx.solve(g)
    assert r["value"] == 0
    for gg in (path_graph([7, 3, 9, 2, 8]), planted_matching(64, 200, 3)):
        _compare(ctx, gg)
    # preflow-only mode
    g = make_config("c1")
    r = ctx.solve(g, mf.options(preflow_only=True))
    B = oracle.sync_maxflow(g, preflow_only=True)
    assert r["value"] == B["value"] and r["rounds2"] == 0 and r["flow"] is None


def test_invalid_graphs_rejected(ctx):
    import paper_1507_01926_amd as mf
    base = path_graph([3, 4, 5])
    cases = []
    b = path_graph([3, 4, 5]); b.cap = b.cap.copy(); b.cap[0] = -1; cases.append(b)
    b = path_graph([3, 4, 5]); b.rev = b.rev.copy(); b.rev[0], b.rev[1] = b.rev[1], b.rev[0]; cases.append(b)
    b = path_graph([3, 4, 5]); b.rev = b.rev.copy(); b.rev[0] = 10**6; cases.append(b)
    b = path_graph([3, 4, 5]); b.head = b.head.copy(); b.head[0] = 99; cases.append(b)
    b = path_graph([2**31 - 1, 4]); b.cap = b.cap.copy(); b.cap[b.rev[0]] = 1; cases.append(b)
    b = path_graph([3, 4, 5]); b.off = b.off.copy(); b.off[1] = b.off[2] + 1; cases.append(b)
    for b in cases:
        with pytest.raises(mf.MaxflowError) as ei:
            ctx.solve(b)
        assert ei.value.status == mf.MF_EINVAL
    b = path_graph([3, 4, 5]); b.t = b.s
    with pytest.raises(mf.MaxflowError):
        ctx.solve(b)
    # the context still works after rejections
    assert ctx.solve(base)["value"] == 3


def test_device_entry_point_with_torch_buffers(ctx):
    import torch
    g = make_config("c2", 16)
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.off).to(dev)
    head = torch.from_numpy(g.head).to(dev)
    rev = torch.from_numpy(g.rev).to(dev)
    cap = torch.from_numpy(g.cap).to(dev)
    flow = torch.zeros(g.slots, dtype=torch.int32, device=dev)
    side = torch.zeros(g.n, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    r = ctx.solve_device(off, head, rev, cap, g.s, g.t, flow=flow, side=side)
    B = oracle.sync_maxflow(g)
    assert r["value"] == B["value"]
    assert (flow.cpu().numpy().astype(np.int64) == B["flow"]).all()
    assert (side.cpu().numpy() == B["tstar"]).all()


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 32), ("c4b", 16)])
def test_persistent_mode_matches(ctx, name, f):
    """Each phase as one persistent cooperative kernel gives the same results
    as one launch per round and level (both must equal the oracle bit for bit)."""
    g = make_config(name, f)
    _note(f"persistent {name}/{f}")
    _compare(ctx, g, persistent=True, check_a=False)
    _compare(ctx, g, persistent=True, check_a=False, sched=dict(round_charge=20000, level_charge=50000))


@pytest.mark.parametrize("dense_threshold", [1, 64, 1 << 30])
def test_dense_threshold_does_not_change_results(ctx, dense_threshold):
    g = make_config("c2", 8)
    _note(f"dense_threshold={dense_threshold}")
    _compare(ctx, g, dense_threshold=dense_threshold, check_a=False)
    _compare(ctx, g, dense_threshold=dense_threshold, check_a=False, persistent=True)


@pytest.mark.parametrize("bpc", [1, 2])
def test_persistent_grid_size(ctx, bpc):
    g = make_config("c4a", 16)
    _note(f"blocks_per_cu={bpc}")
    _compare(ctx, g, blocks_per_cu=bpc, check_a=False, persistent=True)


def _star_graph(k, seed):
    """s -> hub (cap big), hub -> leaf_i (random caps), leaf_i -> t (random
    caps), plus leaf_i -> leaf_{i+1} arcs: one vertex of degree ~2k."""
    rng = np.random.default_rng(seed)
    n = k + 3
    s, hub, t = 0, 1, n - 1
    leaves = np.arange(2, 2 + k)
    u = np.concatenate([[s], np.full(k, hub), leaves, leaves[:-1]])
    v = np.concatenate([[hub], leaves, np.full(k, t), leaves[1:]])
    c = np.concatenate([[10**6], rng.integers(1, 50, k), rng.integers(1, 50, k), rng.integers(0, 20, k - 1)])
    return from_pairs(n, u, v, c, np.zeros(len(c), int), s, t, m_arcs=len(c))


@pytest.mark.parametrize("name,f,lanes", [("c4b", 16, 32), ("c4b", 16, 1), ("c4b", 32, 4), ("star", 3000, 4),
                                          ("star", 700, 1)])
def test_hub_vertices_by_blocks(ctx, name, f, lanes):
    """Vertices above 64 lanes' worth of slots are discharged and merged by a
    block each; results stay those of the oracle."""
    g = _star_graph(f, 7) if name == "star" else make_config(name, f)
    _note(f"hub kernels {name}/{f} lanes={lanes}")
    _compare(ctx, g, lanes=lanes, check_a=False)
