"""Pins for the CPU oracle: brute force, closed forms, library cross-checks,
a hand-traced worked example and preflow invariants.  CPU only.

The oracle must agree with facts fixed by the paper and by mathematics, not
with itself: max-flow = min-cut over every s-t cut (Sec. 2), Eq. 1-2, exact
BFS distances (Sec. 2.1), closed forms, and an independent library solver.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.brute import brute_mincut
from workloads import make_config, random_graph, from_pairs
from tests._graphs import (path_graph, disjoint_paths, uniform_row_grid, planted_matching,
                           graph_from_json)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cert_ok(g, flow, side):
    code, val, cut = oracle.check_certificate(g, flow, side)
    assert code == 0, oracle.CERT_CODES[code]
    return val


# ---------------------------------------------------------------- validation

def test_validate_rejects_bad_inputs():
    g = path_graph([3, 4, 5])
    assert oracle.validate(g) == 0
    bad = path_graph([3, 4, 5]); bad.s = bad.t
    assert oracle.validate(bad) == -2
    bad = path_graph([3, 4, 5]); bad.cap = bad.cap.copy(); bad.cap[0] = -1
    assert oracle.validate(bad) == -7
    bad = path_graph([3, 4, 5]); bad.rev = bad.rev.copy(); bad.rev[0], bad.rev[1] = bad.rev[1], bad.rev[0]
    assert oracle.validate(bad) == -6
    bad = path_graph([3, 4, 5]); bad.head = bad.head.copy(); bad.head[0] = 0   # self-loop at s
    assert oracle.validate(bad) in (-5, -6)
    bad = path_graph([2**31 - 1, 4]); bad.cap = bad.cap.copy(); bad.cap[bad.rev[0]] = 1
    assert oracle.validate(bad) == -8
    with pytest.raises(ValueError):
        b2 = path_graph([3, 4]); b2.t = b2.s
        oracle.fifo_maxflow(b2)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("chunk", range(4))
def test_brute_force_random_graphs(chunk):
    for seed in range(chunk * 60, chunk * 60 + 60):
        n = 4 + seed % 14
        g = random_graph(n, (2 + seed % 4) * n, seed)
        best, tstar, smin = brute_mincut(g)
        A = oracle.fifo_maxflow(g)
        B = oracle.sync_maxflow(g)
        assert A["value"] == best, seed
        assert B["value"] == best, seed
        assert A["cut_tstar"] == best and A["cut_smin"] == best and B["cut_tstar"] == best
        assert (A["tstar"] == tstar).all(), seed
        assert (B["tstar"] == tstar).all(), seed
        assert (A["smin"] == smin).all(), seed
        assert _cert_ok(g, A["flow"], A["tstar"]) == best
        assert _cert_ok(g, B["flow"], B["tstar"]) == best


def test_literal_listing_termination_can_end_early():
    """With the listing's own ending (filter the old working set after a global
    relabel, stop as soon as it is empty) a vertex that a loser's relabel left
    at label n keeps excess that could still reach t.  The rebuilt working set
    reaches the maximum."""
    g = random_graph(15, 45, 59)
    best = brute_mincut(g)[0]
    literal = oracle.sync_maxflow(g, schedule=dict(literal_termination=1))
    fixed = oracle.sync_maxflow(g)
    assert literal["value"] < best
    assert fixed["value"] == best


# ---------------------------------------------------------------- closed forms

def test_path_bottleneck_and_rounds():
    g = path_graph([9, 4, 7, 5])
    for res in (oracle.fifo_maxflow(g), oracle.sync_maxflow(g)):
        assert res["value"] == 4
    # uniform capacities: the excess moves one arc per synchronous round
    k = 12
    g = path_graph([6] * (k + 1))
    B = oracle.sync_maxflow(g)
    assert B["value"] == 6
    assert B["rounds"] == k and B["pushes"] == k and B["relabels"] == 0


def test_disjoint_paths_sum_of_bottlenecks():
    paths = [[5, 3, 8], [2, 9], [7, 7, 7, 1], [4]]
    g = disjoint_paths(paths)
    expect = sum(min(p) for p in paths)
    for res in (oracle.fifo_maxflow(g), oracle.sync_maxflow(g)):
        assert res["value"] == expect
        assert _cert_ok(g, res["flow"], res["tstar"]) == expect


@pytest.mark.parametrize("H,W,c", [(5, 7, 3), (16, 16, 11), (9, 40, 1)])
def test_uniform_row_grid(H, W, c):
    g = uniform_row_grid(H, W, c)
    for res in (oracle.fifo_maxflow(g), oracle.sync_maxflow(g)):
        assert res["value"] == H * c


@pytest.mark.parametrize("k,extra", [(10, 15), (200, 800)])
def test_planted_perfect_matching(k, extra):
    g = planted_matching(k, extra, seed=k)
    for res in (oracle.fifo_maxflow(g), oracle.sync_maxflow(g)):
        assert res["value"] == k


def test_disconnected_and_direct_arc():
    # t unreachable: value 0, T* = {t}
    g = from_pairs(5, np.array([0, 1, 3]), np.array([1, 2, 4]), np.array([5, 5, 5]),
                   np.zeros(3, int), 0, 4, m_arcs=3)
    g.t = 4
    g2 = from_pairs(5, np.array([0, 1]), np.array([1, 2]), np.array([5, 5]), np.zeros(2, int), 0, 4,
                    m_arcs=2)
    for gg in (g2,):
        for res in (oracle.fifo_maxflow(gg), oracle.sync_maxflow(gg)):
            assert res["value"] == 0
            assert res["tstar"].tolist() == [0, 0, 0, 0, 1]
    # a direct s->t arc plus a parallel path
    g3 = from_pairs(3, np.array([0, 0, 1]), np.array([2, 1, 2]), np.array([7, 4, 3]),
                    np.zeros(3, int), 0, 2, m_arcs=3)
    for res in (oracle.fifo_maxflow(g3), oracle.sync_maxflow(g3)):
        assert res["value"] == 10


# ---------------------------------------------------------------- independent library

def _scipy_value(g):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_flow
    tl = g.tails()
    keep = g.cap > 0
    M = sp.csr_matrix((g.cap[keep].astype(np.int32), (tl[keep], g.head[keep])), shape=(g.n, g.n))
    M.sum_duplicates()
    return int(maximum_flow(M, g.s, g.t).flow_value)


@pytest.mark.parametrize("seed", range(6))
def test_scipy_crosscheck_random(seed):
    g = random_graph(300 + 50 * seed, 2000 + 400 * seed, 1000 + seed, cap_max=1000)
    v = _scipy_value(g)
    assert oracle.fifo_maxflow(g)["value"] == v
    assert oracle.sync_maxflow(g)["value"] == v


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 16), ("c4b", 16)])
def test_scipy_crosscheck_families(name, f):
    g = make_config(name, f)
    v = _scipy_value(g)
    A = oracle.fifo_maxflow(g)
    B = oracle.sync_maxflow(g)
    assert A["value"] == v and B["value"] == v
    assert _cert_ok(g, A["flow"], A["tstar"]) == v
    assert _cert_ok(g, B["flow"], B["tstar"]) == v


def test_residual_distance_matches_scipy_bfs():
    from scipy.sparse.csgraph import shortest_path
    import scipy.sparse as sp
    g = make_config("c3", 16)
    B = oracle.sync_maxflow(g, max_rounds=5)
    res = B["res"]
    dist = oracle.residual_distance(g, res, g.t, g.s)
    # reverse residual graph: edge v -> w for every residual arc w -> v, s removed
    tl = g.tails()
    keep = (res > 0) & (tl != g.s) & (g.head != g.s)
    M = sp.csr_matrix((np.ones(int(keep.sum())), (g.head[keep], tl[keep])), shape=(g.n, g.n))
    ref = shortest_path(M, unweighted=True, indices=g.t)
    ref = np.where(np.isinf(ref), g.n, ref).astype(np.int64)
    ref[g.s] = g.n
    assert (dist == ref).all()


# ---------------------------------------------------------------- worked example

def test_hand_traced_two_rounds():
    with open(os.path.join(GOLDEN, "prsn_two_vertex_trace.json")) as fh:
        gold = json.load(fh)
    g = graph_from_json(gold["graph"])
    r1 = oracle.sync_maxflow(g, preflow_only=True, max_rounds=1)
    assert r1["stopped"]
    assert r1["d"].tolist() == gold["after_round_1"]["d"]
    assert r1["e"].tolist() == gold["after_round_1"]["e"]
    assert r1["res"].tolist() == gold["after_round_1"]["res"]
    p1 = oracle.sync_maxflow(g, preflow_only=True)
    ph = gold["phase1"]
    assert p1["value"] == ph["value"] and p1["rounds"] == ph["rounds"]
    assert p1["pushes"] == ph["pushes"] and p1["relabels"] == ph["relabels"]
    assert p1["global_relabels"] == ph["global_relabels"] and p1["work"] == ph["work"]
    assert p1["d"].tolist() == ph["d"] and p1["res"].tolist() == ph["res"]
    assert p1["tstar"].tolist() == ph["tstar"] and p1["cut_tstar"] == ph["cut"]
    full = oracle.sync_maxflow(g)
    assert full["rounds2"] == gold["phase2"]["rounds"]
    assert full["res"].tolist() == gold["phase2"]["res"]
    assert full["flow"].tolist() == gold["phase2"]["flow"]


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("name,f", [("c1", 1), ("c4a", 32), ("c4b", 16)])
def test_preflow_invariants_between_rounds(name, f):
    g = make_config(name, f)
    tl = g.tails()
    pair = g.cap.astype(np.int64) + g.cap[g.rev]
    for k in (1, 3, 10, 40):
        B = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k)
        res, e = B["res"], B["e"]
        flow = g.cap - res
        assert (res >= 0).all()                       # f <= c
        assert (res + res[g.rev] == pair).all()       # f(v,w) = -f(w,v)
        inflow = -np.bincount(tl, weights=flow, minlength=g.n).astype(np.int64)
        assert (inflow == e).all()                    # e = net inflow
        others = np.ones(g.n, bool); others[[g.s]] = False
        assert (e[others] >= 0).all()                 # a preflow


def test_schedules_change_rounds_not_results():
    g = make_config("c2", 16)
    base = oracle.sync_maxflow(g)
    thr = 12 * g.n + 2 * g.slots
    grs = {base["global_relabels"]}
    for sched in (dict(round_charge=thr // 100), dict(freq_num=1, freq_den=1), dict(alpha=30),
                  dict(level_charge=thr // 8), dict(level_charge=thr, round_charge=thr // 100)):
        r = oracle.sync_maxflow(g, schedule=sched)
        assert r["value"] == base["value"]
        assert (r["tstar"] == base["tstar"]).all()
        _cert_ok(g, r["flow"], r["tstar"])
        grs.add(r["global_relabels"])
    assert len(grs) > 2          # the schedules do change how often the labels are recomputed


# ---------------------------------------------------------------- simple rounds

def test_simple_rounds_one_pass_and_one_relabel():
    """The simple synchronous variant Sec. 3 starts from: in a round each
    active vertex checks its arcs once and relabels at most once.  In c1's
    first round the 64 active vertices are the left column, each with
    excess 1000 and one admissible arc (to its right neighbour, capacity at
    most 100): one push and one relabel each.  Listing 1's full discharge
    goes on pushing after the relabel."""
    g = make_config("c1")
    S = oracle.sync_maxflow(g, preflow_only=True, max_rounds=1, schedule=dict(simple=1))
    B = oracle.sync_maxflow(g, preflow_only=True, max_rounds=1)
    assert S["rounds"] == 1 and S["pushes"] == 64 and S["relabels"] == 64
    assert B["pushes"] > 64


@pytest.mark.parametrize("chunk", range(2))
def test_simple_rounds_brute_force(chunk):
    for seed in range(chunk * 50, chunk * 50 + 50):
        n = 4 + seed % 14
        g = random_graph(n, (2 + seed % 4) * n, seed)
        best, tstar, smin = brute_mincut(g)
        S = oracle.sync_maxflow(g, schedule=dict(simple=1))
        assert S["value"] == best, seed
        assert (S["tstar"] == tstar).all(), seed
        _cert_ok(g, S["flow"], S["tstar"])


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 32), ("c4b", 16)])
def test_simple_rounds_families(name, f):
    """Same maximum and sink side as the FIFO oracle; more rounds than
    Listing 1's rounds on every family but the shallow R-MAT."""
    g = make_config(name, f)
    A = oracle.fifo_maxflow(g, preflow_only=True)
    S = oracle.sync_maxflow(g, schedule=dict(simple=1))
    B = oracle.sync_maxflow(g)
    assert S["value"] == A["value"] == B["value"]
    assert (S["tstar"] == A["tstar"]).all()
    _cert_ok(g, S["flow"], S["tstar"])
    assert S["rounds"] >= B["rounds"]


def test_certificate_rejects_non_maximum_and_invalid():
    g = path_graph([4, 2, 6])
    A = oracle.fifo_maxflow(g)
    code, val, cut = oracle.check_certificate(g, A["flow"], A["tstar"])
    assert code == 0 and val == 2 and cut == 2
    zero = np.zeros(g.slots, np.int64)
    assert oracle.check_certificate(g, zero, A["tstar"])[0] == 6          # cut != value
    over = A["flow"].copy(); over[0] += 1; over[g.rev[0]] -= 1
    assert oracle.check_certificate(g, over, A["tstar"])[0] in (2, 3)
    asym = A["flow"].copy(); asym[0] += 1
    assert oracle.check_certificate(g, asym, A["tstar"])[0] == 1


# ---------------------------------------------------------------- labels after a global relabel

@pytest.mark.parametrize("name,f", [("c1", 1), ("c3", 16), ("c4a", 32), ("c4b", 16)])
def test_labels_exact_and_valid_after_each_global_relabel(name, f):
    """Right after a global relabel the labels are the exact residual
    distances to t (Sec. 2.1), hence valid: d(v) <= d(w) + 1 on every
    residual arc v -> w.  A round charge far above the threshold puts a
    global relabel before every round, so the state returned after k rounds
    is a post-relabel state; the distances come from the checker's own BFS,
    and validity and the excess identity are checked on the arrays."""
    g = make_config(name, f)
    tl = g.tails()
    sched = dict(round_charge=10 ** 15)
    for k in (1, 2, 5, 13):
        B = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k, schedule=sched)
        res, d, e = B["res"], B["d"], B["e"]
        dist = oracle.residual_distance(g, res, g.t, g.s)
        dist[g.s] = g.n
        assert (d == dist).all(), k
        resid = res > 0
        assert (d[tl[resid]] <= d[g.head[resid]] + 1).all(), k
        flow = g.cap.astype(np.int64) - res
        assert (-np.bincount(tl, weights=flow, minlength=g.n).astype(np.int64) == e).all()


def test_labels_between_relabels_can_be_invalid():
    """Between global relabels a vertex that gives way on an edge may raise
    its label past the neighbour pushing into it in the same round (Sec. 3.1
    allows this), so validity d(v) <= d(w) + 1 can fail mid-phase (here on a
    seeded random graph after its first round).  The global relabels restore
    it, and the termination rule does not rely on it."""
    g = random_graph(16, 48, 108)
    tl = g.tails()
    broken = False
    for k in range(1, 40):
        B = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k)
        if not B["stopped"]:
            break
        d, res = B["d"], B["res"]
        resid = (res > 0) & (tl != g.s) & (tl != g.t)
        if not (d[tl[resid]] <= d[g.head[resid]] + 1).all():
            broken = True
            break
    assert broken


# ---------------------------------------------------------------- gap rule

def test_gap_rule_hand_trace():
    with open(os.path.join(GOLDEN, "gap_rule_trace.json")) as fh:
        gold = json.load(fh)
    g = graph_from_json(gold["graph"])
    off = gold["without_gap"]
    r1 = oracle.sync_maxflow(g, preflow_only=True, max_rounds=1)
    assert r1["stopped"]
    for key in ("d", "e", "res"):
        assert r1[key].tolist() == off["after_round_1"][key], key
    for sched, ref in ((None, off["phase1"]), (dict(gap=1), gold["with_gap"]["phase1"])):
        p1 = oracle.sync_maxflow(g, preflow_only=True, schedule=sched)
        for key in ("value", "rounds", "pushes", "relabels", "global_relabels", "work", "gap_lifts"):
            assert p1[key] == ref[key], (sched, key)
        if "d" in ref:
            assert p1["d"].tolist() == ref["d"]
        full = oracle.sync_maxflow(g, schedule=sched)
        assert full["rounds2"] == gold["phase2"]["rounds"] and full["pushes2"] == gold["phase2"]["pushes"]
        assert full["res"].tolist() == gold["phase2"]["res"]
        assert full["flow"].tolist() == gold["phase2"]["flow"]


def test_gap_rule_no_hole_after_rounds_random():
    """The no-hole property round by round on seeded random graphs, among
    them one (seed 79) where a round opens gaps at two labels at once: the
    rule must take the smaller."""
    for seed in list(range(40)) + [79]:
        n = 6 + seed % 12 if seed < 40 else 25
        g = random_graph(n, 3 * n if seed < 40 else 5 * n, seed)
        inner = np.ones(g.n, bool)
        inner[[g.s, g.t]] = False
        for k in range(1, 12):
            G = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k, schedule=dict(gap=1))
            labs = np.unique(G["d"][inner & (G["d"] < g.n)])
            if labs.size:
                assert labs[0] >= 1 and labs[-1] == labs.size, (seed, k)
            if not G["stopped"]:
                break


@pytest.mark.parametrize("chunk", range(2))
def test_gap_rule_brute_force(chunk):
    lifted = 0
    for seed in range(chunk * 60, chunk * 60 + 60):
        n = 4 + seed % 14
        g = random_graph(n, (2 + seed % 4) * n, seed)
        best, tstar, _ = brute_mincut(g)
        for simple in (0, 1):
            G = oracle.sync_maxflow(g, schedule=dict(gap=1, simple=simple))
            assert G["value"] == best, seed
            assert (G["tstar"] == tstar).all(), seed
            _cert_ok(g, G["flow"], G["tstar"])
            lifted += G["gap_lifts"]
    assert lifted > 0


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 16), ("c4a", 32), ("c4b", 16)])
def test_gap_rule_leaves_no_gap(name, f):
    """After every round with the gap rule, the labels below n of the
    vertices other than the terminals fill 1 .. max without a hole; the
    value and T* are those of the FIFO oracle."""
    g = make_config(name, f)
    A = oracle.fifo_maxflow(g, preflow_only=True)
    inner = np.ones(g.n, bool)
    inner[[g.s, g.t]] = False
    for k in (1, 2, 4, 8, 16, 32, 64):
        G = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k, schedule=dict(gap=1))
        labs = np.unique(G["d"][inner & (G["d"] < g.n)])
        if labs.size:
            assert labs[0] >= 1 and labs[-1] == labs.size, (k, labs[:10])
        if not G["stopped"]:
            break
    G = oracle.sync_maxflow(g, schedule=dict(gap=1))
    assert G["value"] == A["value"]
    assert (G["tstar"] == A["tstar"]).all()
    _cert_ok(g, G["flow"], G["tstar"])


# ---------------------------------------------------------------- phase 2 (R17)

@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 16), ("c4a", 64), ("c4b", 64)])
def test_phase2_leaves_the_sink_side_alone(name, f):
    """Phase 2 (returning the stranded excess to s, Sec. 2.1's second phase,
    reading R17) runs over V minus T* and never changes the residual of a
    slot with an end in T*: the preflow's flow on every such slot is the
    final flow's, so the value and the minimum cut carry over unchanged.
    After phase 2 every vertex other than s and t has zero excess."""
    g = make_config(name, f)
    P = oracle.sync_maxflow(g, preflow_only=True)
    F = oracle.sync_maxflow(g)
    assert (P["tstar"] == F["tstar"]).all() and P["value"] == F["value"]
    tails = np.repeat(np.arange(g.n), np.diff(g.off))
    touches = (F["tstar"][tails] == 1) | (F["tstar"][g.head] == 1)
    assert touches.any() and (~touches).any()
    assert (P["res"][touches] == F["res"][touches]).all()
    inner = np.ones(g.n, bool)
    inner[[g.s, g.t]] = False
    assert (F["e"][inner] == 0).all()
    assert (P["e"][inner] > 0).any()                   # phase 1 strands excess that phase 2 returns
