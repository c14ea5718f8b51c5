"""Run a quick subset of the oracle pins; exit 1 on the first failure.

Used by the mutation test: a copy of the oracle with one planted mistake is
loaded through ORACLE_LIB, and some pin here must fail."""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle                                   # noqa: E402
from oracle.brute import brute_mincut           # noqa: E402
from workloads import random_graph              # noqa: E402
from tests._graphs import graph_from_json, path_graph   # noqa: E402


def full_value(g):
    return oracle.fifo_maxflow(g, preflow_only=True)["value"]


def main():
    try:
        for seed in range(40):
            n = 4 + seed % 10
            g = random_graph(n, 3 * n, seed)
            best = brute_mincut(g)[0]
            for res in (oracle.fifo_maxflow(g), oracle.sync_maxflow(g)):
                if res["value"] != best:
                    return 1
                if oracle.check_certificate(g, res["flow"], res["tstar"])[0] != 0:
                    return 1
        g = path_graph([6] * 13)
        B = oracle.sync_maxflow(g)
        if B["rounds"] != 12 or B["relabels"] != 0:
            return 1
        gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                           "prsn_two_vertex_trace.json")))
        g = graph_from_json(gold["graph"])
        r1 = oracle.sync_maxflow(g, preflow_only=True, max_rounds=1)
        if r1["res"].tolist() != gold["after_round_1"]["res"] or r1["d"].tolist() != gold["after_round_1"]["d"]:
            return 1
        full = oracle.sync_maxflow(g)
        if full["flow"].tolist() != gold["phase2"]["flow"]:
            return 1
        # simple rounds (Sec. 3's first design): c1's first round is one push
        # and one relabel for each of its 64 active vertices
        from workloads import make_config
        c1 = make_config("c1")
        s1 = oracle.sync_maxflow(c1, preflow_only=True, max_rounds=1, schedule=dict(simple=1))
        if (s1["pushes"], s1["relabels"]) != (64, 64):
            return 1
        # the per-level charge (a schedule term) changes when labels are
        # recomputed, never the value
        lv = oracle.sync_maxflow(c1, schedule=dict(level_charge=100000))
        if lv["value"] != full_value(c1) or lv["global_relabels"] == oracle.sync_maxflow(c1)["global_relabels"]:
            return 1
        # the gap rule: the hand trace, and no hole left below the top label
        gg = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gap_rule_trace.json")))
        g = graph_from_json(gg["graph"])
        p1 = oracle.sync_maxflow(g, preflow_only=True, schedule=dict(gap=1))
        if (p1["rounds"], p1["gap_lifts"]) != (1, 2):
            return 1
        for seed in list(range(30)) + [79]:
            n = 6 + seed % 12 if seed < 30 else 25
            g = random_graph(n, 3 * n if seed < 30 else 5 * n, seed)
            inner = np.ones(g.n, bool)
            inner[[g.s, g.t]] = False
            for k in range(1, 10):
                G = oracle.sync_maxflow(g, preflow_only=True, max_rounds=k, schedule=dict(gap=1))
                labs = np.unique(G["d"][inner & (G["d"] < g.n)])
                if labs.size and (labs[0] < 1 or labs[-1] != labs.size):
                    return 1
    except Exception:
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
