"""Brute-force minimum cut by enumerating every s-t cut.  Test infrastructure only.

Max-flow = min-cut (Sec. 2): the value of a maximum flow equals the smallest
capacity over all partitions (S, T) with s in S and t in T, where the
capacity sums c over arcs from S to T.  For n <= ~20 every partition is
enumerated.  The unique smallest sink side of a minimum cut (T*: the
intersection of the sink sides of all minimum cuts) and the unique smallest
source side (S_min: the intersection of the source sides) follow directly.
"""
from __future__ import annotations

import numpy as np


def brute_mincut(g, chunk: int = 1 << 14):
    """Returns (min_cut_capacity, tstar[n] uint8, smin[n] uint8)."""
    n = g.n
    if n > 22:
        raise ValueError("brute force is for tiny graphs")
    others = [v for v in range(n) if v not in (g.s, g.t)]
    k = len(others)
    tails = np.repeat(np.arange(n), np.diff(g.off))
    heads = np.asarray(g.head, dtype=np.int64)
    caps = np.asarray(g.cap, dtype=np.int64)
    best = None
    sink_inter = None    # AND of sink-side masks over minimum cuts
    src_inter = None     # AND of source-side masks
    total = 1 << k
    for lo in range(0, total, chunk):
        masks = np.arange(lo, min(total, lo + chunk), dtype=np.int64)
        # side[m, v] = 1 if v on the source side
        side = np.zeros((masks.shape[0], n), dtype=bool)
        side[:, g.s] = True
        for j, v in enumerate(others):
            side[:, v] = (masks >> j) & 1
        cross = side[:, tails] & ~side[:, heads]
        caps_m = cross.astype(np.int64) @ caps
        mval = int(caps_m.min())
        if best is None or mval < best:
            best = mval
            sink_inter = np.ones(n, dtype=bool)
            src_inter = np.ones(n, dtype=bool)
        if mval == best:
            sel = side[caps_m == best]
            sink_inter &= (~sel).all(axis=0)
            src_inter &= sel.all(axis=0)
    return best, sink_inter.astype(np.uint8), src_inter.astype(np.uint8)
