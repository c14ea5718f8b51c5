"""Small hand-built graphs with closed-form maximum flows (test helpers)."""
import numpy as np

from workloads import from_pairs, grid2d4


def path_graph(caps):
    """s -> 1 -> 2 -> ... -> k -> t with the given capacities (k+1 arcs)."""
    k = len(caps) - 1
    n = k + 2
    s, t = 0, n - 1
    u = np.arange(0, n - 1)
    v = np.arange(1, n)
    return from_pairs(n, u, v, np.array(caps), np.zeros(len(caps), int), s, t, m_arcs=len(caps))


def disjoint_paths(paths):
    """Vertex-disjoint s-t paths; paths[i] is the list of its arc capacities."""
    s, t = 0, 1
    nxt = 2
    U, V, C = [], [], []
    for caps in paths:
        prev = s
        for j, c in enumerate(caps):
            if j == len(caps) - 1:
                w = t
            else:
                w = nxt
                nxt += 1
            U.append(prev); V.append(w); C.append(c)
            prev = w
    return from_pairs(nxt, np.array(U), np.array(V), np.array(C), np.zeros(len(C), int), s, t,
                      m_arcs=len(C))


def uniform_row_grid(H, W, c, vert_cap=7, term_cap=10**6):
    """H x W 4-grid: every forward horizontal arc has capacity c, backward
    horizontal arcs 0, vertical pairs vert_cap both ways; s feeds column 0 and
    column W-1 feeds t.  The maximum flow is H*c (H disjoint row paths of
    bottleneck c; the cut between two columns has capacity H*c)."""
    N = H * W
    s, t = N, N + 1
    ids = np.arange(N).reshape(H, W)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    U = np.concatenate([hu, vu, np.full(H, s), ids[:, -1]])
    V = np.concatenate([hv, vv, ids[:, 0], np.full(H, t)])
    Cuv = np.concatenate([np.full(hu.size, c), np.full(vu.size, vert_cap), np.full(2 * H, term_cap)])
    Cvu = np.concatenate([np.zeros(hu.size, int), np.full(vu.size, vert_cap), np.zeros(2 * H, int)])
    return from_pairs(N + 2, U, V, Cuv, Cvu, s, t, m_arcs=int((Cuv > 0).sum() + (Cvu > 0).sum()))


def planted_matching(k, extra, seed):
    """Unit-capacity bipartite graph L (k) x R (k) with a planted perfect
    matching plus `extra` random L->R arcs; s -> L, R -> t, unit capacities.
    The maximum flow is k."""
    rng = np.random.default_rng(seed)
    s, t = 0, 1
    L = 2 + np.arange(k)
    R = 2 + k + np.arange(k)
    perm = rng.permutation(k)
    pairs = set((int(i), int(perm[i])) for i in range(k))
    while len(pairs) < k + extra:
        pairs.add((int(rng.integers(0, k)), int(rng.integers(0, k))))
    pl = np.array(sorted(pairs))
    U = np.concatenate([np.full(k, s), L[pl[:, 0]], R])
    V = np.concatenate([L, R[pl[:, 1]], np.full(k, t)])
    C = np.ones(U.size, int)
    return from_pairs(2 + 2 * k, U, V, C, np.zeros(U.size, int), s, t, m_arcs=U.size)


def graph_from_json(d):
    from workloads import Graph
    return Graph(n=d["n"], off=np.array(d["off"], np.int64), head=np.array(d["head"], np.int32),
                 rev=np.array(d["rev"], np.int64), cap=np.array(d["cap"], np.int32),
                 s=d["s"], t=d["t"], m_arcs=int(sum(1 for c in d["cap"] if c > 0)))
