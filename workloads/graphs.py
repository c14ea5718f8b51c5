"""Seeded synthetic max-flow instances in CSR form with paired reverse slots.

This module builds inputs only: it holds none of the max-flow method's
arithmetic and is shared by the oracle tests, the HIP-path tests and the
benchmark.  Every random draw comes from a numpy PCG64 stream seeded
explicitly, so the same call returns the same arrays on every machine.

Graph representation (the paper's adjacency arrays in which each edge also
knows its reverse edge, Sec. 4.2):

* ``off``  int64[n+1]  slots of tail v are ``off[v] .. off[v+1]-1``
* ``head`` int32[S]    head w of slot (v, w)
* ``rev``  int64[S]    paired reverse slot, ``rev[rev[a]] == a`` and
                        ``head[rev[a]] == v``
* ``cap``  int32[S]    capacity c(v, w) >= 0 (a reverse-only slot has 0)
* ``s``, ``t``         source and sink, ``s != t``

The instance families stand in for the paper's benchmark suite (Sec. 4.1,
Table 1), whose datasets are not available: a 4-connected 2D grid (small
smoke case), an 8-connected image-segmentation grid (vision, like
BL06-camel-lrg), a 6-connected 3D grid (like rmf_wide / vision volumes), a
random layered graph (like rlg_wide) and an R-MAT web-like graph with unit
capacities (like pld_spam).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 150701926


@dataclasses.dataclass
class Graph:
    n: int
    off: np.ndarray
    head: np.ndarray
    rev: np.ndarray
    cap: np.ndarray
    s: int
    t: int
    m_arcs: int           # directed arcs as generated (both directions of a pair count)
    family: str = ""
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def slots(self) -> int:
        return int(self.head.shape[0])

    def degree(self) -> np.ndarray:
        return np.diff(self.off)

    def tails(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.off))


def _stable_order(keys: np.ndarray) -> np.ndarray:
    """np.argsort(keys, kind="stable") for non-negative int32 keys.  Keys in
    a few sorted runs (grids, layered graphs) go to numpy's merge sort, which
    takes such runs in linear time; scattered keys (R-MAT) take two 16-bit
    radix passes (numpy sorts 16-bit keys by radix).  Both give the same
    order: a stable sort's result is unique."""
    if keys.shape[0] < (1 << 16) or np.count_nonzero(keys[1:] < keys[:-1]) < keys.shape[0] // 64:
        return np.argsort(keys, kind="stable")
    lo = (keys & 0xFFFF).astype(np.uint16)
    o1 = np.argsort(lo, kind="stable")
    del lo
    hi = (keys >> 16).astype(np.uint16)[o1]
    o2 = np.argsort(hi, kind="stable")
    return o1[o2]


def from_pairs(n, u, v, cap_uv, cap_vu, s, t, m_arcs, family="", params=None) -> Graph:
    """Build the CSR-pair arrays from a list of slot pairs.

    Pair i becomes slot (u[i] -> v[i]) with capacity cap_uv[i] and slot
    (v[i] -> u[i]) with capacity cap_vu[i]; the two are each other's reverse.
    Within a tail the slots keep the order of the pair list, the u-side
    occurrences first, then the v-side ones.
    """
    u = np.asarray(u, dtype=np.int32)
    v = np.asarray(v, dtype=np.int32)
    P = u.shape[0]
    tail = np.concatenate([u, v])
    head = np.concatenate([v, u])
    cap = np.concatenate([np.asarray(cap_uv, dtype=np.int32), np.asarray(cap_vu, dtype=np.int32)])
    del u, v
    order = _stable_order(tail)
    cnt = np.bincount(tail, minlength=n)
    del tail
    pos = np.empty(2 * P, dtype=np.int64)
    pos[order] = np.arange(2 * P, dtype=np.int64)
    head_s = head[order]
    del head
    cap_s = cap[order]
    del cap
    partner = order.astype(np.int64)
    del order
    partner += P
    partner[partner >= 2 * P] -= 2 * P
    rev = pos[partner]
    del partner, pos
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    return Graph(n=int(n), off=off, head=head_s, rev=rev, cap=cap_s, s=int(s), t=int(t),
                 m_arcs=int(m_arcs), family=family, params=dict(params or {}))


def from_arcs(n, tail, head, cap, s, t, family="", params=None) -> Graph:
    """Each directed input arc gets its own slot pair with a capacity-0 reverse."""
    cap = np.asarray(cap, dtype=np.int32)
    return from_pairs(n, tail, head, cap, np.zeros_like(cap), s, t, m_arcs=len(cap),
                      family=family, params=params)


# --------------------------------------------------------------------------
# Families
# --------------------------------------------------------------------------

def grid2d4(H, W, seed, cap_lo=1, cap_hi=100, term_cap=1000) -> Graph:
    """H x W 4-connected grid, row-major ids; s feeds column 0, column W-1 feeds t.

    Each neighbour pair is one slot pair with an independent uniform capacity
    in [cap_lo, cap_hi] per direction.
    """
    rng = np.random.default_rng(seed)
    N = H * W
    s, t = N, N + 1
    ids = np.arange(N, dtype=np.int32).reshape(H, W)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    gu = np.concatenate([hu, vu])
    gv = np.concatenate([hv, vv])
    P = gu.shape[0]
    c1 = rng.integers(cap_lo, cap_hi + 1, size=P, dtype=np.int32)
    c2 = rng.integers(cap_lo, cap_hi + 1, size=P, dtype=np.int32)
    left, right = ids[:, 0], ids[:, -1]
    tu = np.concatenate([np.full(H, s, np.int32), right])
    tv = np.concatenate([left, np.full(H, t, np.int32)])
    tc = np.full(2 * H, term_cap, dtype=np.int32)
    u = np.concatenate([gu, tu])
    v = np.concatenate([gv, tv])
    cuv = np.concatenate([c1, tc])
    cvu = np.concatenate([c2, np.zeros(2 * H, np.int32)])
    return from_pairs(N + 2, u, v, cuv, cvu, s, t, m_arcs=2 * P + 2 * H, family="grid2d4",
                      params=dict(H=H, W=W, seed=seed))


def seg_lut() -> np.ndarray:
    """Neighbour capacity table for the segmentation grid: round(100*exp(-d^2/200))."""
    d = np.arange(256, dtype=np.float64)
    return np.rint(100.0 * np.exp(-(d * d) / 200.0)).astype(np.int32)


def seg_intensity(H, W, rng, cell=64) -> np.ndarray:
    """Smooth uint8 intensity field: a coarse uniform lattice, bilinearly
    upsampled in exact integer arithmetic, plus small per-pixel noise."""
    LH = (H + cell - 1) // cell + 1
    LW = (W + cell - 1) // cell + 1
    lat = rng.integers(0, 256, size=(LH, LW), dtype=np.int64)
    r = np.arange(H, dtype=np.int64)
    c = np.arange(W, dtype=np.int64)
    r0, fr = r // cell, r % cell
    c0, fc = c // cell, c % cell
    a = lat[r0][:, c0]
    b = lat[r0][:, c0 + 1]
    cc = lat[r0 + 1][:, c0]
    dd = lat[r0 + 1][:, c0 + 1]
    wr = fr[:, None]
    wc = fc[None, :]
    num = (a * (cell - wr) * (cell - wc) + b * (cell - wr) * wc
           + cc * wr * (cell - wc) + dd * wr * wc)
    base = (num + (cell * cell) // 2) // (cell * cell)
    noise = rng.integers(-4, 5, size=(H, W), dtype=np.int64)
    return np.clip(base + noise, 0, 255).astype(np.uint8)


def grid2d8_seg(H, W, seed, term_max=500) -> Graph:
    """H x W 8-connected segmentation grid.

    Neighbour capacities (both directions, diagonals included) are
    LUT[|I(a)-I(b)|] from ``seg_lut``; every pixel gets a terminal arc
    s->p if I(p) >= 128 else p->t with capacity uniform in [0, term_max]
    (zero-capacity arcs are kept).
    """
    rng = np.random.default_rng(seed)
    N = H * W
    s, t = N, N + 1
    I = seg_intensity(H, W, rng).astype(np.int32)
    lut = seg_lut()
    ids = np.arange(N, dtype=np.int32).reshape(H, W)
    parts_u, parts_v, parts_c = [], [], []
    for (sa, sb) in (((slice(None), slice(0, -1)), (slice(None), slice(1, None))),      # right
                     ((slice(0, -1), slice(None)), (slice(1, None), slice(None))),      # down
                     ((slice(0, -1), slice(0, -1)), (slice(1, None), slice(1, None))),  # down-right
                     ((slice(0, -1), slice(1, None)), (slice(1, None), slice(0, -1)))):  # down-left
        parts_u.append(ids[sa].ravel())
        parts_v.append(ids[sb].ravel())
        parts_c.append(lut[np.abs(I[sa] - I[sb]).ravel()])
    gu = np.concatenate(parts_u)
    gv = np.concatenate(parts_v)
    gc = np.concatenate(parts_c)
    del parts_u, parts_v, parts_c
    P = gu.shape[0]
    flat = I.ravel()
    tcap = rng.integers(0, term_max + 1, size=N, dtype=np.int32)
    pix = np.arange(N, dtype=np.int32)
    src_side = flat >= 128
    tu = np.where(src_side, s, pix).astype(np.int32)
    tv = np.where(src_side, pix, t).astype(np.int32)
    u = np.concatenate([gu, tu])
    v = np.concatenate([gv, tv])
    cuv = np.concatenate([gc, tcap])
    cvu = np.concatenate([gc, np.zeros(N, np.int32)])
    del gu, gv
    return from_pairs(N + 2, u, v, cuv, cvu, s, t, m_arcs=2 * P + N, family="grid2d8_seg",
                      params=dict(H=H, W=W, seed=seed))


def grid3d6(X, Y, Z, seed, cap_lo=1, cap_hi=10000, term_cap=10**6) -> Graph:
    """X x Y x Z 6-connected grid, z-major ids (id = (z*Y + y)*X + x).

    Independent uniform capacity per direction; s feeds the z=0 plane and the
    z=Z-1 plane feeds t.
    """
    rng = np.random.default_rng(seed)
    N = X * Y * Z
    s, t = N, N + 1
    ids = np.arange(N, dtype=np.int32).reshape(Z, Y, X)
    gu = np.concatenate([ids[:, :, :-1].ravel(), ids[:, :-1, :].ravel(), ids[:-1, :, :].ravel()])
    gv = np.concatenate([ids[:, :, 1:].ravel(), ids[:, 1:, :].ravel(), ids[1:, :, :].ravel()])
    P = gu.shape[0]
    c1 = rng.integers(cap_lo, cap_hi + 1, size=P, dtype=np.int32)
    c2 = rng.integers(cap_lo, cap_hi + 1, size=P, dtype=np.int32)
    bot = ids[0].ravel()
    top = ids[-1].ravel()
    K = bot.shape[0]
    u = np.concatenate([gu, np.full(K, s, np.int32), top])
    del gu
    v = np.concatenate([gv, bot, np.full(K, t, np.int32)])
    del gv
    tc = np.full(2 * K, term_cap, np.int32)
    cuv = np.concatenate([c1, tc])
    cvu = np.concatenate([c2, np.zeros(2 * K, np.int32)])
    del c1, c2
    return from_pairs(N + 2, u, v, cuv, cvu, s, t, m_arcs=2 * P + 2 * K, family="grid3d6",
                      params=dict(X=X, Y=Y, Z=Z, seed=seed))


def _distinct_k(rng, rows, k, width):
    """rows x k draws from [0, width) with distinct values in every row."""
    out = rng.integers(0, width, size=(rows, k), dtype=np.int64)
    while True:
        srt = np.sort(out, axis=1)
        bad = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            return out
        out[bad] = rng.integers(0, width, size=(bad.size, k), dtype=np.int64)


def layered(layers, width, seed, fwd=4, cap_lo=1, cap_hi=10000, term_cap=10**6) -> Graph:
    """Random layered graph, layer-major ids (id = layer*width + i).

    Every vertex of layers 0..layers-2 has ``fwd`` arcs to distinct uniform
    vertices of the next layer; every vertex has one arc to a uniform other
    vertex of its own layer.  s feeds layer 0, the last layer feeds t.  Each
    arc gets its own capacity-0 reverse slot.
    """
    rng = np.random.default_rng(seed)
    N = layers * width
    s, t = N, N + 1
    nf = (layers - 1) * width
    tgt = _distinct_k(rng, nf, fwd, width)
    src = np.arange(nf, dtype=np.int64)
    f_tail = np.repeat(src, fwd)
    f_head = ((src // width + 1) * width)[:, None] + tgt
    f_head = f_head.ravel()
    del tgt
    allv = np.arange(N, dtype=np.int64)
    i = allv % width
    j = rng.integers(0, width - 1, size=N, dtype=np.int64)
    j = j + (j >= i)
    i_head = allv - i + j
    cap_f = rng.integers(cap_lo, cap_hi + 1, size=f_tail.shape[0], dtype=np.int32)
    cap_i = rng.integers(cap_lo, cap_hi + 1, size=N, dtype=np.int32)
    first = np.arange(width, dtype=np.int64)
    last = np.arange((layers - 1) * width, N, dtype=np.int64)
    tail = np.concatenate([f_tail, allv, np.full(width, s), last]).astype(np.int32)
    head = np.concatenate([f_head, i_head, first, np.full(width, t)]).astype(np.int32)
    cap = np.concatenate([cap_f, cap_i, np.full(2 * width, term_cap, np.int32)])
    del f_tail, f_head, i_head
    return from_arcs(N + 2, tail, head, cap, s, t, family="layered",
                     params=dict(layers=layers, width=width, seed=seed))


def rmat(scale, seed, edge_factor=16, a=0.57, b=0.19, c=0.19, top_frac=0.01) -> Graph:
    """R-MAT graph with 2^scale vertices and edge_factor*2^scale arc draws.

    Self-loops and duplicate (u, v) arcs are dropped, vertex ids are permuted
    at random, capacities are 1.  s is drawn uniformly among the top
    ``top_frac`` of vertices by out-degree, t among the top by in-degree,
    s != t.  s and t are ordinary vertices of V.
    """
    rng = np.random.default_rng(seed)
    N = 1 << scale
    M = edge_factor * N
    u = np.zeros(M, dtype=np.int32)
    v = np.zeros(M, dtype=np.int32)
    ab, abc = a + b, a + b + c
    # one bit of each endpoint per level: the quadrant q = [r >= a] + [r >=
    # a+b] + [r >= a+b+c] of a uniform r (a, b, c, d in that order) gives
    # the tail's bit (q >= 2) and the head's bit (q odd)
    for _ in range(scale):
        r = rng.random(M)
        q = (r >= a).view(np.uint8) + (r >= ab).view(np.uint8)
        q += (r >= abc).view(np.uint8)
        del r
        u <<= 1
        u |= q >> 1
        v <<= 1
        v |= q & 1
        del q
    perm = rng.permutation(N).astype(np.int64)
    u = perm[u]
    v = perm[v]
    keep = u != v
    key = np.unique(u[keep] * N + v[keep])
    del u, v, keep
    tail = (key // N).astype(np.int32)
    head = (key % N).astype(np.int32)
    del key
    outdeg = np.bincount(tail, minlength=N)
    indeg = np.bincount(head, minlength=N)
    k = max(2, int(math.ceil(top_frac * N)))
    top_out = np.argsort(-outdeg, kind="stable")[:k]
    top_in = np.argsort(-indeg, kind="stable")[:k]
    s = int(top_out[rng.integers(0, k)])
    t = s
    while t == s:
        t = int(top_in[rng.integers(0, k)])
    cap = np.ones(tail.shape[0], dtype=np.int32)
    return from_arcs(N, tail, head, cap, s, t, family="rmat",
                     params=dict(scale=scale, edge_factor=edge_factor, seed=seed))


def random_graph(n, m, seed, cap_max=20, p_zero=0.1, p_anti=0.3, p_par=0.1, st_arc=True) -> Graph:
    """Small random directed graph for property tests: parallel arcs,
    antiparallel pairs, zero capacities and a possible direct s->t arc."""
    rng = np.random.default_rng(seed)
    s, t = 0, n - 1
    tails, heads = [], []
    while len(tails) < m:
        x, y = (int(z) for z in rng.integers(0, n, size=2))
        if x == y:
            continue
        tails.append(x)
        heads.append(y)
        if rng.random() < p_par and len(tails) < m:
            tails.append(x)
            heads.append(y)
        if rng.random() < p_anti and len(tails) < m:
            tails.append(y)
            heads.append(x)
    if st_arc and rng.random() < 0.5:
        tails.append(s)
        heads.append(t)
    tails = np.array(tails, dtype=np.int32)
    heads = np.array(heads, dtype=np.int32)
    cap = rng.integers(1, cap_max + 1, size=tails.shape[0]).astype(np.int32)
    cap[rng.random(cap.shape[0]) < p_zero] = 0
    # Half the pairs carry capacity both ways (a merged antiparallel pair).
    both = rng.random(cap.shape[0]) < 0.3
    cap_r = np.where(both, rng.integers(1, cap_max + 1, size=cap.shape[0]), 0).astype(np.int32)
    return from_pairs(n, tails, heads, cap, cap_r, s, t, m_arcs=int((cap > 0).sum() + (cap_r > 0).sum()),
                      family="random", params=dict(n=n, m=m, seed=seed))


# --------------------------------------------------------------------------
# The workload configurations
# --------------------------------------------------------------------------

CONFIGS = {
    "c1": dict(desc="2D 4-connected grid 64x64, caps U[1,100], terminals 1000"),
    "c2": dict(desc="2D 8-connected segmentation grid 2048x2048"),
    "c3": dict(desc="3D 6-connected grid 256^3, caps U[1,1e4], terminals 1e6"),
    "c4a": dict(desc="random layered graph 512 x 16384, 4 forward + 1 intra arc per vertex"),
    "c4b": dict(desc="R-MAT scale 22, edge factor 16, unit capacities"),
}


def make_config(name: str, scale_down: int = 1, seed_offset: int = 0) -> Graph:
    """Instance of a named configuration.

    ``scale_down`` shrinks every linear dimension by that factor (same
    generator, same seed) for tests that need the same family at a size the
    oracle finishes quickly.  ``seed_offset`` draws another instance of the
    same family and size (the schedule autotuner tunes on one of those, not on
    the instance the benchmark times).
    """
    k = {"c1": 0, "c2": 1, "c3": 2, "c4a": 3, "c4b": 3}[name]
    seed = SEED_BASE + k + (100 if name == "c4b" else 0) + int(seed_offset)
    f = int(scale_down)
    if name == "c1":
        return grid2d4(max(2, 64 // f), max(2, 64 // f), seed)
    if name == "c2":
        return grid2d8_seg(max(2, 2048 // f), max(2, 2048 // f), seed)
    if name == "c3":
        d = max(2, 256 // f)
        return grid3d6(d, d, d, seed)
    if name == "c4a":
        return layered(max(2, 512 // f), max(2, 16384 // f), seed)
    if name == "c4b":
        sc = 22 - int(round(math.log2(f))) * 2 if f > 1 else 22
        return rmat(max(4, sc), seed)
    raise KeyError(name)


STREAM_FAMILIES = ("grid2d4", "grid2d8_seg", "grid3d6", "layered", "rmat")


def stream_instance(i: int, seed: int = SEED_BASE + 4, n_lo=1e3, n_hi=1e6):
    """Instance ``i`` of the batched/served stream: family uniform over the
    five rules, vertex count log-uniform in [n_lo, n_hi]."""
    ss = np.random.SeedSequence([seed, i])
    rng = np.random.default_rng(ss)
    fam = STREAM_FAMILIES[int(rng.integers(0, len(STREAM_FAMILIES)))]
    n_t = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    gseed = int(rng.integers(0, 2**62))
    if fam == "grid2d4":
        sd = max(2, int(round(math.sqrt(n_t))))
        return grid2d4(sd, sd, gseed)
    if fam == "grid2d8_seg":
        sd = max(2, int(round(math.sqrt(n_t))))
        return grid2d8_seg(sd, sd, gseed)
    if fam == "grid3d6":
        sd = max(2, int(round(n_t ** (1.0 / 3.0))))
        return grid3d6(sd, sd, sd, gseed)
    if fam == "layered":
        w = max(2, int(round(math.sqrt(32 * n_t))))
        L = max(2, int(round(n_t / w)))
        return layered(L, w, gseed)
    sc = max(4, int(round(math.log2(n_t))))
    return rmat(sc, gseed)


def stream_arrivals(count: int, rate: float, seed: int = SEED_BASE + 5) -> np.ndarray:
    """Poisson arrival times (seconds) for ``count`` requests at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    if rate <= 0 or math.isinf(rate):
        return np.zeros(count)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
