"""The seeded input generators against the shapes they are specified to
have: vertex, arc and slot counts from each configuration's formula,
degrees, terminal wiring and capacity ranges, at reduced sizes (the counts at
full size are checked against the goldens by the GPU tests) and at full size
for the small grid.  CPU only."""
import numpy as np
import pytest

import oracle
from workloads import make_config, stream_instance
from workloads.graphs import STREAM_FAMILIES


def _tails(g):
    return np.repeat(np.arange(g.n), np.diff(g.off))


def _common(g):
    """CSR-pair structure every generator must produce."""
    assert oracle.validate(g) == 0
    assert g.off[0] == 0 and g.off[-1] == g.slots == g.head.shape[0]
    t = _tails(g)
    assert (g.rev[g.rev] == np.arange(g.slots)).all()
    assert (g.head[g.rev] == t).all()
    assert (t != g.head).all()                            # no self-loops
    assert (g.cap >= 0).all()
    return t


def test_c1_full_size():
    g = make_config("c1")
    t = _common(g)
    W = 64
    assert (g.n, g.m_arcs, g.slots) == (W * W + 2, 4 * W * (W - 1) + 2 * W, 16384)
    grid = (t < W * W) & (g.head < W * W)
    assert ((g.cap[grid] >= 1) & (g.cap[grid] <= 100)).all()
    out_s = g.head[t == g.s]
    assert sorted(out_s) == list(range(0, W * W, W))    # the left column
    assert (g.cap[t == g.s] == 1000).all()
    into_t = t[(g.head == g.t) & (g.cap > 0)]
    assert sorted(into_t) == list(range(W - 1, W * W, W))   # the right column


@pytest.mark.parametrize("f", [16, 32])
def test_c3_shape(f):
    g = make_config("c3", f)
    t = _common(g)
    L = 256 // f
    pairs = 3 * L * L * (L - 1) + 2 * L * L
    assert (g.n, g.m_arcs, g.slots) == (L ** 3 + 2, 2 * 3 * L * L * (L - 1) + 2 * L * L, 2 * pairs)
    inner = (t != g.s) & (t != g.t) & (g.head != g.s) & (g.head != g.t)
    assert ((g.cap[inner] >= 1) & (g.cap[inner] <= 10000)).all()
    assert sorted(g.head[t == g.s]) == list(range(L * L))                     # the z = 0 plane
    assert sorted(t[(g.head == g.t) & (g.cap > 0)]) == list(range(L ** 3 - L * L, L ** 3))
    assert (g.cap[(t == g.s) | (g.head == g.t)] % 10 ** 6 == 0).all()
    deg = np.diff(g.off)[: L ** 3]
    assert deg.max() == 6 and deg.min() == 3 + (1 if L > 1 else 0)            # corners: 3 neighbours + terminal


@pytest.mark.parametrize("f", [32, 64])
def test_c2_shape(f):
    g = make_config("c2", f)
    t = _common(g)
    W = 2048 // f
    grid_pairs = 2 * W * (W - 1) + 2 * (W - 1) ** 2
    assert (g.n, g.m_arcs, g.slots) == (W * W + 2, 2 * grid_pairs + W * W, 2 * grid_pairs + 2 * W * W)
    # each pixel has exactly one terminal arc (to t or from s), capacity 0..500
    term = (t == g.s) | (g.head == g.t)
    ends = np.concatenate([g.head[t == g.s], t[g.head == g.t]])
    assert (np.bincount(ends, minlength=W * W) == 1).all()
    assert ((g.cap[term] >= 0) & (g.cap[term] <= 500)).all()
    grid = ~term & (t != g.t) & (g.head != g.s)
    assert (g.cap[grid] <= 100).all()                    # round(100 exp(-d^2 / 200)) <= 100
    assert (np.diff(g.off)[: W * W] <= 9).all()


@pytest.mark.parametrize("f", [32, 64])
def test_c4a_shape(f):
    g = make_config("c4a", f)
    t = _common(g)
    Lr, Wd = 512 // f, 16384 // f
    arcs = (Lr - 1) * Wd * 4 + Lr * Wd + 2 * Wd
    assert (g.n, g.m_arcs, g.slots) == (Lr * Wd + 2, arcs, 2 * arcs)
    fwd = (g.cap > 0) & (t < Lr * Wd) & (g.head < Lr * Wd)
    layer_t, layer_h = t[fwd] // Wd, g.head[fwd] // Wd
    assert ((layer_h == layer_t) | (layer_h == layer_t + 1)).all()
    nxt = layer_h == layer_t + 1
    per_vertex = np.bincount(t[fwd][nxt], minlength=Lr * Wd)
    assert (per_vertex[: (Lr - 1) * Wd] == 4).all() and (per_vertex[(Lr - 1) * Wd:] == 0).all()
    key = t[fwd][nxt].astype(np.int64) * g.n + g.head[fwd][nxt]
    assert np.unique(key).size == key.size               # the 4 forward heads are distinct
    assert (np.bincount(t[fwd][~nxt], minlength=Lr * Wd) == 1).all()   # one arc in its own layer
    assert ((g.cap[fwd] >= 1) & (g.cap[fwd] <= 10000)).all()


def test_c4b_shape():
    g = make_config("c4b", 64)                           # scale 22 - 2 log2(64) = 10
    t = _common(g)
    N = 1 << 10
    assert g.n == N and (g.cap[g.cap > 0] == 1).all()
    fwd = g.cap > 0
    key = t[fwd].astype(np.int64) * N + g.head[fwd]
    assert np.unique(key).size == key.size               # duplicates dropped
    assert g.m_arcs == int(fwd.sum()) <= 16 * N
    outdeg = np.bincount(t[fwd], minlength=N)
    indeg = np.bincount(g.head[fwd], minlength=N)
    k = max(2, int(np.ceil(0.01 * N)))
    assert g.s != g.t
    assert outdeg[g.s] >= np.sort(outdeg)[-k] and indeg[g.t] >= np.sort(indeg)[-k]


def test_stream_instances_span_the_families_and_sizes():
    gs = [stream_instance(i, n_hi=2e4) for i in range(60)]
    fams = {g.family for g in gs}
    assert fams == set(STREAM_FAMILIES)
    for g in gs[:12]:
        _common(g)
    ns = np.array([g.n for g in gs])
    assert ns.min() >= 500 and ns.max() <= 4e4
