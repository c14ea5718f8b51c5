"""Large instances in the batched and served forms, and re-solves of
resident graphs in the served form.  Needs a GPU.

Instances of 10^5 - 10^6 vertices, one per generator family of the stream
(drawn by stream_instance with n in [1e5, 1e6]), are routed to the grid-wide
kernels (above the routing size) in both forms; each result must equal
oracle B element by element (value, T*, per-slot flow, round, push, relabel,
global-relabel and level counts), and a served request gives the same alone
and in a mix with small ones.  A resident graph re-solved with new
capacities gives oracle A's value and T* on the new graph with a flow that
passes the certificate, continuing from its previous flow when every new
capacity holds it.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, stream_instance

pytestmark = pytest.mark.gpu

# stream_instance(i, n_lo=1e5, n_hi=1e6) of each family: layered, 3D grid,
# R-MAT, 4-connected grid, segmentation grid
LARGE = (0, 1, 4, 12, 20)


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def large():
    out = []
    for i in LARGE:
        g = stream_instance(i, n_lo=1e5, n_hi=1e6)
        _note(f"oracle B on stream instance {i}: {g.family} n={g.n} slots={g.slots}")
        out.append((g, oracle.sync_maxflow(g)))
    return out


def _same_as_oracle(r, g, B, tag):
    assert r["status"] == 0, tag
    assert r["value"] == B["value"], tag
    assert r["cut_capacity"] == B["value"], tag
    assert (r["sink_side"] == B["tstar"]).all(), tag
    assert (r["flow"].astype(np.int64) == B["flow"]).all(), tag
    for k in ("rounds", "rounds2", "pushes", "relabels", "global_relabels", "bfs_levels"):
        assert r[k] == B[k], (tag, k, r[k], B[k])


ROUTE = 1 << 18        # routing size of these tests: every LARGE instance goes to the grid-wide kernels


def test_batch_large_instances_match_oracle(ctx, large):
    import paper_1507_01926_amd as mf
    small = [make_config("c1"), make_config("c2", 64), make_config("c4a", 64)]
    graphs = [g for g, _ in large] + small
    res, _ = mf.batch_solve(ctx, graphs, opts=[mf.options(batch_grid_slots=ROUTE) for _ in graphs])
    for k, (g, B) in enumerate(large):
        assert res[k]["lanes_per_vertex"] == 0          # solved by the grid-wide kernels
        _same_as_oracle(res[k], g, B, f"batch large {k} {g.family}")
    for j, g in enumerate(small):
        B = oracle.sync_maxflow(g)
        r = res[len(large) + j]
        assert r["lanes_per_vertex"] > 0                # one workgroup each
        _same_as_oracle(r, g, B, f"batch small {j}")


def test_batch_default_routing(ctx, large):
    """With the default routing size, instances above it go to the grid-wide
    kernels while the batch launch runs, the rest run in it."""
    import paper_1507_01926_amd as mf
    graphs = [g for g, _ in large]
    res, _ = mf.batch_solve(ctx, graphs)
    for k, (g, B) in enumerate(large):
        assert (res[k]["lanes_per_vertex"] == 0) == (g.slots > mf.MF_BATCH_GRID_SLOTS)
        _same_as_oracle(res[k], g, B, f"default routing {k} {g.family}")


def test_batch_routing_size_does_not_change_results(ctx, large):
    """The same large instance solved by one workgroup (routing size above
    its slot count) and by the grid-wide kernels gives identical results."""
    import paper_1507_01926_amd as mf
    g, B = large[4]                                     # segmentation grid, 1.8M slots
    for route in (1 << 30, 1 << 16):
        res, _ = mf.batch_solve(ctx, [g], opts=[mf.options(batch_grid_slots=route)])
        _same_as_oracle(res[0], g, B, f"route {route}")


def test_server_large_requests_alone_and_in_mix(ctx, large):
    import paper_1507_01926_amd as mf
    small = [stream_instance(i, n_hi=2e4) for i in range(12)]
    srv = mf.Server(ctx, hbm_budget_bytes=24 << 30)
    try:
        tickets = []
        for k, (g, _) in enumerate(large):
            tickets.append(("L", k, srv.submit(g, mf.options(batch_grid_slots=ROUTE))))
            tickets.append(("S", 2 * k, srv.submit(small[2 * k])))
            tickets.append(("S", 2 * k + 1, srv.submit(small[2 * k + 1])))
        mix = {}
        for kind, k, t in tickets:
            mix[(kind, k)] = srv.wait(t, 600000)
        for k, (g, B) in enumerate(large):
            _same_as_oracle(mix[("L", k)], g, B, f"served large {k} {g.family}")
        for kind, k, _ in tickets:
            if kind == "S":
                g = small[k]
                _same_as_oracle(mix[(kind, k)], g, oracle.sync_maxflow(g), f"served small {k}")
        # alone: the same requests one at a time
        for k in (0, 3):
            g, _ = large[k]
            alone = srv.wait(srv.submit(g, mf.options(batch_grid_slots=ROUTE)), 600000)
            m = mix[("L", k)]
            assert alone["value"] == m["value"]
            assert (alone["flow"] == m["flow"]).all() and (alone["sink_side"] == m["sink_side"]).all()
        st = srv.stats()
        assert st["completed"] == len(tickets) + 2
    finally:
        srv.close()


def _changed_caps(g, rng, frac, raise_only=False):
    cap = g.cap.astype(np.int64).copy()
    idx = rng.choice(g.slots, size=max(1, int(frac * g.slots)), replace=False)
    delta = rng.integers(1, 41, size=idx.size)
    if not raise_only:
        delta = np.where(rng.random(idx.size) < 0.5, delta, -delta)
    cap[idx] = np.maximum(0, cap[idx] + delta)
    pair = cap + cap[g.rev]
    cap = np.where(pair >= 2 ** 31, g.cap, cap)
    return cap.astype(np.int32)


@pytest.mark.parametrize("name,f", [("c2", 4), ("c4a", 8), ("c3", 4)])
def test_served_resident_graph_resolves(ctx, name, f):
    import paper_1507_01926_amd as mf
    from workloads import Graph
    g0 = make_config(name, f)
    rng = np.random.default_rng(7)
    srv = mf.Server(ctx, hbm_budget_bytes=8 << 30)
    try:
        gid = srv.register_graph(g0)
        caps = [g0.cap, _changed_caps(g0, rng, 0.01, raise_only=True), _changed_caps(g0, rng, 0.01),
                _changed_caps(g0, rng, 0.1)]
        prev = None
        for step, cap in enumerate(caps):
            _note(f"resident {name}/{f} step {step}")
            g = Graph(n=g0.n, off=g0.off, head=g0.head, rev=g0.rev, cap=cap, s=g0.s, t=g0.t, m_arcs=g0.m_arcs)
            r = srv.wait(srv.submit_caps(gid, cap), 600000)
            assert r["status"] == 0
            A = oracle.fifo_maxflow(g, preflow_only=True)
            assert r["value"] == A["value"] and r["cut_capacity"] == A["value"]
            assert (r["sink_side"] == A["tstar"]).all()
            code, _, _ = oracle.check_certificate(g, r["flow"].astype(np.int64), r["sink_side"])
            assert code == 0, oracle.CERT_CODES[code]
            if step == 0:
                assert r["resumed"] == 0                  # no previous flow
            elif step == 1:
                assert r["resumed"] == 1                  # raises only: the old flow still fits
            else:
                fits = bool((prev["flow"] <= cap).all())
                assert r["resumed"] == int(fits)
            prev = r
        # a cut below the kept flow: not resumable, still the new graph's maximum
        cap = prev_cap = caps[-1].copy()
        a = int(np.argmax(prev["flow"]))
        cap[a] = max(0, int(prev["flow"][a]) - 1)
        g = Graph(n=g0.n, off=g0.off, head=g0.head, rev=g0.rev, cap=cap, s=g0.s, t=g0.t, m_arcs=g0.m_arcs)
        r = srv.wait(srv.submit_caps(gid, cap), 600000)
        assert r["resumed"] == 0
        assert r["value"] == oracle.fifo_maxflow(g, preflow_only=True)["value"]
        # invalid capacities complete with MF_EINVAL and leave the graph as it was
        bad = cap.copy()
        bad[0] = -1
        r = srv.wait(srv.submit_caps(gid, bad), 600000)
        assert r["status"] == mf.MF_EINVAL
        r = srv.wait(srv.submit_caps(gid, cap), 600000)
        assert r["status"] == 0 and r["resumed"] == 1    # unchanged capacities: the flow fits
        srv.release_graph(gid)
        with pytest.raises(mf.MaxflowError):
            srv.submit_caps(gid, cap)
        del prev_cap
    finally:
        srv.close()
