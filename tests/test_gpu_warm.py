"""Re-solving an uploaded graph whose capacities change (mf_graph_set_caps)
from the flow the last solve left on the device (MF_WARM_START).  Value, cut
and sink side must be the oracle's for the new graph, and the flow must pass
the certificate (valid flow, no residual s-t path, cut = value).  Needs a
GPU."""
import copy

import numpy as np
import pytest

import oracle
from workloads import make_config, random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


def _solve(dg, g, **kw):
    import torch
    import paper_1507_01926_amd as mf
    flow = torch.empty(max(1, g.slots), dtype=torch.int32, device="cuda:0")
    side = torch.empty(g.n, dtype=torch.uint8, device="cuda:0")
    r = dg.solve(mf.options(grid_path=True, **kw), flow.data_ptr(), side.data_ptr())
    torch.cuda.synchronize()
    return r, flow.cpu().numpy()[: g.slots].astype(np.int64), side.cpu().numpy()


def _with_caps(g, cap):
    g2 = copy.copy(g)
    g2.cap = np.ascontiguousarray(cap, dtype=np.int32)
    return g2


def _check(g, r, flow, side):
    A = oracle.fifo_maxflow(g, preflow_only=True)
    assert r["value"] == A["value"] and r["cut_capacity"] == A["value"]
    assert (side == A["tstar"]).all()
    code, val, cut = oracle.check_certificate(g, flow, side)
    assert code == 0, oracle.CERT_CODES[code]
    assert val == cut == A["value"]


def _graphs():
    return [("c1", make_config("c1")), ("c2/16", make_config("c2", 16)), ("c3/8", make_config("c3", 8)),
            ("c4a/32", make_config("c4a", 32)), ("c4b/16", make_config("c4b", 16)),
            ("random", random_graph(300, 1500, 7, cap_max=50))]


@pytest.mark.parametrize("idx", range(6))
def test_warm_resolve_after_changes(ctx, idx):
    """Three rounds of changes, each followed by a resumed solve: raises on a
    random fifth of the slots, then cuts that keep every flow within its new
    capacity, then raises again."""
    import paper_1507_01926_amd as mf
    name, g = _graphs()[idx]
    print(f"warm {name} n={g.n} slots={g.slots}", flush=True)
    rng = np.random.default_rng(1000 + idx)
    dg = ctx.upload(g)
    other = mf.Context(0)          # cold solves for comparison, on their own workspace
    try:
        r, flow, side = _solve(dg, g)
        _check(g, r, flow, side)
        cap = g.cap.astype(np.int64)
        for step in range(3):
            pick = rng.random(g.slots) < 0.2
            if step == 1:
                # lower capacities, never below the slot's flow
                lower = np.maximum(np.maximum(flow, 0), cap - rng.integers(0, 40, g.slots))
                cap = np.where(pick, lower, cap)
            else:
                cap = np.where(pick, cap + rng.integers(0, 40, g.slots), cap)
            g2 = _with_caps(g, cap)
            assert dg.set_caps(g2.cap) is True
            r, flow, side = _solve(dg, g2, warm_start=True)
            _check(g2, r, flow, side)
            cold = other.solve(g2)
            assert cold["value"] == r["value"] and (cold["sink_side"] == side).all()
    finally:
        dg.free()
        other.close()


def test_cut_below_flow_is_not_resumable(ctx):
    import paper_1507_01926_amd as mf
    g = make_config("c2", 16)
    dg = ctx.upload(g)
    try:
        r, flow, side = _solve(dg, g)
        a = int(np.flatnonzero(flow > 0)[0])
        cap = g.cap.astype(np.int64).copy()
        cap[a] = flow[a] - 1
        g2 = _with_caps(g, cap)
        assert dg.set_caps(g2.cap) is False
        with pytest.raises(mf.MaxflowError):
            dg.solve(mf.options(warm_start=True))
        r, flow, side = _solve(dg, g2)               # from zero flow
        _check(g2, r, flow, side)
    finally:
        dg.free()


def test_warm_start_needs_the_last_solve_of_this_graph(ctx):
    import paper_1507_01926_amd as mf
    g, h = make_config("c2", 16), make_config("c3", 8)
    dg, dh = ctx.upload(g), ctx.upload(h)
    try:
        with pytest.raises(mf.MaxflowError):          # no solve yet
            dg.solve(mf.options(warm_start=True))
        _solve(dg, g)
        _solve(dh, h)                                  # another graph used the workspace
        assert dg.set_caps(g.cap) is False
        with pytest.raises(mf.MaxflowError):
            dg.solve(mf.options(warm_start=True))
        _solve(dg, g)
        assert dg.set_caps(g.cap) is True              # unchanged capacities: resumable
        r, flow, side = _solve(dg, g, warm_start=True)
        _check(g, r, flow, side)
    finally:
        dg.free()
        dh.free()


def test_invalid_capacities_leave_the_graph_unchanged(ctx):
    import paper_1507_01926_amd as mf
    g = make_config("c2", 16)
    dg = ctx.upload(g)
    try:
        r0, _, _ = _solve(dg, g)
        bad = g.cap.astype(np.int64).copy()
        bad[3] = -1
        with pytest.raises(mf.MaxflowError):
            dg.set_caps(bad)
        r1, flow, side = _solve(dg, g)
        assert r1["value"] == r0["value"]
        _check(g, r1, flow, side)
    finally:
        dg.free()
