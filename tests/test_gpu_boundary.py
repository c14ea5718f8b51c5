"""The boundary's stream ordering and its invariant-check mode, through the
C ABI.  Needs a GPU.

* mf_solve_device / mf_graph_upload / mf_solve_uploaded take the caller's
  stream: a torch kernel on a non-default stream that is still writing the
  capacities when the call is made must finish first, with no device-wide
  synchronize in between; the results equal oracle B's bit for bit.
* MF_CHECK_INVARIANTS checks the state after every round and every global
  relabel (Eq. 1-2, the preflow's excesses, terminal labels, label validity
  after a relabel); it passes on every family, leaves the results unchanged,
  and stops a solve whose state the test hook breaks from the host.
"""
import sys

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


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _slow_producer(dev, stream, cap_true):
    """On `stream`: keep the GPU busy for a while (a chain of matrix
    products), then write the real capacities into a tensor that holds
    zeros until then."""
    import torch
    with torch.cuda.stream(stream):
        cap = torch.zeros(cap_true.shape[0], dtype=torch.int32, device=dev)
        x = torch.randn(2048, 2048, device=dev, dtype=torch.float32)
        for _ in range(12):
            x = torch.tanh(x @ x)
        src = torch.from_numpy(cap_true).to(dev, non_blocking=False)
        # the write depends on x, so it cannot start before the products end
        cap.copy_(src + (x[0, 0] * 0).to(torch.int32))
    return cap


def test_solve_device_ordered_after_caller_stream(ctx):
    import torch
    g = make_config("c2", 16)
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.off).to(dev)
    head = torch.from_numpy(g.head).to(dev)
    rev = torch.from_numpy(g.rev).to(dev)
    torch.cuda.synchronize()
    side_stream = torch.cuda.Stream()
    cap = _slow_producer(dev, side_stream, g.cap)
    with torch.cuda.stream(side_stream):
        flow = torch.empty(g.slots, dtype=torch.int32, device=dev)
        side = torch.empty(g.n, dtype=torch.uint8, device=dev)
        flow.fill_(-7)
        # no synchronize: the call must wait for the products and the copy
        r = ctx.solve_device(off, head, rev, cap, g.s, g.t, flow=flow, side=side, stream=side_stream)
        f_host = flow.to("cpu", non_blocking=False)
        s_host = side.to("cpu", non_blocking=False)
    B = oracle.sync_maxflow(g)
    assert r["value"] == B["value"]
    assert (f_host.numpy().astype(np.int64) == B["flow"]).all()
    assert (s_host.numpy() == B["tstar"]).all()
    assert r["rounds"] == B["rounds"] and r["pushes"] == B["pushes"]


def test_upload_and_solve_uploaded_ordered_after_caller_stream(ctx):
    import torch
    import paper_1507_01926_amd as mf
    g = make_config("c4a", 32)
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.off).to(dev)
    head = torch.from_numpy(g.head).to(dev)
    rev = torch.from_numpy(g.rev).to(dev)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    cap = _slow_producer(dev, st, g.cap)
    dg = ctx.upload_device(off, head, rev, cap, g.s, g.t, stream=st)
    with torch.cuda.stream(st):
        flow = torch.full((g.slots,), -3, dtype=torch.int32, device=dev)
        side = torch.zeros(g.n, dtype=torch.uint8, device=dev)
    r = dg.solve(mf.options(grid_path=True), flow.data_ptr(), side.data_ptr(), stream=st)
    with torch.cuda.stream(st):
        f_host = flow.to("cpu")
    B = oracle.sync_maxflow(g)
    assert r["value"] == B["value"]
    assert (f_host.numpy().astype(np.int64) == B["flow"]).all()
    dg.free()


@pytest.mark.parametrize("name,f", [("c1", 1), ("c2", 16), ("c3", 8), ("c4a", 32), ("c4b", 16)])
def test_check_invariants_families(ctx, name, f):
    import paper_1507_01926_amd as mf
    g = make_config(name, f)
    _note(f"check invariants {name}/{f}")
    r = ctx.solve(g, mf.options(check_invariants=True))
    B = oracle.sync_maxflow(g)
    assert r["value"] == B["value"]
    assert (r["flow"].astype(np.int64) == B["flow"]).all()
    assert (r["sink_side"] == B["tstar"]).all()
    assert r["rounds"] == B["rounds"] and r["rounds2"] == B["rounds2"]
    assert r["global_relabels"] == B["global_relabels"]


def test_check_invariants_random_and_simple(ctx):
    import paper_1507_01926_amd as mf
    for seed in range(40):
        n = 4 + seed % 30
        g = random_graph(n, 3 * n, seed)
        simple = seed % 2 == 1
        r = ctx.solve(g, mf.options(check_invariants=True, simple_rounds=simple))
        B = oracle.sync_maxflow(g, schedule=dict(simple=int(simple)))
        assert r["value"] == B["value"], seed
        assert (r["flow"].astype(np.int64) == B["flow"]).all(), seed


@pytest.mark.parametrize("fault_round", [1, 3])
def test_check_invariants_stops_a_broken_state(ctx, fault_round):
    """The test hook raises one residual by 1 after `fault_round` rounds of
    phase 1 (from the host, between rounds); the next check must stop the
    solve with MF_EINVARIANT and name the broken pair sum."""
    import paper_1507_01926_amd as mf
    g = make_config("c2", 16)
    with pytest.raises(mf.MaxflowError) as ei:
        ctx.solve(g, mf.options(check_invariants=True, check_fault_round=fault_round))
    assert ei.value.status == mf.MF_EINVARIANT
    assert "res[a] + res[rev a]" in str(ei.value)
    # the context stays usable
    assert ctx.solve(g)["value"] == oracle.fifo_maxflow(g, preflow_only=True)["value"]
