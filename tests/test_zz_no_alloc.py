"""mf_solve_device_noalloc (the entry point that allocates nothing: its
per-solve buffers live in the library's fixed scratch array) against
mf_solve_device on the same inputs, bit for bit, on two calls in a row, the
second with a smaller graph; plus the size limit.  Needs a GPU."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_config, random_graph

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(g):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(g.off).to(dev), torch.from_numpy(g.head).to(dev),
            torch.from_numpy(g.rev).to(dev), torch.from_numpy(g.cap).to(dev))


def _both(ctx, g, **kw):
    import torch
    import paper_1507_01926_amd as mf
    off, head, rev, cap = _dev(g)
    dev = off.device
    f1 = torch.full((max(1, g.slots),), -5, dtype=torch.int32, device=dev)
    s1 = torch.full((g.n,), 9, dtype=torch.uint8, device=dev)
    f2 = torch.full((max(1, g.slots),), -6, dtype=torch.int32, device=dev)
    s2 = torch.full((g.n,), 8, dtype=torch.uint8, device=dev)
    opt = mf.options(**kw)
    if kw.get("preflow_only"):
        f1 = f2 = None           # no flow without phase 2
    a = ctx.solve_device(off, head, rev, cap, g.s, g.t, flow=f1, side=s1, opt=opt)
    b = ctx.solve_device_noalloc(off, head, rev, cap, g.s, g.t, flow=f2, side=s2, opt=opt)
    for k in ("value", "cut_capacity", "rounds", "rounds2", "pushes", "relabels", "global_relabels",
              "bfs_levels"):
        assert a[k] == b[k], k
    if f1 is not None:
        assert torch.equal(f1, f2)
    assert torch.equal(s1, s2)
    return b, None if f2 is None else f2.cpu().numpy(), s2.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    import paper_1507_01926_amd as mf
    c = mf.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("big,small", [(("c2", 4), ("c1", 1)), (("c3", 4), ("c4a", 8)),
                                       (("c4b", 8), ("rand", 40))])
def test_noalloc_matches_solve_device_twice(ctx, big, small):
    for name, f in (big, small):
        g = random_graph(f, 3 * f, 11) if name == "rand" else make_config(name, f)
        _note(f"noalloc {name}/{f} n={g.n} slots={g.slots}")
        r, flow, side = _both(ctx, g)
        B = oracle.sync_maxflow(g)
        assert r["value"] == B["value"]
        assert (flow[: g.slots].astype(np.int64) == B["flow"]).all()
        assert (side == B["tstar"]).all()


def test_noalloc_simple_rounds_and_preflow(ctx):
    g = make_config("c2", 32)
    _both(ctx, g, simple_rounds=True)
    _both(ctx, g, preflow_only=True)


def test_noalloc_rejects_oversize_and_bad_graphs(ctx):
    import torch
    import paper_1507_01926_amd as mf
    g = make_config("c2", 2)            # 10.5M slots, 1M vertices: beyond the fixed scratch
    off, head, rev, cap = _dev(g)
    with pytest.raises(mf.MaxflowError) as ei:
        ctx.solve_device_noalloc(off, head, rev, cap, g.s, g.t)
    assert ei.value.status == mf.MF_ENOMEM
    small = make_config("c1")
    off, head, rev, cap = _dev(small)
    bad = cap.clone()
    bad[3] = -1
    with pytest.raises(mf.MaxflowError) as ei:
        ctx.solve_device_noalloc(off, head, rev, bad, small.s, small.t)
    assert ei.value.status == mf.MF_EINVAL
    r, _, _ = _both(ctx, small)          # still usable afterwards
    assert r["value"] == oracle.fifo_maxflow(small, preflow_only=True)["value"]
