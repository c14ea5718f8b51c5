"""Property-based pins of both oracles on arbitrary small graphs (CPU).

Hypothesis draws graphs of 2-9 vertices with any arc list: parallel and
antiparallel arcs, zero capacities, arcs into s and out of t, a direct s-t
arc, t unreachable.  For each, the value of oracle A (sequential FIFO) and
oracle B (the synchronous rounds, with and without the gap rule, and the
simple rounds) equals the brute-force minimum cut over all s-t cuts (Sec. 2,
max-flow = min-cut), T* equals the intersection of the sink sides of all
minimum cuts, and every flow passes the certificate (Eq. (1)-(2), no
residual s-t path, cut capacity = value)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle.brute import brute_mincut
from workloads import from_pairs


@st.composite
def small_graphs(draw):
    n = draw(st.integers(2, 9))
    m = draw(st.integers(0, 24))
    arcs = []
    for _ in range(m):
        u = draw(st.integers(0, n - 1))
        v = draw(st.integers(0, n - 1).filter(lambda x, u=u: x != u))
        c = draw(st.one_of(st.just(0), st.integers(1, 25)))
        arcs.append((u, v, c))
    # s = 0, t = n - 1
    if arcs:
        U, V, C = (np.array(x) for x in zip(*arcs))
    else:
        U = V = C = np.zeros(0, dtype=np.int64)
    return from_pairs(n, U, V, C, np.zeros(len(C), dtype=np.int64), 0, n - 1, m_arcs=int(np.count_nonzero(C)))


def _check(g, r, best, tstar):
    assert r["value"] == best
    assert (r["tstar"] == tstar).all()
    code, val, cut = oracle.check_certificate(g, r["flow"], r["tstar"])
    assert code == 0, oracle.CERT_CODES[code]
    assert val == best and cut == best


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.filter_too_much])
@given(small_graphs())
def test_oracles_equal_brute_force(g):
    assert oracle.validate(g) == 0
    best, tstar, _ = brute_mincut(g)
    _check(g, oracle.fifo_maxflow(g), best, tstar)
    _check(g, oracle.sync_maxflow(g), best, tstar)
    _check(g, oracle.sync_maxflow(g, schedule=dict(gap=1)), best, tstar)
    _check(g, oracle.sync_maxflow(g, schedule=dict(simple=1)), best, tstar)
    _check(g, oracle.sync_maxflow(g, schedule=dict(round_charge=10 ** 15)), best, tstar)
