"""CPU oracle for the maximum-flow library.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library and never imports it.

* ``fifo_maxflow``  oracle A: sequential FIFO push-relabel (Sec. 2.1) with
  global relabeling every ~12n+2m units of relabel work (Sec. 3), int64.
* ``sync_maxflow``  oracle B: the paper's synchronous rounds (Sec. 3.1)
  with global relabeling by a breadth-first search from the sink (Sec. 2.1,
  Sec. 3), executed sequentially; each round is a function of its start
  state.
* ``check_certificate``  max-flow / min-cut certificate (Sec. 2, Eq. 1-2).
* ``brute_mincut`` (in ``brute``)  enumeration of every s-t cut.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _OgGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("off", ctypes.c_void_p), ("head", ctypes.c_void_p),
                ("rev", ctypes.c_void_p), ("cap", ctypes.c_void_p),
                ("s", ctypes.c_int64), ("t", ctypes.c_int64)]


class _OgSched(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "freq_num", "freq_den", "alpha", "beta", "round_charge", "literal_termination",
        "level_charge", "simple", "gap")]


PAPER_SCHEDULE = dict(freq_num=1, freq_den=2, alpha=6, beta=12, round_charge=0,
                      literal_termination=0, level_charge=0, simple=0, gap=0)


class _OgResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "value", "cut_tstar", "cut_smin", "pushes", "relabels", "global_relabels", "rounds",
        "pushes2", "relabels2", "global_relabels2", "rounds2", "work", "bfs_levels",
        "gap_lifts", "gap_lifts2")]


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE_LIB lets the mutation tests load a deliberately broken copy
        path = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.og_validate.argtypes = [P]
        L.og_validate.restype = ctypes.c_int
        L.og_fifo_maxflow.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.og_fifo_maxflow.restype = ctypes.c_int
        L.og_sync_maxflow.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P]
        L.og_sync_maxflow.restype = ctypes.c_int
        L.og_check_certificate.argtypes = [P, P, P, ctypes.c_int, P, P]
        L.og_check_certificate.restype = ctypes.c_int
        L.og_residual_distance.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, P]
        L.og_residual_distance.restype = None
        _LIB = L
    return _LIB


class _Bound:
    """ctypes view of a graph; keeps the contiguous arrays alive."""

    def __init__(self, g):
        self.off = np.ascontiguousarray(g.off, dtype=np.int64)
        self.head = np.ascontiguousarray(g.head, dtype=np.int32)
        self.rev = np.ascontiguousarray(g.rev, dtype=np.int64)
        self.cap = np.ascontiguousarray(g.cap, dtype=np.int32)
        self.st = _OgGraph(int(g.n), int(self.head.shape[0]), self.off.ctypes.data,
                           self.head.ctypes.data, self.rev.ctypes.data, self.cap.ctypes.data,
                           int(g.s), int(g.t))

    @property
    def ptr(self):
        return ctypes.addressof(self.st)


def _ptr(a):
    return None if a is None else a.ctypes.data


def validate(g) -> int:
    b = _Bound(g)
    return int(lib().og_validate(b.ptr))


def _stats(r: _OgResult) -> dict:
    return {k: int(getattr(r, k)) for k, _ in _OgResult._fields_}


def fifo_maxflow(g, preflow_only: bool = False) -> dict:
    """Oracle A.  Returns value, cut capacities, residuals, T*, S_min, counters."""
    b = _Bound(g)
    res = np.zeros(max(1, b.head.shape[0]), dtype=np.int64)
    tstar = np.zeros(g.n, dtype=np.uint8)
    smin = np.zeros(g.n, dtype=np.uint8)
    r = _OgResult()
    rc = lib().og_fifo_maxflow(b.ptr, int(preflow_only), _ptr(res), _ptr(tstar), _ptr(smin),
                               ctypes.addressof(r))
    if rc < 0:
        raise ValueError(f"oracle rejected the graph (code {rc})")
    out = _stats(r)
    out.update(res=res[: b.head.shape[0]], tstar=tstar, smin=None if preflow_only else smin,
               flow=b.cap.astype(np.int64) - res[: b.head.shape[0]])
    return out


def sync_maxflow(g, preflow_only: bool = False, max_rounds: int = 0, schedule=None) -> dict:
    """Oracle B.  Returns value, cut capacity, residuals, labels, excesses, T*, counters.

    ``schedule`` overrides entries of ``PAPER_SCHEDULE`` (the global-relabel
    rule and the termination reading)."""
    b = _Bound(g)
    sc = dict(PAPER_SCHEDULE)
    sc.update(schedule or {})
    sched = _OgSched(**{k: int(v) for k, v in sc.items()})
    S = b.head.shape[0]
    res = np.zeros(max(1, S), dtype=np.int64)
    d = np.zeros(g.n, dtype=np.int64)
    e = np.zeros(g.n, dtype=np.int64)
    tstar = np.zeros(g.n, dtype=np.uint8)
    r = _OgResult()
    rc = lib().og_sync_maxflow(b.ptr, int(preflow_only), int(max_rounds), ctypes.addressof(sched),
                               _ptr(res), _ptr(d), _ptr(e), _ptr(tstar), ctypes.addressof(r))
    if rc < 0:
        raise ValueError(f"oracle rejected the graph (code {rc})")
    out = _stats(r)
    out.update(res=res[:S], d=d, e=e, tstar=tstar, stopped=bool(rc == 1),
               flow=b.cap.astype(np.int64) - res[:S])
    return out


CERT_CODES = {0: "ok", 1: "antisymmetry", 2: "capacity", 3: "conservation", 4: "value",
              5: "side", 6: "cut", 7: "reachability"}


def check_certificate(g, flow, side, reach_check: bool = True):
    """(code, value, cut): code 0 means flow is a maximum flow and side a minimum cut."""
    b = _Bound(g)
    f = np.ascontiguousarray(flow, dtype=np.int64)
    sd = np.ascontiguousarray(side, dtype=np.uint8)
    val = ctypes.c_int64(0)
    cut = ctypes.c_int64(0)
    rc = lib().og_check_certificate(b.ptr, _ptr(f), _ptr(sd), int(reach_check),
                                    ctypes.addressof(val), ctypes.addressof(cut))
    return int(rc), int(val.value), int(cut.value)


def residual_distance(g, res, target: int, blocked: int = -1):
    """Exact BFS distance to ``target`` over residual arcs; unreachable = n."""
    b = _Bound(g)
    r = np.ascontiguousarray(res, dtype=np.int64)
    dist = np.zeros(g.n, dtype=np.int64)
    lib().og_residual_distance(b.ptr, _ptr(r), int(target), int(blocked), _ptr(dist))
    return dist
