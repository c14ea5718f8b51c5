"""Python binding of the MI355X maximum-flow library (libmaxflow.so).

Argument marshalling only: every step of the solve runs in the HIP library.
The binding raises ``RuntimeError`` if the built library is missing; there is
no CPU fallback.  PyTorch, when used, only provides device buffers.

The functions carry the names of the C ABI (``include/maxflow.h``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmaxflow.so")

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_ETIMEOUT, MF_EAGAIN, MF_ECANCELED, MF_ENOTFOUND, \
    MF_EINVARIANT = range(9)
STATUS_NAMES = {0: "MF_OK", 1: "MF_EINVAL", 2: "MF_ENOMEM", 3: "MF_EDEVICE", 4: "MF_ETIMEOUT",
                5: "MF_EAGAIN", 6: "MF_ECANCELED", 7: "MF_ENOTFOUND", 8: "MF_EINVARIANT"}
MF_PREFLOW_ONLY = 0x1
MF_PROFILE = 0x2
MF_PERSISTENT = 0x4
MF_GRID_PATH = 0x8
MF_SIMPLE_ROUNDS = 0x10
MF_WARM_START = 0x20
MF_CHECK_INVARIANTS = 0x40
MF_GAP_RELABEL = 0x80
MF_BATCH_GRID_SLOTS = 2097152     # default routing size of the batched and served forms


class MaxflowError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class mf_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("slots", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("head", ctypes.c_void_p),
                ("rev", ctypes.c_void_p), ("cap", ctypes.c_void_p),
                ("s", ctypes.c_int32), ("t", ctypes.c_int32)]


class mf_options(ctypes.Structure):
    _fields_ = [("gr_freq_num", ctypes.c_int64), ("gr_freq_den", ctypes.c_int64),
                ("gr_alpha", ctypes.c_int64), ("gr_beta", ctypes.c_int64),
                ("gr_round_charge", ctypes.c_int64), ("gr_level_charge", ctypes.c_int64),
                ("max_rounds", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("lanes_per_vertex", ctypes.c_int32),
                ("lanes_per_merge", ctypes.c_int32), ("dense_threshold", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("lanes_per_bfs", ctypes.c_int32),
                ("profile_mask", ctypes.c_uint32), ("bfs_bottom_up_factor", ctypes.c_int32),
                ("profile_stride", ctypes.c_int32), ("check_fault_round", ctypes.c_int32),
                ("batch_grid_slots", ctypes.c_int32), ("block_round_max", ctypes.c_int32),
                ("grid_workers", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mf_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "value", "cut_capacity", "rounds", "global_relabels", "bfs_levels", "rounds2",
        "global_relabels2", "pushes", "relabels", "arc_scans", "work")] + [
        ("ms_preflow", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("ms_discharge", ctypes.c_double), ("ms_merge", ctypes.c_double),
        ("ms_global_relabel", ctypes.c_double)] + [(k, ctypes.c_int64) for k in (
        "discharge_launches", "merge_launches", "global_relabel_launches", "discharge_bytes",
        "merge_bytes", "global_relabel_bytes")] + [
        ("ms_phase_kernel", ctypes.c_double), ("phase_launches", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double * 12), ("kernel_launches", ctypes.c_int64 * 12),
        ("kernel_bytes", ctypes.c_int64 * 12), ("kernel_timed", ctypes.c_int64 * 12),
        ("gap_lifts", ctypes.c_int64), ("gap_lifts2", ctypes.c_int64)]

# kernel names of mf_stats.kernel_* in index order (mf_kernel_id)
KERNEL_NAMES = ("k_discharge_list", "k_discharge_dense", "k_merge_list", "k_merge_dense", "k_gr_td",
                "k_gr_hub", "k_gr_bu", "k_compact_flags", "k_discharge_hubs", "k_merge_hubs", "k_batch",
                "k_rounds_block")


class mf_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("lanes_per_vertex", ctypes.c_int32)] + [
        (k, ctypes.c_int64) for k in ("value", "cut_capacity", "rounds", "rounds2", "global_relabels",
                                      "global_relabels2", "bfs_levels", "pushes", "relabels")] + [
        ("ms_start", ctypes.c_double), ("ms_end", ctypes.c_double), ("ms_latency", ctypes.c_double),
        ("resumed", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mf_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("idle_ms", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("host_staging_mib", ctypes.c_int32), ("grid_workers", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class mf_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "canceled",
                                              "rejected", "inflight", "queued")] + [
        ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
        ("kernel_launches", ctypes.c_int64)]


_LIB = None

# (name, restype, argtypes) of every symbol include/maxflow.h declares
_P = ctypes.c_void_p
SIGNATURES = [
    ("mf_options_default", None, [_P]),
    ("mf_version", ctypes.c_char_p, []),
    ("mf_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("mf_last_error", ctypes.c_char_p, [_P]),
    ("mf_context_create", ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, _P]),
    ("mf_context_destroy", None, [_P]),
    ("mf_graph_upload", ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P]),
    ("mf_graph_free", None, [_P, _P]),
    ("mf_graph_set_caps", ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P]),
    ("mf_solve_uploaded", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    ("mf_solve", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    ("mf_solve_device", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    ("mf_solve_device_noalloc", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    ("mf_batch_solve", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P]),
    ("mf_server_create", ctypes.c_int, [_P, _P, _P]),
    ("mf_server_destroy", None, [_P]),
    ("mf_server_submit", ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    ("mf_server_poll", ctypes.c_int, [_P, ctypes.c_uint64, _P, _P, _P]),
    ("mf_server_wait", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int64, _P, _P, _P]),
    ("mf_server_cancel", ctypes.c_int, [_P, ctypes.c_uint64]),
    ("mf_server_get_stats", ctypes.c_int, [_P, _P]),
    ("mf_server_register_graph", ctypes.c_int, [_P, _P, _P]),
    ("mf_server_submit_caps", ctypes.c_int, [_P, ctypes.c_uint64, _P, _P, ctypes.c_int, _P]),
    ("mf_server_release_graph", ctypes.c_int, [_P, ctypes.c_uint64]),
]


def lib():
    """Load libmaxflow.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # A process must hold one HIP runtime.  PyTorch ships its own copy; if
        # it is importable, load it first so that libmaxflow.so binds to the
        # same runtime (same soname) and torch device buffers can be passed in.
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1507_01926_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def mf_version() -> str:
    return lib().mf_version().decode()


def options(**kw) -> mf_options:
    """mf_options with the paper's defaults, overridden by keyword."""
    o = mf_options()
    lib().mf_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "preflow_only":
            o.flags = (o.flags | MF_PREFLOW_ONLY) if v else (o.flags & ~MF_PREFLOW_ONLY)
        elif k == "profile":
            o.flags = (o.flags | MF_PROFILE) if v else (o.flags & ~MF_PROFILE)
        elif k == "persistent":
            o.flags = (o.flags | MF_PERSISTENT) if v else (o.flags & ~MF_PERSISTENT)
        elif k == "grid_path":
            o.flags = (o.flags | MF_GRID_PATH) if v else (o.flags & ~MF_GRID_PATH)
        elif k == "simple_rounds":
            o.flags = (o.flags | MF_SIMPLE_ROUNDS) if v else (o.flags & ~MF_SIMPLE_ROUNDS)
        elif k == "warm_start":
            o.flags = (o.flags | MF_WARM_START) if v else (o.flags & ~MF_WARM_START)
        elif k == "gap":
            o.flags = (o.flags | MF_GAP_RELABEL) if v else (o.flags & ~MF_GAP_RELABEL)
        elif k == "check_invariants":
            o.flags = (o.flags | MF_CHECK_INVARIANTS) if v else (o.flags & ~MF_CHECK_INVARIANTS)
        else:
            setattr(o, k, int(v))
    return o


def _stream(stream):
    """The HIP stream handle to order a call against: an explicit handle (int
    or torch stream), else torch's current stream, else the null stream."""
    if stream is None:
        try:
            import torch
            return int(torch.cuda.current_stream().cuda_stream) or None
        except Exception:
            return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream) or None
    return int(stream) or None


def _stats_dict(s: mf_stats) -> dict:
    d = {}
    for k, _ in mf_stats._fields_:
        v = getattr(s, k)
        d[k] = list(v) if k.startswith("kernel_") else v
    return d


class _HostGraph:
    """ctypes view of a host graph (numpy arrays kept alive)."""

    def __init__(self, g):
        self.off = np.ascontiguousarray(g.off, dtype=np.int64)
        self.head = np.ascontiguousarray(g.head, dtype=np.int32)
        self.rev = np.ascontiguousarray(g.rev, dtype=np.int64)
        self.cap = np.ascontiguousarray(g.cap, dtype=np.int32)
        self.st = mf_graph(int(g.n), int(self.head.shape[0]), self.off.ctypes.data,
                           self.head.ctypes.data, self.rev.ctypes.data, self.cap.ctypes.data,
                           int(g.s), int(g.t))


class Context:
    """An mf_context: one device, one HIP stream, an optional HBM budget."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        st = lib().mf_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h))
        if st != MF_OK:
            raise MaxflowError(st, lib().mf_last_error(None).decode())
        self.h = h

    def close(self):
        if self.h:
            lib().mf_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st not in (MF_OK,):
            raise MaxflowError(st, lib().mf_last_error(self.h).decode())

    # -- mf_solve: host buffers in, host buffers out -----------------------
    def solve(self, g, opt: mf_options | None = None, want_flow=True, want_side=True,
              allow_timeout=False) -> dict:
        hg = _HostGraph(g)
        opt = opt or options()
        if opt.flags & MF_PREFLOW_ONLY:
            want_flow = False
        flow = np.zeros(max(1, hg.head.shape[0]), dtype=np.int32) if want_flow else None
        side = np.zeros(g.n, dtype=np.uint8) if want_side else None
        val = ctypes.c_int64(0)
        stats = mf_stats()
        st = lib().mf_solve(self.h, ctypes.byref(hg.st), ctypes.byref(opt), ctypes.byref(val),
                            None if flow is None else flow.ctypes.data,
                            None if side is None else side.ctypes.data, ctypes.byref(stats))
        if not (allow_timeout and st == MF_ETIMEOUT):
            self._check(st)
        out = _stats_dict(stats)
        out.update(status=st, value=int(val.value), sink_side=side,
                   flow=None if flow is None else flow[: hg.head.shape[0]])
        return out

    # -- upload once, solve many times (device-resident graph) -------------
    def upload(self, g) -> "DeviceGraph":
        hg = _HostGraph(g)
        h = ctypes.c_void_p()
        self._check(lib().mf_graph_upload(self.h, ctypes.byref(hg.st), 0, None, ctypes.byref(h)))
        return DeviceGraph(self, h, g.n, hg.head.shape[0])

    def upload_device(self, off, head, rev, cap, s, t, stream=None) -> "DeviceGraph":
        """Graph arrays given as device pointers (e.g. torch tensors on cuda),
        read in the order of `stream` (default: torch's current stream)."""
        n = int(off.numel()) - 1
        S = int(head.numel())
        gst = mf_graph(n, S, off.data_ptr(), head.data_ptr(), rev.data_ptr(), cap.data_ptr(),
                       int(s), int(t))
        h = ctypes.c_void_p()
        self._check(lib().mf_graph_upload(self.h, ctypes.byref(gst), 1, _stream(stream), ctypes.byref(h)))
        return DeviceGraph(self, h, n, S)

    def solve_device(self, off, head, rev, cap, s, t, flow=None, side=None,
                     opt: mf_options | None = None, stream=None, allow_status=()) -> dict:
        """mf_solve_device: inputs and outputs are device buffers (torch tensors),
        ordered against `stream` (default: torch's current stream)."""
        n = int(off.numel()) - 1
        S = int(head.numel())
        gst = mf_graph(n, S, off.data_ptr(), head.data_ptr(), rev.data_ptr(), cap.data_ptr(),
                       int(s), int(t))
        val = ctypes.c_int64(0)
        stats = mf_stats()
        st = lib().mf_solve_device(self.h, ctypes.byref(gst), _stream(stream), ctypes.byref(opt or options()),
                                   ctypes.byref(val), None if flow is None else flow.data_ptr(),
                                   None if side is None else side.data_ptr(), ctypes.byref(stats))
        if st not in allow_status:
            self._check(st)
        out = _stats_dict(stats)
        out.update(status=st, value=int(val.value))
        return out

    def solve_device_noalloc(self, off, head, rev, cap, s, t, flow=None, side=None,
                             opt: mf_options | None = None, stream=None, allow_status=()) -> dict:
        """mf_solve_device_noalloc: as solve_device, with no device allocation
        (per-solve buffers in the library's fixed scratch array)."""
        n = int(off.numel()) - 1
        S = int(head.numel())
        gst = mf_graph(n, S, off.data_ptr(), head.data_ptr(), rev.data_ptr(), cap.data_ptr(),
                       int(s), int(t))
        val = ctypes.c_int64(0)
        stats = mf_stats()
        st = lib().mf_solve_device_noalloc(self.h, ctypes.byref(gst), _stream(stream),
                                           ctypes.byref(opt or options()), ctypes.byref(val),
                                           None if flow is None else flow.data_ptr(),
                                           None if side is None else side.data_ptr(), ctypes.byref(stats))
        if st not in allow_status:
            self._check(st)
        out = _stats_dict(stats)
        out.update(status=st, value=int(val.value))
        return out


def _result_dict(r: mf_result) -> dict:
    return {k: getattr(r, k) for k, _ in mf_result._fields_}


def batch_solve(ctx: "Context", graphs, opts=None, want_flow=True, want_side=True):
    """mf_batch_solve over host graphs; opts: None or one mf_options per graph."""
    k = len(graphs)
    hgs = [_HostGraph(g) for g in graphs]
    garr = (mf_graph * k)(*[h.st for h in hgs])
    oarr = None
    if opts is not None:
        oarr = (mf_options * k)(*opts)
    flows = [np.zeros(max(1, h.head.shape[0]), dtype=np.int32) if want_flow else None for h in hgs]
    if opts is not None:
        flows = [None if (o.flags & MF_PREFLOW_ONLY) else f for f, o in zip(flows, opts)]
    sides = [np.zeros(g.n, dtype=np.uint8) if want_side else None for g in graphs]
    fptrs = (ctypes.c_void_p * k)(*[None if f is None else f.ctypes.data for f in flows])
    sptrs = (ctypes.c_void_p * k)(*[None if x is None else x.ctypes.data for x in sides])
    res = (mf_result * k)()
    stats = mf_stats()
    st = lib().mf_batch_solve(ctx.h, k, garr, oarr, fptrs, sptrs, res, ctypes.byref(stats))
    ctx._check(st)
    out = []
    for i in range(k):
        d = _result_dict(res[i])
        d["flow"] = None if flows[i] is None else flows[i][: hgs[i].head.shape[0]]
        d["sink_side"] = sides[i]
        out.append(d)
    return out, stats.ms_total


class DeviceGraph:
    """An mf_dgraph: a validated graph resident in the context's device memory."""

    def __init__(self, ctx: Context, h, n: int, slots: int):
        self.ctx, self.h, self.n, self.slots = ctx, h, n, slots

    def free(self):
        if self.h and self.ctx.h:
            lib().mf_graph_free(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_caps(self, cap) -> bool:
        """mf_graph_set_caps from a host array of int32[slots]; returns whether
        the next solve can resume from the kept flow (MF_WARM_START)."""
        c = np.ascontiguousarray(cap, dtype=np.int32)
        if c.shape[0] != self.slots:
            raise ValueError("cap must have one entry per slot")
        res = ctypes.c_int(0)
        self.ctx._check(lib().mf_graph_set_caps(self.ctx.h, self.h, c.ctypes.data, 0, None, ctypes.byref(res)))
        return bool(res.value)

    def solve(self, opt: mf_options | None = None, flow_ptr=None, side_ptr=None,
              allow_timeout=False, stream=None, allow_status=()) -> dict:
        """mf_solve_uploaded; flow_ptr / side_ptr are device addresses or None,
        written in the order of `stream` (default: torch's current stream)."""
        val = ctypes.c_int64(0)
        stats = mf_stats()
        st = lib().mf_solve_uploaded(self.ctx.h, self.h, _stream(stream), ctypes.byref(opt or options()),
                                     ctypes.byref(val), flow_ptr, side_ptr, ctypes.byref(stats))
        if not (allow_timeout and st == MF_ETIMEOUT) and st not in allow_status:
            self.ctx._check(st)
        out = _stats_dict(stats)
        out.update(status=st, value=int(val.value))
        return out


class Server:
    """An mf_server: admission by HBM budget, continuous batching, latency per request."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_inflight: int = 0, idle_ms: int = 0,
                 blocks_per_cu: int = 0, host_staging_mib: int = 0, grid_workers: int = 0):
        cfg = mf_server_config(int(hbm_budget_bytes), int(max_inflight), int(idle_ms), int(blocks_per_cu),
                               int(host_staging_mib), int(grid_workers))
        h = ctypes.c_void_p()
        ctx._check(lib().mf_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.ctx, self.h = ctx, h
        self._shapes = {}

    def close(self):
        if self.h:
            lib().mf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, g, opt: mf_options | None = None, want_flow: bool = True) -> int:
        hg = _HostGraph(g)
        t = ctypes.c_uint64()
        st = lib().mf_server_submit(self.h, ctypes.byref(hg.st), None if opt is None else ctypes.byref(opt),
                                    int(want_flow), ctypes.byref(t))
        if st != MF_OK:
            raise MaxflowError(st, "submit failed")
        self._shapes[t.value] = (g.n, hg.head.shape[0], want_flow)
        return t.value

    def _collect(self, fn, ticket, *extra):
        if ticket not in self._shapes:
            st = fn(self.h, ctypes.c_uint64(ticket), *extra, None, None, None)
            raise MaxflowError(st, "unknown ticket")
        n, S, wf = self._shapes[ticket]
        res = mf_result()
        flow = np.zeros(max(1, S), dtype=np.int32) if wf else None
        side = np.zeros(n, dtype=np.uint8)
        st = fn(self.h, ctypes.c_uint64(ticket), *extra, ctypes.byref(res),
                None if flow is None else flow.ctypes.data, side.ctypes.data)
        if st == MF_EAGAIN:
            return None
        if st != MF_OK:
            raise MaxflowError(st, "poll failed")
        del self._shapes[ticket]
        d = _result_dict(res)
        d["flow"] = None if flow is None else flow[:S]
        d["sink_side"] = side
        return d

    def register_graph(self, g) -> int:
        """mf_server_register_graph: keep `g` resident for re-solves with new capacities."""
        hg = _HostGraph(g)
        gid = ctypes.c_uint64()
        st = lib().mf_server_register_graph(self.h, ctypes.byref(hg.st), ctypes.byref(gid))
        if st != MF_OK:
            raise MaxflowError(st, "register failed")
        self._graphs = getattr(self, "_graphs", {})
        self._graphs[gid.value] = (g.n, hg.head.shape[0])
        return gid.value

    def submit_caps(self, graph_id: int, cap, opt: mf_options | None = None, want_flow: bool = True) -> int:
        """mf_server_submit_caps: re-solve a resident graph with capacities `cap` (int32[slots])."""
        n, S = self._graphs[graph_id]
        c = np.ascontiguousarray(cap, dtype=np.int32)
        if c.shape[0] != S:
            raise ValueError("cap must have one entry per slot")
        t = ctypes.c_uint64()
        st = lib().mf_server_submit_caps(self.h, ctypes.c_uint64(graph_id), c.ctypes.data,
                                         None if opt is None else ctypes.byref(opt), int(want_flow), ctypes.byref(t))
        if st != MF_OK:
            raise MaxflowError(st, "submit_caps failed")
        self._shapes[t.value] = (n, S, want_flow)
        return t.value

    def release_graph(self, graph_id: int):
        st = lib().mf_server_release_graph(self.h, ctypes.c_uint64(graph_id))
        if st != MF_OK:
            raise MaxflowError(st, "release failed")

    def poll(self, ticket: int):
        return self._collect(lib().mf_server_poll, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        return self._collect(lib().mf_server_wait, ticket, ctypes.c_int64(timeout_ms))

    def cancel(self, ticket: int):
        st = lib().mf_server_cancel(self.h, ctypes.c_uint64(ticket))
        if st != MF_OK:
            raise MaxflowError(st, "cancel failed")

    def stats(self) -> dict:
        s = mf_server_stats()
        lib().mf_server_get_stats(self.h, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in mf_server_stats._fields_}
