#!/usr/bin/env python3
"""Benchmark of the MI355X maximum-flow library.

A step is one complete solve of one instance (source saturation, synchronous
push-relabel rounds with global relabels up to the maximum preflow, flow
reconstruction, value, per-slot flow and sink side), with the graph already
resident in HBM (uploaded and validated before the timed region, as the
paper excludes data-structure initialisation).

Default workload: the largest single-GPU configuration, the 256^3
6-connected grid (16,777,218 vertices, 100,401,152 arcs).  Prints one JSON
line.  The 2048x2048 segmentation grid is timed too and reported beside it.

The global-relabel schedule (the relabel frequency of Sec. 3's work rule,
a per-round and a per-level charge) comes from the committed schedule cache
(paper_1507_01926_amd/schedules.json), which the autotuner wrote from timed
solves of ANOTHER instance of the same family and size; the fixed rule is
timed beside it.  --schedule fixed uses the fixed rule, --schedule tune
tunes on another instance first.  The schedule never changes the value, the
cut or the sink side.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "max-flow arcs/s + HBM GB/s (% peak); batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c1": "2D 4-connected grid 64x64, caps U[1,100], s->left column, right column->t cap 1000",
    "c2": "2D 8-connected segmentation grid 2048x2048, caps round(100*exp(-|a-b|^2/200)), terminal caps U[0,500]",
    "c3": "3D 6-connected grid 256^3, caps U[1,1e4], s->z=0 plane, z=255 plane->t cap 1e6",
    "c4a": "random layered graph 512 layers x 16384, 4 forward + 1 intra-layer arc per vertex, caps U[1,1e4]",
    "c4b": "R-MAT scale 22, edge factor 16, (a,b,c)=(0.57,0.19,0.19), unit caps",
}


def fixed_schedule(g, level_charge: int = 0) -> dict:
    """Global-relabel schedule used by the benchmark: the paper's rule (freq
    1/2, alpha 6, beta 12) plus a per-round work charge of (12n+2m)/128, which
    bounds the rounds between two global relabels, and optionally a charge
    per breadth-first level of the last relabel (for graphs whose searches
    run thousands of levels deep)."""
    thr = 12 * g.n + 2 * g.slots
    sched = dict(gr_round_charge=max(1, thr // 128))
    if level_charge:
        sched["gr_level_charge"] = int(level_charge)
    return sched


def kernel_source_sha() -> str:
    """sha256 over the HIP sources of the library (counters taken on other
    sources no longer describe the kernels)."""
    from paper_1507_01926_amd.profiling import source_sha
    return source_sha()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary kept under profiles/, if it was taken on the current
    sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_source_sha():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth_gbs(dev, mib: int = 2048, reps: int = 10) -> float:
    """Device-to-device copy bandwidth on this GPU (torch's copy kernel over
    `mib` MiB, read and written), the achievable streaming rate beside the
    nominal peak."""
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    gbs = 2 * reps * (mib << 20) / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


# The CPU oracle's sample of each workload: the same generator rule at a
# size whose sequential solve takes about 10-30 s (the full 256^3 grid takes
# tens of minutes on one core).
CPU_SAMPLE = {"c1": 1, "c2": 1, "c3": 2, "c4a": 4, "c4b": 1}


def cpu_baseline_leg(workload: str) -> dict:
    """The CPU oracle (sequential FIFO push-relabel, exact int64, one thread)
    timed on this host: one complete solve (preflow and flow) of a bounded
    sample of the workload, reported as arcs/s of that sample."""
    import oracle
    from workloads import make_config
    f = CPU_SAMPLE.get(workload, 1)
    g = make_config(workload, f)
    t0 = time.perf_counter()
    A = oracle.fifo_maxflow(g)
    dt = time.perf_counter() - t0
    what = "the full instance" if f == 1 else (f"the same generator rule with every side divided by {f} "
                                               f"({g.n:,} vertices, {g.m_arcs:,} arcs)")
    return {"value": g.m_arcs / dt, "unit": "arcs/s", "cores": 1, "kind": "oracle",
            "sample": f"{workload}: one complete solve (preflow + flow) of {what}, sequential FIFO "
                      f"push-relabel with global relabels, 1 thread, {dt:.1f} s; host CPU: {cpu_model()}, "
                      f"{os.cpu_count()} logical cores",
            "seconds": dt, "oracle_value": A["value"], "sample_arcs": g.m_arcs}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def _gen_instance(args):
    """Pool worker: stream instance i as plain arrays (no GPU in the workers)."""
    i, n_hi = args
    from workloads import stream_instance
    g = stream_instance(i, n_hi=n_hi)
    return i, g


def _instances(count: int, n_hi: float, procs: int, ahead: int = 96):
    """Stream instances 0 .. count-1 in order, generated by a pool of worker
    processes at most `ahead` instances ahead of their use (the whole stream
    does not fit host memory at 1e6 vertices: about 190 GB of arrays)."""
    if procs <= 1:
        from workloads import stream_instance
        for i in range(count):
            yield i, stream_instance(i, n_hi=n_hi)
        return
    import collections
    import multiprocessing as mp
    ctx = mp.get_context("spawn")          # the workers never touch the GPU
    with ctx.Pool(procs) as pool:
        window = collections.deque()
        nxt = 0
        while nxt < count and len(window) < ahead:
            window.append(pool.apply_async(_gen_instance, ((nxt, n_hi),)))
            nxt += 1
        while window:
            i, g = window.popleft().get()
            if nxt < count:
                window.append(pool.apply_async(_gen_instance, ((nxt, n_hi),)))
                nxt += 1
            yield i, g


def stream_leg(count: int, n_hi: float, seed_note: str, chunk: int = 256, procs: int = 0,
               oracle_every: int = 0, route: int = 0) -> dict:
    """Batched and served forms on a stream of `count` instances (family
    uniform over the five generator rules, n log-uniform in [1e3, n_hi]),
    with the lane knob from the autotuner, next to the plain solver run one
    request at a time in arrival order.  Instances are generated by a pool
    of worker processes ahead of their use; the closed-loop batched form
    takes them in chunks of `chunk` (each chunk one mf_batch_solve call, the
    chunks one after another), the served form at their Poisson arrival
    times.  A stream whose arrays fit in a few GB of host memory (n_hi up to
    2e5) is generated once and replayed in every leg; a larger one is
    generated again for each leg, and a request then waits for its instance
    if the pool falls behind (its latency counts from its actual submission,
    and requests_submitted_late counts such requests)."""
    import numpy as np
    import paper_1507_01926_amd as mf
    from paper_1507_01926_amd.autotune import Autotuner, bucket_of
    from workloads import stream_arrivals

    procs = procs or min(15, max(1, (os.cpu_count() or 2) - 1))
    held = list(_instances(count, n_hi, procs)) if n_hi <= 2e5 else None

    def source():
        return iter(held) if held is not None else _instances(count, n_hi, procs)

    ctx = mf.Context(0)
    tuner = Autotuner(ctx, cache_path=None)
    t_all = time.perf_counter()
    # closed loop: every request present at t = 0, processed in chunks
    done_ms, plain_ms, values, plain_vals, arcs, fam = [], [], [], [], 0, {}
    t_gpu = 0.0
    buf = []
    tuned = set()
    checked = []
    tune_s = 0.0

    def flush(buf):
        nonlocal t_gpu, tune_s
        graphs = [g for _, g in buf]
        fresh = []
        # one autotuning sample per new bucket (knobs never change results)
        for g in graphs:
            b = bucket_of(g)
            if b not in tuned:
                tuned.add(b)
                if g.slots <= 262144:
                    fresh.append(g)
        if fresh:
            t0 = time.perf_counter()
            tuner.tune(fresh, mode="batch", reps=1, round_divisors=(0, 128, 32))
            tune_s += time.perf_counter() - t0
        opts = [tuner.options_for(g, "batch", batch_grid_slots=route) for g in graphs]
        t0 = time.perf_counter()
        res, _ = mf.batch_solve(ctx, graphs, opts=opts, want_flow=False, want_side=False)
        dt = time.perf_counter() - t0
        for r in res:
            assert r["status"] == 0
            done_ms.append(1e3 * t_gpu + r["ms_end"])
            values.append(r["value"])
        t_gpu += dt
        for g, o in zip(graphs, opts):
            t1 = time.perf_counter()
            pr = ctx.solve(g, o, want_flow=False, want_side=False)
            plain_ms.append(1e3 * (time.perf_counter() - t1))
            plain_vals.append(pr["value"])

    for i, g in source():
        arcs += g.m_arcs
        fam[g.family] = fam.get(g.family, 0) + 1
        if oracle_every and i % oracle_every == 0 and g.n <= 2e5:
            import oracle
            t1 = time.perf_counter()
            A = oracle.fifo_maxflow(g)             # the whole solve, both phases, on one host core
            checked.append((i, A["value"], time.perf_counter() - t1))
        buf.append((i, g))
        if len(buf) == chunk:
            flush(buf)
            buf = []
        if i % 256 == 255:
            print(f"[bench] stream closed loop: {i + 1} instances", file=sys.stderr, flush=True)
    if buf:
        flush(buf)
    assert plain_vals == values
    for i, v, _ in checked:
        assert values[i] == v, (i, values[i], v)
    oracle_s = sum(x[2] for x in checked)
    gpu_s = sum(plain_ms[i] for i, _, _ in checked) / 1e3
    oracle_sample = {"instances": len(checked), "oracle_seconds": oracle_s, "oracle_cores": 1,
                     "oracle_solves_per_s": len(checked) / oracle_s if oracle_s else None,
                     "plain_gpu_solves_per_s": len(checked) / gpu_s if gpu_s else None,
                     "note": f"every {oracle_every}-th instance with at most 2e5 vertices, solved whole by oracle A "
                             "(sequential FIFO push-relabel) on one host core and by the plain GPU solver"}
    closed_rate = count / t_gpu
    batched = {"solves_per_s": closed_rate, "arcs_per_s": arcs / t_gpu,
               "p50_ms": _pct(done_ms, 50), "p99_ms": _pct(done_ms, 99), "gpu_wall_s": t_gpu,
               "note": f"latency = completion time from the stream start with every request present at t=0; "
                       f"the stream runs as {-(-count // chunk)} mf_batch_solve calls of up to {chunk} "
                       f"instances, one after another (generation time excluded)"}
    served = {}
    plain_total_s = sum(plain_ms) / 1e3
    for frac in (0.5, 0.8):
        rate = frac * closed_rate
        arr = stream_arrivals(count, rate)
        srv = mf.Server(ctx, hbm_budget_bytes=64 << 30)
        tickets, submit_late = [], 0
        t_start = time.perf_counter()
        for i, g in source():
            delay = arr[i] - (time.perf_counter() - t_start)
            if delay > 0:
                time.sleep(delay)
            elif delay < -0.005:
                submit_late += 1
            tickets.append(srv.submit(g, tuner.options_for(g, "batch", batch_grid_slots=route), want_flow=False))
            if i % 512 == 511:
                print(f"[bench] stream served {frac}x: {i + 1} submitted", file=sys.stderr, flush=True)
        out = []
        for j, t in enumerate(tickets):
            out.append(srv.wait(t, 1800000))
            if j % 512 == 511:
                print(f"[bench] stream served {frac}x: {j + 1} done", file=sys.stderr, flush=True)
        span = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        assert [r["value"] for r in out] == values
        lat = [r["ms_latency"] for r in out]
        fin, plat = 0.0, []
        for a, sv in zip(arr, plain_ms):
            fin = max(fin, a) + sv / 1e3
            plat.append(1e3 * (fin - a))
        served[f"poisson_{frac}x"] = {
            "rate_per_s": rate, "solves_per_s": count / span, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
            "requests_submitted_late": submit_late, "peak_hbm_bytes": st["peak_bytes"],
            "kernel_launches": st["kernel_launches"],
            "plain_one_at_a_time": {"solves_per_s": count / fin if fin else None,
                                    "p50_ms": _pct(plat, 50), "p99_ms": _pct(plat, 99)}}
    ctx.close()
    return {"stream": f"{count} instances, n log-uniform in [1e3, {n_hi:.0e}], families uniform over "
                      f"the five generator rules ({seed_note}); instances above "
                      f"{route or mf.MF_BATCH_GRID_SLOTS:,} slots run on "
                      f"the grid-wide kernels in both forms",
            "families": fam, "arcs_total": arcs, "generator_processes": procs,
            "instances_generated": "once, held in host memory" if held is not None else "again for every leg",
            "autotune_s": tune_s, "autotuned_buckets": len(tuned), "batched": batched, "served": served,
            "plain_one_at_a_time_solves_per_s": count / plain_total_s,
            "oracle_checked_instances": len(checked), "oracle_sample": oracle_sample,
            "wall_s": time.perf_counter() - t_all}


def _changed_caps(cap, flow, frac: float, rng):
    """New capacities on a random `frac` of the slots that carry capacity:
    half raised by U{1..40}, half cut by U{1..40} but never below the slot's
    flow in the last solve (so that the kept flow stays feasible)."""
    import numpy as np
    new = cap.copy()
    cand = np.flatnonzero(cap > 0)
    pick = rng.choice(cand, size=max(2, int(frac * cand.size)), replace=False)
    up, down = pick[: pick.size // 2], pick[pick.size // 2:]
    new[up] += rng.integers(1, 41, size=up.size, dtype=np.int32)
    slack = cap[down] - np.maximum(flow[down], 0)
    new[down] -= np.minimum(rng.integers(1, 41, size=down.size, dtype=np.int32), slack)
    return new


def resolve_leg(name: str, fracs=(0.001, 0.01, 0.1), seed: int = 11) -> dict:
    """Served re-solves of a resident graph against cold requests of the
    same graph: the graph is registered once (mf_server_register_graph);
    each step changes a random fraction of the capacities and submits them
    both as a re-solve of the resident graph (mf_server_submit_caps, which
    resumes from the flow the server kept) and as a new request carrying the
    whole graph (mf_server_submit).  Latency is the server's, from submit to
    completion."""
    import dataclasses
    import numpy as np
    import paper_1507_01926_amd as mf
    from workloads import make_config
    g = make_config(name)
    ctx = mf.Context(0)
    sc, sc_from = pick_schedule("cache", name, g, ctx, 0)
    opt = mf.options(**sc)
    srv = mf.Server(ctx, hbm_budget_bytes=64 << 30)
    rng = np.random.default_rng(seed)
    gid = srv.register_graph(g)
    first = srv.wait(srv.submit_caps(gid, g.cap, opt), 600000)
    cold0 = srv.wait(srv.submit(g, opt), 600000)
    assert first["value"] == cold0["value"]
    steps, cap, flow = [], g.cap, first["flow"]
    for frac in fracs:
        cap = _changed_caps(cap, flow, frac, rng)
        warm = srv.wait(srv.submit_caps(gid, cap, opt), 600000)
        cold = srv.wait(srv.submit(dataclasses.replace(g, cap=cap), opt), 600000)
        assert warm["value"] == cold["value"] and warm["cut_capacity"] == cold["cut_capacity"]
        steps.append({"changed_fraction": frac, "value": warm["value"], "resumed": bool(warm["resumed"]),
                      "resolve_ms": warm["ms_latency"], "cold_request_ms": cold["ms_latency"],
                      "resolve_rounds": [warm["rounds"], warm["rounds2"]],
                      "cold_rounds": [cold["rounds"], cold["rounds2"]]})
        flow = warm["flow"]
        print(f"[bench] resolve {name} {frac}: {warm['ms_latency']:.1f} ms resumed, "
              f"{cold['ms_latency']:.1f} ms cold", file=sys.stderr, flush=True)
    srv.release_graph(gid)
    srv.close()
    ctx.close()
    return {"workload": WORKLOADS[name], "schedule": sc, "schedule_from": sc_from,
            "first_resident_solve_ms": first["ms_latency"], "cold_request_ms": cold0["ms_latency"],
            "steps": steps,
            "note": "each step raises half of the changed slots by U{1..40} and cuts the other half by "
                    "U{1..40}, never below the slot's flow; steps follow one another on the same resident graph"}


def schedule_options(g, knobs: dict) -> dict:
    thr = 12 * g.n + 2 * g.slots
    return dict(gr_round_charge=max(1, thr // knobs["round_divisor"]) if knobs.get("round_divisor") else 0,
                gr_freq_num=1, gr_freq_den=knobs.get("freq_den", 2), gr_level_charge=knobs.get("level_charge", 0))


def pick_schedule(mode: str, workload: str, g, ctx, level_charge: int):
    """(schedule options, where they came from)."""
    fixed = fixed_schedule(g, level_charge)
    if mode == "fixed":
        return fixed, "fixed rule"
    if mode == "paper":
        return {}, "the paper's rule"
    from paper_1507_01926_amd.autotune import cached_schedule, tune_workload_schedules
    if mode == "tune":
        print("[bench] autotuning the schedule on another instance of the family", file=sys.stderr, flush=True)
        entry = tune_workload_schedules([workload], path=os.path.join(ROOT, "_tuned_schedules.json"))[workload]
        return schedule_options(g, entry["knobs"]), "autotuner, " + entry["tuned_on"]
    entry = cached_schedule(workload)
    if entry is None:
        return fixed, "fixed rule (no cached schedule for this workload)"
    return schedule_options(g, entry["knobs"]), "schedule cache: autotuner on " + entry["tuned_on"]


def time_solves(dg, g, opt, flow, side, steps: int, warmup: int, pick_dominant: bool, mf):
    """Warm-up and timed solves of an uploaded graph; returns the timing and
    the per-kernel tables."""
    import torch

    def per_kernel(rs):
        out = {}
        for i, name in enumerate(mf.KERNEL_NAMES):
            out[name] = (sum(r["kernel_ms"][i] for r in rs), sum(r["kernel_bytes"][i] for r in rs),
                         sum(r["kernel_launches"][i] for r in rs), sum(r["kernel_timed"][i] for r in rs))
        return out

    # Warm-up solves time every kernel with HIP events and name the dominant
    # one; the timed solves then bracket only that kernel's launches, and of
    # a kernel launched thousands of times per solve only every 16th launch
    # (an event pair costs a few microseconds of device time).
    warm = [dg.solve(opt, flow.data_ptr(), side.data_ptr()) for _ in range(warmup)]
    torch.cuda.synchronize()
    dom_idx = None
    if warm and pick_dominant:
        wk = per_kernel(warm[-1:])
        dom_idx = mf.KERNEL_NAMES.index(max(wk, key=lambda k: wk[k][0]))
        opt.profile_mask = 1 << dom_idx
        opt.profile_stride = 16 if wk[mf.KERNEL_NAMES[dom_idx]][2] >= 256 else 1
    t0 = time.perf_counter()
    runs = [dg.solve(opt, flow.data_ptr(), side.data_ptr()) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernels = per_kernel(runs)
    table = per_kernel(warm[-1:]) if warm and dom_idx is not None else kernels
    return dict(dt=dt, runs=runs, kernels=kernels, table=table, dom_idx=dom_idx,
                table_steps=1 if warm and dom_idx is not None else steps)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--extra", default="c2",
                    help="comma-separated workloads timed beside the headline (5 solves each; '' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--persistent", action="store_true",
                    help="run each phase as one persistent cooperative kernel instead of one launch per round")
    ap.add_argument("--schedule", default="cache", choices=("cache", "fixed", "tune", "paper"),
                    help="global-relabel schedule: the committed cache (tuned on another instance of the "
                         "family), the fixed rule, a fresh tuning on another instance, or the paper's rule")
    ap.add_argument("--simple-rounds", action="store_true",
                    help="rounds of the simple synchronous variant of Sec. 3 (ablation of Listing 1's rounds)")
    ap.add_argument("--gap", action="store_true", help="the gap rule at every round end (ablation)")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-rule solve beside the tuned schedule")
    ap.add_argument("--level-charge", type=int, default=0,
                    help="with --schedule fixed: global-relabel threshold charge per level of the last search")
    ap.add_argument("--stream", type=int, default=256,
                    help="instances of the batched/served stream leg (0 = skip)")
    ap.add_argument("--stream-nmax", type=float, default=1e5)
    ap.add_argument("--stream-chunk", type=int, default=256,
                    help="instances per mf_batch_solve call of the closed-loop stream")
    ap.add_argument("--stream-oracle-every", type=int, default=64,
                    help="check every k-th stream instance (up to 2e5 vertices) against the CPU oracle")
    ap.add_argument("--route-slots", type=int, default=0,
                    help="stream leg: instances above this many slots go to the grid-wide kernels "
                         "(0 = the library's default)")
    ap.add_argument("--resolve", default="",
                    help="workload of a served re-solve leg (resident graph, capacity changes; '' = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the solves, copy a buffer of this size on the device (a dispatch of known "
                         "traffic that scales the HBM counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X "
              "(no sharding across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1507_01926_amd as mf
    from workloads import make_config

    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    g = make_config(args.workload)
    ctx = mf.Context(0)
    dg = ctx.upload(g)                       # residency + validation: not timed
    dev = torch.device("cuda:0")
    flow = torch.empty(max(1, g.slots), dtype=torch.int32, device=dev)
    side = torch.empty(g.n, dtype=torch.uint8, device=dev)
    sched, sched_from = pick_schedule(args.schedule, args.workload, g, ctx, args.level_charge)
    mode = dict(simple_rounds=args.simple_rounds)
    if args.gap:
        mode["gap"] = True
    opt = mf.options(profile=True, persistent=args.persistent, **mode, **sched)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # (not in a counter run: its copies would be taken for the probe's)
    copy_gbs = copy_bandwidth_gbs(dev) if args.copy_probe_mib == 0 else None
    print(f"[bench] warmup x{args.warmup}, timing x{args.steps}", file=sys.stderr, flush=True)
    T = time_solves(dg, g, opt, flow, side, args.steps, args.warmup, not args.persistent, mf)
    dt, runs, kernels, table = T["dt"], T["runs"], T["kernels"], T["table"]
    ms_per_step = 1e3 * dt / args.steps
    value = g.m_arcs * args.steps / dt

    # dominant kernel over the timed region, from the library's HIP events
    # (recorded around each launch on the stream the kernels run on)
    tot = {k: sum(r[k] for r in runs) for k in runs[0] if isinstance(runs[0][k], (int, float))}
    table_steps = T["table_steps"]
    if args.persistent:
        kernels = {"k_phase": (tot["ms_phase_kernel"], tot["discharge_bytes"] + tot["merge_bytes"]
                               + tot["global_relabel_bytes"], tot["phase_launches"], tot["phase_launches"])}
        table, table_steps = kernels, args.steps
    dom = mf.KERNEL_NAMES[T["dom_idx"]] if T["dom_idx"] is not None else max(kernels, key=lambda k: kernels[k][0])
    ms_k, bytes_k, launches_k, timed_k = kernels[dom]
    avg_launch_ms = ms_k / max(1, timed_k)
    achieved = bytes_k / max(1, launches_k) / (avg_launch_ms * 1e-3) / 1e9 if ms_k > 0 else 0.0
    alg_bytes_total = tot["discharge_bytes"] + tot["merge_bytes"] + tot["global_relabel_bytes"]
    r0 = runs[0]
    fixed = None
    if args.schedule != "fixed" and not args.persistent and not args.no_fixed:
        # the fixed rule beside the tuned schedule (one solve)
        fopt = mf.options(persistent=False, **mode, **fixed_schedule(g, 0))
        t1 = time.perf_counter()
        fr = dg.solve(fopt, flow.data_ptr(), side.data_ptr())
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t1
        assert fr["value"] == r0["value"]
        fixed = {"ms_per_solve": 1e3 * fdt, "arcs_per_s": g.m_arcs / fdt, "solves": 1,
                 "schedule": fixed_schedule(g, 0), "rounds": fr["rounds"], "rounds_phase2": fr["rounds2"],
                 "global_relabels": fr["global_relabels"] + fr["global_relabels2"]}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "arcs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32 capacities/residuals, int64 excess",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "n": g.n, "arcs": g.m_arcs, "slots": g.slots,
                   "schedule": sched or "paper (freq 1/2, alpha 6, beta 12)",
                   "schedule_from": sched_from,
                   "rounds": "simple synchronous variant (Sec. 3)" if args.simple_rounds
                             else "Listing 1 (win criterion, full discharge)",
                   "gap_rule": bool(args.gap)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, args.workload),
                     "launches_per_step": launches_k / args.steps,
                     "alg_bytes_per_launch": bytes_k / max(1, launches_k),
                     "avg_launch_us": 1e3 * avg_launch_ms,
                     "launches_timed": timed_k,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None},
        "solve": {"value": r0["value"], "cut_capacity": r0["cut_capacity"],
                  "value_equals_cut": r0["value"] == r0["cut_capacity"],
                  "rounds": r0["rounds"], "rounds_phase2": r0["rounds2"],
                  "global_relabels": r0["global_relabels"] + r0["global_relabels2"],
                  "bfs_levels_phase1": r0["bfs_levels"],
                  "ms_preflow": sum(r["ms_preflow"] for r in runs) / len(runs),
                  "preflow_arcs_per_s": g.m_arcs / (1e-3 * sum(r["ms_preflow"] for r in runs) / len(runs)),
                  "kernels_per_step": {k: {"ms": v[0] / table_steps, "launches": v[2] / table_steps,
                                           "alg_GBps": (v[1] / v[2] / (v[0] / v[3] * 1e-3) / 1e9)
                                           if v[0] > 0 and v[3] > 0 else None}
                                       for k, v in table.items() if v[2] > 0},
                  "kernels_per_step_note": "event-timed in the last warm-up solve (every kernel timed)"
                                           if table is not kernels else "event-timed in the timed solves",
                  "alg_GBps_whole_solve": alg_bytes_total / dt / 1e9,
                  "alg_frac_whole_solve": alg_bytes_total / dt / 1e9 / HBM_PEAK_GBS},
        "fixed_schedule": fixed,
    }
    dg.free()
    del flow, side
    extra = {}
    for name in [x for x in args.extra.split(",") if x and x != args.workload]:
        print(f"[bench] extra workload {name}", file=sys.stderr, flush=True)
        ge = make_config(name)
        dge = ctx.upload(ge)
        fe = torch.empty(max(1, ge.slots), dtype=torch.int32, device=dev)
        se = torch.empty(ge.n, dtype=torch.uint8, device=dev)
        sc_e, from_e = pick_schedule("cache" if args.schedule in ("cache", "tune") else args.schedule, name, ge, ctx, 0)
        Te = time_solves(dge, ge, mf.options(**mode, **sc_e), fe, se, 5, 1, False, mf)
        re0 = Te["runs"][0]
        extra[name] = {"workload": WORKLOADS[name], "arcs": ge.m_arcs, "arcs_per_s": ge.m_arcs * 5 / Te["dt"],
                       "ms_per_solve": 1e3 * Te["dt"] / 5, "solves": 5, "value": re0["value"],
                       "value_equals_cut": re0["value"] == re0["cut_capacity"], "schedule": sc_e,
                       "schedule_from": from_e, "rounds": re0["rounds"], "rounds_phase2": re0["rounds2"],
                       "ms_preflow": re0["ms_preflow"]}
        dge.free()
        del fe, se
    if extra:
        line["extra"] = extra
    ctx.close()
    if args.stream > 0:
        print(f"[bench] stream leg x{args.stream}", file=sys.stderr, flush=True)
        line["stream"] = stream_leg(args.stream, args.stream_nmax, "seeded", chunk=args.stream_chunk,
                                    oracle_every=args.stream_oracle_every, route=args.route_slots)
    if args.resolve:
        print(f"[bench] served re-solve leg on {args.resolve}", file=sys.stderr, flush=True)
        line["resolve"] = resolve_leg(args.resolve)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline_leg(args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
