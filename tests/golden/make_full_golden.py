"""Write the expected results of the full-size workloads, computed by the CPU
oracle only (test infrastructure; never by the HIP path).

    python tests/golden/make_full_golden.py c2 [c3 c4a c4b c1]

For each workload it writes tests/golden/full_<name>.json with
  - from oracle A (sequential FIFO push-relabel): value, cut capacity of T*,
    sha256 of T* (uint8[n]);
  - from oracle B (the synchronous rounds) under the benchmark's schedule
    (the paper's rule plus a per-round charge of (12n+2m)/128): value, round,
    push, relabel and global-relabel counts and sha256 of the per-slot flow
    (int32[slots], little endian).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import make_config  # noqa: E402


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def bench_schedule(g):
    return dict(round_charge=max(1, (12 * g.n + 2 * g.slots) // 128))


def main(names):
    for name in names:
        t0 = time.time()
        g = make_config(name)
        A = oracle.fifo_maxflow(g, preflow_only=True)
        ta = time.time() - t0
        sc = bench_schedule(g)
        B = oracle.sync_maxflow(g, schedule=sc)
        tb = time.time() - t0 - ta
        assert A["value"] == B["value"] == A["cut_tstar"] == B["cut_tstar"]
        assert (A["tstar"] == B["tstar"]).all()
        out = {
            "workload": name, "n": g.n, "slots": g.slots, "arcs": g.m_arcs, "s": g.s, "t": g.t,
            "value": A["value"], "cut": A["cut_tstar"], "tstar_sha256": sha(A["tstar"]),
            "tstar_count": int(A["tstar"].sum()),
            "sync": {"schedule": sc, "rounds": B["rounds"], "rounds2": B["rounds2"],
                     "pushes": B["pushes"], "relabels": B["relabels"],
                     "global_relabels": B["global_relabels"], "bfs_levels": B["bfs_levels"],
                     "flow_sha256": sha(B["flow"].astype("<i4"))},
            "oracle_seconds": {"fifo_preflow": round(ta, 1), "sync_full": round(tb, 1)},
        }
        with open(os.path.join(HERE, f"full_{name}.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print(name, out["value"], out["sync"]["rounds"], f"{ta:.0f}s {tb:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c3", "c4a", "c4b"])
