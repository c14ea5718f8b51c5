"""The rocprofv3 summarizer (paper_1507_01926_amd/profiling.py) on small
hand-made trace and counter files: the per-kernel table covers the last
solve only, the sampled-launch split follows the benchmark's stride, and the
traffic per launch scales each counter by the probe copy launched last before
the solve.  CPU only."""
import os

import pytest

from paper_1507_01926_amd import profiling


def _write(path, header, rows):
    with open(path, "w") as fh:
        fh.write(",".join(header) + "\n")
        for r in rows:
            fh.write(",".join(str(x) for x in r) + "\n")


def _trace(tmp_path):
    # two solves; durations in ns.  Solve 2: k_gr_td launches of 1000, 2000,
    # 3000, 4000 ns and one merge of 500 ns.
    hdr = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows, t, i = [], 0, 0
    for solve, tds in ((1, [9000, 9000]), (2, [1000, 2000, 3000, 4000])):
        for name, dur in [("mf::k_init_state(x)", 100)] + [("void mf::k_gr_td<8>(y)", d) for d in tds] + \
                         [("void mf::k_merge_list<4>(z)", 500)]:
            i += 1
            rows.append((i, name, t, t + dur))
            t += dur + 10
    d = tmp_path / "trace"
    d.mkdir()
    _write(d / "run_kernel_trace.csv", hdr, rows)
    return str(d)


def test_kernel_summary_covers_the_last_solve(tmp_path):
    out = profiling.kernel_summary(_trace(tmp_path), "t", "k_gr_td", 2)
    lines = [ln for ln in out.splitlines() if not ln.startswith("#")]
    td = next(ln for ln in lines if "k_gr_td" in ln).split()
    assert td[-4:] == ["4", "0.01", "2.50", f"{100 * 10000 / 10600:.2f}"]   # calls, ms, us, pct
    merge = next(ln for ln in lines if "k_merge_list" in ln).split()
    assert merge[-4] == "1"
    assert "2 solves traced" in out
    # launches 0 and 2 of the solve (stride 2): 1000 and 3000 ns; the others 2000 and 4000
    split = out.splitlines()[-1]
    assert "2 launches, avg 2.00 us" in split and "the other 2: avg 3.00 us" in split


def _counters(tmp_path, name, probe_kib, vals):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [(1, "__amd_rocclr_copyBuffer", name, 999999.0),        # an earlier, larger copy
            (2, "__amd_rocclr_copyBuffer", name, probe_kib),       # the probe: last copy before the solve
            (3, "mf::k_init_state(x)", name, 1.0)]
    rows += [(4 + j, "void mf::k_gr_td<8>(y)", name, v) for j, v in enumerate(vals)]
    rows.append((10, "__amd_rocclr_copyBuffer", name, 5.0))          # a readback after the solve began
    d = tmp_path / name
    d.mkdir()
    _write(d / "run_counter_collection.csv", hdr, rows)
    return str(d)


def test_traffic_scales_by_the_probe_copy(tmp_path):
    # the probe is 256 MiB read and written; FETCH_SIZE reads half of it, WRITE_SIZE all of it
    f = _counters(tmp_path, "FETCH_SIZE", 131072.0, [100.0, 300.0])
    w = _counters(tmp_path, "WRITE_SIZE", 262144.0, [50.0, 50.0])
    out = profiling.traffic_summary(f, w, "k_gr_td", "c3", 256, "rocprofv3 --pmc PMC -- cmd")
    fields = dict(ln.split(": ", 1) for ln in out.splitlines() if not ln.startswith("#"))
    assert fields["dispatches"] == "2"
    assert float(fields["fetch_scale"]) == pytest.approx(2.0)
    assert float(fields["write_scale"]) == pytest.approx(1.0)
    # per launch: (2 * 400 + 1 * 100) KiB / 2 launches = 450 KiB
    assert int(fields["hbm_bytes_per_launch"]) == 450 * 1024
    assert fields["source_sha256"] == profiling.source_sha()
    assert "--pmc FETCH_SIZE" in out and "--pmc WRITE_SIZE" in out


def test_source_sha_covers_the_hip_sources():
    csrc = os.path.join(os.path.dirname(profiling.__file__), "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".h")))
    assert "kernels.hip" in names and "mf_device.h" in names
    assert len(profiling.source_sha()) == 64
