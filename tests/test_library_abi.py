"""The C-ABI library builds, loads without a GPU and exports every symbol
include/maxflow.h declares; the binding fails loudly without a device.
CPU only."""
import ctypes
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maxflow.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mf_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("mf_context_create", "mf_solve", "mf_solve_device", "mf_graph_upload",
                 "mf_solve_uploaded", "mf_batch_solve", "mf_server_submit", "mf_server_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1507_01926_amd as mf
    L = mf.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding covers the whole ABI too
    bound = {n for n, _, _ in mf.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_version_and_status_strings():
    import paper_1507_01926_amd as mf
    assert "gfx950" in mf.mf_version()
    L = mf.lib()
    assert L.mf_status_str(mf.MF_EINVAL).decode() == "invalid argument"


def test_defaults_are_the_papers_schedule():
    import paper_1507_01926_amd as mf
    o = mf.options()
    assert (o.gr_freq_num, o.gr_freq_den, o.gr_alpha, o.gr_beta, o.gr_round_charge) == (1, 2, 6, 12, 0)
    assert o.gr_level_charge == 0 and o.bfs_bottom_up_factor == 0 and o.profile_stride == 0


def test_no_device_fails_loudly():
    import paper_1507_01926_amd as mf
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    with pytest.raises(mf.MaxflowError) as ei:
        mf.Context(0)
    assert ei.value.status == mf.MF_EDEVICE


def test_struct_sizes_match_header():
    """Compile a tiny C program against the header and compare struct sizes
    with the ctypes mirrors."""
    import subprocess
    import tempfile
    import paper_1507_01926_amd as mf
    src = r'''
#include <stdio.h>
#include "maxflow.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(mf_graph), sizeof(mf_options), sizeof(mf_stats),
         sizeof(mf_result), sizeof(mf_server_config), sizeof(mf_server_stats), sizeof(mf_status));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(x) for x in out]
    mine = [ctypes.sizeof(mf.mf_graph), ctypes.sizeof(mf.mf_options), ctypes.sizeof(mf.mf_stats),
            ctypes.sizeof(mf.mf_result), ctypes.sizeof(mf.mf_server_config),
            ctypes.sizeof(mf.mf_server_stats), 4]
    assert sizes == mine


def test_autotuner_buckets_and_defaults(tmp_path):
    """Bucketing and the cache are host logic (no device needed)."""
    from paper_1507_01926_amd import autotune
    from workloads import make_config
    g1 = make_config("c1")
    g2 = make_config("c4b", 16)
    assert autotune.bucket_of(g1) != autotune.bucket_of(g2)
    assert autotune.bucket_of(g2).endswith("h1")          # R-MAT hubs
    tuner = autotune.Autotuner(ctx=None, cache_path=str(tmp_path / "cache.json"))
    k = tuner.knobs_for(g1)
    assert k["lanes_per_vertex"] in autotune.LANES
    tuner.cache["plain:" + autotune.bucket_of(g1)] = {"knobs": {"lanes_per_vertex": 16, "round_divisor": 32,
                                                                "dense_divisor": 64}}
    tuner.save()
    again = autotune.Autotuner(ctx=None, cache_path=str(tmp_path / "cache.json"))
    assert again.knobs_for(g1)["lanes_per_vertex"] == 16
    o = again.options_for(g1)
    assert o.lanes_per_vertex == 16 and o.gr_round_charge == (12 * g1.n + 2 * g1.slots) // 32


def test_schedule_knobs_and_mode_flags_map_to_options():
    """The autotuner's schedule knobs and the mode keywords of options()
    land in the fields and flags the header defines (host logic)."""
    import paper_1507_01926_amd as mf
    from paper_1507_01926_amd import autotune
    from workloads import make_config
    g = make_config("c1")
    thr = 12 * g.n + 2 * g.slots
    for rd, fd, lc in autotune.SCHEDULES:
        o = autotune.knobs_to_options(g, dict(round_divisor=rd, freq_den=fd, level_charge=lc))
        assert (o.gr_round_charge, o.gr_freq_num, o.gr_freq_den, o.gr_level_charge) == (thr // rd, 1, fd, lc)
    assert autotune.SCHEDULES[0] == (128, 2, 0)          # the benchmark's fixed rule comes first
    o = mf.options(simple_rounds=True, warm_start=True, grid_path=True)
    assert o.flags == mf.MF_SIMPLE_ROUNDS | mf.MF_WARM_START | mf.MF_GRID_PATH
    o = mf.options(simple_rounds=False)
    assert o.flags & mf.MF_SIMPLE_ROUNDS == 0
    header = open(os.path.join(ROOT, "include", "maxflow.h")).read()
    for name, val in (("MF_SIMPLE_ROUNDS", mf.MF_SIMPLE_ROUNDS), ("MF_WARM_START", mf.MF_WARM_START),
                      ("MF_GRID_PATH", mf.MF_GRID_PATH)):
        assert f"#define {name}" in header and hex(val) in header.split(f"#define {name}")[1].split("u")[0]


def test_bench_refuses_several_gpus():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_traffic_only_for_the_profiled_sources(monkeypatch):
    """The benchmark reports the counter-measured traffic of the dominant
    kernel only while the profile was taken on the current HIP sources."""
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "k_gr_td_c3_traffic.txt")
    recorded = [l.split(":", 1)[1].strip() for l in open(path) if l.startswith("source_sha256:")][0]
    per_launch = [float(l.split(":", 1)[1]) for l in open(path) if l.startswith("hbm_bytes_per_launch:")][0]
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: recorded)
    assert bench.measured_traffic("k_gr_td", "c3") == per_launch
    assert bench.measured_traffic("k_gr_td", "c2") is None     # no profile for that workload
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.measured_traffic("k_gr_td", "c3") is None     # sources changed since the counters


def test_committed_traffic_profile_matches_the_sources():
    """The committed k_gr_td traffic summary of the headline workload was
    taken on the HIP sources as they stand."""
    from paper_1507_01926_amd.profiling import source_sha
    path = os.path.join(ROOT, "profiles", "k_gr_td_c3_traffic.txt")
    recorded = [l.split(":", 1)[1].strip() for l in open(path) if l.startswith("source_sha256:")][0]
    assert recorded == source_sha()


def test_bench_fixed_schedule():
    sys.path.insert(0, ROOT)
    import bench
    from workloads import make_config
    g = make_config("c1")
    thr = 12 * g.n + 2 * g.slots
    assert bench.fixed_schedule(g) == {"gr_round_charge": thr // 128}
    assert bench.fixed_schedule(g, 1 << 17) == {"gr_round_charge": thr // 128, "gr_level_charge": 1 << 17}
