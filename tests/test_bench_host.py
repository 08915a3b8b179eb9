"""Host logic of bench.py, without a GPU: the algorithmic byte count of the
spread workload, the kernel named for each launch plan, the traffic
summary written from two rocprofv3 counter collections (calibrated by the
plain copy of known size), and when a summary is reported."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_spread_rollout():
    # actions 8 B per agent-step, state read 24 B per entity, state written
    # 24 B per agent, static 12 B per entity
    n = bench.algorithmic_bytes(30000, 4, 2, 100)
    assert n == 30000 * (100 * 4 * 8 + 6 * 24 + 4 * 24 + 6 * 12) == 105_360_000


def test_kernel_of_plan():
    assert bench.kernel_of("quad-ordered/64") == "k_rollout_quad_ord"
    assert bench.kernel_of("quad/256") == "k_rollout_quad"
    assert bench.kernel_of("entity-lane/256/size-sorted") == "k_rollout_sph"
    assert bench.kernel_of("pair-queue/256/natural", spheres_only=False) == "k_rollout"


def _collection(path, counter, rows):
    hdr = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(hdr)
        for d, grid, name, vals in rows:
            for v in vals:  # several instances of the counter per dispatch
                wr.writerow([d, grid, name, counter, v])


def test_traffic_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    k = "void vmas::(anonymous namespace)::k_rollout_quad_ord<false, 2, false>(vmas::StepArgs)"
    other = "void vmas::(anonymous namespace)::k_rollout_quad<false, 2, false>(vmas::StepArgs)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    # the 256 MiB copy reads as half its bytes on FETCH_SIZE and its bytes on
    # WRITE_SIZE; a small copy and a kernel whose name shares a prefix are
    # not taken
    _collection(fetch, "FETCH_SIZE", [(1, 512, copy, [5.0]), (2, 1 << 26, copy, [65536.0, 65536.0]),
                                      (3, 30016, k, [25000.0, 25000.0]), (4, 30016, k, [26000.0, 26000.0]),
                                      (5, 30016, other, [1.0])])
    _collection(write, "WRITE_SIZE", [(1, 512, copy, [5.0]), (2, 1 << 26, copy, [262144.0]),
                                      (3, 30016, k, [4000.0]), (4, 30016, k, [4000.0])])
    bench.write_traffic_summary("k_rollout_quad_ord", "t", str(fetch), str(write), "s", "w")
    d = json.load(open(tmp_path / "k_rollout_quad_ord_t_traffic.json"))
    assert d["dispatches"] == 2
    assert d["fetch_scale_from_copy"] == 2.0 and d["write_scale_from_copy"] == 1.0
    assert d["fetch_kib_per_dispatch_raw"] == 51000.0
    assert d["hbm_bytes_per_launch"] == 51000.0 * 1024 * 2.0 + 4000.0 * 1024
    assert d["kernel_source_sha"] == bench.kernel_sha()


def test_traffic_taken_only_for_the_same_sources_and_plan(tmp_path, monkeypatch):
    """A traffic summary is reported only for the kernel sources it was taken
    on and, when a plan is named, for the plan it was taken under."""
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    d = {"kernel": "k_rollout", "schedule": "pair-queue/256/natural/even",
         "kernel_source_sha": bench.kernel_sha(), "hbm_bytes_per_launch": 123.0}
    (tmp_path / "k_rollout_mixed4096_traffic.json").write_text(json.dumps(d))
    assert bench.traffic_per_launch("k_rollout", "mixed4096") == 123.0
    assert bench.traffic_per_launch("k_rollout", "mixed4096", "pair-queue/256/natural/even") == 123.0
    assert bench.traffic_per_launch("k_rollout", "mixed4096", "pair-queue/256/natural") is None
    d["kernel_source_sha"] = "0" * 16
    (tmp_path / "k_rollout_mixed4096_traffic.json").write_text(json.dumps(d))
    assert bench.traffic_per_launch("k_rollout", "mixed4096") is None
    assert bench.traffic_per_launch("k_rollout", "spread30k") is None  # no summary at all
