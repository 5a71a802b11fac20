"""Host-side pieces of bench.py: the one-GPU refusal, the traffic lookup that
feeds roofline.traffic, and the algorithmic byte counts behind roofline.achieved."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_lookup_follows_the_kernel_source_hash(tmp_path):
    rec = {"kernels_hip_sha": "abc123", "fetch_scale": 2.0, "write_scale": 1.0,
           "fp32": {"patch_forward": {"kernel": "void kmv::k_step<float, 2, 18, false>(kmv::StepArgs<float>)",
                                      "fetch_kib": 1.0, "write_kib": 2.0, "bytes_per_launch": 12345},
                    "patch_adjoint": {"kernel": "void kmv::k_step<float, 2, 18, true>(kmv::StepArgs<float>)",
                                      "fetch_kib": 1.0, "write_kib": 2.0, "bytes_per_launch": 67890}}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    assert bench.traffic_from_profiles("patch_forward", "abc123", "fp32", str(p)) == 12345
    assert bench.traffic_from_profiles("patch_adjoint", "abc123", "fp32", str(p)) == 67890
    assert bench.traffic_from_profiles("patch_forward", "other", "fp32", str(p)) is None
    assert bench.traffic_from_profiles("missing", "abc123", "fp32", str(p)) is None
    assert bench.traffic_from_profiles("patch_forward", "abc123", "fp32", str(tmp_path / "none.json")) is None


def test_fp64_roofline_never_takes_fp32_traffic(tmp_path):
    """Counter bytes are per precision: an FP64 lookup finds nothing when only FP32
    counters were taken, and a record filed under fp64 whose kernel is the float
    instance is refused too."""
    fwd32 = {"kernel": "void kmv::k_step<float, 2, 18, false>(kmv::StepArgs<float>)",
             "fetch_kib": 1.0, "write_kib": 2.0, "bytes_per_launch": 111}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"kernels_hip_sha": "h", "fp32": {"patch_forward": fwd32}}))
    assert bench.traffic_from_profiles("patch_forward", "h", "fp32", str(p)) == 111
    assert bench.traffic_from_profiles("patch_forward", "h", "fp64", str(p)) is None
    p.write_text(json.dumps({"kernels_hip_sha": "h", "fp64": {"patch_forward": fwd32}}))
    assert bench.traffic_from_profiles("patch_forward", "h", "fp64", str(p)) is None
    fwd64 = dict(fwd32, kernel="void kmv::k_step<double, 2, 18, false>(kmv::StepArgs<double>)",
                 bytes_per_launch=222)
    p.write_text(json.dumps({"kernels_hip_sha": "h", "fp32": {"patch_forward": fwd32},
                             "fp64": {"patch_forward": fwd64}}))
    assert bench.traffic_from_profiles("patch_forward", "h", "fp64", str(p)) == 222
    assert bench.traffic_from_profiles("patch_forward", "h", "fp32", str(p)) == 111
    # the roofline of an FP64 result asks for the fp64 record
    res = {"n_dofs": 1000, "n_cells": 300,
           "prof": {"patch_forward": {"timed": 1, "launches": 1, "mean_ms": 0.01},
                    "patch_adjoint": {"timed": 0, "launches": 0, "mean_ms": 0.0}}}
    orig = bench.traffic_from_profiles
    seen = []
    try:
        bench.traffic_from_profiles = lambda v, h, prec="fp32", path=None: seen.append(prec)
        bench.roofline(res, 8)
        bench.roofline(dict(res), 4)
    finally:
        bench.traffic_from_profiles = orig
    assert seen == ["fp64", "fp32"]


def test_committed_traffic_summary_is_per_precision():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert len(d["kernels_hip_sha"]) == 16
    for prec, ctype in (("fp32", "float"), ("fp64", "double")):
        for v, rec in (d.get(prec) or {}).items():
            assert rec["bytes_per_launch"] > 0
            assert f"k_step<{ctype}," in rec["kernel"].replace(" ", "")


def test_host_cpu_is_stated():
    h = bench.host_cpu()
    assert h["os_cpu_count"] == os.cpu_count()
    assert h["cpus_allowed"] is None or 1 <= h["cpus_allowed"] <= os.cpu_count()


def test_algorithmic_bytes():
    N, E = 1000, 300
    topo2, geom2 = 4 * 6, 3 * 4
    # one shot: 7 values per DOF forward, 8 values + a float64 read-modify-write adjoint
    assert bench.algorithmic_bytes("patch_forward", N, E, 2, 4) == N * 7 * 4 + E * (topo2 + geom2)
    assert bench.algorithmic_bytes("patch_adjoint", N, E, 2, 4) == N * (8 * 4 + 16) + E * (topo2 + geom2)
    # several shots share c^2, gamma, beta and the cell tables
    f1 = bench.algorithmic_bytes("patch_forward", N, E, 2, 4, 1)
    f8 = bench.algorithmic_bytes("patch_forward", N, E, 2, 4, 8)
    assert f8 - f1 == 7 * N * 4 * 4
    a1 = bench.algorithmic_bytes("patch_adjoint", N, E, 3, 8, 1)
    a3 = bench.algorithmic_bytes("patch_adjoint", N, E, 3, 8, 3)
    assert a3 - a1 == 2 * N * (5 * 8 + 16)


def test_trace_busy_summary(tmp_path):
    """The serving trace summary: a set-up stream, then two server streams whose
    kernels overlap and leave two idle stretches (20 and 100 time units)."""
    import csv
    S = 1000000
    rows = [("1", 0, 100, "k_dot"), ("2", 1000, 1100, "k_step<float>"), ("2", 1150, 1250, "k_step<float>"),
            ("3", 1120, 1300, "k_step<float>"), ("2", 1400, 1500, "k_misfit")]
    path = tmp_path / "kernel_trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kind", "Stream_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for sid, a, b, name in rows:
            w.writerow(["KERNEL_DISPATCH", sid, name, a * S, b * S])
    r = bench.trace_busy_summary(str(path))
    assert r["window_ms"] == 500 and r["busy_ms"] == 380 and r["idle_frac"] == 0.24
    s2 = r["streams"]["2"]
    assert s2["kernels"] == 3 and s2["kernel_ms"] == 300 and s2["gap_ms"] == 200 and s2["gap_frac"] == 0.4
    assert s2["median_step_us"] == 100000.0
    assert "1" not in r["streams"]
