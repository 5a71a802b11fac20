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
           "patch_forward": {"kernel": "k", "fetch_kib": 1.0, "write_kib": 2.0, "bytes_per_launch": 12345},
           "patch_adjoint": {"kernel": "k", "fetch_kib": 1.0, "write_kib": 2.0, "bytes_per_launch": 67890}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    assert bench.traffic_from_profiles("patch_forward", "abc123", str(p)) == 12345
    assert bench.traffic_from_profiles("patch_adjoint", "abc123", str(p)) == 67890
    assert bench.traffic_from_profiles("patch_forward", "other", str(p)) is None
    assert bench.traffic_from_profiles("missing", "abc123", str(p)) is None
    assert bench.traffic_from_profiles("patch_forward", "abc123", str(tmp_path / "none.json")) is None


def test_committed_traffic_summary_has_both_variants():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert len(d["kernels_hip_sha"]) == 16
    for v in ("patch_forward", "patch_adjoint"):
        assert d[v]["bytes_per_launch"] > 0


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
