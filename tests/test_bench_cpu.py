"""Host logic of bench.py, no GPU: the one-GPU guard, the kernel named for
each profiled operation, the roofline arithmetic (algorithmic bytes per launch
over event-timed launch time, against the 8 TB/s HBM peak) and the rule that
measured traffic is reported only for the kernel source it was taken on."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("op,kernel", [
    ("edgejoin_dense", "k_ejv"),
    ("edgejoin2_sparse_op5+6", "k_ejv"),
    ("edgejoin_sparse_op10", "k_ejv"),
    ("merge_edge_dense_op6", "k_medge_v / k_medge"),
    ("merge_root_terms_sparse", "k_mroot_rows / k_mroot_terms"),
    ("level_build_sparse", "k_mark_* / k_cmp_*"),
    ("light", "k_light"),
])
def test_kernel_of(op, kernel):
    assert bench.kernel_of(op) == kernel


def test_roofline_arithmetic():
    # op -> (launches, seconds, ...): the untimed profiled solve and the timed steps
    pstats = {"edgejoin_dense": (10, 2.0, 0, 0), "edgejoin_sparse": (30, 0.5, 0, 0),
              "merge_root_dense": (10, 1.0, 0, 0), "level_build_sparse": (30, 0.1, 0, 0)}
    tstats = {"edgejoin_dense": (20, 3.0, 0, 0), "edgejoin_sparse": (60, 1.0, 0, 0)}
    # op -> (launches, seconds, algorithmic bytes, (triples scanned, rows relaxed, rows written))
    cstats = {"edgejoin_dense": (10, 0.0, 1.0e10, (100, 200, 300)),
              "edgejoin_sparse": (30, 0.0, 3.0e9, (30, 60, 90)),
              "merge_root_dense": (10, 0.0, 5.0e9, (0, 0, 0))}
    roof, kern = bench.roofline(tstats, pstats, cstats, "no_such_workload")
    assert roof["kernel"] == "k_ejv"  # 2.5 s of the profiled solve against 1.0 s
    # timed: 20 dense launches at 1e9 B and 60 sparse launches at 1e8 B over 4.0 s
    assert roof["launches"] == 80
    assert roof["alg_bytes_per_launch"] == pytest.approx((20 * 1e9 + 60 * 1e8) / 80)
    assert roof["achieved"] == pytest.approx((20 * 1e9 + 60 * 1e8) / 4.0 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)
    assert roof["avg_launch_ms"] == pytest.approx(4000.0 / 80)
    assert roof["traffic"] is None
    allk = roof["all_kernels"]
    assert allk["kernel_s"] == pytest.approx(3.6)
    assert allk["alg_GB"] == pytest.approx((1e10 + 3e9 + 5e9) / 1e9)
    assert allk["kernels_without_byte_count"] == ["k_mark_* / k_cmp_*"]
    assert kern["edgejoin_dense"]["per_launch_rows_written"] == pytest.approx(30.0)
    assert kern["merge_root_dense"]["alg_GBps"] == pytest.approx(5.0)


def test_traffic_only_for_the_source_it_was_taken_on(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1602_04478_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "heavy.hip"
    src.write_bytes(b"// kernel source A\n")
    rec = {"source": "heavy.hip", "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "hbm_bytes_per_launch": 1234.5}
    (tmp_path / "profiles" / "k_ejv_wl_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record("k_ejv", "wl") == 1234.5
    assert bench.traffic_record("k_ejv", "other") is None
    src.write_bytes(b"// kernel source B\n")
    assert bench.traffic_record("k_ejv", "wl") is None
