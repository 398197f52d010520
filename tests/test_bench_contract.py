"""Host-side parts of the benchmark's contract (no GPU): the refusal of more
than one GPU, and the guard that keeps counter-derived figures (HBM traffic,
VALU issue) out of the report unless they were taken on the current kernel
sources and the same workload."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

WORKLOAD = bench.HEADLINE_WORKLOAD


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def _record(tmp_path, monkeypatch, sha, workload):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_sha": sha, "records": [{
        "kernel": "k", "workload": workload, "bytes_per_launch": 123.0, "valu_busy": 0.5,
        "valu_lane_utilisation": 0.9, "valu_instructions_per_path_step": 100.0}]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))


def test_counters_reported_for_current_sources_and_workload(tmp_path, monkeypatch):
    _record(tmp_path, monkeypatch, bench.kernel_source_hash(), WORKLOAD)
    assert bench.measured_traffic("k", WORKLOAD) == 123.0
    assert bench._issue(bench.measured_counters("k", WORKLOAD)) == {
        "busy": 0.5, "lane_utilisation": 0.9, "instructions_per_path_step": 100.0}


@pytest.mark.parametrize("what", ["stale_sources", "other_workload", "other_kernel", "no_file"])
def test_counters_withheld_otherwise(tmp_path, monkeypatch, what):
    sha = "0" * 16 if what == "stale_sources" else bench.kernel_source_hash()
    _record(tmp_path, monkeypatch, sha, WORKLOAD + " (other)" if what == "other_workload" else WORKLOAD)
    if what == "no_file":
        monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    kernel = "other" if what == "other_kernel" else "k"
    assert bench.measured_traffic(kernel, WORKLOAD) is None
    assert bench._issue(bench.measured_counters(kernel, WORKLOAD)) is None



def test_headline_kernel_names_follow_the_library_choice():
    # the plain FP64 kernel with a row-major copy has its own four-wave build;
    # every other instance runs the kernel of its feature set
    assert bench.path_kernel_name(64, 0, True) == "fk_stream_f64_l1"
    assert bench.path_kernel_name(64, 2, False) == "fk_stream_f64<2>"
    assert bench.path_kernel_name(32, 0, True) == "fk_stream_f32<0>"
    assert bench.path_kernel_name(32, 2, True, lds=True) == "fk_stream_f32_lds<2>"
    assert bench.flops_per_step(64, True) == 60.0
    # disc domains run the curved-edge builds (feature bit 6 with a hole and
    # the reflecting edge)
    from paper_2308_11469_amd import workloads as W
    p = W.annulus_shape2(k=0.5, n=91)
    assert bench._features(p) == 73
    assert bench.path_kernel_name(64, bench._features(p), False) == "fk_stream_f64<73>"
    assert bench.path_kernel_name(32, bench._features(p), True) == "fk_stream_f32<73>"
    assert bench._features(W.annulus_shape3(nx=21, ny=33)) == 9


def test_only_parts_parse():
    for name in bench.ONLY:
        assert bench.parse(["--only", name]).only == name
