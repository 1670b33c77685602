"""Host logic of bench.py (no GPU): the one-GPU guard, the HBM traffic
summary's calibration arithmetic on synthetic counter files, the hash gate
on committed counter summaries, and the step-kind table against the
library's StepKind enum."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert not any(l.startswith("{") for l in r.stdout.splitlines())


def test_step_kinds_follow_the_enum():
    src = open(os.path.join(ROOT, "paper_1202_1350_amd", "csrc", "steps.hpp")).read()
    body = src[src.index("enum StepKind"):]
    body = body[body.index("{") + 1:body.index("};")]
    names = re.findall(r"^\s*ST_([A-Z0-9]+)", body, re.M)
    assert [n.lower() for n in names][:len(bench.STEP_KINDS)] == bench.STEP_KINDS
    assert bench.rocprof_kernel_name("step_wt") == "void gkr::k_step_one<12u, *, *>(gkr::StepDesc)"
    # every specialization of a kind is its kernel, no other kind's
    assert bench.kernel_matches("void gkr::k_step_one<12u, 1, 0>(gkr::StepDesc)", "step_wt")
    assert bench.kernel_matches("void gkr::k_step_one<12u, 0, 0>(gkr::StepDesc)", "step_wt")
    assert not bench.kernel_matches("void gkr::k_step_one<1u, -1, 0>(gkr::StepDesc)", "step_wt")
    assert not bench.kernel_matches("void gkr::k_step_one<12u, 1, 0>(gkr::StepDesc)", "step_start")


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (name, v) in enumerate(rows):
            f.write(f'{i},"{name}",{counter},{v}\n')


def test_traffic_summary_scales_each_counter_by_the_copy(tmp_path):
    k = "void gkr::k_step_one<12u, 1, 0>(gkr::StepDesc)"
    cp = 1 << 30  # the calibration copy moves 1 GiB each way
    # FETCH_SIZE reads half of the copy (factor 2), WRITE_SIZE all of it
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 512 * 1024), (k, 100.0), (k, 300.0)])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1024 * 1024), (k, 50.0), (k, 50.0)])
    text = bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "step_wt", cp, "cmd")
    vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith("#"))
    assert float(vals["fetch_calibration_factor"]) == pytest.approx(2.0)
    assert float(vals["write_calibration_factor"]) == pytest.approx(1.0)
    assert float(vals["fetch_bytes_per_launch"]) == pytest.approx(200 * 1024 * 2, abs=1)
    assert float(vals["write_bytes_per_launch"]) == pytest.approx(50 * 1024, abs=1)
    assert float(vals["hbm_bytes_per_launch"]) == pytest.approx(400 * 1024 + 50 * 1024, abs=1)
    assert vals["kernel_source_hash"] == bench.kernel_source_hash()
    with pytest.raises(SystemExit):  # no calibration copy: refused
        _counter_csv(tmp_path / "g", "FETCH_SIZE", [(k, 1.0)])
        bench.traffic_summary(str(tmp_path / "g"), str(tmp_path / "w"), "step_wt", cp, "cmd")


def test_measured_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    p = tmp_path / "t.txt"
    monkeypatch.setattr(bench, "traffic_path", lambda cls: str(p))
    p.write_text(f"hbm_bytes_per_launch: 12345\nkernel_source_hash: {bench.kernel_source_hash()}\n")
    assert bench.measured_traffic("step_wt") == 12345.0
    p.write_text("hbm_bytes_per_launch: 12345\nkernel_source_hash: 0000000000000000\n")
    assert bench.measured_traffic("step_wt") is None
    p.unlink()
    assert bench.measured_traffic("step_wt") is None
