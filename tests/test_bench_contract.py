"""Host-side parts of bench.py's contract (no GPU): the one-GPU rule, the
algorithmic byte model, and the gating of measured traffic on sources,
workload and launch schedule."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_algorithmic_bytes_follow_the_truncated_layout():
    import bench
    # 1024^2 mixed: K = 341, 342 x 683 spectral entries, row fields 1024 x 342
    ab = bench.algorithmic_bytes(1024, True)
    rowfield = 1024 * 342 * 8
    phys4 = 1024 * 1024 * 16
    assert ab["rows_dyn"] == 9 * rowfield + phys4
    assert ab["rows_rhs"] == 24 * rowfield + phys4
    state = 342 * 683 * (9 * 8 + 4 * 16)
    comp = 0.5 * 9 * 342 * 683 * 8  # trailing words of the compensated float32 state, stage 4 only
    assert abs(ab["columns"] - (33 * rowfield + 2.75 * state + 6 * 342 * 683 * 8 + comp)) < 1
    # float64 doubles every float32 stream
    ab64 = bench.algorithmic_bytes(1024, False)
    assert ab64["rows_dyn"] == 2 * ab["rows_dyn"]


def test_measured_traffic_is_gated(tmp_path, monkeypatch):
    import bench
    lines = ["workload: sw1024_fp32", f"source_sha256: {bench.kernel_source_hash()}", "schedule: 1,1",
             "traffic_bytes_columns: 123"]
    f = tmp_path / "t.md"
    f.write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("columns", "sw1024_fp32", (1, 1)) == 123.0
    assert bench.measured_traffic("columns", "sw1024_fp32", (0, 1)) is None      # another schedule
    assert bench.measured_traffic("columns", "sw256_fp64", (1, 1)) is None       # another workload
    lines[1] = "source_sha256: " + "0" * 64
    f.write_text("\n".join(lines) + "\n")
    assert bench.measured_traffic("columns", "sw1024_fp32", (1, 1)) is None      # other kernel sources
