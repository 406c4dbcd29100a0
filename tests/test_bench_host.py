"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the
phase table of the bench line, and the rule that recorded HBM traffic is
reported only for the kernel sources it was measured on."""
import os
import shutil
import subprocess
import sys

import bench
import paper_1604_01632_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_phase_passes_name_every_timed_phase():
    assert set(bench.PHASE_PASSES) == {p + "_ms" for p in pkg.PHASES}
    assert all(v for v in bench.PHASE_PASSES.values())


def test_recorded_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """The recorded bytes come back only while the HIP sources hash to the
    value stored beside them, and only for the workload they were taken on."""
    src = tmp_path / "csrc"
    shutil.copytree(bench.CSRC, src)
    monkeypatch.setattr(bench, "CSRC", str(src))
    h = bench.kernel_source_hash()
    prof = tmp_path / "traffic.md"
    prof.write_text(f"# t\n\n- hbm_bytes_per_launch: `2.5e+09`\n- kernel_source_sha256: `{h}`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    assert bench.recorded_traffic("fp32", "p1") == 2.5e9
    assert bench.recorded_traffic("fp16dev", "p1") is None
    assert bench.recorded_traffic("fp32", "c2") is None
    # any change to a kernel source voids it
    name = sorted(n for n in os.listdir(src) if n.endswith(".hpp"))[0]
    with open(src / name, "a") as fh:
        fh.write("\n// changed\n")
    assert bench.kernel_source_hash() != h
    assert bench.recorded_traffic("fp32", "p1") is None
