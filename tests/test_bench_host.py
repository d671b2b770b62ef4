"""Host logic of bench.py (CPU): the counter-profile lookup that gates the
reported HBM traffic on the hash of the kernel sources, the recorded launch
configuration, and the one-GPU rule of the command line."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PROFILE = """# a summary
Machine-readable (bench.py reads these while the kernel sources hash to the value below):

    source_sha256: {sha}
    traffic_bytes_per_sweep_f64: 57581645632
    mean_duration_us_per_sweep_f64: 11752.9
    launch_smooth_f64: split=1 tile=28
    launch_tuning_raw: 0,1,732752,1,732752,1,0,28,28
"""


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A repository root with one kernel source and one profile written for it."""
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    (csrc / "k.hip").write_text("// kernel v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "CSRC", str(csrc))
    sha = bench._sha(["k.hip"])
    (tmp_path / "profiles" / "p.md").write_text(PROFILE.format(sha=sha))
    return tmp_path


def test_traffic_read_while_sources_match(tree):
    assert bench.counter_traffic("p.md", ["k.hip"], "traffic_bytes_per_sweep_f64") == 57581645632.0
    # a launch configuration that matches the recorded one keeps the figure
    assert bench.counter_traffic("p.md", ["k.hip"], "traffic_bytes_per_sweep_f64",
                                 require={"launch_smooth_f64": "split=1 tile=28"}) == 57581645632.0


def test_traffic_null_when_sources_or_launch_differ(tree):
    (tree / "csrc" / "k.hip").write_text("// kernel v2\n")
    assert bench.counter_traffic("p.md", ["k.hip"], "traffic_bytes_per_sweep_f64") is None
    assert bench.recorded_launch("p.md", ["k.hip"]) is None


def test_traffic_null_for_other_launch_missing_key_or_file(tree):
    assert bench.counter_traffic("p.md", ["k.hip"], "traffic_bytes_per_sweep_f64",
                                 require={"launch_smooth_f64": "split=0 tile=28"}) is None
    assert bench.counter_traffic("p.md", ["k.hip"], "traffic_bytes_per_sweep_f32") is None
    assert bench.counter_traffic("missing.md", ["k.hip"], "traffic_bytes_per_sweep_f64") is None
    assert bench.counter_traffic("p.md", ["missing.hip"], "traffic_bytes_per_sweep_f64") is None


def test_recorded_launch(tree):
    assert bench.recorded_launch("p.md", ["k.hip"]) == [0, 1, 732752, 1, 732752, 1, 0, 28, 28]


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "exactly one GPU" in res.stdout


def test_profiling_timeline_picks_the_last_iteration(tmp_path, capsys):
    """The timeline summary keeps the dispatches after the second-to-last
    marker up to the last one, with the idle gaps between them."""
    from paper_2510_00998_amd import profiling
    hdr = "Kind,Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp\n"
    ev = [("k_update_ur(double*)", 0, 1000),            # an earlier iteration's marker
          ("void hpmg::k_a<float>(int)", 1000, 3000),
          ("k_update_ur(double*)", 3000, 4000),         # second-to-last marker: iteration starts at 4000
          ("void hpmg::(anonymous namespace)::k_a<float>(int)", 6000, 8000),   # gap 2 us
          ("void hpmg::k_b(int)", 8000, 9000),
          ("k_update_ur(double*)", 9500, 10500)]        # last marker, gap 0.5 us
    path = tmp_path / "trace.csv"
    path.write_text(hdr + "".join(f"KERNEL_DISPATCH,{i},\"{k}\",{a},{b}\n" for i, (k, a, b) in enumerate(ev)))
    profiling.timeline(str(path), "k_update_ur", "t", "cmd")
    out = capsys.readouterr().out
    assert "the 3 dispatches after" in out
    assert "| 0 | `hpmg::k_a<float>` | 2.0 | 2.0 | 2.0 |" in out
    assert "| 2 | `k_update_ur` | 5.5 | 1.0 | 0.5 |" in out
    assert "Iteration span 6.5 us: kernels 4.0 us, idle gaps 2.5 us." in out
