"""CPU checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and the PMC traffic figure is used only while the
committed summary was taken on the current sweep source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_current_kernel(tmp_path, monkeypatch):
    import bench
    good = "kernel source sha256[:16]: `%s`\n\nHBM bytes per launch (scaled): 3.5e+09\n" % bench.kernel_source_hash()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "fw_sweep_w_pmc.md").write_text(good)
    (tmp_path / "profiles" / "fw_sweep_old_pmc.md").write_text(good.replace(bench.kernel_source_hash(), "0" * 16))
    src = tmp_path / "paper_2504_10937_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "fw.hip").write_bytes(open(os.path.join(ROOT, "paper_2504_10937_amd", "csrc", "fw.hip"), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w") == 3.5e9
    assert bench.measured_traffic("old") is None
    assert bench.measured_traffic("missing") is None
