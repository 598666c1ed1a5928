"""CPU checks of bench.py's contract that need no GPU: it refuses more than
one GPU with a message, and the counter figures it reports are used only
while they were taken from the kernel sources that run (profiles/traffic.json
keyed by the hash of every kernel source and the tuning table)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_figures_follow_the_source_hash(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    (tmp_path / "profiles").mkdir()
    entry = {"kernel_hash": h, "bytes_per_level_launch": 123.0, "bytes_per_build": 456.0}
    stale = dict(entry, kernel_hash="0" * 16 if h != "0" * 16 else "1" * 16)
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(
        {"c2": entry, "c3": stale, "c4": {"kernel_hash": h, "bytes_per_batched_build": 7.0}, "kernel_hash": h}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("c2") == 123.0
    assert bench.load_traffic("c3") is None          # taken from other sources: not reported
    assert bench.load_traffic("c1") is None          # never taken
    assert bench.load_batch_traffic() == 7.0


def test_source_hash_changes_with_any_kernel_source_or_the_tuning_table(tmp_path, monkeypatch):
    import shutil
    from paper_1610_05994_amd import profiling
    pkg = os.path.join(ROOT, "paper_1610_05994_amd")
    copy = tmp_path / "pkg"
    shutil.copytree(os.path.join(pkg, "csrc"), copy / "csrc")
    shutil.copy(os.path.join(pkg, "tune_table.json"), copy / "tune_table.json")
    monkeypatch.setattr(profiling, "_PKG", str(copy))
    base = profiling.kernel_source_hash()
    assert base == bench.kernel_source_hash()  # (bench asks the same function)
    seen = {base}
    for name in sorted(os.listdir(copy / "csrc")) + ["../tune_table.json"]:
        path = copy / "csrc" / name
        old = path.read_bytes()
        path.write_bytes(old + b"\n")
        h = profiling.kernel_source_hash()
        assert h not in seen, name
        seen.add(h)
        path.write_bytes(old)
    assert profiling.kernel_source_hash() == base
