"""bench.py on the CPU: it refuses more than one GPU (the library has no multi-GPU
path) before touching a device, and the source hash that ties stored HBM counters
to the library ignores comments."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_2502_17789_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("int f() { return 1; }  // one\n/* block */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.library_source_hash()
    (csrc / "k.hip").write_text("// header\nint f() {\n  return 1;  // changed comment\n}\n")
    assert bench.library_source_hash() == h0
    (csrc / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.library_source_hash() != h0
