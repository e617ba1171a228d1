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


def test_committed_bench_line_keeps_the_contract():
    """The committed bench line carries every field of the output contract, its roofline
    fraction is achieved / peak, its value is the visibilities of one step over the step
    time, and its traffic is the committed counter record's bytes for that kernel."""
    import json
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_mwa_line.json")))
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    n_vis = d["config"]["n_vis"]
    assert abs(d["value"] - n_vis / (d["ms_per_step"] * 1e-3) / 1e6) < 1e-2 * d["value"]
    rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic_mwa.json")))
    assert r["traffic"] == round(rec["kernels"][r["kernel"]]["bytes_per_launch"])
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
