"""Host logic of bench.py, no GPU: the kernel-source digest that ties a
recorded HBM traffic figure to the kernel it was measured on, the lookup of
that figure, the roofline arithmetic of the dominant kernel, and the refusal
of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2304_01728_amd import workloads  # noqa: E402

KA = "template <typename T>\n__global__ void k_a(int x) {\n  x += 1;\n}\n"
KB = "__global__ __launch_bounds__(256) void k_b(int y) {\n  y += 2;\n}\n"


def test_source_digest_covers_only_the_named_kernel(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text(KA + "\n" + KB)
    da, db = bench.source_digest(str(src), "k_a<float>"), bench.source_digest(str(src), "k_b")
    assert da != db
    src.write_text(KA + "\n" + KB.replace("2", "3"))
    assert bench.source_digest(str(src), "k_a<float>") == da
    assert bench.source_digest(str(src), "k_b") != db
    src.write_text("// a comment before\n" + KA + "\n" + KB)
    assert bench.source_digest(str(src), "k_a<float>") == da


def test_measured_traffic_needs_the_workload_and_the_unchanged_kernel(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text(KA + "\n" + KB)
    rec = {"k_a<float>": {"workload": "w1", "bytes_per_launch": 123.0, "source": str(src),
                          "source_sha256_16": bench.source_digest(str(src), "k_a<float>")}}
    tf = tmp_path / "traffic.json"
    tf.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    assert bench.measured_traffic("k_a<float>", "w1") == 123.0
    assert bench.measured_traffic("k_a<float>", "w2") is None
    assert bench.measured_traffic("k_b", "w1") is None
    src.write_text(KA.replace("1", "4") + "\n" + KB)
    assert bench.measured_traffic("k_a<float>", "w1") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("k_a<float>", "w1") is None


def test_recorded_traffic_entries_are_consistent():
    """Each recorded figure names a workload the bench runs and a source
    file that exists, and lies between the algorithmic bytes (every tile is
    read once) and 1.3 times them."""
    with open(bench.TRAFFIC_FILE) as f:
        recs = json.load(f)
    names = {w().name for w in workloads.ALL.values()}
    for sym, r in recs.items():
        assert r["workload"] in names, sym
        assert os.path.exists(os.path.join(ROOT, r["source"])), sym
        ratio = r["bytes_per_launch"] / r["algorithmic_bytes_per_launch"]
        assert 1.0 <= ratio <= 1.3, (sym, ratio)
        assert 1.9 < r["fetch_factor"] < 2.1 and r["write_factor"] == 1.0, sym


def test_roofline_of_the_dominant_apply_kernel(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda sym, w: 7.0e9)
    # (launches, total ms, algorithmic bytes): apply32 dominates by time
    stats = {"apply32": (10, 20.0, 10 * 8.0e9), "apply64": (5, 4.0, 5 * 1.0e9),
             "gram": (3, 1.0, 0.0), "potrf": (9, 50.0, 1e12)}
    r = bench.roofline_for(stats, "any")
    assert r["kernel"] == "k_strips<float>" and r["bound"] == "hbm"
    assert r["avg_ms"] == pytest.approx(2.0)
    assert r["achieved"] == pytest.approx(8.0e9 / 2.0e-3 / 1e9)   # 4000 GB/s
    assert r["frac"] == pytest.approx(4000.0 / bench.HBM_PEAK_GBS)
    assert r["traffic"] == 7.0e9 and r["work_per_launch"] == pytest.approx(8.0e9)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_serving_child_failure_is_loud(monkeypatch):
    """The serving leg runs bench.py --serving in a child process; a child
    that fails (here a stand-in interpreter that exits with status 3) raises
    instead of leaving the leg out of the line."""
    import subprocess as sp
    real = sp.run

    def fake(cmd, **kw):
        assert cmd[2:4] == ["--serving", "--requests"] and cmd[4] == "5"
        return real([sys.executable, "-c", "import sys; sys.exit(3)"], **kw)

    monkeypatch.setattr(sp, "run", fake)
    with pytest.raises(RuntimeError, match="status 3"):
        bench.serving_child(5, 4, 8, 0.7)
