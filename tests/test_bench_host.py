"""Host-side logic of bench.py that needs no GPU: the refusal of more than
one GPU, and the fields of the oracle's CPU baseline."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_cpu_baseline_fields():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1908_02681_amd import gen
    cloud, view = gen.config1(n=5000)
    out = bench.cpu_baseline(cloud, view, (1, 100), min_s=0.0, budget_s=60.0)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "Gpoints/s"
    assert out["value"] > 0
    assert out["sample"].startswith("3 full frames") and "host cores" in out["sample"]
