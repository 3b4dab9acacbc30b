"""Host-side parts of bench.py (no GPU): the one-GPU guard, the roofline
arithmetic of both paths, and the lookup of counted HBM bytes in the
committed counter summaries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_of_both_paths():
    import bench
    g = bench.roofline_of("gather", {"alg_bytes": 4e9}, 1.0)
    assert g["bound"] == "hbm" and g["unit"] == "GB/s"
    assert abs(g["achieved"] - 4000.0) < 1e-9 and abs(g["frac"] - 0.5) < 1e-12
    b = bench.roofline_of("band", {"alg_ops": 2.5e12}, 1.0, counted=1.0e9)
    assert b["bound"] == "mfma" and b["unit"] == "TOP/s" and b["traffic"] == 1.0e9
    assert abs(b["achieved"] - 2500.0) < 1e-9 and abs(b["frac"] - 0.5) < 1e-12


def test_counted_traffic_needs_matching_workload_and_sources():
    import bench
    # a workload no summary covers
    assert bench.counted_traffic("n=1 nq=1 k=1 w=1", "band") == (None, None)
    # a found summary names the workload and the md5 of the sources built here
    for path in ("band", "gather"):
        tb, src = bench.counted_traffic("n=10000000 nq=100000 k=10 w=27648", path)
        if tb is not None:
            text = open(os.path.join(ROOT, src)).read()
            assert "workload: n=10000000 nq=100000 k=10 w=27648" in text
            assert f"kernel_sources_md5: {bench.sources_md5(path)}" in text
            assert tb > 0
