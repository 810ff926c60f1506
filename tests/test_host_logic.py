"""Host-side logic that needs no GPU: the benchmark's one-GPU guard and the
served-latency summary."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_latency_summary():
    from paper_2410_15227_amd import serve
    jobs = []
    for k in range(100):
        j = serve.Job(key="g", tess=None, pos=np.zeros((1, 3)), h=np.ones(1), m=np.ones(1))
        j.arrival = float(k)
        j.start = j.arrival + 0.5
        j.end = j.arrival + 1.0 + 0.01 * k
        j.n_pairs = 1000
        j.resident_hit = k % 2 == 0
        jobs.append(j)
    s = serve.latency_summary(jobs)
    lat = np.array([1.0 + 0.01 * k for k in range(100)])
    assert s["requests"] == 100 and s["pairs"] == 100000 and s["resident_hits"] == 50
    assert abs(s["p50_ms"] - np.percentile(lat, 50) * 1e3) < 1e-9
    assert abs(s["p99_ms"] - np.percentile(lat, 99) * 1e3) < 1e-9
    assert abs(s["makespan_s"] - (99 + 1.99)) < 1e-12
