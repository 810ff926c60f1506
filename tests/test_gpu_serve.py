"""Served mapping: jobs admitted while others run overlap on the device and
each gives the same cell masses as when run alone; a memory budget that fits
one job at a time still completes every job; resident grids are reused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pool(workloads):
    out = []
    for k, (n, kind) in enumerate([(1200, "uniform"), (5000, "turbulent"), (3000, "uniform")]):
        pos, m, h, rho = workloads.make_cloud(kind, n, 700 + k)
        out.append(dict(key=f"g{k}", pos=pos, m=m, h=h, rho=rho, tess=workloads.voronoi(pos)))
    return out


def jobs_for(serve, workloads, pool, count=12):
    jobs = []
    for i in range(count):
        g = pool[i % len(pool)]
        pos = g["pos"] if i < len(pool) else workloads.jitter(g["pos"], g["m"], g["rho"], seed=i)
        jobs.append(serve.Job(g["key"], g["tess"], pos, g["h"], g["m"]))
    return jobs


def test_same_alone_and_in_mix(pool, workloads):
    from paper_2410_15227_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("case: 12 jobs on 3 slots against each alone")
    srv = serve.MappingServer(0, slots=3, hbm_budget=8 << 30)
    mix = [srv.submit(j) for j in jobs_for(serve, workloads, pool)]
    srv.drain()
    assert not [j.error for j in mix if j.error]
    assert sum(j.resident_hit for j in mix) >= len(mix) - 3 * len(pool)
    for j in mix:
        solo = srv.submit(serve.Job(j.key, j.tess, j.pos, j.h, j.m))
        solo.done.wait()
        assert solo.error is None
        assert torch.equal(solo.mass, j.mass)
        assert torch.equal(solo.coverage, j.coverage)
    s = serve.latency_summary(mix)
    assert s["requests"] == 12 and s["pairs"] > 0 and s["p99_ms"] >= s["p50_ms"]
    srv.close()


def test_budget_of_one_job(pool, workloads):
    from paper_2410_15227_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("case: budget below two jobs")
    g = pool[1]
    import paper_2410_15227_amd as pkg
    c = pkg.Context(0)
    fp = c.estimate_footprint(len(g["m"]), g["tess"])
    c.close()
    one = fp["workspace"] + fp["pairs"] + fp["tessellation"]
    srv = serve.MappingServer(0, slots=3, hbm_budget=one)
    mix = [srv.submit(serve.Job(g["key"], g["tess"], workloads.jitter(g["pos"], g["m"], g["rho"], seed=50 + i),
                                g["h"], g["m"])) for i in range(6)]
    srv.drain()
    assert not [j.error for j in mix if j.error]
    # admitted one at a time: no two jobs overlap in time
    spans = sorted((j.start, j.end) for j in mix)
    assert all(b[0] >= a[1] for a, b in zip(spans, spans[1:]))
    srv.close()
