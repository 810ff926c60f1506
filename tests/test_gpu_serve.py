"""Served mapping: jobs admitted while others run overlap on the device and
each gives the same cell masses as when run alone; repeat-timestep jobs map
the resident particles with a jitter drawn on the device and copy nothing
from the host; a memory budget that fits one job at a time still completes
every job; resident grids are reused.  One grid holds 120,000 particles."""
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
    for k, (n, kind) in enumerate([(1200, "uniform"), (5000, "turbulent"), (3000, "uniform"), (120000, "turbulent")]):
        pos, m, h, rho = workloads.make_cloud(kind, n, 700 + k)
        out.append(dict(key=f"g{k}", pos=pos, m=m, h=h, rho=rho, tess=workloads.voronoi(pos)))
    return out


def job(serve, g, seed=None):
    return serve.Job(g["key"], g["tess"], g["pos"], g["h"], g["m"], rho=g["rho"], jitter_seed=seed)


def test_same_alone_and_in_mix(pool, oracle):
    from paper_2410_15227_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("case: 16 jobs (4 grids, 12 repeat timesteps) on 3 slots against each alone")
    srv = serve.MappingServer(0, slots=3, hbm_budget=16 << 30)
    first = [srv.submit(job(serve, g)) for g in pool]
    srv.drain()
    mix = first + [srv.submit(job(serve, pool[i % len(pool)], seed=100 + i)) for i in range(12)]
    srv.drain()
    assert not [j.error for j in mix if j.error]
    reps = mix[len(pool):]
    assert all(j.resident_hit for j in reps)
    # repeat timesteps copy nothing from the host
    assert all(j.host_bytes == 0 for j in reps)
    assert all(j.host_bytes > 0 for j in first)
    for j in mix:
        solo = srv.submit(job(serve, next(g for g in pool if g["key"] == j.key), seed=j.jitter_seed))
        solo.done.wait()
        assert solo.error is None
        assert torch.equal(solo.mass, j.mass)
        assert torch.equal(solo.coverage, j.coverage)
    # a repeat job moved its particles: its masses differ from the grid's first job
    g3 = [j for j in mix if j.key == "g3"]
    assert not torch.equal(g3[0].mass, g3[1].mass)
    # the 120,000-particle job against the oracle on sampled cells
    g = pool[3]
    cells = np.random.default_rng(9).choice(g["tess"].n_cells, 60, replace=False)
    Mref, _, _ = oracle.map_cells(g["tess"], g["pos"], g["h"], g["m"], cells)
    got = g3[0].mass.cpu().numpy()[cells]
    assert np.max(np.abs(got - Mref) / Mref) < 1e-5
    s = serve.latency_summary(mix)
    assert s["requests"] == 16 and s["pairs"] > 0 and s["p99_ms"] >= s["p50_ms"]
    assert s["repeat_jobs"] == 12 and s["repeat_host_bytes"] == 0
    srv.close()


def test_budget_of_one_job(pool):
    from paper_2410_15227_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("case: budget below two jobs")
    g = pool[1]
    srv = serve.MappingServer(0, slots=3, hbm_budget=1 << 40)
    one = srv.footprint_bytes(job(serve, g, seed=1))
    srv.close()
    srv = serve.MappingServer(0, slots=3, hbm_budget=one)
    mix = [srv.submit(job(serve, g, seed=50 + i)) for i in range(6)]
    srv.drain()
    assert not [j.error for j in mix if j.error]
    # admitted one at a time: no two jobs overlap in time
    spans = sorted((j.start, j.end) for j in mix)
    assert all(b[0] >= a[1] for a, b in zip(spans, spans[1:]))
    srv.close()
