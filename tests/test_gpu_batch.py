"""Batched forward mapping: several independent instances in one call give,
instance by instance, the same cell masses, coverages and weights as the
single-instance call, bit for bit (each weight depends on its own pair
only), for both precisions."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_15227_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def instances(workloads):
    out = []
    for n, kind, seed in [(1500, "uniform", 40), (6000, "turbulent", 41), (300, "uniform", 42),
                          (12000, "turbulent", 43), (2500, "uniform", 44)]:
        pos, m, h, rho = workloads.make_cloud(kind, n, seed)
        out.append((pos, h, m, workloads.voronoi(pos)))
    return out


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_equals_single(ctx, instances, precision):
    import paper_2410_15227_amd as pkg
    say(f"case: batch of {len(instances)} instances, precision={precision}")
    dts = [pkg.DeviceTessellation(ctx, t) for (_, _, _, t) in instances]
    singles = []
    for (pos, h, m, _), dt in zip(instances, dts):
        r = pkg.map_particles_to_cells(ctx, dt, pos, h, m, precision=precision, keep_pairs=True)
        singles.append((r.mass.cpu().numpy(), r.coverage.cpu().numpy(), [x.cpu().numpy() for x in r.pairs.export()]))
        r.pairs.free()
    batch = pkg.map_particles_to_cells_batch(ctx, dts, [i[0] for i in instances], [i[1] for i in instances],
                                             [i[2] for i in instances], precision=precision, keep_pairs=True)
    torch.cuda.synchronize()
    for k, (res, (M, cov, (off, idx, w))) in enumerate(zip(batch, singles)):
        goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
        assert np.array_equal(goff, off) and np.array_equal(gidx, idx), k
        assert np.array_equal(gw, w), k                      # weights bit for bit
        assert np.array_equal(res.mass.cpu().numpy(), M), k
        assert np.array_equal(res.coverage.cpu().numpy(), cov), k
        res.pairs.free()
    # the batch again without keeping the lists (scratch lists reused)
    again = pkg.map_particles_to_cells_batch(ctx, dts, [i[0] for i in instances], [i[1] for i in instances],
                                             [i[2] for i in instances], precision=precision)
    for res, (M, _, _) in zip(again, singles):
        assert np.array_equal(res.mass.cpu().numpy(), M)
    for dt in dts:
        dt.free()


def test_batch_rejects_bad_input(ctx, instances):
    import paper_2410_15227_amd as pkg
    pos, h, m, t = instances[0]
    dt = pkg.DeviceTessellation(ctx, t)
    with pytest.raises(Exception):
        pkg.map_particles_to_cells_batch(ctx, [dt], [pos], [h[:-1]], [m])
    dt.free()


def test_graph_plan(ctx, instances):
    """The batch captured as one HIP graph: each replay equals the single
    calls bit for bit; after the particle arrays are updated in place a
    replay equals a fresh uncaptured batch on the new values; a step whose
    pair counts pass the lists' capacity (every h enlarged in place) leaves
    the lists empty and raises the overflow flag instead of writing past
    them, and a new plan maps the enlarged supports correctly."""
    import paper_2410_15227_amd as pkg
    say(f"case: graph plan of {len(instances)} instances")
    dts = [pkg.DeviceTessellation(ctx, t) for (_, _, _, t) in instances]
    xs = [torch.tensor(i[0], device="cuda") for i in instances]
    hs = [torch.tensor(i[1], device="cuda") for i in instances]
    ms = [torch.tensor(i[2], device="cuda") for i in instances]
    singles = []
    for dt, x, h, m in zip(dts, xs, hs, ms):
        r = pkg.map_particles_to_cells(ctx, dt, x, h, m, keep_pairs=True)
        singles.append((r.mass.clone(), r.coverage.clone(), r.density.clone(), r.pairs.n_pairs))
        r.pairs.free()
    plan = pkg.BatchPlan(ctx, dts, xs, hs, ms)
    for rep in range(3):
        plan.run()
        counts, over = plan.check()
        assert not over
        for k, (M, cov, rho, npairs) in enumerate(singles):
            assert counts[k] == npairs, (rep, k)
            assert torch.equal(plan.mass[k], M), (rep, k)
            assert torch.equal(plan.coverage[k], cov), (rep, k)
            assert torch.equal(plan.density[k], rho), (rep, k)
    # new positions in the same buffers (a timestep: each moved by about 2e-3)
    g = np.random.default_rng(77)
    for x, (pos, h, m, t) in zip(xs, instances):
        x.copy_(torch.tensor(np.clip(pos + g.normal(size=pos.shape) * 2e-3, 0.0, np.nextafter(1.0, 0.0)),
                             device="cuda"))
    plan.run()
    counts, over = plan.check()
    assert not over
    fresh = pkg.map_particles_to_cells_batch(ctx, dts, xs, hs, ms)
    for k, r in enumerate(fresh):
        assert torch.equal(plan.mass[k], r.mass), k
        assert torch.equal(plan.coverage[k], r.coverage), k
    # supports 1.6 times larger: more pairs than the lists hold
    for h in hs:
        h.mul_(1.6)
    plan.run()
    counts, over = plan.check()
    assert over
    assert all(float(M.abs().sum()) == 0.0 for M, n in zip(plan.mass, counts) if n == 0)
    assert any(n == 0 for n in counts)
    plan.free()
    plan = pkg.BatchPlan(ctx, dts, xs, hs, ms)
    plan.run()
    counts, over = plan.check()
    assert not over
    fresh = pkg.map_particles_to_cells_batch(ctx, dts, xs, hs, ms)
    for k, r in enumerate(fresh):
        assert torch.equal(plan.mass[k], r.mass), k
    plan.free()
    for dt in dts:
        dt.free()


def test_batch_mix_subset_against_oracle(ctx, workloads, oracle):
    """Eight instances of the 64-instance batch mix (round(2^U(12,18))
    particles, uniform or turbulent, seeds 4000 + k), one of them above 2^17
    particles: the captured graph, the uncaptured batch and the single calls
    give the same masses bit for bit, and sampled cells of every instance
    (30 seeded plus the 10 most degenerate) match the oracle within 1e-5."""
    import paper_2410_15227_amd as pkg
    mix = workloads.batch_mix(64, 4000, 12, 18)
    big = next(k for k, (n, _, _) in enumerate(mix) if n >= (1 << 17))
    rest = [k for k in np.random.default_rng(5).permutation(len(mix)) if k != big and mix[k][0] < (1 << 16)][:7]
    pick = [big] + sorted(rest)
    say(f"case: batch mix subset {[mix[k] for k in pick]}")
    inst = []
    for k in pick:
        n, kind, seed = mix[k]
        pos, m, h, rho = workloads.make_cloud(kind, n, seed)
        inst.append((pos, h, m, workloads.voronoi(pos)))
    dts = [pkg.DeviceTessellation(ctx, t) for (_, _, _, t) in inst]
    xs = [torch.tensor(i[0], device="cuda") for i in inst]
    hs = [torch.tensor(i[1], device="cuda") for i in inst]
    ms = [torch.tensor(i[2], device="cuda") for i in inst]
    plan = pkg.BatchPlan(ctx, dts, xs, hs, ms)
    plan.run()
    counts, over = plan.check()
    assert not over
    batch = pkg.map_particles_to_cells_batch(ctx, dts, xs, hs, ms)
    for k, (dt, x, h, m) in enumerate(zip(dts, xs, hs, ms)):
        single = pkg.map_particles_to_cells(ctx, dt, x, h, m)
        assert torch.equal(plan.mass[k], batch[k].mass) and torch.equal(plan.mass[k], single.mass), k
    for k, (pos, h, m, t) in enumerate(inst):
        g = np.random.default_rng(100 + k)
        cells = np.unique(np.concatenate([g.choice(t.n_cells, 30, replace=False),
                                          np.argsort(workloads.degeneracy_scores(t))[-10:]]))
        Mref, _, _ = oracle.map_cells(t, pos, h, m, cells)
        rel = np.abs(plan.mass[k].cpu().numpy()[cells] - Mref) / Mref
        say(f"  instance {pick[k]} n={len(pos)} pairs={counts[k]} max_rel={rel.max():.2e}")
        assert rel.max() < 1e-5
    plan.free()
    for dt in dts:
        dt.free()
