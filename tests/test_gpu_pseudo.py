"""Parity of the HIP pseudo-particle builder (Sec. 2.4) with the oracle's.

Bars: the emitted set is identical (order, kind, lowest member, member count
and bit-identical position, mass and node size); each pseudo-particle takes
the same h-solve branch and |h - h_oracle| <= 1e-9 h0 (both iterate the same
binary64 recurrence; only the power function may differ in the last bit)."""
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


def compare(ctx, oracle, pos, m, h, src, **kw):
    import paper_2410_15227_amd as pkg
    ref = oracle.pseudo_build(pos, m, h, src, **{k: v for k, v in kw.items() if k != "bypass_threshold"},
                              **({"bypass": kw["bypass_threshold"]} if "bypass_threshold" in kw else {}))
    got = pkg.build_pseudo_particles(ctx, pos, m=m, h=h, xyz=None, sources=src, **kw) if False else \
        pkg.build_pseudo_particles(ctx, pos, h, m, src, **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in got.items() if k != "stats"}
    n = len(ref["kind"])
    assert len(g["kind"]) == n
    assert np.array_equal(g["kind"], ref["kind"])
    assert np.array_equal(g["first"], ref["first"])
    assert np.array_equal(g["count"], ref["count"])
    assert np.array_equal(g["xyz"], ref["pos"])          # bit-identical
    assert np.array_equal(g["m"], ref["mass"])
    assert np.array_equal(g["s"], ref["s"])
    assert np.array_equal(g["branch"], ref["branch"])
    ps = ref["kind"] == 1
    real = ~ps
    assert np.array_equal(g["h"][real], ref["h"][real])
    h0 = 1.2 * 2 * ref["s"][ps]
    if ps.any():
        assert np.max(np.abs(g["h"][ps] - ref["h"][ps]) / h0) <= 1e-9
    st = got["stats"]
    assert st["n_pseudo"] == int(ps.sum()) and st["n_units"] == len(ref["upos"])
    assert st["n_nodes"] == ref["n_nodes"]
    return ref, g, st


def test_uniform_cloud(ctx, oracle, workloads):
    say("case: pseudo uniform 6000, one source")
    pos, m, h, rho = workloads.make_cloud("uniform", 6000, seed=21)
    ref, g, st = compare(ctx, oracle, pos, m, h, np.array([[0.5, 0.5, 0.5]]), r_part=0.2, theta=0.5)
    assert abs(g["m"].sum() - m.sum()) < 1e-12
    say(f"  entries={len(g['m'])} pseudo={st['n_pseudo']} branches={st['branch_count']}")


def test_turbulent_two_sources(ctx, oracle, workloads):
    say("case: pseudo turbulent 40000, two sources")
    pos, m, h, rho = workloads.make_cloud("turbulent", 40000, seed=31)
    src = np.array([pos[workloads.densest_particle(rho)], [0.1, 0.8, 0.3]])
    compare(ctx, oracle, pos, m, h, src, r_part=0.15, theta=0.4)


def test_small_and_degenerate(ctx, oracle, workloads):
    say("case: pseudo tiny inputs and bypass")
    g = np.random.default_rng(5)
    for n in [1, 2, 7, 8, 9, 50]:
        pos = g.random((n, 3))
        m = g.uniform(0.5, 1.5, n)
        h = np.full(n, 0.05)
        compare(ctx, oracle, pos, m, h, np.array([[0.9, 0.9, 0.9]]), r_part=0.05, theta=0.8)
    pos, m, h, rho = workloads.make_cloud("uniform", 3000, seed=8)
    ref, gg, st = compare(ctx, oracle, pos, m, h, np.array([[0.2, 0.2, 0.2]]), r_part=0.1, theta=0.5,
                          bypass_threshold=3)
    assert np.all(gg["branch"][gg["kind"] == 1] == 3)


@pytest.mark.slow
def test_turbulent_1m_densest_source(ctx, oracle, workloads):
    """Pseudo-particles of the 1,048,576-particle turbulent cloud with one
    source at the densest particle (r_part 0.2, theta 0.5, leaf <= 8)."""
    say("case: pseudo turbulent 1048576, densest source")
    pos, m, h, rho = workloads.make_cloud("turbulent", 1 << 20, seed=3)
    src = pos[workloads.densest_particle(rho)][None, :]
    ref, g, st = compare(ctx, oracle, pos, m, h, src, r_part=0.2, theta=0.5)
    say(f"  entries={len(g['m'])} pseudo={st['n_pseudo']} real={st['n_real']} nodes={st['n_nodes']} "
        f"branches={st['branch_count']}")
