"""Parity of the HIP k-d tree pseudo-particles (Sec. 2.2.1, 2.4) with the
oracle's.

Bars: the emitted set is identical (order, kind, lowest member, member
count, label, level, owner map) with bit-identical positions, masses and
sizes (both sides split through the same fixed-point centres of mass); the
same h-solve branch per pseudo-particle and |h - h_oracle| <= 1e-9 h0 (the
same binary64 iteration; only pow may differ in the last bit); the same
k_mid when the neighbour-find runs."""
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
    ref = oracle.kd_build(pos, m, h, src, **kw)
    kw2 = dict(kw)
    if "bypass" in kw2:
        kw2["bypass_threshold"] = kw2.pop("bypass")
    if "hfact" in kw2:
        kw2["h_fact"] = kw2.pop("hfact")
    got = pkg.build_pseudo_particles(ctx, pos, h, m, src, tree="kd", **kw2)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in got.items() if k != "stats"}
    n = len(ref["kind"])
    assert len(g["kind"]) == n
    for key in ("kind", "first", "count", "branch", "level"):
        assert np.array_equal(g[key], ref[key]), key
    assert np.array_equal(g["label"].view(np.uint64), ref["label"])
    assert np.array_equal(g["owner"], ref["owner"])
    assert np.array_equal(g["xyz"], ref["pos"])
    assert np.array_equal(g["m"], ref["mass"])
    assert np.array_equal(g["s"], ref["s"])
    ps = ref["kind"] == 1
    assert np.array_equal(g["h"][~ps], ref["h"][~ps])
    if ps.any():
        h0 = 1.2 * 2 * ref["s"][ps]
        assert np.max(np.abs(g["h"][ps] - ref["h"][ps]) / h0) <= 1e-9
    st = got["stats"]
    assert st["n_pseudo"] == ref["stats"]["n_pseudo"] and st["n_units"] == ref["stats"]["n_units"]
    assert st["n_nodes"] == ref["stats"]["n_nodes"] and st["k_mid"] == ref["stats"]["k_mid"]
    assert st["s_root"] == ref["s_root"]
    return ref, g, st


def test_uniform_and_turbulent(ctx, oracle, workloads):
    say("case: kd uniform 6000; turbulent 40000 with annulus, brute force and neighbour-find")
    pos, m, h, rho = workloads.make_cloud("uniform", 6000, seed=91)
    compare(ctx, oracle, pos, m, h, np.array([[0.5, 0.5, 0.5]]), r_part=0.1, r_leaf=0.2, theta=0.5)
    pos, m, h, rho = workloads.make_cloud("turbulent", 40000, seed=92)
    src = np.array([pos[workloads.densest_particle(rho)], [0.2, 0.7, 0.4]])
    ref, g, st = compare(ctx, oracle, pos, m, h, src, r_part=0.05, r_leaf=0.15, theta=0.4)
    say(f"  entries={len(g['kind'])} pseudo={st['n_pseudo']} units={st['n_units']} k_mid={st['k_mid']}")
    ref, g, st = compare(ctx, oracle, pos, m, h, src, r_part=0.05, r_leaf=0.15, theta=0.4, nf_threshold=100)
    assert st["k_mid"] >= 0
    say(f"  neighbour-find: k_mid={st['k_mid']} branches={st['branch_count']}")
    compare(ctx, oracle, pos, m, h, src, r_part=0.05, r_leaf=0.15, theta=0.4, nf_threshold=100, up_levels=2)


def test_forced_open_and_degenerate(ctx, oracle, workloads):
    say("case: kd forced opening, small and coincident inputs, bad masses")
    pos, m, h, rho = workloads.make_cloud("turbulent", 20000, seed=93)
    src = pos[workloads.densest_particle(rho)][None, :]
    ref, g, st = compare(ctx, oracle, pos, m, h, src, r_part=0.05, r_leaf=0.1, theta=0.5)
    lab = ref["label"][ref["kind"] == 1][::3]
    compare(ctx, oracle, pos, m, h, src, r_part=0.05, r_leaf=0.1, theta=0.5,
            open_labels=np.concatenate([lab, np.array([5, 1 << 62], np.uint64)]))
    rng = np.random.default_rng(9)
    for n in (1, 2, 9, 10, 11, 64):
        p = rng.random((n, 3))
        compare(ctx, oracle, p, rng.uniform(0.5, 1.5, n), np.full(n, 0.05), np.array([[0.9, 0.1, 0.5]]),
                r_part=0.05, r_leaf=0.3, theta=0.5)
    # 30 coincident particles: no split separates them, so they stay one leaf
    p = np.concatenate([np.full((30, 3), 0.25), rng.random((40, 3))])
    compare(ctx, oracle, p, np.ones(70), np.full(70, 0.05), np.array([[0.9, 0.9, 0.9]]), r_part=0.05,
            r_leaf=0.1, theta=0.5)
    import paper_2410_15227_amd as pkg
    with pytest.raises(Exception):
        pkg.build_pseudo_particles(ctx, p, np.full(70, 0.05), np.zeros(70), [[0.5, 0.5, 0.5]], tree="kd")


@pytest.mark.slow
def test_turbulent_1m(ctx, oracle, workloads):
    """The 1,048,576-particle turbulent cloud with one source at the densest
    particle, r_part 0.2, r_leaf 0.3, theta 0.5."""
    say("case: kd turbulent 1048576")
    pos, m, h, rho = workloads.make_cloud("turbulent", 1 << 20, seed=3)
    src = pos[workloads.densest_particle(rho)][None, :]
    ref, g, st = compare(ctx, oracle, pos, m, h, src, r_part=0.2, r_leaf=0.3, theta=0.5)
    say(f"  entries={len(g['kind'])} pseudo={st['n_pseudo']} units={st['n_units']} nodes={st['n_nodes']} "
        f"k_mid={st['k_mid']} branches={st['branch_count']}")
