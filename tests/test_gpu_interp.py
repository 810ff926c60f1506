"""Parity of the HIP per-particle interpolation from the mixed set (Sec. 3.3)
and of the builder's owner map with the oracle's.

Bars: the owner map is identical; interpolated values agree with the oracle's
on the same entries within 1e-12 times the largest entry value (the same
binary64 terms, summed in another order); particles emitted as themselves and
particles no sphere reaches get their owner's value bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12


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


def mixed_set(ref, dev="cuda"):
    """The oracle's mixed set as the device dict the interpolation reads."""
    return dict(xyz=torch.tensor(ref["pos"], device=dev), h=torch.tensor(ref["h"], device=dev),
                kind=torch.tensor(ref["kind"], device=dev), owner=torch.tensor(ref["owner"], device=dev))


def check(ctx, oracle, pos, ref, values, sample=None):
    import paper_2410_15227_amd as pkg
    got = pkg.interpolate_to_particles(ctx, pos, mixed_set(ref), values).cpu().numpy()
    idx = np.arange(len(pos)) if sample is None else sample
    want = oracle.interpolate(pos[idx], ref["owner"][idx], ref["pos"], ref["h"], ref["kind"], values)
    scale = max(np.abs(values).max(), 1e-300)
    err = np.abs(got[idx] - want).max() / scale
    real = ref["kind"][ref["owner"][idx]] == 0
    assert np.array_equal(got[idx][real], want[real])
    assert err <= TOL, err
    return got, err


def test_owner_map_matches(ctx, oracle, workloads):
    import paper_2410_15227_amd as pkg
    say("case: owner map, turbulent 40000, r_part 0.2 / 0.05")
    pos, m, h, rho = workloads.make_cloud("turbulent", 40000, seed=51)
    src = pos[workloads.densest_particle(rho)][None, :]
    for r_part in (0.2, 0.05):
        ref = oracle.pseudo_build(pos, m, h, src, r_part=r_part, theta=0.5)
        got = pkg.build_pseudo_particles(ctx, pos, h, m, src, r_part=r_part, theta=0.5)
        assert np.array_equal(got["owner"].cpu().numpy(), ref["owner"])
    # with forced opening as well
    lab = ref["label"][ref["kind"] == 1][::2]
    ref = oracle.pseudo_build(pos, m, h, src, r_part=0.05, theta=0.5, open_labels=lab)
    got = pkg.build_pseudo_particles(ctx, pos, h, m, src, r_part=0.05, theta=0.5, open_labels=lab)
    assert np.array_equal(got["owner"].cpu().numpy(), ref["owner"])


def test_interpolation_parity(ctx, oracle, workloads):
    say("case: interpolation, turbulent 40000, 1 and 3 and 5 components")
    pos, m, h, rho = workloads.make_cloud("turbulent", 40000, seed=52)
    src = pos[workloads.densest_particle(rho)][None, :]
    ref = oracle.pseudo_build(pos, m, h, src, r_part=0.15, theta=0.5)
    g = np.random.default_rng(3)
    ne = len(ref["kind"])
    _, e1 = check(ctx, oracle, pos, ref, g.random(ne))
    _, e3 = check(ctx, oracle, pos, ref, g.random((ne, 3)))
    _, e5 = check(ctx, oracle, pos, ref, g.normal(size=(ne, 5)))
    say(f"  entries={ne} max rel err {e1:.2e} {e3:.2e} {e5:.2e}")


def test_interpolation_repeats_and_constants(ctx, oracle, workloads):
    import paper_2410_15227_amd as pkg
    say("case: interpolation determinism and constant field, uniform 20000")
    pos, m, h, rho = workloads.make_cloud("uniform", 20000, seed=53)
    ref = oracle.pseudo_build(pos, m, h, [[0.5, 0.5, 0.5]], r_part=0.1, theta=0.6)
    ms = mixed_set(ref)
    v = np.random.default_rng(4).random(len(ref["kind"]))
    a = pkg.interpolate_to_particles(ctx, pos, ms, v).cpu().numpy()
    b = pkg.interpolate_to_particles(ctx, pos, ms, v).cpu().numpy()
    assert np.array_equal(a, b)
    c = pkg.interpolate_to_particles(ctx, pos, ms, np.full(len(ref["kind"]), 0.625)).cpu().numpy()
    assert np.max(np.abs(c - 0.625)) <= 1e-13


def test_interpolation_edge_cases(ctx, oracle, workloads):
    import paper_2410_15227_amd as pkg
    say("case: interpolation edge cases")
    # every particle emitted as itself: values pass through unchanged
    pos, m, h, rho = workloads.make_cloud("uniform", 3000, seed=54)
    ref = oracle.pseudo_build(pos, m, h, [[0.5, 0.5, 0.5]], r_part=2.0, theta=0.5)
    assert (ref["kind"] == 0).all()
    v = np.random.default_rng(5).random(len(ref["kind"]))
    got = pkg.interpolate_to_particles(ctx, pos, mixed_set(ref), v).cpu().numpy()
    assert np.array_equal(got, v[ref["owner"]])
    # hand-made mixed set: fewer than one hierarchy group of entries, a
    # particle no sphere reaches, spheres touching at exactly 2h
    ex = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.5, 0.5, 0.7], [0.9, 0.9, 0.9]])
    eh = np.array([0.05, 0.1, 0.1, 0.01])
    ek = np.array([1, 1, 1, 0], dtype=np.int32)
    px = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.6], [0.3, 0.3, 0.3], [0.9, 0.9, 0.9], [0.1, 0.1, 0.2]])
    own = np.array([1, 2, 0, 3, 0])
    ref = dict(pos=ex, h=eh, kind=ek, owner=own)
    vals = np.array([0.2, 0.4, 0.8, 0.9])
    got, _ = check(ctx, oracle, px, ref, vals)
    assert got[2] == 0.2 and got[3] == 0.9
    # bad input is refused
    ms = mixed_set(ref)
    ms["owner"] = torch.tensor([1, 2, 0, 3, 4], device="cuda")
    with pytest.raises(Exception):
        pkg.interpolate_to_particles(ctx, px, ms, vals)
    with pytest.raises(Exception):
        pkg.interpolate_to_particles(ctx, px + 1.0, mixed_set(ref), vals)
    with pytest.raises(ValueError):
        pkg.interpolate_to_particles(ctx, px, mixed_set(ref), vals[:3])


def test_interpolation_1m_sampled(ctx, oracle, workloads):
    """The 1,048,576-particle turbulent cloud with one source at the densest
    particle (r_part 0.2, theta 0.5): 20,000 sampled particles against the
    oracle, the whole cloud through the same launch as the benchmark."""
    import paper_2410_15227_amd as pkg
    say("case: interpolation turbulent 1048576, 20000 sampled")
    pos, m, h, rho = workloads.make_cloud("turbulent", 1 << 20, seed=3)
    src = pos[workloads.densest_particle(rho)][None, :]
    ref = oracle.pseudo_build(pos, m, h, src, r_part=0.2, theta=0.5)
    g = np.random.default_rng(6)
    sample = g.choice(len(m), 20000, replace=False)
    _, err = check(ctx, oracle, pos, ref, g.random(len(ref["kind"])), sample=sample)
    say(f"  entries={len(ref['kind'])} max rel err {err:.2e}")
