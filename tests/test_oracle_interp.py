"""Pins of the per-particle interpolation from the mixed set (Sec. 3.3: each
SPH particle's value taken from the entries whose smoothing spheres reach it,
the refinement the paper proposes over giving every member its node's value).
The SPH interpolant with entry volumes (h/h_fact)^3 (eq. h_node) weights each
entry by the dimensionless kernel w(r/h) alone; closed forms use the M4
kernel's textbook values w(0) = 1, w(1) = 1/4, w(3/2) = 1/32."""
import numpy as np
import pytest


def one(oracle, px, ex, eh, ek, val, owner=0):
    return oracle.interpolate(np.array([px], float), np.array([owner]), np.array(ex, float), np.array(eh, float),
                              np.array(ek, np.int32), np.array(val, float))[0]


def test_closed_forms(oracle):
    # a member of pseudo-particle A at A's centre; B is another entry
    # same h: weights 1 and 1/4 -> (0 * 1 + 1 * 1/4) / (5/4)
    assert abs(one(oracle, [0, 0, 0], [[0, 0, 0], [1, 0, 0]], [1, 1], [1, 0], [0, 1]) - 0.2) < 1e-15
    # h_B = 1/2 at r = 1/2: the same q = 1, so the same weight 1/4 whatever h is
    assert abs(one(oracle, [0, 0, 0], [[0, 0, 0], [0, 0.5, 0]], [1, 0.5], [1, 1], [0, 1]) - 0.2) < 1e-15
    # h_A = 3 at r = 0 and h_B = 0.4 at r = 0.6 (q = 3/2): weights 1 and 1/32
    assert abs(one(oracle, [0, 0, 0], [[0, 0, 0], [0.6, 0, 0]], [3, 0.4], [1, 1], [0, 1]) - 1.0 / 33.0) < 1e-15
    # q = 3/2: weights 1 and 1/32
    assert abs(one(oracle, [0, 0, 0], [[0, 0, 0], [0, 0, 1.5]], [1, 1], [1, 1], [0, 1]) - 1.0 / 33.0) < 1e-15
    # at exactly r = 2h an entry adds nothing
    assert one(oracle, [0, 0, 0], [[0, 0, 0], [2, 0, 0]], [1, 1], [1, 1], [3, 7]) == 3.0


def test_owner_rules(oracle):
    # a particle that is an entry itself keeps that entry's value exactly
    assert one(oracle, [0, 0, 0], [[0, 0, 0], [0.1, 0, 0]], [1, 1], [0, 1], [0.25, 0.75]) == 0.25
    # no sphere reaches it: its owner's value
    assert one(oracle, [5, 5, 5], [[0, 0, 0], [0.1, 0, 0]], [1, 1], [1, 1], [0.25, 0.75], owner=1) == 0.75


def test_constant_and_convexity(oracle):
    g = np.random.default_rng(1)
    ex = g.random((200, 3))
    eh = g.uniform(0.02, 0.2, 200)
    ek = np.ones(200, np.int32)
    px = g.random((500, 3))
    owner = g.integers(0, 200, 500)
    c = oracle.interpolate(px, owner, ex, eh, ek, np.full(200, 0.375))
    assert np.max(np.abs(c - 0.375)) < 1e-15
    v = g.random(200)
    f = oracle.interpolate(px, owner, ex, eh, ek, v)
    for i in range(0, 500, 7):
        r = np.linalg.norm(ex - px[i], axis=1)
        reach = r < 2 * eh
        if reach.any():
            assert v[reach].min() - 1e-15 <= f[i] <= v[reach].max() + 1e-15
        else:
            assert f[i] == v[owner[i]]
    # components are independent
    v3 = g.random((200, 3))
    f3 = oracle.interpolate(px, owner, ex, eh, ek, v3)
    for k in range(3):
        assert np.array_equal(f3[:, k], oracle.interpolate(px, owner, ex, eh, ek, v3[:, k]))


def test_owner_of_walk(oracle, workloads):
    pos, m, h, rho = workloads.make_cloud("turbulent", 6000, 71)
    b = oracle.pseudo_build(pos, m, h, [pos[workloads.densest_particle(rho)]], r_part=0.2, theta=0.5)
    own = b["owner"]
    assert own.min() >= 0 and own.max() < len(b["kind"])
    assert np.array_equal(np.bincount(own, minlength=len(b["kind"])), b["count"])
    real = np.flatnonzero(b["kind"] == 0)
    assert np.array_equal(own[b["first"][real]], real)
    ps = np.flatnonzero(b["kind"] == 1)
    for e in ps[:50]:
        mem = np.flatnonzero(own == e)
        assert mem.min() == b["first"][e]
        assert np.allclose(np.average(pos[mem], axis=0, weights=m[mem]), b["pos"][e], rtol=0, atol=1e-12)
    # every member of a pseudo-particle with h from the solve: interpolated values stay in [0, 1]
    f = oracle.interpolate(pos, own, b["pos"], b["h"], b["kind"], np.linspace(0, 1, len(b["kind"])))
    assert f.min() >= 0 and f.max() <= 1
