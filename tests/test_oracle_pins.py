"""Pins of oracle parts that no other test reaches independently:
  - the signed point-to-cell distance that decides the exact 0/1 shortcuts
    of the mapping (a kernel support clear of every face gives w = 0 outside
    the cell and 1 inside), against closed forms on a box and brute-force
    sampling of the faces of random Voronoi cells;
  - the octree node size s (Sec. 2.2.1: distance from the centre of mass to
    the furthest member), the node mass and centre of mass, against brute
    force over each pseudo-particle's members;
  - the canonical binary32 bounding radius R_c of the candidate-pair test
    (the smallest binary32 R with R*R >= max_v |v - g_c|^2 in binary64),
    against its definition evaluated in numpy."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from conftest import rng


def _box_tess(lo, hi):
    from paper_2410_15227_amd.workloads import box_cells, tess_from_cells
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return tess_from_cells(np.array([(lo + hi) / 2]), [box_cells(lo, hi)], box_lo=lo, box_hi=hi)


def test_cell_distance_box_closed_form(oracle):
    lo, hi = np.array([0.2, 0.1, 0.3]), np.array([0.7, 0.4, 0.9])
    t = _box_tess(lo, hi)
    c, a = (lo + hi) / 2, (hi - lo) / 2
    x = np.concatenate([rng(5).uniform(-0.5, 1.5, size=(4000, 3)), rng(8).uniform(lo, hi, size=(500, 3))])
    got = oracle.cell_distance(t, np.zeros(len(x), dtype=np.int64), x)
    out = np.maximum(np.abs(x - c) - a, 0.0)
    inside = np.all(np.abs(x - c) < a, axis=1)
    ref = np.where(inside, -np.min(a - np.abs(x - c), axis=1), np.sqrt((out ** 2).sum(axis=1)))
    assert inside.sum() > 100 and (~inside).sum() > 1000
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-15)


def _face_samples(t, c, g, k=3000):
    """Random points on every face polygon of cell c (fan triangles)."""
    pts = []
    for f in range(t.cell_face_off[c], t.cell_face_off[c + 1]):
        V = t.vertices[t.face_vtx[t.face_vtx_off[f]:t.face_vtx_off[f + 1]]]
        for q in range(1, len(V) - 1):
            u = g.uniform(size=(k, 2))
            flip = u.sum(axis=1) > 1
            u[flip] = 1 - u[flip]
            pts.append(V[0] + u[:, :1] * (V[q] - V[0]) + u[:, 1:] * (V[q + 1] - V[0]))
        pts.append(V)  # the vertices themselves
    return np.concatenate(pts)


def test_cell_distance_random_cells(oracle, small_tess):
    pos, m, h, t = small_tess
    g = rng(6)
    for c in g.choice(t.n_cells, 12, replace=False):
        surf = _face_samples(t, c, g)
        # points around the cell at distances up to a few cell sizes
        x = t.generators[c] + g.normal(scale=0.08, size=(300, 3))
        got = oracle.cell_distance(t, np.full(len(x), c, dtype=np.int64), x)
        brute = cKDTree(surf).query(x)[0]
        # inside test from the Voronoi definition: in the unit box and no
        # generator closer than c's
        dg = np.linalg.norm(x[:, None, :] - t.generators[None, :, :], axis=2)
        inside = (np.argmin(dg, axis=1) == c) & np.all((x > 0.0) & (x < 1.0), axis=1)
        assert np.array_equal(got <= 0, inside)
        out = ~inside
        # outside: the distance to the nearest point of the cell, which a
        # dense sample of its faces approaches from above
        assert np.all(got[out] <= brute[out] + 1e-12)
        assert np.max(brute[out] - got[out]) < 3e-3
        # inside: minus the distance to the boundary (the nearest face plane
        # of a convex cell), never more than the sampled surface distance
        assert np.all(-got[inside] <= brute[inside] + 1e-12)


def test_octree_node_size_and_moments(oracle, workloads):
    pos, m, h, rho = workloads.make_cloud("turbulent", 6000, seed=23)
    m = m * (1.0 + 0.5 * rng(7).uniform(size=len(m)))  # unequal masses: the centre of mass is weighted
    for src in ([0.5, 0.5, 0.5], [0.2, 0.8, 0.3]):
        out = oracle.pseudo_build(pos, m, h, [src], r_part=0.15, theta=0.5)
        ps = np.flatnonzero(out["kind"] == 1)
        assert len(ps) > 20
        owner = out["owner"]
        assert np.array_equal(np.bincount(owner, minlength=len(out["kind"])), out["count"])
        for e in ps:
            mem = np.flatnonzero(owner == e)
            com = np.average(pos[mem], axis=0, weights=m[mem])
            assert np.max(np.abs(out["pos"][e] - com)) < 1e-14
            assert abs(out["mass"][e] - m[mem].sum()) < 1e-15
            # s: the furthest member from the centre of mass (not from the
            # cell centre, not squared)
            s_ref = np.max(np.linalg.norm(pos[mem] - out["pos"][e], axis=1))
            assert abs(out["s"][e] - s_ref) < 1e-14
        # the node's cube (from its label) holds all its members, and the
        # size is at most the cube's half diagonal from any inner point
        # doubled: a coarse but independent bound
        for e in ps[:50]:
            lab = int(out["label"][e])
            depth = (lab.bit_length() - 1) // 3
            assert out["s"][e] <= np.sqrt(3.0) * 0.5 ** depth + 1e-15


def test_canonical_radius_definition(oracle, small_tess, workloads):
    for t in (small_tess[3], workloads.uniform_4096(seed=1).tess):
        vol, rad = oracle.cell_info(t)
        assert rad.dtype == np.float32
        r2 = np.empty(t.n_cells)
        for c in range(t.n_cells):
            vs = t.face_vtx[t.face_vtx_off[t.cell_face_off[c]]:t.face_vtx_off[t.cell_face_off[c + 1]]]
            d = t.vertices[vs] - t.generators[c]
            r2[c] = np.max((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
        R = rad.astype(np.float64)
        below = np.nextafter(rad, np.float32(0)).astype(np.float64)
        # a binary32 value squared is exact in binary64: the comparisons are exact
        assert np.all(R * R >= r2)
        assert np.all(below * below < r2)


@pytest.mark.parametrize("hh, want", [
    (0.4, [1, 6, 0, 0, 0, 0, 0]),      # support inside the cube: nothing to integrate
    (0.6, [1, 6, 6, 24, 0, 0, 0]),     # reaches the six faces (distance 1) but no edge (sqrt 2)
    (0.75, [1, 6, 6, 24, 24, 0, 24]),  # reaches every edge, never within U < 1 of one
    (1.5, [1, 6, 6, 24, 24, 24, 24]),  # edge line at 0.943 h: U = 1 crossed on both sides
])
def test_work_counts_cube(oracle, hh, want):
    """The algorithmic work histogram on a cube of half-side 1 about the
    particle, in closed form: faces at distance 1, edges at sqrt(2), corners
    at sqrt(3); an edge line at a = sqrt(2)/h (units of h) crosses U = 1 at
    t = +-sqrt(1 - a^2), inside the edge's span +-1/h."""
    t = _box_tess([-1.0, -1.0, -1.0], [1.0, 1.0, 1.0])
    got = oracle.work_counts(t, np.zeros((1, 3)), np.array([hh]), np.array([0]))
    assert list(got) == want


def test_work_counts_shared_face(oracle, workloads):
    """Two cubes of half-side 1 sharing the face x = 1, the particle at the
    first one's centre with h = 0.6: the first cell's six faces are reached
    at distance 1 (their edges at sqrt 2 are not); of the second cell only
    the shared face is.  Counted for both pairs, the shared face appears
    twice; counted once per (particle, face), only for the lower-numbered
    cell."""
    box0 = workloads.box_cells([-1.0, -1.0, -1.0], [1.0, 1.0, 1.0])
    box1 = workloads.box_cells([1.0, -1.0, -1.0], [3.0, 1.0, 1.0])
    t = workloads.tess_from_cells([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]], [box0, box1],
                                  box_lo=(-1, -1, -1), box_hi=(3, 1, 1))
    # face 1 of each box is its x+ face, face 0 its x- face
    nbr = -np.ones(12, dtype=np.int32)
    nbr[1] = 1
    nbr[6 + 0] = 0
    t.face_nbr = nbr
    x, h = np.zeros((1, 3)), np.array([0.6])
    both = oracle.work_counts(t, x, h, np.array([0, 1]))
    once = oracle.work_counts(t, x, h, np.array([0, 1]), owned=True)
    assert list(both) == [2, 12, 7, 28, 0, 0, 0]
    assert list(once) == [2, 12, 6, 24, 0, 0, 0]
    # the second cell alone evaluates nothing of its own
    assert list(oracle.work_counts(t, x, h, np.array([1]), owned=True)) == [1, 6, 0, 0, 0, 0, 0]
