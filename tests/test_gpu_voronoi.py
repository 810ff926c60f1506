"""Parity of the device Voronoi grid and Lloyd iterations (Sec. 2.3) with the
oracle's bisector-clipping construction.

Bars: per cell, the volume (the grid's own divergence-theorem volume after
upload preparation) within 1e-11 relative; the set of faces larger than
1e-10 with their neighbours, and their areas within 1e-11; every vertex no
closer to another site than to its own (1e-12); Lloyd sites within 1e-12
after one iteration and 1e-10 after five; the forward mapping on the device
grid equals the oracle's mapping on the oracle's grid (binary64 path, 1e-10
relative cell mass)."""
import sys
import types

import numpy as np
import pytest
from scipy.spatial import cKDTree

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


def face_areas(t):
    out = np.empty(len(t.face_vtx_off) - 1)
    for f in range(len(out)):
        p = t.vertices[t.face_vtx[t.face_vtx_off[f]:t.face_vtx_off[f + 1]]]
        a = np.zeros(3)
        for i in range(1, len(p) - 1):
            a += np.cross(p[i] - p[0], p[i + 1] - p[0])
        out[f] = 0.5 * np.linalg.norm(a)
    return out


def compare_grid(ctx, oracle, gen, lo=(0, 0, 0), hi=(1, 1, 1), sample=None):
    import paper_2410_15227_amd as pkg
    dt, g_out = pkg.build_voronoi(ctx, gen, lo, hi, n_lloyd=0)
    t = dt.export()
    vol = dt.cell_info()[0].cpu().numpy()
    assert np.array_equal(g_out.cpu().numpy(), gen)
    ref = oracle.voronoi(gen, np.asarray(lo, float), np.asarray(hi, float))
    box = np.prod(np.asarray(hi, float) - np.asarray(lo, float))
    assert abs(vol.sum() - box) < 1e-11 * box
    assert np.max(np.abs(vol - ref["volume"]) / ref["volume"]) < 1e-11
    ga = face_areas(t)
    cells = range(len(gen)) if sample is None else sample
    tree = cKDTree(gen)
    for c in cells:
        mine = {}
        for f in range(t.cell_face_off[c], t.cell_face_off[c + 1]):
            if ga[f] > 1e-10:
                mine[int(t.face_nbr[f])] = mine.get(int(t.face_nbr[f]), 0.0) + ga[f]
        theirs = {}
        for f in range(ref["cell_face_off"][c], ref["cell_face_off"][c + 1]):
            if ref["face_area"][f] > 1e-10:
                k = int(ref["face_id"][f])
                theirs[k] = theirs.get(k, 0.0) + ref["face_area"][f]
        assert mine.keys() == theirs.keys(), (c, sorted(mine), sorted(theirs))
        for k in mine:
            assert abs(mine[k] - theirs[k]) < 1e-11, (c, k)
        vs = t.vertices[t.face_vtx[t.face_vtx_off[t.cell_face_off[c]]:t.face_vtx_off[t.cell_face_off[c + 1]]]]
        dmin, _ = tree.query(vs)
        assert np.all(np.linalg.norm(vs - gen[c], axis=1) <= dmin + 1e-12)
    dt.free()
    return t, ref


def test_small_grids(ctx, oracle, workloads):
    say("case: voronoi uniform 2000, turbulent 3000, non-unit box 500")
    g = workloads.make_cloud("uniform", 2000, seed=71)[0]
    t, ref = compare_grid(ctx, oracle, g)
    say(f"  uniform: faces/cell {len(t.face_nbr) / len(g):.2f}, vertices/cell {len(t.vertices) / len(g):.2f}")
    g = workloads.make_cloud("turbulent", 3000, seed=72)[0]
    compare_grid(ctx, oracle, g)
    lo, hi = np.array([-0.5, 0.0, 0.25]), np.array([1.5, 1.0, 1.0])
    g = lo + np.random.default_rng(73).random((500, 3)) * (hi - lo)
    compare_grid(ctx, oracle, g, lo, hi)


def test_degenerate_grids(ctx, oracle):
    import paper_2410_15227_amd as pkg
    say("case: voronoi single site, two slabs, eight octants, lattice")
    compare_grid(ctx, oracle, np.array([[0.3, 0.6, 0.2]]))
    compare_grid(ctx, oracle, np.array([[0.3, 0.5, 0.5], [0.7, 0.5, 0.5]]))
    octs = np.array([[(i + 0.5) / 2, (j + 0.5) / 2, (k + 0.5) / 2] for k in range(2) for j in range(2) for i in range(2)])
    compare_grid(ctx, oracle, octs)
    lat = np.array([[(i + 0.5) / 5, (j + 0.5) / 5, (k + 0.5) / 5] for k in range(5) for j in range(5) for i in range(5)])
    dt, _ = pkg.build_voronoi(ctx, lat, n_lloyd=0)
    vol = dt.cell_info()[0].cpu().numpy()
    assert np.allclose(vol, 1 / 125, rtol=1e-12)
    dt.free()
    # bad input is refused
    with pytest.raises(Exception):
        pkg.build_voronoi(ctx, np.array([[0.2, 0.2, 0.2], [0.2, 0.2, 0.2], [0.7, 0.1, 0.4]]))
    with pytest.raises(Exception):
        pkg.build_voronoi(ctx, np.array([[0.2, 0.2, 0.2], [1.2, 0.2, 0.2]]))
    with pytest.raises(Exception):
        pkg.build_voronoi(ctx, np.array([[0.2, 0.2, 0.2]]), box_lo=(0, 0, 0), box_hi=(1, 0, 1))


def test_lloyd(ctx, oracle, workloads):
    import paper_2410_15227_amd as pkg
    say("case: lloyd 1 and 5 iterations, turbulent 2000")
    g = workloads.make_cloud("turbulent", 2000, seed=74)[0]
    for it, tol in ((1, 1e-12), (5, 1e-10)):
        dt, out = pkg.build_voronoi(ctx, g, n_lloyd=it)
        want = oracle.lloyd(g, it)
        err = np.abs(out.cpu().numpy() - want).max()
        say(f"  {it} iterations: max site difference {err:.2e}")
        assert err < tol
        vol = dt.cell_info()[0].cpu().numpy()
        assert abs(vol.sum() - 1.0) < 1e-11
        dt.free()
    # the line case of the oracle pins: slabs converge as x <- b/2, (1+b)/2
    dt, out = pkg.build_voronoi(ctx, [[0.3, 0.5, 0.5], [0.4, 0.5, 0.5]], n_lloyd=5)
    assert np.abs(out.cpu().numpy() - oracle.lloyd([[0.3, 0.5, 0.5], [0.4, 0.5, 0.5]], 5)).max() < 1e-14
    dt.free()


def test_mapping_on_device_grid(ctx, oracle, workloads):
    import paper_2410_15227_amd as pkg
    say("case: forward mapping on the device grid, uniform 600")
    pos, m, h, rho = workloads.make_cloud("uniform", 600, seed=75)
    dt, _ = pkg.build_voronoi(ctx, pos, n_lloyd=0)
    res = pkg.map_particles_to_cells(ctx, dt, pos, h, m, precision="fp64")
    got = res.mass.cpu().numpy()
    ref = oracle.voronoi(pos)
    t = types.SimpleNamespace(n_cells=len(pos), generators=np.ascontiguousarray(pos), vertices=ref["face_pts"],
                              cell_face_off=ref["cell_face_off"], face_vtx_off=ref["face_vtx_off"],
                              face_vtx=np.arange(len(ref["face_pts"]), dtype=np.int32))
    want = oracle.map_cells(t, pos, h, m)[0]
    err = np.max(np.abs(got - want) / np.maximum(want, 1e-300))
    say(f"  max relative cell-mass difference {err:.2e}")
    assert err < 1e-10
    dt.free()


def test_turbulent_262144_sampled(ctx, oracle, workloads):
    """The 262,144-site turbulent grid: 300 sampled cells against the oracle
    (volume, centroid through one Lloyd step), and the five-iteration grid's
    invariants (box partition, vertices no closer to another site)."""
    import paper_2410_15227_amd as pkg
    say("case: voronoi turbulent 262144 sampled")
    g = workloads.make_cloud("turbulent", 1 << 18, seed=2)[0]
    dt, out = pkg.build_voronoi(ctx, g, n_lloyd=1)
    rng = np.random.default_rng(9)
    cells = rng.choice(len(g), 300, replace=False)
    vol_ref, cen_ref = oracle.voronoi_cells(g, cells)
    err = np.abs(out.cpu().numpy()[cells] - cen_ref).max()
    say(f"  one Lloyd step: max centroid difference {err:.2e}")
    assert err < 1e-12
    dt.free()
    dt, _ = pkg.build_voronoi(ctx, g, n_lloyd=0)
    vol = dt.cell_info()[0].cpu().numpy()
    assert np.max(np.abs(vol[cells] - vol_ref) / vol_ref) < 1e-11
    dt.free()
    dt, out = pkg.build_voronoi(ctx, g, n_lloyd=5)
    vol = dt.cell_info()[0].cpu().numpy()
    assert abs(vol.sum() - 1.0) < 1e-10 and (vol > 0).all()
    t = dt.export()
    s5 = out.cpu().numpy()
    tree = cKDTree(s5)
    for c in cells[:50]:
        vs = t.vertices[t.face_vtx[t.face_vtx_off[t.cell_face_off[c]]:t.face_vtx_off[t.cell_face_off[c + 1]]]]
        dmin, _ = tree.query(vs)
        assert np.all(np.linalg.norm(vs - s5[c], axis=1) <= dmin + 1e-12)
    dt.free()
