"""Parity of the HIP forward and inverse mapping with the FP64 oracle.

Bars: candidate-pair lists bit-exact; FP64 path weights within 1e-12
absolute and cell masses within 1e-10 relative; mixed path cell masses
within 1e-5 relative (max over cells with M_c > 0)."""
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
def c1(workloads):
    return workloads.uniform_4096(seed=1)


@pytest.fixture(scope="module")
def c1_oracle(oracle, c1):
    say("oracle: full pair list and weights of uniform_4096")
    off, idx, w = oracle.pairs_weights(c1.tess, c1.pos, c1.h)
    M = np.add.reduceat(c1.m[idx] * w, off[:-1]) if len(idx) else np.zeros(c1.tess.n_cells)
    vol, rad = oracle.cell_info(c1.tess)
    return off, idx, w, M, vol, rad


def run_map(pkg, ctx, wl, precision, keep=True):
    dt = pkg.DeviceTessellation(ctx, wl.tess)
    res = pkg.map_particles_to_cells(ctx, dt, wl.pos, wl.h, wl.m, precision=precision, keep_pairs=keep)
    torch.cuda.synchronize()
    return dt, res


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_shortcuts(ctx, c1, c1_oracle, oracle, precision):
    """A support that stays clear of every face of the cell gives exactly 0
    (particle outside) or exactly 1 (inside), on both paths: the point-to-cell
    distance of every candidate pair of uniform_4096 decides which pairs are
    such, independently of the device path.  A margin of 1e-5 h keeps pairs
    whose support touches an edge to within binary32 geometry out of it."""
    import paper_2410_15227_amd as pkg
    say(f"case: uniform_4096 exact 0/1 shortcuts, precision={precision}")
    off, idx, w, M, vol, rad = c1_oracle
    cells = np.repeat(np.arange(c1.tess.n_cells), np.diff(off))
    dist = oracle.cell_distance(c1.tess, cells, c1.pos[idx])
    hh = c1.h[idx]
    clear_out = dist >= 2.0 * hh * (1.0 + 1e-5)
    clear_in = dist <= -2.0 * hh * (1.0 + 1e-5)
    say(f"pairs {len(idx)}: support clear outside {clear_out.sum()}, clear inside {clear_in.sum()}")
    # uniform_4096's supports are larger than its cells, so no support fits
    # inside one (the exact 1 is pinned by the lattice cases with tiny h)
    assert clear_out.sum() > 100000
    dt, res = run_map(pkg, ctx, c1, precision)
    goff, gidx, gw = (t.cpu().numpy() for t in res.pairs.export())
    assert np.array_equal(gidx, idx)
    bad_out = np.flatnonzero(clear_out & (gw != 0.0))
    bad_in = np.flatnonzero(clear_in & (gw != 1.0))
    assert len(bad_out) == 0, (len(bad_out), gw[bad_out[:5]], dist[bad_out[:5]] / hh[bad_out[:5]])
    assert len(bad_in) == 0, (len(bad_in), gw[bad_in[:5]])
    # the oracle agrees that these weights vanish (it sums every face)
    assert np.max(np.abs(w[clear_out])) < 1e-13
    if clear_in.any():
        assert np.max(np.abs(w[clear_in] - 1.0)) < 1e-13
    res.pairs.free()
    dt.free()


def test_cell_info_matches(ctx, c1, c1_oracle):
    import paper_2410_15227_amd as pkg
    say("case: uniform_4096 cell info")
    off, idx, w, M, vol, rad = c1_oracle
    dt = pkg.DeviceTessellation(ctx, c1.tess)
    gv, gr = dt.cell_info()
    gv, gr = gv.cpu().numpy(), gr.cpu().numpy()
    assert np.array_equal(gr, rad)                       # canonical radius bit-exact
    assert np.max(np.abs(gv - vol) / vol) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform_4096_full(ctx, c1, c1_oracle, precision):
    import paper_2410_15227_amd as pkg
    say(f"case: uniform_4096 full parity, precision={precision}")
    off, idx, w, M, vol, rad = c1_oracle
    dt, res = run_map(pkg, ctx, c1, precision)
    goff, gidx, gw = (t.cpu().numpy() for t in res.pairs.export())
    torch.cuda.synchronize()
    assert np.array_equal(goff, off)                     # bit-exact CSR
    assert np.array_equal(gidx, idx)
    gm = res.mass.cpu().numpy()
    rel = np.abs(gm - M) / M
    if precision == "fp64":
        assert np.max(np.abs(gw - w)) < 1e-12
        assert np.max(rel) < 1e-10
    else:
        assert np.max(np.abs(gw - w)) < 1e-5
        assert np.max(rel) < 1e-5
    # the oracle sums every face (no shortcut): its exact zeros are pairs
    # whose terms all vanish; the mixed path's angle terms there carry the
    # 2e-9 relative error of its binary32-core atan (the exact 0/1 cases
    # themselves are pinned in test_exact_shortcuts)
    assert np.all(np.abs(gw[w == 0.0]) < (1e-15 if precision == "fp64" else 1e-8))
    np.testing.assert_allclose(res.density.cpu().numpy(), gm / vol, rtol=1e-12)
    # coverage: sum over the particle's cells of the oracle weights
    cov_ref = np.bincount(idx, weights=w, minlength=len(c1.pos))
    assert np.max(np.abs(res.coverage.cpu().numpy() - cov_ref)) < (1e-11 if precision == "fp64" else 1e-5)


def test_shared_faces_once(ctx, c1, c1_oracle):
    """Mixed path, faces shared by two cells: with the grid's neighbours
    declared, the device verifies each face against its twin (same bounding
    sphere, opposite normal), and each shared face is evaluated once per
    particle -- by the lower-numbered cell -- and given to the twin pair with
    the opposite sign (w = S - sum_f sgn(d_f) C_f; C_f depends on the polygon
    and the particle only).  Against the same grid evaluated face by face from
    each side: identical pair lists, weights within 2e-7 (two binary32 views
    of one polygon), both within the mixed bars of the oracle; repeats are
    bit-identical (integer sums)."""
    import paper_2410_15227_amd as pkg
    say("case: uniform_4096 shared faces once vs every face from its own side")
    off, idx, w, M, vol, rad = c1_oracle
    interior = int(np.sum(c1.tess.face_nbr >= 0))
    dt_own = pkg.DeviceTessellation(ctx, c1.tess, neighbours=False)
    dt_tw = pkg.DeviceTessellation(ctx, c1.tess)
    say(f"  interior faces {interior}, shared after verification {dt_tw.n_shared}")
    assert dt_own.n_shared == 0
    assert interior * 0.99 <= dt_tw.n_shared <= interior
    out = {}
    for name, dt in (("own", dt_own), ("twin", dt_tw), ("twin2", dt_tw)):
        res = pkg.map_particles_to_cells(ctx, dt, c1.pos, c1.h, c1.m, precision="mixed", keep_pairs=True)
        torch.cuda.synchronize()
        goff, gidx, gw = (t.cpu().numpy() for t in res.pairs.export())
        assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
        out[name] = (gw, res.mass.cpu().numpy(), res.coverage.cpu().numpy())
    cov_ref = np.bincount(idx, weights=w, minlength=len(c1.pos))
    for name in ("own", "twin"):
        gw, gm, cov = out[name]
        say(f"  {name}: max|dw| {np.max(np.abs(gw - w)):.3e}  max rel dM {np.max(np.abs(gm - M) / M):.3e}  "
            f"max|dcov| {np.max(np.abs(cov - cov_ref)):.3e}")
        assert np.max(np.abs(gw - w)) < 1e-5
        assert np.max(np.abs(gm - M) / M) < 1e-5
        assert np.max(np.abs(cov - cov_ref)) < 1e-5
    assert np.max(np.abs(out["twin"][0] - out["own"][0])) < 2e-7
    assert np.array_equal(out["twin"][0].view(np.int64), out["twin2"][0].view(np.int64))


def test_reverse_map(ctx, c1, c1_oracle, oracle):
    import paper_2410_15227_amd as pkg
    say("case: uniform_4096 inverse mapping")
    off, idx, w, M, vol, rad = c1_oracle
    dt, res = run_map(pkg, ctx, c1, "fp64")
    g = c1.tess.generators
    q = np.stack([np.sin(9 * g[:, 0]) * np.cos(5 * g[:, 1]), g[:, 2] ** 2], axis=1)
    out = pkg.map_cells_to_particles(ctx, res.pairs, q).cpu().numpy()
    parts = np.arange(0, len(c1.pos), 97)
    cov, qref = oracle.particles(c1.tess, c1.pos, c1.h, parts, q)
    assert np.max(np.abs(out[parts] - qref)) < 1e-11
    # a constant field comes back unchanged
    one = pkg.map_cells_to_particles(ctx, res.pairs, np.full(c1.tess.n_cells, 2.5)).cpu().numpy()
    assert np.max(np.abs(one - 2.5)) < 1e-12
    # sum_i m_i c_i q_i = sum_c M_c q_c
    single = pkg.map_cells_to_particles(ctx, res.pairs, q[:, 0]).cpu().numpy()
    lhs = np.dot(c1.m * res.coverage.cpu().numpy(), single)
    assert abs(lhs - np.dot(res.mass.cpu().numpy(), q[:, 0])) < 1e-12


def lattice(n):
    from paper_2410_15227_amd.workloads import box_cells, tess_from_cells
    a = 1.0 / n
    gens, cells = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                lo = np.array([i, j, k]) * a
                gens.append(lo + 0.5 * a)
                cells.append(box_cells(lo, lo + a))
    return tess_from_cells(np.array(gens), cells)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lattice_special_positions(ctx, oracle, precision):
    """Cubic cells with particles on faces, edges, corners, cell centres and
    generic points; h from tiny (exact 0/1) to several cells."""
    import paper_2410_15227_amd as pkg
    say(f"case: lattice special positions, precision={precision}")
    t = lattice(6)
    a = 1.0 / 6
    g = np.random.default_rng(4)
    pts = [[0.5, 0.5, 0.5], [2 * a, 0.5, 0.5], [2 * a, 3 * a, 0.5], [2 * a, 3 * a, 4 * a], [a * 2.5, a * 2.5, a * 2.5],
           [0.31, 0.47, 0.62], [1e-9, 0.5, 0.5], [0.0, 0.0, 0.0]]
    pts += list(g.random((24, 3)))
    pts = np.array(pts)
    hs = np.concatenate([np.full(8, 0.9 * a), g.uniform(0.01 * a, 3 * a, 24)])
    hs[2] = 1e-4
    hs[3] = 2.5 * a
    m = g.uniform(0.5, 2.0, len(pts))
    wl = type("W", (), dict(tess=t, pos=pts, h=hs, m=m))
    dt, res = run_map(pkg, ctx, wl, precision)
    goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
    off, idx, w = oracle.pairs_weights(t, pts, hs)
    assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert np.max(np.abs(gw - w)) < tol
    cov = res.coverage.cpu().numpy()
    inner = np.all((pts - 2 * hs[:, None] > 0) & (pts + 2 * hs[:, None] < 1), axis=1)
    assert np.max(np.abs(cov[inner] - 1.0)) < (1e-12 if precision == "fp64" else 2e-6)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_near_degenerate_positions(ctx, oracle, precision):
    """Particles 3e-5 h, 1e-7 h and 1e-11 h off a face plane, an edge line
    and a corner of the cubic lattice, and particles whose foot point on a
    face plane 0.3 h away lies on an edge line or 1e-9 h beside it: cases
    near the mixed path's binary64 routing (edge lines within 1e-2 h of the
    particle, p = 0, face planes through the particle), against the oracle."""
    import paper_2410_15227_amd as pkg
    say(f"case: near-degenerate positions, precision={precision}")
    t = lattice(6)
    a = 1.0 / 6
    h0 = 0.7 * a
    pts, hs = [], []
    for eps in (3e-5, 1e-7, 1e-11):
        dlt = eps * h0
        pts += [[2 * a + dlt, 0.513, 0.479],          # face x = 2a
                [2 * a - dlt, 3 * a + dlt, 0.371],     # edge x = 2a, y = 3a
                [2 * a + dlt, 3 * a - dlt, 4 * a + dlt]]  # corner
        hs += [h0, h0, h0]
    # 0.3 h off the face plane x = 2a with the foot point on the edge line
    # y = 3a of that face (p = 0 exactly) and 1e-9 h beside it: only the edge
    # is degenerate, the face is not
    yb = t.vertices[np.argmin(np.abs(t.vertices[:, 1] - 3 * a)), 1]
    xb = t.vertices[np.argmin(np.abs(t.vertices[:, 0] - 2 * a)), 0]
    for eps in (0.0, 1e-9):
        pts += [[xb + 0.3 * h0, yb + eps * h0, 0.371], [xb - 0.3 * h0, yb - eps * h0, 0.629]]
        hs += [h0, h0]
    pts = np.array(pts)
    hs = np.array(hs)
    m = np.ones(len(pts))
    wl = type("W", (), dict(tess=t, pos=pts, h=hs, m=m))
    dt, res = run_map(pkg, ctx, wl, precision)
    goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
    off, idx, w = oracle.pairs_weights(t, pts, hs)
    assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert np.all(np.isfinite(gw))
    assert np.max(np.abs(gw - w)) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_near_edge_lines(ctx, oracle, workloads, precision):
    """Particles 3e-4 h to 3e-3 h off a face plane whose foot point lies
    1e-4 h to 1e-3 h beside an edge line of the face, so the edge's line
    passes within about 3e-3 h of the particle (Voronoi cells of 300 random
    sites): the mixed path takes such edges from binary64 geometry (d^2 +
    p^2 below (1e-2 h)^2); per-pair weights against the oracle."""
    import paper_2410_15227_amd as pkg
    say(f"case: particles near edge lines, precision={precision}")
    g = np.random.default_rng(7)
    t = workloads.voronoi(g.random((300, 3)))
    h = 0.09
    cfo, fvo, fv, V = t.cell_face_off, t.face_vtx_off, t.face_vtx, t.vertices
    pts = []
    for f in g.choice(t.n_faces, 20, replace=False):
        vs = V[fv[fvo[f]:fvo[f + 1]]]
        c = np.searchsorted(cfo, f, side="right") - 1
        n = np.cross(vs[1] - vs[0], vs[2] - vs[0])
        n /= np.linalg.norm(n)
        if np.dot(n, vs.mean(0) - t.generators[c]) < 0:
            n = -n
        A, B = vs[0], vs[1]
        mdir = np.cross(n, (B - A) / np.linalg.norm(B - A))
        if np.dot(mdir, vs.mean(0) - A) < 0:
            mdir = -mdir
        for d in (3e-4, 1e-3, 3e-3):
            for p in (1e-4, 3e-4, 1e-3):
                for sd in (1.0, -1.0):
                    x = A + (0.3 + 0.4 * g.random()) * (B - A) + p * h * mdir - sd * d * h * n
                    if np.all(x > 0.0) and np.all(x < 1.0):
                        pts.append(x)
    pts = np.array(pts)
    hs = np.full(len(pts), h)
    wl = type("W", (), dict(tess=t, pos=pts, h=hs, m=np.ones(len(pts))))
    dt, res = run_map(pkg, ctx, wl, precision)
    goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
    off, idx, w = oracle.pairs_weights(t, pts, hs)
    assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
    err = float(np.max(np.abs(gw - w)))
    say(f"  {len(pts)} particles, {len(w)} pairs, max |w - w_oracle| = {err:.2e}")
    assert err < (1e-12 if precision == "fp64" else 5e-6)


def test_transpose_three_sort_passes(ctx):
    """More than 2^20 particles: the particle-major copy is then sorted in
    three passes.  Particles with tiny supports inside a 4^3 lattice each
    lie in one cell with weight exactly 1, so the inverse mapping of
    q_c = c must return each particle's own cell index exactly, and its
    coverage must be exactly 1."""
    import paper_2410_15227_amd as pkg
    n = (1 << 20) + 4097
    say(f"case: transpose of {n} particles (three sort passes)")
    t = lattice(4)
    a = 0.25
    g = np.random.default_rng(11)
    pos = g.uniform(0.01, 0.99, (n, 3))
    h = np.full(n, 1e-6)
    m = np.ones(n)
    wl = type("W", (), dict(tess=t, pos=pos, h=h, m=m))
    dt, res = run_map(pkg, ctx, wl, "mixed")
    ijk = np.floor(pos / a).astype(np.int64)
    cell = (ijk[:, 0] * 4 + ijk[:, 1]) * 4 + ijk[:, 2]  # lattice() order: i, then j, then k
    frac = pos / a - ijk
    inner = np.all((frac > 1e-4) & (frac < 1 - 1e-4), axis=1)
    assert inner.sum() > n - 1000
    assert np.array_equal(t.generators[cell[inner]] // a, ijk[inner].astype(float))
    cov = res.coverage.cpu().numpy()
    assert np.all(cov[inner] == 1.0)
    out = pkg.map_cells_to_particles(ctx, res.pairs, np.arange(t.n_cells, dtype=np.float64)).cpu().numpy()
    assert np.array_equal(out[inner], cell[inner].astype(np.float64))


def test_exact_zero_and_one(ctx):
    """A support inside the cell gives exactly 1, a candidate whose support
    misses the cell exactly 0 (every face beyond 2h contributes nothing)."""
    import paper_2410_15227_amd as pkg
    say("case: exact 0 / 1 limits")
    t = lattice(3)
    a = 1.0 / 3
    c = 13  # the central cube [a, 2a]^3
    pts = np.array([[1.5 * a, 1.5 * a, 1.5 * a], [1.5 * a + 0.01, 1.45 * a, 1.52 * a], [0.5 * a, 1.5 * a, 1.5 * a]])
    hs = np.array([0.2 * a, 0.12 * a, 0.2 * a])
    wl = type("W", (), dict(tess=t, pos=pts, h=hs, m=np.ones(3)))
    for prec in ["fp64", "mixed"]:
        dt, res = run_map(pkg, ctx, wl, prec)
        off, idx, w = (x.cpu().numpy() for x in res.pairs.export())
        ws = dict(zip(idx[off[c]:off[c + 1]].tolist(), w[off[c]:off[c + 1]].tolist()))
        assert ws[0] == 1.0 and ws[1] == 1.0
        # particle 2 (centre of the face neighbour) is a candidate of cell 13
        # (distance a < R + 2h = 0.87a + 0.4a) but its support stops 0.1a
        # short of the shared face
        assert ws.get(2, 0.0) == 0.0
        assert 2 in ws


@pytest.fixture(scope="module")
def c2(workloads):
    say("building turbulent_262144 inputs")
    return workloads.turbulent(262144, seed=2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_turbulent_262144_sampled(ctx, c2, oracle, precision):
    import paper_2410_15227_amd as pkg
    say(f"case: turbulent_262144 sampled cells, precision={precision}")
    dt, res = run_map(pkg, ctx, c2, precision)
    goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
    gm = res.mass.cpu().numpy()
    g = np.random.default_rng(12)
    cells = np.sort(g.choice(c2.tess.n_cells, 160, replace=False))
    # plus the cells with the most pairs, the smallest / largest volumes and
    # the 200 most degenerate (thinnest, shortest-edged) cells
    npairs = np.diff(goff)
    vol = dt.cell_info()[0].cpu().numpy()
    from paper_2410_15227_amd.workloads import degeneracy_scores
    extra = np.concatenate([np.argsort(npairs)[-20:], np.argsort(vol)[:10], np.argsort(vol)[-10:],
                            np.argsort(degeneracy_scores(c2.tess))[-200:]])
    cells = np.unique(np.concatenate([cells, extra]))
    off, idx, w = oracle.pairs_weights(c2.tess, c2.pos, c2.h, cells)
    Mref = np.add.reduceat(c2.m[idx] * w, off[:-1])
    for k, c in enumerate(cells):
        assert np.array_equal(gidx[goff[c]:goff[c + 1]], idx[off[k]:off[k + 1]]), c
    gws = np.concatenate([gw[goff[c]:goff[c + 1]] for c in cells])
    rel = np.abs(gm[cells] - Mref) / Mref
    say(f"  pairs={int(goff[-1])} cells={len(cells)} max_rel={np.max(rel):.3e} max|dw|={np.max(np.abs(gws - w)):.3e}")
    if precision == "fp64":
        assert np.max(np.abs(gws - w)) < 1e-12
        assert np.max(rel) < 1e-10
    else:
        # per pair: binary32 edge geometry (relative 6e-8 of the vertex
        # coordinates, a few h) moves a weight by at most a few 1e-7
        assert np.max(np.abs(gws - w)) < 1e-6
        assert np.max(rel) < 1e-5
    # whole-grid properties: mass is lost only through the walls
    tot = gm.sum()
    assert 0.95 < tot <= 1.0 + 1e-9
    assert abs(tot - np.dot(c2.m, res.coverage.cpu().numpy())) < 1e-9


def test_long_cell_lists(ctx, oracle):
    """Three slab cells and 12,000 particles: every cell's candidate list is
    longer than one LDS sort run (4096), so the lists go through the merged
    path of the per-cell sort.  Lists bit-exact; the cell masses add up to
    the particles' coverage-weighted mass."""
    import types

    import paper_2410_15227_amd as pkg
    say("case: long cell lists, 3 slab cells, 12000 particles")
    gen = np.array([[0.2, 0.5, 0.5], [0.5, 0.5, 0.5], [0.8, 0.5, 0.5]])
    v = oracle.voronoi(gen)
    t = types.SimpleNamespace(n_cells=3, generators=gen, vertices=v["face_pts"], cell_face_off=v["cell_face_off"],
                              face_vtx_off=v["face_vtx_off"],
                              face_vtx=np.arange(len(v["face_pts"]), dtype=np.int32))
    g = np.random.default_rng(31)
    pos = 0.1 + 0.8 * g.random((12000, 3))  # supports (2h <= 0.06) inside the box
    h = g.uniform(0.01, 0.03, 12000)
    m = np.full(12000, 1.0 / 12000)
    dt = pkg.DeviceTessellation(ctx, t)
    res = pkg.map_particles_to_cells(ctx, dt, pos, h, m, precision="fp64", keep_pairs=True)
    goff, gidx, gw = (x.cpu().numpy() for x in res.pairs.export())
    off, idx = oracle.pair_lists(t, pos, h)
    assert np.min(np.diff(off)) > 4096
    assert np.array_equal(goff, off) and np.array_equal(gidx, idx)
    cov = res.coverage.cpu().numpy()
    assert abs(res.mass.sum().item() - (m * cov).sum()) < 1e-12
    assert np.all(np.abs(cov - 1.0) < 1e-12)  # every support lies inside the box and the cells tile it
    res.pairs.free()
    dt.free()
