"""Pins of the oracle's Exact-mapping weights (Sec. 1, Sec. 2.3: the analytic
volume integral of the SPH kernel over a Voronoi cell; kernel of Sec. 2.4.2)
against routes that do not go through the oracle: slab integration of the
half-space, 3-D quadrature of a cube, Monte-Carlo sampling of the kernel over
random convex cells, symmetry, partition of unity, additivity and
invariances."""
import math

import numpy as np
import pytest
from scipy import integrate

from conftest import rng


def m4(q):
    q = np.asarray(q, float)
    return np.where(q < 1, 1 - 1.5 * q**2 + 0.75 * q**3, np.where(q < 2, 0.25 * (2 - q) ** 3, 0.0))


def W(r):
    return m4(r) / math.pi


def box(lo, hi):
    from paper_2410_15227_amd.workloads import box_cells
    return box_cells(lo, hi)


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("d", [0.0, 0.25, 0.5, 0.99, 1.0, 1.4, 1.9, 2.0, 2.6])
def test_half_space_slab(oracle, d):
    # mass beyond a plane at distance d: int_d^2 dz  2pi int_z^2 W(r) r dr
    def slab(z):
        return 2 * math.pi * integrate.quad(lambda r: W(r) * r, z, 2.0, points=[1.0] if z < 1 else None,
                                            epsabs=1e-14)[0]

    beyond = integrate.quad(slab, d, 2.0, points=[1.0] if d < 1 else None, epsabs=1e-14)[0] if d < 2 else 0.0
    # particle at the origin, the cell is the (huge) slab z < d
    w_in = oracle.weight_poly([0, 0, 0], 1.0, box([-50, -50, -50], [50, 50, d]))
    assert abs(w_in - (1.0 - beyond)) < 1e-11


def test_half_space_known_values(oracle):
    # w_beyond(0) = 1/2, w_beyond(1) = 1/30 (closed form of the slab integral)
    assert abs(oracle.weight_poly([0, 0, 0], 1.0, box([-50] * 3, [50, 50, 0.0 + 1e-300])) - 0.5) < 1e-12
    assert abs((1 - oracle.weight_poly([0, 0, 0], 1.0, box([-50] * 3, [50, 50, 1.0]))) - 1.0 / 30.0) < 1e-12


def test_cube_by_cubature(oracle):
    # cube of half-side a centred on the particle, 8 x the positive octant by
    # nested adaptive quadrature of the kernel (independent of the cone route)
    for a in [0.5, 1.0, 1.5]:
        def fz(x, y):
            return integrate.quad(lambda z: W(math.sqrt(x * x + y * y + z * z)), 0, a, epsabs=1e-12)[0]

        def fy(x):
            return integrate.quad(lambda y: fz(x, y), 0, a, epsabs=1e-11)[0]

        ref = 8 * integrate.quad(fy, 0, a, epsabs=1e-10)[0]
        got = oracle.weight_poly([0, 0, 0], 1.0, box([-a] * 3, [a] * 3))
        assert abs(got - ref) < 5e-8, (a, got, ref)


def test_continuity_near_degenerate_positions(oracle):
    """w is an integral of a bounded kernel over a fixed cell, hence smooth in
    the particle position: approaching a face plane whose foot point sits on a
    face corner (edges with p -> 0), w(delta) must follow its tangent line."""
    a, h = 1.0 / 6.0, 0.15
    faces = box([0, 0.5, 0.5], [a, 0.5 + a, 0.5 + a])
    w0 = oracle.weight_poly([0.0, 0.5, 0.5], h, faces)
    slope = (oracle.weight_poly([2e-6, 0.5, 0.5], h, faces) - oracle.weight_poly([1e-6, 0.5, 0.5], h, faces)) / 1e-6
    for dl in [1e-13, 1e-11, 1e-9, 1e-8, 1e-7]:
        got = oracle.weight_poly([dl, 0.5, 0.5], h, faces)
        assert abs(got - (w0 + slope * dl)) < 1e-13 + 1e-5 * dl, (dl, got - w0 - slope * dl)
    # the same along an edge line of a generic cell face: x slides onto the
    # plane that contains an edge and is normal to its face
    for dl in [1e-12, 1e-9]:
        g1 = oracle.weight_poly([0.05, 0.5 + dl, 0.6], h, faces)
        g0 = oracle.weight_poly([0.05, 0.5, 0.6], h, faces)
        gs = oracle.weight_poly([0.05, 0.5 + 1e-6, 0.6], h, faces)
        assert abs(g1 - (g0 + (gs - g0) * dl / 1e-6)) < 1e-13 + 1e-5 * dl


def test_symmetry_and_limits(oracle):
    x0 = [0.0, 0.0, 0.0]
    assert abs(oracle.weight_poly(x0, 1.0, box([-9, -9, 0], [0, 9, 9])) - 0.25) < 1e-12   # edge
    assert abs(oracle.weight_poly(x0, 1.0, box([0, 0, 0], [9, 9, 9])) - 0.125) < 1e-12     # corner
    assert abs(oracle.weight_poly(x0, 1.0, box([-2.5] * 3, [2.5] * 3)) - 1.0) < 1e-12        # ball inside
    assert abs(oracle.weight_poly(x0, 1.0, box([2.01, -1, -1], [3, 1, 1]))) < 1e-14          # disjoint
    # monotone in the cube size and 1 once the ball fits
    vals = [oracle.weight_poly(x0, 1.0, box([-a] * 3, [a] * 3)) for a in np.linspace(0.2, 2.0, 10)]
    assert all(np.diff(vals) > 0) and abs(vals[-1] - 1.0) < 1e-12


# ------------------------------------------------------------- Monte Carlo
def _radial_sampler():
    q = np.linspace(0.0, 2.0, 200001)
    pdf = 4 * q * q * m4(q)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(q))])
    cdf /= cdf[-1]
    return lambda u: np.interp(u, cdf, q)


def _planes(faces, inside):
    ns, cs = [], []
    for F in faces:
        F = np.asarray(F, float)
        c = F.mean(axis=0)
        n = np.zeros(3)
        for k in range(len(F)):
            n += np.cross(F[k] - c, F[(k + 1) % len(F)] - c)
        n /= np.linalg.norm(n)
        if np.dot(n, c - inside) < 0:
            n = -n
        ns.append(n)
        cs.append(np.dot(n, c))
    return np.array(ns), np.array(cs)


def test_monte_carlo_random_cells(oracle, small_tess):
    pos, m, h, tess = small_tess
    inv = _radial_sampler()
    g = rng(7)
    n_samp = 2_000_000
    checked = 0
    for c in [3, 50, 121, 200, 277]:
        faces = tess.cell_faces(c)
        gen = tess.generators[c]
        N, C = _planes(faces, gen)
        for trial in range(2):
            # particle near the cell (inside or outside), h ~ cell size
            x = gen + g.normal(size=3) * 0.05
            hh = g.uniform(0.03, 0.09)
            wq = oracle.weight_poly(x, hh, faces, inside=gen)
            d = g.normal(size=(n_samp, 3))
            d /= np.linalg.norm(d, axis=1)[:, None]
            r = inv(g.random(n_samp)) * hh
            X = x + d * r[:, None]
            inside = np.all(X @ N.T <= C + 1e-15, axis=1)
            est = inside.mean()
            sig = math.sqrt(max(wq * (1 - wq), 1e-12) / n_samp)
            assert abs(est - wq) < 5 * sig + 2e-6, (c, wq, est, sig)
            checked += 1
    assert checked == 10


# ------------------------------------------------------ tessellation sums
def test_partition_of_unity(oracle, small_tess):
    pos, m, h, tess = small_tess
    # particles whose 2h ball lies inside the box: coverage sums to 1
    inner = np.where(np.all((pos - 2 * h[:, None] > 0) & (pos + 2 * h[:, None] < 1), axis=1))[0][:25]
    assert len(inner) >= 10
    cov, _ = oracle.particles(tess, pos, h, inner)
    assert np.max(np.abs(cov - 1.0)) < 1e-11
    # and a particle next to a wall loses exactly its mass beyond the wall
    # (half-space closed form at the distance to the single nearest wall)
    i = int(np.argmin(pos[:, 2] / h))
    d = pos[i, 2] / h[i]
    others = min(pos[i, 0], 1 - pos[i, 0], pos[i, 1], 1 - pos[i, 1], 1 - pos[i, 2]) / h[i]
    if d < 2 and others > 2:
        wb = (d**6 / 20 - 3 * d**5 / 20 + d**3 / 3 - 7 * d / 10 + 0.5) if d < 1 else \
            (-d**6 / 60 + 3 * d**5 / 20 - d**4 / 2 + 2 * d**3 / 3 - 4 * d / 5 + 8 / 15)
        cov1, _ = oracle.particles(tess, pos, h, [i])
        assert abs(cov1[0] - (1 - wb)) < 1e-11


def test_mass_conservation_and_reverse_constant(oracle, small_tess):
    pos, m, h, tess = small_tess
    M, rho, npairs = oracle.map_cells(tess, pos, h, m)
    cov, q = oracle.particles(tess, pos, h, None, np.full(tess.n_cells, 3.25))
    # sum_c M_c = sum_i m_i c_i (the same pair weights summed two ways)
    assert abs(M.sum() - np.dot(m, cov)) < 1e-13
    # mass is only lost through the non-periodic walls
    assert 0.5 < M.sum() <= 1.0 + 1e-12
    # inverse mapping of a constant field returns the constant
    assert np.max(np.abs(q - 3.25)) < 1e-12
    # sum_i m_i c_i q_i = sum_c M_c q_c for a varying field
    qc = np.sin(7 * tess.generators[:, 0]) + tess.generators[:, 1]
    cov2, qi = oracle.particles(tess, pos, h, None, qc)
    assert abs(np.dot(m * cov2, qi) - np.dot(M, qc)) < 1e-13
    vol, _ = oracle.cell_info(tess)
    assert abs(vol.sum() - 1.0) < 1e-12
    assert np.allclose(rho, M / vol, rtol=1e-15)


def _split(faces, n, c0, inside):
    """Clip a convex cell (list of faces) by the plane n.x = c0 into the two
    convex halves (plain polygon clipping, test-local)."""
    def clip(fs, nn, cc):
        out, cut = [], []
        for F in fs:
            F = np.asarray(F, float)
            s = F @ nn - cc
            P = []
            for k in range(len(F)):
                a, b = F[k], F[(k + 1) % len(F)]
                sa, sb = s[k], s[(k + 1) % len(F)]
                if sa <= 0:
                    P.append(a)
                if (sa < 0 < sb) or (sb < 0 < sa):
                    t = sa / (sa - sb)
                    p = a + t * (b - a)
                    P.append(p)
                    cut.append(p)
            if len(P) >= 3:
                out.append(np.array(P))
        cut = np.array(cut)
        cen = cut.mean(axis=0)
        u = cut[0] - cen
        u /= np.linalg.norm(u)
        v = np.cross(nn / np.linalg.norm(nn), u)
        ang = np.arctan2((cut - cen) @ v, (cut - cen) @ u)
        cap = cut[np.argsort(ang)]
        keep = [cap[0]]
        for p in cap[1:]:
            if np.linalg.norm(p - keep[-1]) > 1e-12:
                keep.append(p)
        out.append(np.array(keep))
        return out

    return clip(faces, n, c0), clip(faces, -n, -c0)


def test_additivity_under_plane_split(oracle, small_tess):
    pos, m, h, tess = small_tess
    g = rng(3)
    for c in [10, 99, 180]:
        faces = tess.cell_faces(c)
        gen = tess.generators[c]
        n = g.normal(size=3)
        n /= np.linalg.norm(n)
        c0 = float(np.dot(n, gen))
        A, B = _split(faces, n, c0, gen)
        ia = np.concatenate(A).mean(axis=0)
        ib = np.concatenate(B).mean(axis=0)
        for _ in range(3):
            x = gen + g.normal(size=3) * 0.04
            hh = g.uniform(0.03, 0.08)
            whole = oracle.weight_poly(x, hh, faces, inside=gen)
            parts = oracle.weight_poly(x, hh, A, inside=ia) + oracle.weight_poly(x, hh, B, inside=ib)
            assert abs(whole - parts) < 1e-11, (c, whole, parts)


def test_invariances(oracle, small_tess):
    pos, m, h, tess = small_tess
    g = rng(5)
    c = 42
    faces = tess.cell_faces(c)
    gen = tess.generators[c]
    x = gen + np.array([0.01, -0.02, 0.015])
    hh = 0.06
    w0 = oracle.weight_poly(x, hh, faces, inside=gen)
    shift = np.array([3.1, -2.2, 0.7])
    assert abs(oracle.weight_poly(x + shift, hh, [F + shift for F in faces], inside=gen + shift) - w0) < 1e-12
    s = 7.5
    assert abs(oracle.weight_poly(x * s, hh * s, [F * s for F in faces], inside=gen * s) - w0) < 1e-12
    # 90-degree rotation about z followed by a reflection of x (reverses orientation)
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]]) @ np.diag([-1.0, 1, 1])
    assert abs(oracle.weight_poly(R @ x, hh, [F @ R.T for F in faces], inside=R @ gen) - w0) < 1e-12
    # vertex order reversed: same cell
    assert abs(oracle.weight_poly(x, hh, [F[::-1] for F in faces], inside=gen) - w0) < 1e-14


# ------------------------------------------------------------ pair list
def test_pair_list_contains_every_overlap(oracle, small_tess):
    pos, m, h, tess = small_tess
    off, idx, w = oracle.pairs_weights(tess, pos, h)
    # every particle overlaps its own cell (the generator is the particle)
    for c in range(tess.n_cells):
        assert c in idx[off[c]:off[c + 1]]
        assert np.all(np.diff(idx[off[c]:off[c + 1]]) > 0)  # ascending
    # pairs left out have zero weight: test the nearest excluded particles
    g = rng(9)
    for c in g.choice(tess.n_cells, 20, replace=False):
        inl = set(idx[off[c]:off[c + 1]].tolist())
        d = np.linalg.norm(pos - tess.generators[c], axis=1) - 2 * h
        for i in np.argsort(d):
            if int(i) in inl:
                continue
            assert abs(oracle.weight(tess, c, pos[i], h[i])) < 1e-14
            break
    assert np.all(w >= -1e-13) and np.all(w <= 1 + 1e-13)
