"""The boundary's inverse map without a retained pair list, the context's
workspace cap, and the summation orders include/sphmap.h states.

  - map_cells_to_particles with no pair list recomputes the weights from the
    particles and the grid: the values equal those from the retained list
    bit for bit (same kernels, same weights), and match the oracle's inverse
    map;
  - a context whose workspace cap is too small refuses a mapping with
    SPHMAP_ENOMEM before allocating and reports an upper bound of what the
    call needs; with that cap the same call succeeds and the scratch stays
    within it;
  - M_c and each particle's inverse-map sum follow the fixed strided-plus-
    butterfly order the header describes: numpy, adding the exported
    weights in that order, reproduces them bit for bit;
  - empty and oversized inputs get the errors the header states (EINVAL
    before any device work, outputs untouched), and interpolation onto no
    particles is a valid call that writes nothing."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def grid(workloads):
    pos, m, h, rho = workloads.make_cloud("turbulent", 6000, seed=31)
    return pos, m, h, workloads.voronoi(pos)


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_15227_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_inverse_map_recomputes_without_pairs(ctx, grid, oracle, precision):
    import paper_2410_15227_amd as pkg
    say(f"case: inverse map without a pair list, turbulent 6000, {precision}")
    pos, m, h, tess = grid
    dt = ctx.upload(tess)
    g = tess.generators
    q = np.stack([np.sin(7 * g[:, 0]) ** 2, g[:, 1] * g[:, 2]], axis=1)
    res = pkg.map_particles_to_cells(ctx, dt, pos, h, m, precision=precision, keep_pairs=True)
    a = pkg.map_cells_to_particles(ctx, res.pairs, q).cpu().numpy()
    b = pkg.map_cells_to_particles(ctx, None, q, tess=dt, xyz=pos, h=h, precision=precision).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b)
    parts = np.arange(0, len(pos), 53)
    cov, qref = oracle.particles(tess, pos, h, parts, q)
    assert np.max(np.abs(b[parts] - qref)) < (1e-11 if precision == "fp64" else 1e-5)
    res.pairs.free()
    dt.free()


def test_workspace_cap(grid):
    import paper_2410_15227_amd as pkg
    say("case: workspace cap, turbulent 6000")
    pos, m, h, tess = grid
    small = pkg.Context(0, workspace_bytes=4 << 20)
    dt = small.upload(tess)
    with pytest.raises(pkg.SphmapError) as e:
        pkg.map_particles_to_cells(small, dt, pos, h, m)
    assert e.value.code == -2  # SPHMAP_ENOMEM
    info = small.workspace_info()
    say(f"refused: {info}")
    assert info["limit"] == 4 << 20 and info["held"] <= info["limit"]
    need = info["required"]
    est = small.estimate_footprint(len(pos), tess)
    assert need > info["limit"] and need <= est["workspace"] + est["pairs"]
    small.set_workspace_limit(need)
    res = pkg.map_particles_to_cells(small, dt, pos, h, m)
    torch.cuda.synchronize()
    info = small.workspace_info()
    assert 0 < info["held"] <= need
    # the capped context computes what an uncapped one does
    big = pkg.Context(0)
    dt2 = big.upload(tess)
    ref = pkg.map_particles_to_cells(big, dt2, pos, h, m)
    assert torch.equal(res.mass, ref.mass)
    dt.free()
    dt2.free()
    small.close()
    big.close()


def _butterfly(parts):
    """Combine partial sums pairwise: l with l + n/2, then l + n/4, ..., as a
    wavefront's xor-shuffle butterfly does; returns lane 0's value."""
    v = np.array(parts, dtype=np.float64)
    n = len(v)
    o = n // 2
    while o >= 1:
        v = v + v[np.arange(n) ^ o]
        o //= 2
    return v[0]


def _strided(terms, lanes):
    """Partial l adds terms l, l + lanes, ... in turn (each product already
    rounded), then the butterfly."""
    parts = np.zeros(lanes)
    for l in range(lanes):
        acc = 0.0
        for t in terms[l::lanes]:
            acc = acc + t
        parts[l] = acc
    return _butterfly(parts)


def test_documented_summation_orders(ctx, grid):
    import paper_2410_15227_amd as pkg
    say("case: summation orders of M_c and of the inverse map")
    pos, m, h, tess = grid
    dt = ctx.upload(tess)
    res = pkg.map_particles_to_cells(ctx, dt, pos, h, m, keep_pairs=True)
    off, idx, w = (t.cpu().numpy() for t in res.pairs.export())
    M = res.mass.cpu().numpy()
    cells = np.random.default_rng(3).choice(tess.n_cells, 300, replace=False)
    for c in cells:
        terms = m[idx[off[c]:off[c + 1]]] * w[off[c]:off[c + 1]]
        assert _strided(terms, 64) == M[c], c
    q = np.cos(5 * tess.generators[:, 0])
    out = pkg.map_cells_to_particles(ctx, res.pairs, q).cpu().numpy()
    cov = res.coverage.cpu().numpy()
    # particle-major order: each particle's pairs in ascending cell index
    cell_of = np.repeat(np.arange(tess.n_cells), np.diff(off))
    order = np.lexsort((cell_of, idx))
    pidx, pcell, pw = idx[order], cell_of[order], w[order]
    starts = np.searchsorted(pidx, np.arange(len(pos) + 1))
    for i in np.random.default_rng(4).choice(len(pos), 300, replace=False):
        s, e = starts[i], starts[i + 1]
        cov_i = _strided(pw[s:e], 64)
        assert cov_i == cov[i], i
        v = _strided(pw[s:e] * q[pcell[s:e]], 16)
        assert (v / cov_i if cov_i > 0 else 0.0) == out[i], i
    res.pairs.free()
    dt.free()


def test_empty_and_oversized_inputs(ctx, grid):
    import paper_2410_15227_amd as pkg
    from paper_2410_15227_amd import _native
    say("case: empty and oversized inputs")
    pos, m, h, tess = grid
    dt = ctx.upload(tess)
    none3 = np.zeros((0, 3))
    none1 = np.zeros(0)
    # forward map of no particles: EINVAL, the mass buffer left as it was
    sentinel = torch.full((tess.n_cells,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.SphmapError) as e:
        pkg.map_particles_to_cells(ctx, dt, none3, none1, none1, out_mass=sentinel)
    assert e.value.code == -1  # SPHMAP_EINVAL
    torch.cuda.synchronize()
    assert bool(torch.all(sentinel == -7.0))
    # n = 2^31 through the C-ABI: refused by its range check before any
    # pointer is used (the buffers hold one particle)
    x = torch.as_tensor(pos[:1], dtype=torch.float64, device="cuda").contiguous()
    hh = torch.as_tensor(h[:1], dtype=torch.float64, device="cuda")
    mm = torch.as_tensor(m[:1], dtype=torch.float64, device="cuda")
    rc = _native.lib().map_particles_to_cells(ctx.handle, dt.handle, 1 << 31, x.data_ptr(), hh.data_ptr(),
                                              mm.data_ptr(), 1, 0, sentinel.data_ptr(), None, None, None, None)
    assert rc == -1
    torch.cuda.synchronize()
    assert bool(torch.all(sentinel == -7.0))
    # inverse map without a list, of no particles
    with pytest.raises(pkg.SphmapError) as e:
        pkg.map_cells_to_particles(ctx, None, np.ones(tess.n_cells), tess=dt, xyz=none3, h=none1)
    assert e.value.code == -1
    # pseudo-particle builders and the Voronoi builder on no points
    for tree in ("octree", "kd"):
        with pytest.raises(pkg.SphmapError) as e:
            pkg.build_pseudo_particles(ctx, none3, none1, none1, [[0.5, 0.5, 0.5]], tree=tree)
        assert e.value.code == -1
    with pytest.raises(pkg.SphmapError) as e:
        pkg.build_voronoi(ctx, none3, n_lloyd=0)
    assert e.value.code == -1
    # interpolation onto no particles is valid and returns an empty array
    ps = pkg.build_pseudo_particles(ctx, pos, h, m, [[0.9, 0.9, 0.9]], r_part=0.05, theta=0.8)
    out = pkg.interpolate_to_particles(ctx, none3, ps, torch.ones(ps["kind"].shape[0], dtype=torch.float64,
                                                                  device="cuda"))
    torch.cuda.synchronize()
    assert out.shape == (0,)
    dt.free()
