"""ORACLE -- test infrastructure only (ctypes wrapper of oracle.c).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The device library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_L = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(_SO):
            build(True)
        L = ctypes.CDLL(_SO)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.ora_threads.restype = ctypes.c_int
        L.ora_threads.argtypes = []
        L.ora_w.restype = dbl
        L.ora_w.argtypes = [dbl]
        L.ora_Phi.restype = dbl
        L.ora_Phi.argtypes = [dbl]
        L.ora_G.restype = dbl
        L.ora_G.argtypes = [dbl]
        L.ora_Psi.restype = dbl
        L.ora_Psi.argtypes = [dbl, dbl]
        L.ora_fan_integral.restype = dbl
        L.ora_fan_integral.argtypes = [dbl, dbl, dbl, dbl]
        L.ora_weight_poly.restype = dbl
        L.ora_weight_poly.argtypes = [vp, dbl, ctypes.c_int, vp, vp, vp]
        tess = [i64, vp, vp, vp, vp, vp]
        L.ora_pairs_weights.restype = None
        L.ora_pairs_weights.argtypes = tess + [i64, vp, vp, i64, vp, vp, vp, vp, vp]
        L.ora_weight.restype = dbl
        L.ora_weight.argtypes = tess + [i64, vp, dbl]
        L.ora_cell_info.restype = None
        L.ora_cell_info.argtypes = tess + [i64, vp, vp, vp]
        L.ora_map_cells.restype = None
        L.ora_map_cells.argtypes = tess + [i64, vp, vp, vp, i64, vp, vp, vp, vp]
        L.ora_particles.restype = None
        L.ora_particles.argtypes = tess + [i64, vp, vp, i64, vp, vp, i32, vp, vp]
        L.ora_node_h.restype = ctypes.c_int
        L.ora_node_h.argtypes = [vp, dbl, i64, vp, dbl, dbl, vp, vp]
        L.ora_pseudo_build.restype = i64
        L.ora_pseudo_build.argtypes = [i64, vp, vp, vp, i32, vp, dbl, dbl, dbl, dbl, i32, i32, i64, i64, vp] + [vp] * 15
        L.ora_fneu_limit.restype = dbl
        L.ora_fneu_limit.argtypes = [dbl, dbl]
        L.ora_underresolved.restype = i64
        L.ora_underresolved.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, vp]
        L.ora_voronoi.restype = ctypes.c_int
        L.ora_voronoi.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ora_kd_build.restype = i64
        L.ora_kd_build.argtypes = ([i64, vp, vp, vp, i32, vp, dbl, dbl, dbl, dbl, dbl, i32, i32, i64, i32, i64, i64, vp]
                                   + [vp] * 13)
        L.ora_voronoi_cells.restype = None
        L.ora_voronoi_cells.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp]
        L.ora_lloyd.restype = None
        L.ora_lloyd.argtypes = [i64, vp, vp, vp, i32, vp]
        L.ora_work_counts.restype = None
        L.ora_work_counts.argtypes = tess + [i64, vp, vp, i64, vp, vp, vp]
        L.ora_cell_distance.restype = None
        L.ora_cell_distance.argtypes = tess + [i64, vp, vp, vp]
        L.ora_interpolate.restype = None
        L.ora_interpolate.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp, i32, vp]
        _L = L
    return _L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _tess_args(t):
    return [t.n_cells, _p(t.generators), _p(t.vertices), _p(t.cell_face_off), _p(t.face_vtx_off), _p(t.face_vtx)]


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_lib().ora_threads())


# ---------------------------------------------------------------- kernel
def w(q: float) -> float:
    return _lib().ora_w(q)


def Phi(q: float) -> float:
    return _lib().ora_Phi(q)


def G(u: float) -> float:
    return _lib().ora_G(u)


def Psi(ad: float, U: float) -> float:
    return _lib().ora_Psi(ad, U)


def fan_integral(ad, p, pa, pb) -> float:
    return _lib().ora_fan_integral(ad, p, pa, pb)


# ---------------------------------------------------------- single cells
def weight_poly(x, h, faces, inside=None) -> float:
    """Kernel integral of particle (x,h) over one convex cell given as a list
    of [k,3] vertex arrays (either orientation)."""
    fsz = np.array([len(f) for f in faces], dtype=np.int32)
    verts = _c(np.concatenate([np.asarray(f, float) for f in faces]), np.float64)
    if inside is None:
        inside = verts.mean(axis=0)
    x = _c(x, np.float64)
    inside = _c(inside, np.float64)
    return _lib().ora_weight_poly(_p(x), float(h), len(faces), _p(fsz), _p(verts), _p(inside))


# --------------------------------------------------------- tessellations
def weight(t, c: int, x, h: float) -> float:
    x = _c(x, np.float64)
    return _lib().ora_weight(*_tess_args(t), int(c), _p(x), float(h))


def work_counts(t, pos, h, cells, owned: bool = False):
    """What the Exact integral of the canonical pairs of the listed cells
    must evaluate, in exact geometry: [pairs, faces, faces the support
    reaches, their edges, edges the support reaches, inner pieces, outer
    pieces] (see ora_work_counts).  owned: a face shared with a cell
    (t.face_nbr) counts only for the lower-numbered of the two."""
    cells = _c(cells, np.int64)
    pos, h = _c(pos, np.float64), _c(h, np.float64)
    out = np.zeros(7, dtype=np.int64)
    nbr = _c(t.face_nbr, np.int32) if owned else None
    _lib().ora_work_counts(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(cells), _p(cells),
                           _p(nbr) if nbr is not None else None, _p(out))
    return out


def cell_distance(t, cells, xyz):
    """Signed distance of point xyz[k] to cell cells[k]: positive outside
    (distance to the nearest point of the cell), minus the distance to the
    nearest face plane inside.  The exact 0/1 shortcuts of the mapping hold
    where it is at least 2h (w = 0) or at most -2h (w = 1)."""
    cells = _c(cells, np.int64)
    xyz = _c(np.asarray(xyz, float).reshape(-1, 3), np.float64)
    assert len(cells) == xyz.shape[0]
    out = np.empty(len(cells))
    _lib().ora_cell_distance(*_tess_args(t), len(cells), _p(cells), _p(xyz), _p(out))
    return out


def cell_info(t, cells=None):
    """(volumes, canonical binary32 radii) of the listed cells."""
    cells = np.arange(t.n_cells, dtype=np.int64) if cells is None else _c(cells, np.int64)
    vol = np.empty(len(cells))
    rad = np.empty(len(cells), dtype=np.float32)
    _lib().ora_cell_info(*_tess_args(t), len(cells), _p(cells), _p(vol), _p(rad))
    return vol, rad


def pair_lists(t, pos, h, cells=None):
    """Canonical candidate pairs of the listed cells without weights:
    (offsets[len(cells)+1], particle idx)."""
    cells = np.arange(t.n_cells, dtype=np.int64) if cells is None else _c(cells, np.int64)
    pos = _c(pos, np.float64)
    h = _c(h, np.float64)
    L = _lib()
    counts = np.zeros(len(cells), dtype=np.int64)
    L.ora_pairs_weights(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(cells), _p(cells), _p(counts),
                        None, None, None)
    off = np.zeros(len(cells) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    idx = np.empty(int(off[-1]), dtype=np.int32)
    L.ora_pairs_weights(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(cells), _p(cells), _p(counts),
                        _p(off), _p(idx), None)
    return off, idx


def pairs_weights(t, pos, h, cells=None):
    """Canonical candidate pairs of the listed cells with their weights:
    (offsets[len(cells)+1], particle idx, w)."""
    cells = np.arange(t.n_cells, dtype=np.int64) if cells is None else _c(cells, np.int64)
    pos = _c(pos, np.float64)
    h = _c(h, np.float64)
    L = _lib()
    counts = np.zeros(len(cells), dtype=np.int64)
    L.ora_pairs_weights(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(cells), _p(cells), _p(counts),
                        None, None, None)
    off = np.zeros(len(cells) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    idx = np.empty(int(off[-1]), dtype=np.int32)
    wv = np.empty(int(off[-1]))
    L.ora_pairs_weights(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(cells), _p(cells), _p(counts),
                        _p(off), _p(idx), _p(wv))
    return off, idx, wv


def map_cells(t, pos, h, m, cells=None):
    """Forward mapping of the listed cells: (M_c, rho_c, n_pairs)."""
    cells = np.arange(t.n_cells, dtype=np.int64) if cells is None else _c(cells, np.int64)
    pos, h, m = _c(pos, np.float64), _c(h, np.float64), _c(m, np.float64)
    mass = np.empty(len(cells))
    rho = np.empty(len(cells))
    npairs = np.empty(len(cells), dtype=np.int64)
    _lib().ora_map_cells(*_tess_args(t), pos.shape[0], _p(pos), _p(h), _p(m), len(cells), _p(cells),
                         _p(mass), _p(rho), _p(npairs))
    return mass, rho, npairs


def particles(t, pos, h, parts=None, q=None):
    """Coverage c_i and inverse-mapped values q_i of the listed particles.
    q: cell values [n_cells] or [n_cells, k]."""
    pos, h = _c(pos, np.float64), _c(h, np.float64)
    parts = np.arange(pos.shape[0], dtype=np.int64) if parts is None else _c(parts, np.int64)
    cov = np.empty(len(parts))
    outq = None
    ncomp = 0
    qq = None
    if q is not None:
        qq = _c(q, np.float64)
        ncomp = 1 if qq.ndim == 1 else qq.shape[1]
        if ncomp > 16:
            raise ValueError("at most 16 components")
        outq = np.empty((len(parts), ncomp))
    _lib().ora_particles(*_tess_args(t), pos.shape[0], _p(pos), _p(h), len(parts), _p(parts), _p(qq), ncomp,
                         _p(cov), _p(outq))
    if outq is not None and qq.ndim == 1:
        outq = outq[:, 0]
    return cov, outq


# ----------------------------------------------------- pseudo-particles
def node_h(a, s, upos, hfact=1.2, eps=1e-2):
    """(h, branch, newton iterations) of one node over the unit positions."""
    a = _c(a, np.float64)
    upos = _c(upos, np.float64)
    h = np.zeros(1)
    it = np.zeros(1, dtype=np.int32)
    br = _lib().ora_node_h(_p(a), float(s), upos.shape[0], _p(upos), hfact, eps, _p(h), _p(it))
    return float(h[0]), int(br), int(it[0])


def pseudo_build(pos, m, h, sources, r_part=0.2, theta=0.5, hfact=1.2, eps=1e-2, leaf_max=8, max_depth=21,
                 bypass=1_000_000, open_labels=None):
    """Tree-walk pseudo-particles and node smoothing lengths.  Returns a dict
    of arrays in emission order.  open_labels: node labels to open whatever
    the walk criterion says (the failed nodes of an earlier walk).  'owner'
    gives, for every particle, the entry that holds it."""
    pos, m, h = _c(pos, np.float64), _c(m, np.float64), _c(h, np.float64)
    src = _c(np.asarray(sources, float).reshape(-1, 3), np.float64)
    n = pos.shape[0]
    kind = np.empty(n, dtype=np.int32)
    first = np.empty(n, dtype=np.int64)
    count = np.empty(n, dtype=np.int64)
    opos = np.empty((n, 3))
    mass = np.empty(n)
    oh = np.empty(n)
    s = np.empty(n)
    branch = np.empty(n, dtype=np.int32)
    unit = np.empty(n, dtype=np.int32)
    label = np.empty(n, dtype=np.uint64)
    owner = np.empty(n, dtype=np.int64)
    nu = np.zeros(1, dtype=np.int64)
    upos = np.empty((n, 3))
    nn = np.zeros(1, dtype=np.int64)
    sroot = np.zeros(1)
    op = np.ascontiguousarray(np.asarray(open_labels if open_labels is not None else [], dtype=np.uint64))
    k = _lib().ora_pseudo_build(n, _p(pos), _p(m), _p(h), src.shape[0], _p(src), r_part, theta, hfact, eps,
                                leaf_max, max_depth, bypass, len(op), _p(op), _p(kind), _p(first), _p(count),
                                _p(opos), _p(mass), _p(oh), _p(s), _p(branch), _p(unit), _p(label), _p(owner), _p(nu),
                                _p(upos), _p(nn), _p(sroot))
    k = int(k)
    return dict(kind=kind[:k], first=first[:k], count=count[:k], pos=opos[:k], mass=mass[:k], h=oh[:k], s=s[:k],
                branch=branch[:k], unit=unit[:k], label=label[:k], owner=owner, upos=upos[:int(nu[0])], n_nodes=int(nn[0]),
                s_root=float(sroot[0]))


def fneu_limit(s_ratio: float, K: float) -> float:
    """eq. resol_param: neutral-fraction threshold of a node of relative size s_ratio."""
    return float(_lib().ora_fneu_limit(float(s_ratio), float(K)))


def underresolved(kind, label, s, fneu, s_root: float, K: float):
    """Labels of the pseudo-particles below their threshold, in entry order."""
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    label = np.ascontiguousarray(label, dtype=np.uint64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    fneu = np.ascontiguousarray(fneu, dtype=np.float64)
    out = np.empty(len(kind), dtype=np.uint64)
    k = _lib().ora_underresolved(len(kind), _p(kind), _p(label), _p(s), _p(fneu), float(s_root), float(K), _p(out))
    return out[:int(k)]


def interpolate(pos, owner, entry_pos, entry_h, entry_kind, values):
    """Per-particle values from the mixed set (Sec. 3.3): a particle that is
    an entry keeps its value, any other takes the Shepard-normalised SPH
    interpolant over the entries whose 2h spheres reach it, each weighted by
    w(r / h_j) (volume (h_j / h_fact)^3 times W; its owner's value when none
    reaches it).  values: [E] or [E][k]."""
    pos = _c(pos, np.float64)
    owner = _c(owner, np.int64)
    ex = _c(entry_pos, np.float64)
    eh = _c(entry_h, np.float64)
    ek = _c(entry_kind, np.int32)
    v = np.asarray(values, dtype=np.float64)
    k = 1 if v.ndim == 1 else v.shape[1]
    assert k <= 16
    v = np.ascontiguousarray(v.reshape(len(eh), k))
    out = np.empty((pos.shape[0], k))
    _lib().ora_interpolate(pos.shape[0], _p(pos), _p(owner), len(eh), _p(ex), _p(eh), _p(ek), _p(v), k, _p(out))
    return out[:, 0] if np.asarray(values).ndim == 1 else out


def voronoi(gen, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0)):
    """Voronoi cells of the generators in the box (Sec. 2.3) by cutting the
    box with every bisector.  Returns volume [C], centroid [C][3] and the
    faces: cell_face_off [C+1], face_id [F] (neighbour, or -1..-6 for the
    box planes x-, x+, y-, y+, z-, z+), face_area [F], face_vtx_off [F+1]
    and face_pts [FV][3] (each face's polygon in cyclic order)."""
    g = _c(np.asarray(gen).reshape(-1, 3), np.float64)
    lo = _c(box_lo, np.float64)
    hi = _c(box_hi, np.float64)
    n = g.shape[0]
    vol = np.empty(n)
    cen = np.empty((n, 3))
    F = np.zeros(1, dtype=np.int64)
    FV = np.zeros(1, dtype=np.int64)
    _lib().ora_voronoi(n, _p(g), _p(lo), _p(hi), _p(vol), _p(cen), None, None, None, None, None, _p(F), _p(FV))
    cfo = np.empty(n + 1, dtype=np.int64)
    fid = np.empty(int(F[0]), dtype=np.int64)
    farea = np.empty(int(F[0]))
    fvo = np.empty(int(F[0]) + 1, dtype=np.int64)
    pts = np.empty((int(FV[0]), 3))
    _lib().ora_voronoi(n, _p(g), _p(lo), _p(hi), _p(vol), _p(cen), _p(cfo), _p(fid), _p(farea), _p(fvo), _p(pts),
                       _p(F), _p(FV))
    return dict(volume=vol, centroid=cen, cell_face_off=cfo, face_id=fid, face_area=farea, face_vtx_off=fvo,
                face_pts=pts)


def lloyd(gen, iters, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0)):
    """Generators after `iters` Lloyd iterations (each moves to the centroid
    of its Voronoi cell, Sec. 2.3)."""
    g = _c(np.asarray(gen).reshape(-1, 3), np.float64)
    out = np.empty_like(g)
    _lib().ora_lloyd(g.shape[0], _p(g), _p(_c(box_lo, np.float64)), _p(_c(box_hi, np.float64)), int(iters), _p(out))
    return out


def voronoi_cells(gen, cells, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0)):
    """Volume and centroid of the listed cells only."""
    g = _c(np.asarray(gen).reshape(-1, 3), np.float64)
    cells = _c(cells, np.int64)
    vol = np.empty(len(cells))
    cen = np.empty((len(cells), 3))
    _lib().ora_voronoi_cells(g.shape[0], _p(g), _p(_c(box_lo, np.float64)), _p(_c(box_hi, np.float64)), len(cells),
                             _p(cells), _p(vol), _p(cen))
    return vol, cen



def kd_build(pos, m, h, sources, r_part=0.2, r_leaf=None, theta=0.5, hfact=1.2, eps=1e-2, leaf_split=10,
             max_depth=62, nf_threshold=10_000, up_levels=1, bypass=1_000_000, open_labels=None):
    """Pseudo-particles from the paper's k-d tree (Sec. 2.2.1, 2.4): the
    entries in emission order, each with its node's label and level, the
    owner of every particle, and stats (nodes, units, k_mid or -1 when all
    units are summed, pseudo-particles)."""
    pos, m, h = _c(pos, np.float64), _c(m, np.float64), _c(h, np.float64)
    src = _c(np.asarray(sources, float).reshape(-1, 3), np.float64)
    n = pos.shape[0]
    r_leaf = r_part if r_leaf is None else r_leaf
    kind = np.empty(n, dtype=np.int32)
    first = np.empty(n, dtype=np.int64)
    count = np.empty(n, dtype=np.int64)
    opos = np.empty((n, 3))
    mass = np.empty(n)
    oh = np.empty(n)
    s = np.empty(n)
    branch = np.empty(n, dtype=np.int32)
    label = np.empty(n, dtype=np.uint64)
    level = np.empty(n, dtype=np.int32)
    owner = np.empty(n, dtype=np.int64)
    st = np.zeros(4, dtype=np.int64)
    sroot = np.zeros(1)
    op = np.ascontiguousarray(np.asarray(open_labels if open_labels is not None else [], dtype=np.uint64))
    k = int(_lib().ora_kd_build(n, _p(pos), _p(m), _p(h), src.shape[0], _p(src), r_part, r_leaf, theta, hfact, eps,
                                leaf_split, max_depth, nf_threshold, up_levels, bypass, len(op), _p(op), _p(kind),
                                _p(first), _p(count), _p(opos), _p(mass), _p(oh), _p(s), _p(branch), _p(label),
                                _p(level), _p(owner), _p(st), _p(sroot)))
    return dict(kind=kind[:k], first=first[:k], count=count[:k], pos=opos[:k], mass=mass[:k], h=oh[:k], s=s[:k],
                branch=branch[:k], label=label[:k], level=level[:k], owner=owner,
                stats=dict(n_nodes=int(st[0]), n_units=int(st[1]), k_mid=int(st[2]), n_pseudo=int(st[3])),
                s_root=float(sroot[0]))
