"""Seeded synthetic inputs for the mapping: particle clouds, their SPH
smoothing lengths and a box-clipped Voronoi tessellation of the generation
sites.

This module is shared by the device path, the CPU oracle's tests and the
benchmark as the common source of inputs.  It holds none of the mapping's
arithmetic: the SPH smoothing-length solve of the INPUT particles is what the
SPH code does before the radiation step (Sec. 2.3, first paragraph of the
pipeline description), and the Voronoi grid with generation sites at the
particle positions is the grid code's input (Sec. 1, Sec. 2.3).

Workload recipes (stand-ins for the paper's glass and turbulent boxes):
  * uniform cloud: n points uniform in the unit cube, equal masses 1/n;
  * turbulent cloud: a Gaussian random field with P(k) ~ k^-4 on a G^3 grid,
    standardised to delta, ln(rho) = sigma*delta - sigma^2/2, particles drawn
    multinomially over grid cells with probability ~ rho and placed uniformly
    inside the drawn cell, equal masses 1/n;
  * h from h = 1.2 (m/rho)^(1/3) with the self-consistent SPH density;
  * Voronoi grid of the same points, clipped to the (non-periodic) unit box.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsphinput.so")
_SRC = os.path.join(_HERE, "hostgeom.cpp")

_lib_handle = None


def build(force: bool = True) -> str:
    """Compile the host input tools (g++, OpenMP) into libsphinput.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        c_i64, c_dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.sph_smoothing_lengths.restype = c_i64
        L.sph_smoothing_lengths.argtypes = [c_i64, vp, vp, c_dbl, c_dbl, vp, vp]
        L.voronoi_build.restype = vp
        L.voronoi_build.argtypes = [c_i64, vp, vp, vp, vp, vp]
        L.voronoi_fill.restype = None
        L.voronoi_fill.argtypes = [vp] * 7
        L.voronoi_free.restype = None
        L.voronoi_free.argtypes = [vp]
        L.tess_check.restype = c_dbl
        L.tess_check.argtypes = [c_i64, vp, vp, vp, vp, vp, vp, vp]
        _lib_handle = L
    return _lib_handle


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------ clouds
def uniform_cloud(n: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1)^3 (PCG64 seeded), float64 [n,3]."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3))


def turbulent_cloud(n: int, seed: int, grid: int | None = None, sigma_lnrho: float = 1.5) -> np.ndarray:
    """Log-normal cloud from a Gaussian random field with P(k) ~ k^-4.

    grid defaults to 128 for n <= 2^18 and 256 above.
    """
    if grid is None:
        grid = 128 if n <= (1 << 18) else 256
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((grid, grid, grid))
    fk = np.fft.rfftn(noise)
    kx = np.fft.fftfreq(grid) * grid
    kz = np.fft.rfftfreq(grid) * grid
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / k2[nz]  # |k|^-2 amplitude -> P(k) ~ k^-4
    fk *= amp
    delta = np.fft.irfftn(fk, s=(grid, grid, grid), axes=(0, 1, 2))
    delta -= delta.mean()
    delta /= delta.std()
    rho = np.exp(sigma_lnrho * delta - 0.5 * sigma_lnrho**2).ravel()
    cdf = np.cumsum(rho)
    cdf /= cdf[-1]
    u = rng.random(n)
    cells = np.searchsorted(cdf, u, side="right")
    cells = np.minimum(cells, grid**3 - 1)
    iz = cells % grid
    iy = (cells // grid) % grid
    ix = cells // (grid * grid)
    off = rng.random((n, 3))
    pos = (np.stack([ix, iy, iz], axis=1) + off) / grid
    return np.ascontiguousarray(pos)


def smoothing_lengths(pos: np.ndarray, m: np.ndarray, hfact: float = 1.2, tol: float = 1e-4):
    """Self-consistent SPH h and rho (Newton, |dh|/h < tol; Sec. 2.4.2 cites
    the SPH relation h = hfact (m/rho)^(1/3)).  Returns (h, rho, n_bisect)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = pos.shape[0]
    h = np.empty(n)
    rho = np.empty(n)
    nb = _lib().sph_smoothing_lengths(n, _p(pos), _p(m), hfact, tol, _p(h), _p(rho))
    return h, rho, int(nb)


# ------------------------------------------------------------ tessellation
@dataclasses.dataclass
class Tessellation:
    """Convex cells given as faces grouped by cell.

    generators   [C,3] f64  generation sites (one per cell)
    vertices     [V,3] f64
    cell_face_off[C+1] i64  faces of cell c are cell_face_off[c]:cell_face_off[c+1]
    face_vtx_off [F+1] i64  vertex ids of face f are face_vtx[face_vtx_off[f]:...]
    face_vtx     [FV]  i32  cyclic polygon (either orientation is accepted)
    face_nbr     [F]   i32  neighbouring cell or -1 for the box wall (informational)
    box_lo, box_hi (3,) f64
    """

    generators: np.ndarray
    vertices: np.ndarray
    cell_face_off: np.ndarray
    face_vtx_off: np.ndarray
    face_vtx: np.ndarray
    face_nbr: np.ndarray
    box_lo: np.ndarray
    box_hi: np.ndarray
    cell_vtx_off: np.ndarray | None = None

    @property
    def n_cells(self) -> int:
        return int(self.generators.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_vtx_off.shape[0] - 1)

    def cell_faces(self, c: int):
        """List of faces of cell c, each an [k,3] array of vertex positions."""
        out = []
        for f in range(int(self.cell_face_off[c]), int(self.cell_face_off[c + 1])):
            ids = self.face_vtx[self.face_vtx_off[f]:self.face_vtx_off[f + 1]]
            out.append(self.vertices[ids])
        return out

    def subset(self, cells) -> "Tessellation":
        """A tessellation holding only the listed cells (same geometry); a
        face's neighbour is renumbered into the subset, or -1 when it is not
        in it."""
        cells = np.asarray(cells, dtype=np.int64)
        gens = self.generators[cells]
        renum = np.full(self.n_cells, -1, dtype=np.int64)
        renum[cells] = np.arange(len(cells))
        verts, fvo, fv, fnb, cfo = [], [0], [], [], [0]
        nv = 0
        for c in cells:
            for f in range(int(self.cell_face_off[c]), int(self.cell_face_off[c + 1])):
                ids = self.face_vtx[self.face_vtx_off[f]:self.face_vtx_off[f + 1]]
                verts.append(self.vertices[ids])
                fv.append(np.arange(nv, nv + len(ids), dtype=np.int32))
                nv += len(ids)
                fvo.append(nv)
                nb = int(self.face_nbr[f])
                fnb.append(int(renum[nb]) if nb >= 0 else nb)
            cfo.append(len(fnb))
        return Tessellation(
            generators=np.ascontiguousarray(gens),
            vertices=np.ascontiguousarray(np.concatenate(verts)) if verts else np.zeros((0, 3)),
            cell_face_off=np.asarray(cfo, dtype=np.int64),
            face_vtx_off=np.asarray(fvo, dtype=np.int64),
            face_vtx=np.concatenate(fv).astype(np.int32) if fv else np.zeros(0, np.int32),
            face_nbr=np.asarray(fnb, dtype=np.int32),
            box_lo=self.box_lo.copy(),
            box_hi=self.box_hi.copy(),
        )


def degeneracy_scores(t: Tessellation) -> np.ndarray:
    """A score per cell of how thin or sliver-like it is, for picking the
    cells that stress the closed forms in samples: the cell's largest vertex
    distance from its generator divided by the smaller of (a) the nearest
    face plane's distance from the generator and (b) the shortest edge.
    Flat cells, cells with a face nearly through the generator and cells
    with tiny edges score high."""
    fvo, fv, cfo = t.face_vtx_off, t.face_vtx.astype(np.int64), t.cell_face_off
    nf = len(fvo) - 1
    face_of_slot = np.repeat(np.arange(nf), np.diff(fvo))
    cell_of_face = np.repeat(np.arange(t.n_cells), np.diff(cfo))
    V = t.vertices[fv]
    nxt = np.arange(len(fv)) + 1
    last = fvo[1:] - 1
    nxt[last] = fvo[:-1]  # the edge from a face's last vertex closes the polygon
    W = V[nxt]
    # face area vector (fan about the first vertex), its unit normal
    V0 = V[fvo[:-1]][face_of_slot]
    cr = np.cross(V - V0, W - V0)
    area = np.zeros((nf, 3))
    np.add.at(area, face_of_slot, cr)
    an = np.linalg.norm(area, axis=1)
    n = area / np.where(an > 0, an, 1.0)[:, None]
    g = t.generators[cell_of_face]
    pd = np.abs(np.einsum("ij,ij->i", n, t.vertices[fv[fvo[:-1]]] - g))
    pd = np.where(an > 0, pd, np.inf)
    elen = np.linalg.norm(W - V, axis=1)
    elen = np.where(elen > 0, elen, np.inf)
    dmin = np.full(t.n_cells, np.inf)
    np.minimum.at(dmin, cell_of_face, pd)
    emin = np.full(t.n_cells, np.inf)
    np.minimum.at(emin, cell_of_face[face_of_slot], elen)
    rv = np.linalg.norm(V - t.generators[cell_of_face[face_of_slot]], axis=1)
    rmax = np.zeros(t.n_cells)
    np.maximum.at(rmax, cell_of_face[face_of_slot], rv)
    return rmax / np.minimum(dmin, emin)


def voronoi(gen: np.ndarray, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0)) -> Tessellation:
    """Box-clipped Voronoi tessellation of the generators (host, OpenMP)."""
    gen = np.ascontiguousarray(gen, dtype=np.float64)
    lo = np.ascontiguousarray(box_lo, dtype=np.float64)
    hi = np.ascontiguousarray(box_hi, dtype=np.float64)
    n = gen.shape[0]
    sizes = np.zeros(3, dtype=np.int64)
    nfail = np.zeros(1, dtype=np.int64)
    L = _lib()
    h = L.voronoi_build(n, _p(gen), _p(lo), _p(hi), _p(sizes), _p(nfail))
    try:
        if nfail[0] != 0:
            raise RuntimeError(f"voronoi: {int(nfail[0])} cells failed to clip")
        V, F, FV = (int(s) for s in sizes)
        verts = np.empty((V, 3))
        cvo = np.empty(n + 1, dtype=np.int64)
        cfo = np.empty(n + 1, dtype=np.int64)
        fvo = np.empty(F + 1, dtype=np.int64)
        fv = np.empty(FV, dtype=np.int32)
        fnb = np.empty(F, dtype=np.int32)
        L.voronoi_fill(h, _p(verts), _p(cvo), _p(cfo), _p(fvo), _p(fv), _p(fnb))
    finally:
        L.voronoi_free(h)
    return Tessellation(gen, verts, cfo, fvo, fv, fnb, lo, hi, cvo)


def tess_check(t: Tessellation):
    """(volumes, max closure defect, max non-planarity, #inward-facing faces)."""
    vol = np.empty(t.n_cells)
    stats = np.zeros(2)
    worst = _lib().tess_check(t.n_cells, _p(t.generators), _p(t.vertices), _p(t.cell_face_off),
                              _p(t.face_vtx_off), _p(t.face_vtx), _p(vol), _p(stats))
    return vol, float(worst), float(stats[0]), int(stats[1])


def box_cells(lo, hi) -> list:
    """Faces of an axis-aligned box cell as a list of [4,3] vertex arrays
    (CCW seen from outside)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    v = np.array([[hi[0] if k & 1 else lo[0], hi[1] if k & 2 else lo[1], hi[2] if k & 4 else lo[2]]
                  for k in range(8)])
    faces = [[0, 4, 6, 2], [1, 3, 7, 5], [0, 1, 5, 4], [2, 6, 7, 3], [0, 2, 3, 1], [4, 5, 7, 6]]
    return [v[f] for f in faces]


def tess_from_cells(gens, cells, box_lo=(0, 0, 0), box_hi=(1, 1, 1)) -> Tessellation:
    """Tessellation from explicit cells: cells[c] is a list of [k,3] faces."""
    verts, fvo, fv, cfo = [], [0], [], [0]
    nv = 0
    for faces in cells:
        for F in faces:
            F = np.asarray(F, float)
            verts.append(F)
            fv.append(np.arange(nv, nv + len(F), dtype=np.int32))
            nv += len(F)
            fvo.append(nv)
        cfo.append(len(fvo) - 1)
    return Tessellation(
        generators=np.ascontiguousarray(np.asarray(gens, float).reshape(-1, 3)),
        vertices=np.ascontiguousarray(np.concatenate(verts)),
        cell_face_off=np.asarray(cfo, dtype=np.int64),
        face_vtx_off=np.asarray(fvo, dtype=np.int64),
        face_vtx=np.concatenate(fv).astype(np.int32),
        face_nbr=-np.ones(len(fvo) - 1, dtype=np.int32),
        box_lo=np.asarray(box_lo, float),
        box_hi=np.asarray(box_hi, float),
    )


# -------------------------------------------------------------- workloads
@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray  # [n,3]
    h: np.ndarray
    m: np.ndarray
    rho: np.ndarray
    tess: Tessellation | None


def make_cloud(kind: str, n: int, seed: int):
    """(positions, masses, h, rho) of a seeded cloud ("uniform"|"turbulent")."""
    if kind == "uniform":
        pos = uniform_cloud(n, seed)
    elif kind == "turbulent":
        pos = turbulent_cloud(n, seed)
    else:
        raise ValueError(kind)
    m = np.full(n, 1.0 / n)
    h, rho, _ = smoothing_lengths(pos, m)
    return pos, m, h, rho


def uniform_4096(seed: int = 1) -> Workload:
    """4,096 uniform particles, m = 1/4096, h = 1.2 (m/rho)^(1/3), Voronoi
    grid of the same points in the unit box (the small FP64 case)."""
    pos, m, h, rho = make_cloud("uniform", 4096, seed)
    return Workload("uniform_4096", pos, h, m, rho, voronoi(pos))


def turbulent(n: int = 262144, seed: int = 2, with_tess: bool = True) -> Workload:
    """Log-normal (sigma_lnrho = 1.5) P(k)~k^-4 cloud of n particles, equal
    masses, SPH h, Voronoi grid of the same points."""
    pos, m, h, rho = make_cloud("turbulent", n, seed)
    return Workload(f"turbulent_{n}", pos, h, m, rho, voronoi(pos) if with_tess else None)


def densest_particle(rho: np.ndarray) -> int:
    """Index of the largest SPH density (ties to the lowest index)."""
    return int(np.argmax(rho))


def batch_mix(count: int = 64, base_seed: int = 4000, lo_exp: int = 12, hi_exp: int = 18):
    """Instance sizes and cloud kinds of the batched workload: n_k =
    round(2^U(lo,hi)), kind ~ Bernoulli(1/2), seed = base + k."""
    rng = np.random.default_rng(base_seed)
    exps = rng.uniform(lo_exp, hi_exp, size=count)
    kinds = rng.random(count) < 0.5
    return [(int(round(2.0**e)), "turbulent" if k else "uniform", base_seed + i)
            for i, (e, k) in enumerate(zip(exps, kinds))]


def jitter(pos: np.ndarray, m: np.ndarray, rho: np.ndarray, seed: int, frac: float = 0.01):
    """Gaussian positional jitter with sigma = frac*(m/rho)^(1/3) per
    component, clamped into the unit box."""
    rng = np.random.default_rng(seed)
    sig = frac * np.cbrt(m / rho)
    out = pos + rng.standard_normal(pos.shape) * sig[:, None]
    return np.clip(out, 0.0, np.nextafter(1.0, 0.0))
