"""Exact SPH <-> Voronoi mapping and tree-node pseudo-particles on MI355X.

Thin Python binding of libsphmap (include/sphmap.h): argument marshalling
only.  Device memory and streams come from PyTorch (ROCm); every step of the
computation runs in the library's HIP kernels.

    ctx  = Context(0)
    tess = ctx.upload(tessellation)                # workloads.Tessellation
    out  = map_particles_to_cells(ctx, tess, xyz, h, m, precision="mixed",
                                  keep_pairs=True)
    q    = map_cells_to_particles(ctx, out.pairs, cell_values)
    ps   = build_pseudo_particles(ctx, xyz, h, m, sources)
"""
from __future__ import annotations

import ctypes
import dataclasses

from . import _native
from ._native import PREC_FP64, PREC_MIXED, SphmapError

__all__ = ["Context", "DeviceTessellation", "Pairs", "MapResult", "map_particles_to_cells",
           "map_cells_to_particles", "build_pseudo_particles", "SphmapError", "PREC_FP64", "PREC_MIXED"]


STATUS_NONFINITE_MASS = 1   # a cell mass was not finite
STATUS_ZERO_COVERAGE = 2    # inverse map: a particle no cell overlaps got 0
STATUS_NONFINITE_VALUE = 4  # inverse map or interpolation wrote a non-finite value


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f64(x, device, shape_last=None):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
    if shape_last is not None and (t.ndim != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected [n,{shape_last}] array")
    return t


class Context:
    """A library context on one HIP device (torch device index).
    workspace_bytes: cap on the context's device scratch (0 = none)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the mapping runs only on the HIP device")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        L = _native.lib()
        h = ctypes.c_void_p()
        _native.check(L.sphmap_create(device, int(workspace_bytes), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _native.lib().sphmap_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        _native.check(rc, self.handle)

    def set_workspace_limit(self, nbytes: int):
        self.check(_native.lib().sphmap_set_workspace_limit(self.handle, int(nbytes)))

    def workspace_info(self) -> dict:
        """held, limit and required (the workspace the last refused call needs)."""
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self.check(_native.lib().sphmap_workspace_info(self.handle, ctypes.byref(a), ctypes.byref(b),
                                                       ctypes.byref(c)))
        return dict(held=a.value, limit=b.value, required=c.value)

    def upload(self, tess, stream=None, neighbours: bool = True) -> "DeviceTessellation":
        """Upload a host grid; with neighbours (default) its face_nbr, when it
        has one, is declared (sphmap_tess_set_face_neighbours), so that the
        mixed path evaluates each shared face once per particle."""
        return DeviceTessellation(self, tess, stream, neighbours)

    # timing / counters -------------------------------------------------
    def sync_status(self, stream=None, clear: bool = True) -> int:
        """Wait for `stream` and return the device status word (bits
        STATUS_*), clearing it unless clear is False."""
        v = ctypes.c_int32()
        self.check(_native.lib().sphmap_sync_status(self.handle, _stream_handle(stream), 1 if clear else 0,
                                                    ctypes.byref(v)))
        return v.value

    def estimate_footprint(self, n_particles: int, tess, n_pairs: int = 0) -> dict:
        """Device bytes of one forward + inverse mapping of n_particles on
        `tess` (host Tessellation or DeviceTessellation's source): the
        context workspace, the retained pair list and the uploaded grid.
        n_pairs: the candidate-pair count if known, else 0 (estimated)."""
        f = _native.Footprint()
        self.check(_native.lib().sphmap_estimate_footprint(
            self.handle, int(n_particles), int(n_pairs), int(tess.n_cells), len(tess.face_vtx_off) - 1,
            len(tess.face_vtx), len(tess.vertices), ctypes.byref(f)))
        return dict(workspace=f.workspace, pairs=f.pairs, tessellation=f.tessellation)

    def set_timing(self, on: bool = True):
        self.check(_native.lib().sphmap_set_timing(self.handle, 1 if on else 0))

    def kernel_time(self, name: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(_native.lib().sphmap_kernel_time(self.handle, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def reset_timing(self):
        self.check(_native.lib().sphmap_reset_timing(self.handle))

    def set_counting(self, on: bool = True):
        self.check(_native.lib().sphmap_set_counting(self.handle, 1 if on else 0))

    def set_pool_limit(self, n_bytes: int):
        """Largest device memory the pool of freed pair-list blocks keeps."""
        self.check(_native.lib().sphmap_set_pool_limit(self.handle, int(n_bytes)))

    def set_autotune(self, on: bool = True):
        """Autotune the Exact launch shape per power-of-two pair-count class."""
        self.check(_native.lib().sphmap_set_autotune(self.handle, 1 if on else 0))

    def tuned_shape(self, n_pairs: int):
        """(workgroups per CU, chunks per fetch, ms) kept for the class of n_pairs, or None."""
        b, f, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self.check(_native.lib().sphmap_tuned_shape(self.handle, int(n_pairs), ctypes.byref(b), ctypes.byref(f),
                                                    ctypes.byref(ms)))
        return None if b.value == 0 else (b.value, f.value, ms.value)

    def work_counters(self):
        arr = (ctypes.c_int64 * 8)()
        self.check(_native.lib().sphmap_work_counters(self.handle, arr))
        return list(arr)


class DeviceTessellation:
    """A tessellation resident on the device (see include/sphmap.h)."""

    def __init__(self, ctx: Context, tess, stream=None, neighbours: bool = True):
        import numpy as np
        self.ctx = ctx
        self.n_cells = int(tess.n_cells)
        g = np.ascontiguousarray(tess.generators, dtype=np.float64)
        v = np.ascontiguousarray(tess.vertices, dtype=np.float64)
        cfo = np.ascontiguousarray(tess.cell_face_off, dtype=np.int64)
        fvo = np.ascontiguousarray(tess.face_vtx_off, dtype=np.int64)
        fv = np.ascontiguousarray(tess.face_vtx, dtype=np.int32)
        h = ctypes.c_void_p()
        L = _native.lib()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        ctx.check(L.sphmap_tess_upload(ctx.handle, self.n_cells, len(fvo) - 1, len(v), p(g), p(v), p(cfo), p(fvo),
                                       p(fv), _stream_handle(stream), ctypes.byref(h)))
        self.handle = h
        self.n_shared = 0
        nbr = getattr(tess, "face_nbr", None)
        if neighbours and nbr is not None and len(nbr) == len(fvo) - 1:
            self.set_face_neighbours(nbr, stream)

    def set_face_neighbours(self, face_nbr, stream=None) -> int:
        """Declare each face's neighbouring cell (negative: wall); None clears.
        Returns the number of faces found shared."""
        import numpy as np
        n = ctypes.c_int64()
        if face_nbr is None:
            arg = None
        else:
            nb = np.ascontiguousarray(face_nbr, dtype=np.int32)
            arg = nb.ctypes.data_as(ctypes.c_void_p)
        self.ctx.check(_native.lib().sphmap_tess_set_face_neighbours(self.ctx.handle, self.handle, arg,
                                                                     _stream_handle(stream), ctypes.byref(n)))
        self.n_shared = n.value
        return n.value

    @classmethod
    def _from_handle(cls, ctx: Context, handle) -> "DeviceTessellation":
        self = cls.__new__(cls)
        self.ctx = ctx
        self.handle = handle
        self.n_shared = None  # a grid built on the device records its neighbours
        c = ctypes.c_int64()
        _native.lib().sphmap_tess_counts(handle, ctypes.byref(c), None, None, None)
        self.n_cells = c.value
        return self

    def counts(self) -> dict:
        c, f, fv, v = (ctypes.c_int64() for _ in range(4))
        self.ctx.check(_native.lib().sphmap_tess_counts(self.handle, ctypes.byref(c), ctypes.byref(f), ctypes.byref(fv),
                                                        ctypes.byref(v)))
        return dict(n_cells=c.value, n_faces=f.value, n_face_vertices=fv.value, n_vertices=v.value)

    def export(self, with_neighbours: bool = True, stream=None):
        """The grid as host arrays (a workloads.Tessellation); face_nbr holds
        each face's neighbouring site (-1..-6: box planes) for grids built by
        build_voronoi."""
        import numpy as np

        from .workloads import Tessellation
        torch = _torch()
        k = self.counts()
        dev = self.ctx.device
        g = torch.empty((k["n_cells"], 3), dtype=torch.float64, device=dev)
        v = torch.empty((max(k["n_vertices"], 1), 3), dtype=torch.float64, device=dev)
        cfo = torch.empty(k["n_cells"] + 1, dtype=torch.int64, device=dev)
        fvo = torch.empty(k["n_faces"] + 1, dtype=torch.int64, device=dev)
        fv = torch.empty(max(k["n_face_vertices"], 1), dtype=torch.int32, device=dev)
        nb = torch.full((max(k["n_faces"], 1),), -7, dtype=torch.int32, device=dev)
        self.ctx.check(_native.lib().sphmap_tess_export(self.ctx.handle, self.handle, _ptr(g), _ptr(v), _ptr(cfo),
                                                        _ptr(fvo), _ptr(fv), _ptr(nb) if with_neighbours else None,
                                                        _stream_handle(stream)))
        torch.cuda.synchronize(dev)
        gn = g.cpu().numpy()
        vn = v.cpu().numpy()[:k["n_vertices"]]
        return Tessellation(generators=gn, vertices=vn, cell_face_off=cfo.cpu().numpy(),
                            face_vtx_off=fvo.cpu().numpy(), face_vtx=fv.cpu().numpy()[:k["n_face_vertices"]],
                            face_nbr=nb.cpu().numpy()[:k["n_faces"]],
                            box_lo=np.min(vn, axis=0) if len(vn) else np.zeros(3),
                            box_hi=np.max(vn, axis=0) if len(vn) else np.ones(3))

    def cell_info(self, stream=None):
        torch = _torch()
        vol = torch.empty(self.n_cells, dtype=torch.float64, device=self.ctx.device)
        rad = torch.empty(self.n_cells, dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(_native.lib().sphmap_tess_cell_info(self.ctx.handle, self.handle, _ptr(vol), _ptr(rad),
                                                            _stream_handle(stream)))
        return vol, rad

    def free(self):
        if self.handle:
            _native.lib().sphmap_tess_free(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.ctx.handle:
                self.free()
        except Exception:
            pass


def build_voronoi(ctx: Context, generators, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), n_lloyd: int = 5,
                  stream=None):
    """The Voronoi grid of the sites on the device (Sec. 2.3), after n_lloyd
    Lloyd iterations.  Returns (DeviceTessellation, final sites [n][3] on the
    device)."""
    torch = _torch()
    g = _dev_f64(generators, ctx.device, 3)
    out = torch.empty_like(g)
    lo = (ctypes.c_double * 3)(*[float(x) for x in box_lo])
    hi = (ctypes.c_double * 3)(*[float(x) for x in box_hi])
    h = ctypes.c_void_p()
    ctx.check(_native.lib().sphmap_tess_build_voronoi(ctx.handle, g.shape[0], _ptr(g), lo, hi, int(n_lloyd),
                                                      _ptr(out), _stream_handle(stream), ctypes.byref(h)))
    return DeviceTessellation._from_handle(ctx, h), out


class Pairs:
    """A retained candidate-pair list with its weights."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        n = ctypes.c_int64()
        c = ctypes.c_int64()
        q = ctypes.c_int64()
        ctx.check(_native.lib().sphmap_pairs_info(handle, ctypes.byref(n), ctypes.byref(c), ctypes.byref(q)))
        self.n_pairs, self.n_cells, self.n_particles = n.value, c.value, q.value

    def export(self, stream=None):
        """(cell_off int64 [C+1], particle int32 [P], w float64 [P]) on the device."""
        torch = _torch()
        dev = self.ctx.device
        off = torch.empty(self.n_cells + 1, dtype=torch.int64, device=dev)
        part = torch.empty(max(self.n_pairs, 1), dtype=torch.int32, device=dev)
        w = torch.empty(max(self.n_pairs, 1), dtype=torch.float64, device=dev)
        self.ctx.check(_native.lib().sphmap_pairs_export(self.ctx.handle, self.handle, _ptr(off), _ptr(part), _ptr(w),
                                                          _stream_handle(stream)))
        return off, part[:self.n_pairs], w[:self.n_pairs]

    def free(self):
        if self.handle:
            _native.lib().sphmap_pairs_free(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.ctx.handle:
                self.free()
        except Exception:
            pass


@dataclasses.dataclass
class MapResult:
    mass: object
    density: object
    coverage: object
    pairs: Pairs | None


def map_particles_to_cells(ctx: Context, tess: DeviceTessellation, xyz, h, m, precision: str | int = "mixed",
                           normalize: bool = False, keep_pairs: bool = False, with_coverage: bool = True,
                           out_mass=None, out_density=None, out_coverage=None, stream=None) -> MapResult:
    """Forward Exact mapping: cell masses M_c, densities M_c/V_c and the
    particle coverage c_i (see include/sphmap.h)."""
    torch = _torch()
    dev = ctx.device
    xyz = _dev_f64(xyz, dev, 3)
    h = _dev_f64(h, dev)
    m = _dev_f64(m, dev)
    n = xyz.shape[0]
    if h.shape != (n,) or m.shape != (n,):
        raise ValueError("h and m must have shape [n]")
    prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}.get(precision, precision)
    mass = out_mass if out_mass is not None else torch.empty(tess.n_cells, dtype=torch.float64, device=dev)
    dens = out_density if out_density is not None else torch.empty(tess.n_cells, dtype=torch.float64, device=dev)
    cov = out_coverage
    if cov is None and with_coverage:
        cov = torch.empty(n, dtype=torch.float64, device=dev)
    ph = ctypes.c_void_p()
    ctx.check(_native.lib().map_particles_to_cells(ctx.handle, tess.handle, n, _ptr(xyz), _ptr(h), _ptr(m), int(prec),
                                                   1 if normalize else 0, _ptr(mass), _ptr(dens), _ptr(cov),
                                                   _stream_handle(stream), ctypes.byref(ph) if keep_pairs else None))
    pairs = Pairs(ctx, ph) if keep_pairs else None
    return MapResult(mass, dens, cov, pairs)


def map_particles_to_cells_batch(ctx: Context, tess, xyz, h, m, precision: str | int = "mixed",
                                 normalize: bool = False, keep_pairs: bool = False, with_coverage: bool = True,
                                 stream=None) -> list:
    """Forward mapping of several independent instances in one call (lists
    of tessellations and per-instance particle arrays); returns one
    MapResult per instance."""
    torch = _torch()
    dev = ctx.device
    k = len(tess)
    if not (len(xyz) == len(h) == len(m) == k) or k < 1:
        raise ValueError("tess, xyz, h and m must be lists of the same non-zero length")
    xs = [_dev_f64(a, dev, 3) for a in xyz]
    hs = [_dev_f64(a, dev) for a in h]
    ms = [_dev_f64(a, dev) for a in m]
    ns = [a.shape[0] for a in xs]
    for x, hh, mm, n in zip(xs, hs, ms, ns):
        if hh.shape != (n,) or mm.shape != (n,):
            raise ValueError("h and m must have shape [n] per instance")
    prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}.get(precision, precision)
    mass = [torch.empty(t.n_cells, dtype=torch.float64, device=dev) for t in tess]
    dens = [torch.empty(t.n_cells, dtype=torch.float64, device=dev) for t in tess]
    cov = [torch.empty(n, dtype=torch.float64, device=dev) for n in ns] if with_coverage else None
    P = ctypes.c_void_p * k
    arr = lambda ts: P(*[_ptr(t) for t in ts])
    th = P(*[t.handle for t in tess])
    nn = (ctypes.c_int64 * k)(*ns)
    ph = P()
    ctx.check(_native.lib().map_particles_to_cells_batch(
        ctx.handle, k, th, nn, arr(xs), arr(hs), arr(ms), int(prec), 1 if normalize else 0, arr(mass), arr(dens),
        arr(cov) if cov is not None else None, _stream_handle(stream), ph if keep_pairs else None))
    out = []
    for j in range(k):
        pairs = Pairs(ctx, ctypes.c_void_p(ph[j])) if keep_pairs else None
        out.append(MapResult(mass[j], dens[j], cov[j] if cov is not None else None, pairs))
    return out


class BatchPlan:
    """A batched forward mapping captured as one HIP graph (sphmap_batch_*):
    run() launches the whole step once; the particle tensors passed at
    creation may be updated in place between steps.  Outputs: .mass,
    .density, .coverage (lists of device tensors, rewritten by each step)."""

    def __init__(self, ctx: Context, tess, xyz, h, m, normalize: bool = False, headroom: float = 0.125,
                 stream=None):
        torch = _torch()
        dev = ctx.device
        k = len(tess)
        if not (len(xyz) == len(h) == len(m) == k) or k < 1:
            raise ValueError("tess, xyz, h and m must be lists of the same non-zero length")
        self.ctx = ctx
        self.xyz = [_dev_f64(a, dev, 3) for a in xyz]
        self.h = [_dev_f64(a, dev) for a in h]
        self.m = [_dev_f64(a, dev) for a in m]
        ns = [a.shape[0] for a in self.xyz]
        self.mass = [torch.empty(t.n_cells, dtype=torch.float64, device=dev) for t in tess]
        self.density = [torch.empty(t.n_cells, dtype=torch.float64, device=dev) for t in tess]
        self.coverage = [torch.empty(n, dtype=torch.float64, device=dev) for n in ns]
        P = ctypes.c_void_p * k
        arr = lambda ts: P(*[_ptr(t) for t in ts])
        self._keep = (tess,)
        h_ = ctypes.c_void_p()
        ctx.check(_native.lib().sphmap_batch_create(
            ctx.handle, k, P(*[t.handle for t in tess]), (ctypes.c_int64 * k)(*ns), arr(self.xyz), arr(self.h),
            arr(self.m), 1 if normalize else 0, arr(self.mass), arr(self.density), arr(self.coverage),
            float(headroom), _stream_handle(stream), ctypes.byref(h_)))
        self.handle = h_
        self.n_inst = k

    def run(self, stream=None):
        self.ctx.check(_native.lib().sphmap_batch_run(self.ctx.handle, self.handle, _stream_handle(stream)))

    def check(self, stream=None):
        """(pair count of each instance in the last step, overflow flag)."""
        counts = (ctypes.c_int64 * self.n_inst)()
        flag = ctypes.c_int32()
        self.ctx.check(_native.lib().sphmap_batch_check(self.ctx.handle, self.handle, _stream_handle(stream), counts,
                                                        ctypes.byref(flag)))
        return list(counts), bool(flag.value)

    def free(self):
        if self.handle:
            _native.lib().sphmap_batch_free(self.ctx.handle, self.handle)
            self.handle = None


def map_cells_to_particles(ctx: Context, pairs, cell_values, out=None, stream=None, *, tess=None, xyz=None,
                           h=None, precision: str | int = "mixed"):
    """Inverse mapping q_i = sum_c w_ic q_c / c_i ([C] or [C,k] -> [n] or [n,k]).
    pairs: a retained list of the forward mapping, or None to recompute the
    weights from the particles (xyz, h) and the grid `tess`."""
    torch = _torch()
    q = torch.as_tensor(cell_values, dtype=torch.float64, device=ctx.device).contiguous()
    k = 1 if q.ndim == 1 else q.shape[1]
    if pairs is not None:
        if q.shape[0] != pairs.n_cells:
            raise ValueError("cell_values must have one row per cell")
        n = pairs.n_particles
        args = (None, 0, None, None, 0, pairs.handle)
    else:
        if tess is None or xyz is None or h is None:
            raise ValueError("without a pair list, tess, xyz and h are needed")
        if q.shape[0] != tess.n_cells:
            raise ValueError("cell_values must have one row per cell")
        xyz = _dev_f64(xyz, ctx.device, 3)
        h = _dev_f64(h, ctx.device)
        n = xyz.shape[0]
        if h.shape != (n,):
            raise ValueError("h must have shape [n]")
        prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}.get(precision, precision)
        args = (tess.handle, n, _ptr(xyz), _ptr(h), int(prec), None)
    shape = (n,) if q.ndim == 1 else (n, k)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=ctx.device)
    ctx.check(_native.lib().map_cells_to_particles(ctx.handle, *args, _ptr(q), k, _ptr(out), _stream_handle(stream)))
    return out


def build_pseudo_particles(ctx: Context, xyz, h, m, sources, r_part: float = 0.2, theta: float = 0.5,
                           h_fact: float = 1.2, eps_h: float = 1e-2, leaf_max: int = 8, max_depth: int | None = None,
                           bypass_threshold: int = 1_000_000, open_labels=None, tree: str = "octree",
                           r_leaf: float | None = None, leaf_split: int = 10, nf_threshold: int = 10_000,
                           up_levels: int = 1, stream=None) -> dict:
    """Tree-node pseudo-particles and their smoothing lengths (Sec. 2.4).
    tree: "octree" (cubic subdivision, at most leaf_max per leaf) or "kd"
    (the paper's k-d tree: recursive coordinate bisection, split while
    holding leaf_split or more; r_leaf annulus; k_mid neighbour-find above
    nf_threshold units).  open_labels: node labels to open whatever the walk
    criterion says (the failed nodes of an earlier walk).  Returns a dict of
    device tensors in emission order (with each entry's node 'label', and
    'level' for the k-d tree), 'owner' (for every input particle, the entry
    that holds it) and 'stats'."""
    if tree not in ("octree", "kd"):
        raise ValueError("tree must be 'octree' or 'kd'")
    if max_depth is None:
        max_depth = 21 if tree == "octree" else 62
    import numpy as np
    torch = _torch()
    dev = ctx.device
    xyz = _dev_f64(xyz, dev, 3)
    h = _dev_f64(h, dev)
    m = _dev_f64(m, dev)
    n = xyz.shape[0]
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).reshape(-1, 3))
    opts = _native.PseudoOpts(r_part, theta, h_fact, eps_h, leaf_max, max_depth, bypass_threshold)
    cap = n
    o = dict(xyz=torch.empty((cap, 3), dtype=torch.float64, device=dev),
             h=torch.empty(cap, dtype=torch.float64, device=dev),
             m=torch.empty(cap, dtype=torch.float64, device=dev),
             s=torch.empty(cap, dtype=torch.float64, device=dev),
             kind=torch.empty(cap, dtype=torch.int32, device=dev),
             first=torch.empty(cap, dtype=torch.int64, device=dev),
             count=torch.empty(cap, dtype=torch.int64, device=dev),
             branch=torch.empty(cap, dtype=torch.int32, device=dev),
             label=torch.empty(cap, dtype=torch.int64, device=dev))  # uint64 bit patterns
    owner = torch.empty(n, dtype=torch.int64, device=dev)
    if open_labels is not None and len(open_labels) > 0:
        ol = torch.as_tensor(np.asarray(open_labels, dtype=np.uint64).view(np.int64), device=dev).contiguous()
    else:
        ol = None
    n_out = ctypes.c_int64()
    st = _native.PseudoStats()
    k_mid = ctypes.c_int32(-1)
    if tree == "octree":
        ctx.check(_native.lib().build_pseudo_particles_open(
            ctx.handle, n, _ptr(xyz), _ptr(h), _ptr(m), src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(opts), 0 if ol is None else ol.shape[0], _ptr(ol), cap, _ptr(o["xyz"]), _ptr(o["h"]),
            _ptr(o["m"]), _ptr(o["s"]), _ptr(o["kind"]), _ptr(o["first"]), _ptr(o["count"]), _ptr(o["branch"]),
            _ptr(o["label"]), _ptr(owner), ctypes.byref(n_out), ctypes.byref(st), _stream_handle(stream)))
    else:
        o["level"] = torch.empty(cap, dtype=torch.int32, device=dev)
        kd = _native.KdOpts(float(r_part if r_leaf is None else r_leaf), int(leaf_split), int(up_levels),
                            int(nf_threshold))
        ctx.check(_native.lib().build_pseudo_particles_kd(
            ctx.handle, n, _ptr(xyz), _ptr(h), _ptr(m), src.shape[0], src.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(opts), ctypes.byref(kd), 0 if ol is None else ol.shape[0], _ptr(ol), cap, _ptr(o["xyz"]),
            _ptr(o["h"]), _ptr(o["m"]), _ptr(o["s"]), _ptr(o["kind"]), _ptr(o["first"]), _ptr(o["count"]),
            _ptr(o["branch"]), _ptr(o["label"]), _ptr(o["level"]), _ptr(owner), ctypes.byref(n_out),
            ctypes.byref(st), ctypes.byref(k_mid), _stream_handle(stream)))
    k = n_out.value
    res = {key: val[:k] for key, val in o.items()}
    res["owner"] = owner
    res["stats"] = dict(n_nodes=st.n_nodes, n_units=st.n_units, n_pseudo=st.n_pseudo, n_real=st.n_real,
                        branch_count=list(st.branch_count), s_root=st.s_root, k_mid=k_mid.value)
    return res


def select_underresolved(ctx: Context, ps: dict, fneu, K: float, stream=None):
    """Labels (uint64, host) of the pseudo-particles of `ps` whose neutral
    fraction `fneu` (one value per entry) is below f_neu,limit of their size
    (eq. resol_param), in entry order."""
    import numpy as np
    torch = _torch()
    fneu = _dev_f64(fneu, ctx.device)
    n = ps["kind"].shape[0]
    out = torch.empty(max(n, 1), dtype=torch.int64, device=ctx.device)
    cnt = ctypes.c_int64()
    ctx.check(_native.lib().select_underresolved(ctx.handle, n, _ptr(ps["kind"]), _ptr(ps["label"]), _ptr(ps["s"]),
                                                 _ptr(fneu), float(ps["stats"]["s_root"]), float(K), _ptr(out),
                                                 ctypes.byref(cnt), _stream_handle(stream)))
    return out[:cnt.value].cpu().numpy().view(np.uint64)


def interpolate_to_particles(ctx: Context, xyz, ps: dict, values, stream=None, out=None, noalloc: bool = False):
    """Per-particle values from the mixed set `ps` (Sec. 3.3): a particle
    emitted as itself keeps its entry's value; a member of a pseudo-particle
    takes the Shepard-normalised SPH interpolant over the entries whose 2h
    spheres reach it, entry j weighted by w(r / h_j) (its volume
    (h_j / h_fact)^3 times W).  values: [E] or [E][k] per entry; returns [n] or
    [n][k] on the device.  noalloc: use the entry point that allocates no
    device memory (its scratch is the library's fixed per-device region; with
    `out` given, the call allocates nothing at all)."""
    torch = _torch()
    dev = ctx.device
    xyz = _dev_f64(xyz, dev, 3)
    v = _dev_f64(values, dev)
    if v.dim() not in (1, 2):
        raise ValueError("values must be [E] or [E][k]")
    ne = ps["kind"].shape[0]
    k = 1 if v.dim() == 1 else v.shape[1]
    if v.shape[0] != ne:
        raise ValueError(f"values has {v.shape[0]} rows for {ne} entries")
    n = xyz.shape[0]
    if out is None:
        out = torch.empty((n, k) if v.dim() == 2 else n, dtype=torch.float64, device=dev)
    fn = _native.lib().interpolate_to_particles_noalloc if noalloc else _native.lib().interpolate_to_particles
    ctx.check(fn(ctx.handle, n, _ptr(xyz), _ptr(ps["owner"]), ne, _ptr(ps["xyz"]), _ptr(ps["h"]), _ptr(ps["kind"]),
                 _ptr(v), k, _ptr(out), _stream_handle(stream)))
    return out


def adaptive_pseudo_particles(ctx: Context, xyz, h, m, sources, cell_fneu, K: float, max_iter: int = 16,
                              precision: str = "mixed", n_lloyd: int = 5, leaf_remedy: str = "open",
                              **walk) -> tuple:
    """The adaptive tree walk of Sec. 2.4.1.  Each iteration builds the
    pseudo-particles with every node that has failed so far opened, builds the
    Voronoi grid of the mixed set on the device (n_lloyd Lloyd iterations,
    Sec. 2.3), asks `cell_fneu(sites)` for the neutral fraction of every cell
    (the radiative transfer's output; here any cell field), maps it back onto
    the entries (map_cells_to_particles of the forward mapping's weights) and
    checks eq. resol_param; it stops when no pseudo-particle is
    under-resolved.  A failed pseudo-particle that is a leaf cannot be
    resolved further: leaf_remedy "open" opens it into its particles (they are
    never checked); "grow" is the paper's remedy, which instead increases
    r_part (and r_leaf by as much) until that leaf lies inside it, so that
    every node within the new radius is emitted at particle level.  Returns
    (final build, history); the build also holds the entries' 'fneu', the
    labels it 'opened' and the final 'r_part' and 'r_leaf'."""
    import numpy as np

    if leaf_remedy not in ("open", "grow"):
        raise ValueError("leaf_remedy must be 'open' or 'grow'")
    src = np.asarray(sources, dtype=np.float64).reshape(-1, 3)
    walk = dict(walk)
    walk.setdefault("r_part", 0.2)
    if walk.get("tree", "octree") == "kd":
        walk.setdefault("r_leaf", walk["r_part"])
        leaf_below = walk.get("leaf_split", 10)  # a k-d leaf holds fewer than leaf_split
    else:
        leaf_below = walk.get("leaf_max", 8) + 1  # an octree leaf holds at most leaf_max
    opened = np.zeros(0, dtype=np.uint64)
    history = []
    for it in range(max_iter):
        ps = build_pseudo_particles(ctx, xyz, h, m, src, open_labels=opened, **walk)
        dt, sites = build_voronoi(ctx, ps["xyz"], n_lloyd=n_lloyd)
        res = map_particles_to_cells(ctx, dt, ps["xyz"], ps["h"], ps["m"], precision=precision, keep_pairs=True)
        f_cells = np.asarray(cell_fneu(sites.cpu().numpy()), dtype=np.float64)
        fneu = map_cells_to_particles(ctx, res.pairs, f_cells)
        bad = select_underresolved(ctx, ps, fneu, K)
        history.append(dict(iteration=it, n_entries=int(ps["kind"].shape[0]), n_pseudo=ps["stats"]["n_pseudo"],
                            n_pairs=res.pairs.n_pairs, n_failed=int(len(bad)), r_part=walk["r_part"]))
        res.pairs.free()
        dt.free()
        ps["fneu"] = fneu
        ps["opened"] = opened
        ps["r_part"] = walk["r_part"]
        ps["r_leaf"] = walk.get("r_leaf", walk["r_part"])
        if len(bad) == 0:
            return ps, history
        if leaf_remedy == "grow":
            lab = ps["label"].cpu().numpy().view(np.uint64)
            cnt = ps["count"].cpu().numpy()
            leaf = np.isin(lab, bad) & (cnt < leaf_below) & (ps["kind"].cpu().numpy() == 1)
            if leaf.any():
                pos_l = ps["xyz"].cpu().numpy()[leaf]
                s_l = ps["s"].cpu().numpy()[leaf]
                # a node reaches r_part when r - s <= r_part for some source
                r = np.min(np.linalg.norm(pos_l[:, None, :] - src[None, :, :], axis=2), axis=1)
                grow = float(np.max(r - s_l)) * (1.0 + 1e-12) + 1e-15
                if grow > walk["r_part"]:
                    d = grow - walk["r_part"]
                    walk["r_part"] = grow
                    if "r_leaf" in walk:
                        walk["r_leaf"] = walk["r_leaf"] + d
                bad = np.setdiff1d(bad, lab[leaf])
        opened = np.union1d(opened, bad)
    return ps, history
