"""Served mapping: continuous batching of mapping jobs on one GPU.

Jobs arrive at any time.  A job names a grid (tessellation) and the particles
to map onto it.  A job is admitted first-come first-served as soon as a slot
is free and its estimated device footprint fits in the memory budget next to
the jobs already running; each slot owns a library context and a HIP stream,
so admitted jobs overlap on the device while later arrivals wait.

State stays on the device across timesteps (the mapping is called every
timestep on the same fluid, Sec. 2.3): a grid, once uploaded, is kept
resident together with its particle arrays (positions, h, m and the jitter
scale of each particle).  A repeat-timestep job carries no particle data: it
names a resident grid and a seed, and its positions are the resident ones
moved by a seeded Gaussian jitter drawn on the device (the stand-in for the
hydrodynamics moving the particles between two calls), so it copies nothing
from the host.  Resident grids are evicted least-recently-used when the
budget needs their memory; a repeat job whose grid has been evicted uploads
it again from the host copy it refers to.

Every step of the mapping runs in the library's kernels; this module only
schedules (the jitter is workload synthesis, drawn with PyTorch's device
generator).  A job's results do not depend on what runs beside it: each
weight is a function of its own pair and each cell sum has a fixed order.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

# device bytes of one particle's resident state: x, y, z, h, m, jitter scale
RESIDENT_BYTES_PER_PARTICLE = 48
# device bytes of one particle's jittered positions while a repeat job runs
JITTER_BYTES_PER_PARTICLE = 24


@dataclass
class Job:
    key: str                 # identity of the grid and its particles
    tess: object             # host Tessellation (uploaded when not resident)
    pos: np.ndarray          # host particles of the grid (uploaded with it)
    h: np.ndarray
    m: np.ndarray
    rho: np.ndarray | None = None    # SPH densities: jitter scale 0.01 (m/rho)^(1/3)
    jitter_seed: int | None = None   # repeat timestep: resident positions + seeded jitter
    jitter_frac: float = 0.01
    arrival: float = 0.0     # time.perf_counter() at submission
    # filled in by the server
    start: float = 0.0
    end: float = 0.0
    n_pairs: int = 0
    resident_hit: bool = False
    host_bytes: int = 0      # bytes copied from the host for this job
    mass: object = None      # device tensor of cell masses
    coverage: object = None  # device tensor of particle coverages
    error: str | None = None
    done: threading.Event = field(default_factory=threading.Event)


@dataclass
class Resident:
    dt: object               # DeviceTessellation
    x: object                # device [n,3] positions of the grid's particles
    h: object
    m: object
    sigma: object            # device [n] jitter scale (None without densities)
    bytes: int
    users: int = 0


class MappingServer:
    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 64 << 30, precision: str = "mixed",
                 inverse_components: int = 1):
        import torch

        import paper_2410_15227_amd as pkg
        self._torch = torch
        self._pkg = pkg
        self.device = device
        self.precision = precision
        self.k = inverse_components
        self.budget = int(hbm_budget)
        self._slots = [(pkg.Context(device), torch.cuda.Stream(device=device)) for _ in range(slots)]
        # freed pair lists keep their blocks for the slot's next jobs: one
        # eighth of the budget over all slots, held beside it
        for ctx, _ in self._slots:
            ctx.set_pool_limit(self.budget // (8 * slots))
        self._est_ctx = pkg.Context(device)  # footprint queries, under the lock only
        self._cv = threading.Condition()
        self._queue: collections.deque[Job] = collections.deque()
        self._running_bytes = 0
        self._resident: collections.OrderedDict[str, Resident] = collections.OrderedDict()
        self._resident_bytes = 0
        self._pairs_seen: dict[str, int] = {}
        self._stop = False
        self.completed: list[Job] = []
        self._threads = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(slots)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------ interface
    def submit(self, job: Job) -> Job:
        job.arrival = job.arrival or time.perf_counter()
        with self._cv:
            self._queue.append(job)
            self._cv.notify_all()
        return job

    def footprint_bytes(self, job: Job, resident: bool = False) -> int:
        """Device bytes admission reserves for `job` (its grid and particle
        state counted unless resident)."""
        with self._cv:
            run, keep = self._footprint(job)
        return run + (0 if resident else keep)

    def resident_keys(self) -> list[str]:
        with self._cv:
            return list(self._resident.keys())

    def drain(self):
        """Wait until every submitted job has finished."""
        with self._cv:
            while self._queue or self._running_bytes:
                self._cv.wait()

    def close(self):
        self.drain()
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        with self._cv:
            for r in self._resident.values():
                r.dt.free()
            self._resident.clear()
        for ctx, _ in self._slots:
            ctx.close()
        self._est_ctx.close()

    # ----------------------------------------------------------- scheduling
    def _footprint(self, job: Job) -> tuple[int, int]:
        """(bytes while the job runs, bytes its grid and particles keep when
        resident), from the library's model; a grid seen before lends its
        last pair count."""
        n = len(job.m)
        fp = self._est_ctx.estimate_footprint(n, job.tess, self._pairs_seen.get(job.key, 0))
        run = fp["workspace"] + fp["pairs"] + (JITTER_BYTES_PER_PARTICLE * n if job.jitter_seed is not None else 0)
        return run, fp["tessellation"] + RESIDENT_BYTES_PER_PARTICLE * n

    def _need(self, job: Job) -> int:
        run, keep = self._footprint(job)
        return run + (0 if job.key in self._resident else keep)

    def _evict_for(self, need: int) -> bool:
        """Free least-recently-used idle grids until `need` fits."""
        while self._running_bytes + self._resident_bytes + need > self.budget:
            victim = next((k for k, r in self._resident.items() if r.users == 0), None)
            if victim is None:
                return False
            r = self._resident.pop(victim)
            r.dt.free()
            self._resident_bytes -= r.bytes
        return True

    def _upload(self, ctx, job: Job, stream, keep: int) -> Resident:
        torch = self._torch
        dev = ctx.device
        dt = ctx.upload(job.tess, stream=stream)
        x = torch.tensor(job.pos, dtype=torch.float64, device=dev)
        h = torch.tensor(job.h, dtype=torch.float64, device=dev)
        m = torch.tensor(job.m, dtype=torch.float64, device=dev)
        sigma = None
        if job.rho is not None:
            sigma = torch.tensor(job.jitter_frac * np.cbrt(job.m / job.rho), dtype=torch.float64, device=dev)
        job.host_bytes = (job.tess.generators.nbytes + job.tess.vertices.nbytes + job.tess.face_vtx.nbytes
                          + job.tess.face_vtx_off.nbytes + job.tess.cell_face_off.nbytes
                          + job.pos.nbytes + job.h.nbytes + job.m.nbytes + (job.rho.nbytes if job.rho is not None else 0))
        return Resident(dt, x, h, m, sigma, keep)

    def _positions(self, r: Resident, job: Job, stream):
        """The job's particle positions on the device: the resident ones, or
        for a repeat timestep the resident ones plus a seeded Gaussian jitter
        of 1% of the local spacing per component, clamped into the unit box."""
        torch = self._torch
        if job.jitter_seed is None:
            return r.x
        if r.sigma is None:
            raise ValueError("a repeat job needs the grid's densities (Job.rho) for its jitter scale")
        g = torch.Generator(device=r.x.device)
        g.manual_seed(int(job.jitter_seed))
        noise = torch.randn(r.x.shape, generator=g, dtype=torch.float64, device=r.x.device)
        return torch.clamp(torch.addcmul(r.x, noise, r.sigma[:, None]), 0.0, float(np.nextafter(1.0, 0.0)))

    def _worker(self, slot: int):
        torch = self._torch
        pkg = self._pkg
        ctx, stream = self._slots[slot]
        while True:
            with self._cv:
                while True:
                    if self._stop and not self._queue:
                        return
                    if self._queue:
                        head = self._queue[0]
                        need = self._need(head)
                        # first come first served: only the oldest job may start;
                        # a job larger than the budget runs alone
                        alone = self._running_bytes == 0
                        if self._evict_for(need) or alone:
                            job = self._queue.popleft()
                            break
                    self._cv.wait()
                run_bytes, keep_bytes = self._footprint(job)
                r = self._resident.pop(job.key, None)
                job.resident_hit = r is not None
                if r is not None:
                    r.users += 1
                    self._resident[job.key] = r  # most recently used
                else:
                    run_bytes += keep_bytes  # held as running until the grid is resident
                self._running_bytes += run_bytes
                job.start = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    if r is None:
                        mine = self._upload(ctx, job, stream, keep_bytes)
                        with self._cv:
                            other = self._resident.pop(job.key, None)
                            if other is not None:  # uploaded meanwhile by another slot
                                other.users += 1
                                self._resident[job.key] = other
                                r = other
                            else:
                                mine.users = 1
                                self._resident[job.key] = mine
                                self._resident_bytes += keep_bytes
                                r = mine
                            self._running_bytes -= keep_bytes
                            run_bytes -= keep_bytes
                        if r is not mine:
                            stream.synchronize()
                            mine.dt.free()
                    x = self._positions(r, job, stream)
                    res = pkg.map_particles_to_cells(ctx, r.dt, x, r.h, r.m, precision=self.precision,
                                                     keep_pairs=True, stream=stream)
                    q = torch.ones((job.tess.n_cells, self.k) if self.k > 1 else job.tess.n_cells,
                                   dtype=torch.float64, device=ctx.device)
                    pkg.map_cells_to_particles(ctx, res.pairs, q, stream=stream)
                    stream.synchronize()
                    job.n_pairs = res.pairs.n_pairs
                    job.mass, job.coverage = res.mass, res.coverage
                    res.pairs.free()
            except Exception as e:  # reported on the job
                job.error = f"{type(e).__name__}: {e}"
            job.end = time.perf_counter()
            with self._cv:
                self._running_bytes -= run_bytes
                if job.n_pairs:
                    self._pairs_seen[job.key] = job.n_pairs
                entry = self._resident.get(job.key)
                if entry is not None and r is entry:
                    entry.users = max(entry.users - 1, 0)
                self.completed.append(job)
                self._cv.notify_all()
            job.done.set()


def latency_summary(jobs: list[Job]) -> dict:
    lat = np.array([j.end - j.arrival for j in jobs])
    t0 = min(j.arrival for j in jobs)
    t1 = max(j.end for j in jobs)
    pairs = sum(j.n_pairs for j in jobs)
    return {"requests": len(jobs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "makespan_s": t1 - t0, "pairs": int(pairs), "pairs_per_s": pairs / (t1 - t0),
            "resident_hits": int(sum(j.resident_hit for j in jobs)),
            "repeat_jobs": int(sum(j.jitter_seed is not None for j in jobs)),
            "repeat_host_bytes": int(sum(j.host_bytes for j in jobs if j.jitter_seed is not None and j.resident_hit))}
