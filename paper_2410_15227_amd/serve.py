"""Served mapping: continuous batching of mapping jobs on one GPU.

Jobs (a tessellation plus a particle set) arrive at any time.  A job is
admitted first-come first-served as soon as a slot is free and its estimated
device footprint fits in the memory budget next to the jobs already running;
each slot owns a library context and a HIP stream, so admitted jobs overlap
on the device while later arrivals wait.  Tessellations stay resident on the
device between jobs (a repeated timestep maps new particle positions onto a
grid that is already there) and are evicted least-recently-used when the
budget needs their memory.

Every step of a job runs in the library's kernels; this module only
schedules.  A job's results do not depend on what runs beside it: each
weight is a function of its own pair and each cell sum has a fixed order.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

@dataclass
class Job:
    key: str                 # identity of the tessellation
    tess: object             # host Tessellation (uploaded when not resident)
    pos: np.ndarray
    h: np.ndarray
    m: np.ndarray
    arrival: float = 0.0     # time.perf_counter() at submission
    # filled in by the server
    start: float = 0.0
    end: float = 0.0
    n_pairs: int = 0
    resident_hit: bool = False
    mass: object = None      # device tensor of cell masses
    coverage: object = None  # device tensor of particle coverages
    error: str | None = None
    done: threading.Event = field(default_factory=threading.Event)


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
        self._resident: collections.OrderedDict[str, tuple] = collections.OrderedDict()  # key -> (dt, bytes, users)
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
        """Device bytes admission reserves for `job` (its grid counted
        unless resident)."""
        with self._cv:
            fp = self._footprint(job)
        return fp["workspace"] + fp["pairs"] + (0 if resident else fp["tessellation"])

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
            for dt, _, _ in self._resident.values():
                dt.free()
            self._resident.clear()
        for ctx, _ in self._slots:
            ctx.close()
        self._est_ctx.close()

    # ----------------------------------------------------------- scheduling
    def _footprint(self, job: Job) -> dict:
        # the library's model; a grid seen before lends its last pair count
        return self._est_ctx.estimate_footprint(len(job.m), job.tess, self._pairs_seen.get(job.key, 0))

    def _need(self, job: Job) -> int:
        fp = self._footprint(job)
        need = fp["workspace"] + fp["pairs"]
        if job.key not in self._resident:
            need += fp["tessellation"]
        return need

    def _evict_for(self, need: int) -> bool:
        """Free least-recently-used idle tessellations until `need` fits."""
        while self._running_bytes + self._resident_bytes + need > self.budget:
            victim = next((k for k, (_, _, users) in self._resident.items() if users == 0), None)
            if victim is None:
                return False
            dt, b, _ = self._resident.pop(victim)
            dt.free()
            self._resident_bytes -= b
        return True

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
                job.resident_hit = job.key in self._resident
                fp = self._footprint(job)
                if job.resident_hit:
                    dt, b, users = self._resident.pop(job.key)
                    self._resident[job.key] = (dt, b, users + 1)  # most recently used
                    run_bytes = fp["workspace"] + fp["pairs"]
                else:
                    dt = None
                    run_bytes = need
                self._running_bytes += run_bytes
                job.start = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    if dt is None:
                        dt = ctx.upload(job.tess, stream=stream)
                        with self._cv:
                            if job.key in self._resident:  # uploaded meanwhile by another slot
                                other, b, users = self._resident.pop(job.key)
                                self._resident[job.key] = (other, b, users + 1)
                                mine, dt = dt, other
                                stream.synchronize()
                                mine.free()
                            else:
                                tb = fp["tessellation"]
                                self._resident[job.key] = (dt, tb, 1)
                                self._resident_bytes += tb
                                self._running_bytes -= tb
                                run_bytes -= tb
                    dev = ctx.device
                    x = torch.tensor(job.pos, dtype=torch.float64, device=dev)
                    h = torch.tensor(job.h, dtype=torch.float64, device=dev)
                    m = torch.tensor(job.m, dtype=torch.float64, device=dev)
                    res = pkg.map_particles_to_cells(ctx, dt, x, h, m, precision=self.precision, keep_pairs=True,
                                                     stream=stream)
                    q = torch.ones((job.tess.n_cells, self.k) if self.k > 1 else job.tess.n_cells,
                                   dtype=torch.float64, device=dev)
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
                dt_entry = self._resident.get(job.key)
                if dt_entry is not None:
                    d, b, users = dt_entry
                    self._resident[job.key] = (d, b, max(users - 1, 0))
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
            "resident_hits": int(sum(j.resident_hit for j in jobs))}
