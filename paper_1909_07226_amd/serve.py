"""Request loop for grid and degrid jobs on one GPU, with continuous batching.

Jobs arrive at any time (``Server.submit``).  The scheduler admits them in
arrival order as soon as a stream slot is free and the device memory they
need fits the budget; admitted jobs run concurrently on their own HIP streams,
so a small job does not wait behind a large one.  Large jobs (more than
``large_cost`` visibility x pixel products) are limited to ``large_slots`` at a
time, so concurrent large jobs do not slow each other down; a job that cannot
start yet is passed over by the jobs behind it that can.  Completion is
detected with HIP events.  Each job's result does not depend on what else is running: the
kernels are deterministic per job and share nothing writable.

Memory admission: a job needs its output (a grid or a visibility array) plus
the gridding scratch its plan may allocate; a job larger than the whole budget
is refused at submission.  A job that fails (bad arguments, library error)
fails only its own future.
"""

import collections
import threading
import time

from . import _lib


class Job:
    """One request: ``kind`` "grid" (visibilities -> new grid) or "degrid" (grid -> new visibilities).

    Inputs are device tensors that stay valid while the job runs (resident
    A-terms, taper and grids may be shared between jobs).  ``plan`` is an
    ``idg.Plan`` for the job's samples.
    """

    def __init__(self, kind, plan, uvw, freqs, aterms, taper, vis=None, grid=None, name=None):
        if kind not in ("grid", "degrid"):
            raise ValueError("kind must be 'grid' or 'degrid'")
        if kind == "grid" and vis is None:
            raise ValueError("a grid job needs visibilities")
        if kind == "degrid" and grid is None:
            raise ValueError("a degrid job needs a grid")
        self.kind, self.plan, self.name = kind, plan, name
        self.uvw, self.freqs, self.aterms, self.taper, self.vis, self.grid = uvw, freqs, aterms, taper, vis, grid
        sh = plan.shapes()
        n_out = 1
        for d in (sh["grid"] if kind == "grid" else sh["vis"]):
            n_out *= d
        self.out_bytes = 8 * n_out
        scratch = plan.params.scratch_bytes if plan.params.scratch_bytes > 0 else 2 << 30
        self.mem_bytes = self.out_bytes + (scratch if kind == "grid" else 0) + (1 << 20)
        self.cost = float(plan.stats()["nr_gridded"]) * plan.subgrid_size ** 2   # visibility x pixel products

    def launch(self, stream):
        """Queue the job on `stream`; returns the output tensor (valid once the stream reaches it)."""
        import torch
        sh = self.plan.shapes()
        with torch.cuda.stream(stream):
            if self.kind == "grid":
                out = torch.zeros(sh["grid"], dtype=torch.complex64, device=self.uvw.device)
                _lib.grid(self.plan, self.uvw, self.freqs, self.vis, self.aterms, self.taper, out, stream)
            else:
                out = torch.empty(sh["vis"], dtype=torch.complex64, device=self.uvw.device)
                _lib.degrid(self.plan, self.uvw, self.freqs, self.grid, self.aterms, self.taper, out, stream)
        return out


class JobFuture:
    def __init__(self, job, arrival):
        self.job = job
        self.arrival = arrival
        self.start = None
        self.finish = None
        self._done = threading.Event()
        self._result = None
        self._error = None

    def done(self):
        return self._done.is_set()

    def result(self, timeout=None):
        if not self._done.wait(timeout):
            raise TimeoutError("job not finished")
        if self._error is not None:
            raise self._error
        return self._result

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival

    def _set(self, result=None, error=None):
        self.finish = time.perf_counter()
        self._result, self._error = result, error
        self._done.set()


class Server:
    """Continuous-batching scheduler: `slots` concurrent jobs (one HIP stream each), `mem_budget` bytes."""

    def __init__(self, slots=4, mem_budget=None, device=None, poll_s=50e-6, large_slots=1, large_cost=4e9,
                 keep_results=True):
        import torch
        self.device = torch.device("cuda" if device is None else device)
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            mem_budget = int(free * 0.6)
        self.mem_budget = int(mem_budget)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.mem_in_use = 0
        self.large_slots, self.large_cost = large_slots, large_cost
        self.large_in_use = 0
        self.poll_s = poll_s
        self.keep_results = keep_results   # False: a finished job's output is dropped (latency measurements)
        self._queue = collections.deque()
        self._inflight = []
        self._cv = threading.Condition()
        self._stop = False
        self.completed = []
        self._thread = threading.Thread(target=self._loop, name="idg-serve", daemon=True)
        self._thread.start()

    def submit(self, job, arrival=None):
        fut = JobFuture(job, time.perf_counter() if arrival is None else arrival)
        if job.mem_bytes > self.mem_budget:
            fut._set(error=MemoryError(f"job needs {job.mem_bytes} bytes, budget is {self.mem_budget}"))
            return fut
        with self._cv:
            self._queue.append(fut)
            self._cv.notify()
        return fut

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify()
        self._thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # scheduler thread
    def _admit(self):
        import torch
        started = False
        i = 0
        while i < len(self._queue) and self.free_slots:
            fut = self._queue[i]
            job = fut.job
            large = job.cost >= self.large_cost
            if self.mem_in_use + job.mem_bytes > self.mem_budget or (large and self.large_in_use >= self.large_slots):
                i += 1          # cannot start yet: let the jobs behind it try
                continue
            del self._queue[i]
            slot = self.free_slots.pop(0)
            stream = self.streams[slot]
            fut.start = time.perf_counter()
            try:
                out = job.launch(stream)
                ev = torch.cuda.Event()
                ev.record(stream)
            except Exception as e:  # noqa: BLE001 - a failing job fails its own future only
                self.free_slots.append(slot)
                fut._set(error=e)
                continue
            self.mem_in_use += job.mem_bytes
            self.large_in_use += int(large)
            self._inflight.append((fut, slot, ev, out))
            started = True
        return started

    def _reap(self):
        done = [x for x in self._inflight if x[2].query()]
        for item in done:
            fut, slot, ev, out = item
            self._inflight.remove(item)
            self.free_slots.append(slot)
            self.mem_in_use -= fut.job.mem_bytes
            self.large_in_use -= int(fut.job.cost >= self.large_cost)
            fut._set(result=out if self.keep_results else None)
            self.completed.append(fut)
        return bool(done)

    def _loop(self):
        while True:
            with self._cv:
                if self._stop and not self._queue and not self._inflight:
                    return
                progressed = self._admit()
            progressed = self._reap() or progressed
            if not progressed:
                with self._cv:
                    self._cv.wait(self.poll_s)


def latency_summary(futures):
    """p50 / p99 / mean latency (ms) and throughput over finished futures."""
    import numpy as np
    lat = np.array([f.latency for f in futures if f.latency is not None and f._error is None])
    if lat.size == 0:
        return {}
    span = max(f.finish for f in futures) - min(f.arrival for f in futures)
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3), "jobs": int(lat.size),
            "jobs_per_s": round(lat.size / span, 2)}


def jobs_from_trace(trace, datasets, device_data, model_grids, scratch_bytes=512 << 20):
    """Build the jobs of a request trace (``synth.serving_trace``).

    datasets:     class -> workload with host arrays (geometry for planning)
    device_data:  class -> dict of device tensors uvw, freqs, vis, aterms, taper (resident)
    model_grids:  class -> device grid that degrid jobs predict from (resident)
    Each distinct (class, window) gets one plan and one device copy of its
    visibilities and uvw; A-terms and taper are views of the resident arrays.
    Returns (jobs, templates).
    """
    import numpy as np
    from ._lib import Plan

    templates = {}
    jobs = []
    for i in range(len(trace["arrivals"])):
        cls, wid, kind = str(trace["classes"][i]), int(trace["window_ids"][i]), str(trace["kinds"][i])
        key = (cls, wid)
        if key not in templates:
            wl, dd = datasets[cls], device_data[cls]
            w = trace["windows"][cls][wid]
            t0, nt, c0, nch = w["t0"], w["nt"], w["c0"], w["nch"]
            uvw = np.ascontiguousarray(wl.uvw[:, t0:t0 + nt])
            freqs = np.ascontiguousarray(wl.freqs[c0:c0 + nch])
            s0 = t0 // wl.aterm_timesteps
            ns = -(-nt // wl.aterm_timesteps)
            plan = Plan(wl.grid_size, wl.image_size, wl.subgrid_size, wl.kernel_size, wl.max_timesteps,
                        wl.aterm_timesteps, wl.nr_stations, wl.baselines, uvw, freqs, scratch_bytes=scratch_bytes)
            templates[key] = dict(
                plan=plan,
                uvw=dd["uvw"][:, t0:t0 + nt].contiguous(),
                freqs=dd["freqs"][c0:c0 + nch].contiguous(),
                vis=dd["vis"][:, t0:t0 + nt, c0:c0 + nch].contiguous(),
                aterms=dd["aterms"][s0:s0 + ns],
                taper=dd["taper"])
        t = templates[key]
        jobs.append(Job(kind, t["plan"], t["uvw"], t["freqs"], t["aterms"], t["taper"],
                        vis=t["vis"] if kind == "grid" else None,
                        grid=model_grids[cls] if kind == "degrid" else None, name=f"{cls}/{wid}/{kind}"))
    return jobs, templates


def replay(server, jobs, arrivals):
    """Submit jobs at their arrival times (seconds from now); wait for all; return the futures."""
    t0 = time.perf_counter()
    futs = []
    for job, at in zip(jobs, arrivals):
        target = t0 + float(at)
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 1e-3))
        futs.append(server.submit(job, arrival=target))
    for f in futs:
        try:
            f.result(timeout=600)
        except Exception:  # noqa: BLE001 - recorded on the future
            pass
    return futs
