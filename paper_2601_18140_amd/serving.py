"""Continuous-batching request loop over the C interface.

Simulation jobs (design, instance count, cycle count) arrive over time.  A
job is admitted when its device footprint fits what is free: its batch's
device memory (plus its design's records if not yet loaded) within the
memory budget, and the LDS its kernels hold for a whole step (RESIDENT
batches whose state lives in LDS) within the device's LDS.  Admitted jobs
stay resident on the device and advance together, a chunk of cycles per
tick, through one rteaal_step_many call per tick, so work of different
designs overlaps on the GPU.  A tick enqueues its step first and admits
waiting jobs while the step runs (batch creation only enqueues its
initialisation); it then waits for the step's event, reads back the jobs
that finished, frees their batches, and the freed memory admits waiting
jobs during the next tick's step.  Latency is arrival -> results readable.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import rteaal as R


@dataclasses.dataclass
class Job:
    job_id: int
    design: int                 # index into the server's design pool
    n_inst: int
    n_cycles: int
    arrival: float = 0.0
    admitted: float | None = None
    finished: float | None = None
    done_cycles: int = 0
    batch: int | None = None
    footprint: int = 0
    lds: int = 0
    regs: np.ndarray | None = None   # packed register limbs [n_inst][words] once finished

    @property
    def seeds(self) -> np.ndarray:
        return (np.uint64(self.job_id) << np.uint64(16)) | np.arange(self.n_inst, dtype=np.uint64)


class Server:
    """pool: list of rtlgen.Design; budget_bytes: device memory the loop may use."""

    def __init__(self, ctx, pool, budget_bytes, tick_seconds=0.05, chunk_cycles=None,
                 max_chunk=4096, log=None, lds_budget_bytes=256 * 160 * 1024, preload=True):
        self.ctx = ctx
        self.pool = pool
        self.budget = int(budget_bytes)
        self.lds_budget = int(lds_budget_bytes)   # MI355X: 256 compute units x 160 KB
        self.used_lds = 0
        self.tick_seconds = tick_seconds
        self.fixed_chunk = chunk_cycles
        self.max_chunk = max_chunk
        self.loaded = {}                       # pool index -> design id
        self.design_bytes = {}                 # pool index -> bytes of its records
        self.users = collections.Counter()     # pool index -> resident jobs using it
        self.queue = collections.deque()
        self.running = []
        self.finished = []
        self.used = 0
        self.rate = {}                         # (design, n_inst) -> observed cycles/s per batch
        self.instance_cycles = 0
        self.log = log                         # optional callable(str) for admit/retire events
        self.gpu_busy_s = 0.0                  # time the steps kept the device busy
        if preload:                            # designs load before any job arrives
            for k in range(len(pool)):
                self._load(k)

    # ---- admission ---------------------------------------------------------
    def _design_bytes(self, k):
        d = self.pool[k]
        return 32 * (d.n_ops + d.n_regs + d.n_inputs + d.n_consts + 16) + 16 * (d.n_layers + 8)

    def _load(self, k):
        did = R.rteaal_load_design(self.ctx, self.pool[k])
        self.loaded[k] = did
        self.design_bytes[k] = self._design_bytes(k)
        self.used += self.design_bytes[k]
        return did

    def _footprint(self, job):
        """(device bytes, LDS bytes held for a whole step) of the job's batch."""
        did = self.loaded.get(job.design)
        if did is None:
            did = self._load(job.design)
        return R.rteaal_batch_resources(self.ctx, did, job.n_inst)

    def submit(self, job, now=None):
        job.arrival = time.perf_counter() if now is None else now
        self.queue.append(job)

    def _admit(self, now, idle):
        """Admits waiting jobs in arrival order while they fit; idle: no job
        is running or being stepped (an LDS demand above the device's is then
        admitted alone, its workgroups taking turns on the device)."""
        admitted = []
        while self.queue:
            job = self.queue[0]
            fp, lds = self._footprint(job)
            alone = idle and not admitted
            if self.used + fp > self.budget:
                if alone:
                    raise RuntimeError(f"job {job.job_id} needs {fp} bytes, budget {self.budget}")
                break
            if self.used_lds + lds > self.lds_budget and not alone:
                break
            self.queue.popleft()
            job.footprint, job.lds = fp, lds
            job.batch = R.rteaal_create_batch(self.ctx, self.loaded[job.design], job.seeds)
            job.admitted = now
            self.used += fp
            self.used_lds += lds
            self.users[job.design] += 1
            admitted.append(job)
            if self.log:
                self.log(f"admit job {job.job_id}: design {job.design}, {job.n_inst} instances, "
                         f"{job.n_cycles} cycles, {fp} bytes, {lds} LDS bytes")
        return admitted

    # ---- one tick ----------------------------------------------------------
    def _chunk(self, job):
        left = job.n_cycles - job.done_cycles
        if self.fixed_chunk:
            return min(left, self.fixed_chunk)
        r = self.rate.get((job.design, job.n_inst))
        c = int(self.tick_seconds * r) if r else 16
        return max(1, min(left, c, self.max_chunk))

    def _wait(self):
        """Waits for the work enqueued so far: by polling an event on the
        context's stream when it is a torch stream, else rteaal_sync."""
        stream = getattr(self.ctx, "stream", None)
        if stream is not None and hasattr(stream, "cuda_stream"):
            import torch
            ev = torch.cuda.Event()
            ev.record(stream)
            while not ev.query():
                time.sleep(0.0002)
        else:
            R.rteaal_sync(self.ctx)

    def tick(self):
        if not self.running:
            self.running += self._admit(time.perf_counter(), idle=True)
            if not self.running:
                return 0
        chunks = [self._chunk(j) for j in self.running]
        t0 = time.perf_counter()
        R.rteaal_step_many(self.ctx, [j.batch for j in self.running], chunks)
        # Admission while the step runs: the new batches' initialisation is
        # enqueued behind the step, and they join the next tick.
        new = self._admit(time.perf_counter(), idle=False)
        self._wait()
        dt = max(time.perf_counter() - t0, 1e-6)
        self.gpu_busy_s += dt
        done = []
        for j, c in zip(self.running, chunks):
            j.done_cycles += c
            self.instance_cycles += c * j.n_inst
            # all batches shared the tick: credit each with the tick's rate
            self.rate[(j.design, j.n_inst)] = c / dt
            if j.done_cycles >= j.n_cycles:
                done.append(j)
        for j in done:
            j.regs = R.rteaal_read_state(self.ctx, j.batch)
            R.rteaal_free_batch(self.ctx, j.batch)
            j.batch = None
            j.finished = time.perf_counter()
            self.used -= j.footprint
            self.used_lds -= j.lds
            self.users[j.design] -= 1
            self.running.remove(j)
            self.finished.append(j)
            if self.log:
                self.log(f"done job {j.job_id}: latency {j.finished - j.arrival:.2f} s, "
                         f"{len(self.finished)} finished, {len(self.queue)} queued")
        self.running += new
        return len(done)

    def drain(self):
        while self.running or self.queue:
            self.tick()

    def close(self):
        for j in self.running:
            R.rteaal_free_batch(self.ctx, j.batch)
        self.running = []
        for k, did in self.loaded.items():
            R.rteaal_unload_design(self.ctx, did)
        self.loaded = {}

    # ---- a timed run with arrivals -----------------------------------------
    def run(self, jobs, arrival_times, duration=None):
        """Replay `jobs` arriving at `arrival_times` (seconds from start); stop
        admitting at `duration` if given; drain; return summary statistics."""
        order = np.argsort(arrival_times)
        start = time.perf_counter()
        k = 0
        next_status = 15.0
        while k < len(order) or self.queue or self.running:
            now = time.perf_counter() - start
            if self.log and now >= next_status:
                self.log(f"t={now:.0f} s: {len(self.running)} running, {len(self.queue)} queued, "
                         f"{len(self.finished)} finished, {self.instance_cycles} instance-cycles")
                next_status += 15.0
            while k < len(order) and arrival_times[order[k]] <= now:
                if duration is None or arrival_times[order[k]] <= duration:
                    self.submit(jobs[order[k]], now=start + arrival_times[order[k]])
                k += 1
            if duration is not None and now > duration:
                k = len(order)   # the admission window has closed
            if not self.running and not self.queue:
                if k < len(order):
                    time.sleep(max(0.0, min(0.01, arrival_times[order[k]] - now)))
                continue
            self.tick()
        wall = time.perf_counter() - start
        return self.summary(wall)

    def summary(self, wall):
        lat = np.array([j.finished - j.arrival for j in self.finished]) if self.finished else np.zeros(0)
        return {
            "jobs": len(self.finished),
            "wall_s": wall,
            "instance_cycles": int(self.instance_cycles),
            "instance_cycles_per_s": self.instance_cycles / wall if wall > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "latency_max_s": float(lat.max()) if lat.size else None,
            "peak_budget_bytes": self.budget,
            "lds_budget_bytes": self.lds_budget,
            "waited_for_admission": int(sum(1 for j in self.finished if j.admitted > j.arrival + 0.5)),
        }


def poisson_arrivals(rate_per_s, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))
