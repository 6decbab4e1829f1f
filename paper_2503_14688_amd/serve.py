"""Continuous-batching service for quench jobs (protocol 1 runs on demand).

A job asks for a T = infinity start of one lattice (model, L, seed, J, Delta)
followed by a number of sweeps at bath temperature T, and returns the final
measurement (energy, magnetisation, C(r) on the sparse separation set, xi).

Scheduling: jobs wait in a FIFO queue.  At every epoch boundary the server
admits queued jobs while a slot is free and the device-memory budget holds
the new lattice; admitted lattices stay resident in HBM until their job ends.
One epoch advances every active job by the same number of sweeps through one
spin_batch (one launch per half-sweep covers all active lattices, captured as
a HIP graph), so work of jobs that arrived at different times overlaps on the
device; the batch is kept across epochs until a job joins or leaves.  A finished job is measured, its lattice freed, and its slot reused
at the next boundary.  Each replica of an epoch continues its own random
stream (descriptor t0 = sweeps already done), so a job's result does not
depend on which other jobs shared its epochs.

The device work sits behind a small backend interface (GpuBackend here); the
scheduler itself is plain host logic.
"""
import time
from collections import deque

import numpy as np

from . import (BATCH_VARIANT, spin_batch_create, spin_batch_destroy, spin_batch_info, spin_batch_run, spin_create,
               spin_destroy, spin_get_spins, spin_init_random, spin_lattice_bytes, spin_measure,
               spin_replica_desc, spin_set_t)
from . import workloads


class Job:
    def __init__(self, id, model, L, sweeps, seed, T, J=1.0, Delta=0.0, arrival=0.0, **_):
        self.id, self.model, self.L, self.sweeps = id, model, L, sweeps
        self.seed, self.T, self.J, self.Delta = seed, T, J, Delta
        self.arrival = arrival
        self.bytes = spin_lattice_bytes(model, L)
        self.done = 0
        self.state = None  # backend-owned lattice state
        self.admitted_at = None
        self.finished_at = None
        self.result = None
        self.spins = None


class GpuBackend:
    """Lattices in torch device buffers, advanced by one spin_batch that lives
    as long as the set of active jobs does not change.

    The batch is created with a schedule that covers the shortest remaining
    job, so consecutive epochs of the same jobs replay its captured graphs
    without rebuilding anything; a job joining or leaving (or the schedule
    running out) makes the next epoch build a new batch whose replicas continue
    each job's stream (t0 = sweeps done).  The sweep strategy is tuned by the
    first batch and kept for the later ones."""

    def __init__(self, device="cuda", variant=None):
        import torch
        self.torch = torch
        self.variant = variant  # None: tuned by the first batch, then kept
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.batch = None
        self.members = None
        self.steps_left = 0
        self.batches_built = 0

    def free_bytes(self):
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return free

    def admit(self, job):
        with self.torch.cuda.stream(self.stream):
            buf = self.torch.empty(job.bytes, dtype=self.torch.uint8, device=self.device)
        h = spin_create(job.model, job.L, job.seed, job.J, job.Delta, buf.data_ptr(), job.bytes,
                        self.stream.cuda_stream)
        spin_init_random(h)
        job.state = (buf, h)

    def _release(self):
        if self.batch is not None:
            spin_batch_destroy(self.batch)  # waits for the batch's work
            self.batch = None
            self.members = None
            self.steps_left = 0

    def epoch(self, jobs, n):
        members = tuple(j.id for j in jobs)
        if self.batch is None or members != self.members or self.steps_left < n:
            self._release()
            steps = min(j.sweeps - j.done for j in jobs)
            temps = sorted({j.T for j in jobs})
            T = np.array([[tk] * steps for tk in temps], dtype=np.float64)
            descs = [spin_replica_desc(j.model, j.L, j.seed, j.J, j.Delta, j.state[0].data_ptr(), j.bytes,
                                       temps.index(j.T), j.done) for j in jobs]
            self.batch = spin_batch_create(descs, T, self.stream.cuda_stream)
            self.members = members
            self.steps_left = steps
            self.batches_built += 1
        spin_batch_run(self.batch, n, 0 if self.variant is None else BATCH_VARIANT(self.variant))
        if self.variant is None:
            self.variant = spin_batch_info(self.batch)["variant"]
        self.steps_left -= n

    def finish(self, job, r, keep_spins):
        if self.members is not None and job.id in self.members:
            self._release()
        buf, h = job.state
        spin_set_t(h, job.done)
        job.result = spin_measure(h, r)
        if keep_spins:
            job.spins = spin_get_spins(h, job.L)
        spin_destroy(h)
        job.state = None

    def close(self):
        self._release()


class Server:
    """Admission by slots and memory budget, epochs of continuous batching."""

    def __init__(self, max_slots=256, mem_budget=None, epoch=64, keep_spins=False, backend=None):
        self.backend = backend if backend is not None else GpuBackend()
        if mem_budget is None:
            mem_budget = int(0.8 * self.backend.free_bytes())
        self.max_slots = max_slots
        self.mem_budget = mem_budget
        self.epoch = epoch
        self.keep_spins = keep_spins
        self.queue = deque()
        self.active = []
        self.finished = []
        self.bytes_in_use = 0
        self.peak_bytes = 0
        self.peak_active = 0
        self.epochs = 0
        self.flips = 0

    def submit(self, job):
        self.queue.append(job)

    def _admit(self, now):
        while self.queue and len(self.active) < self.max_slots:
            job = self.queue[0]
            if self.bytes_in_use + job.bytes > self.mem_budget:
                if not self.active and job.bytes > self.mem_budget:
                    raise MemoryError(f"job {job.id} needs {job.bytes} bytes, budget is {self.mem_budget}")
                break  # FIFO: wait until memory frees up
            self.queue.popleft()
            self.backend.admit(job)
            job.admitted_at = now
            self.bytes_in_use += job.bytes
            self.active.append(job)
        self.peak_bytes = max(self.peak_bytes, self.bytes_in_use)
        self.peak_active = max(self.peak_active, len(self.active))

    def _run_epoch(self):
        n = min(self.epoch, min(j.sweeps - j.done for j in self.active))
        self.backend.epoch(self.active, n)
        for j in self.active:
            j.done += n
            self.flips += n * j.L * j.L
        self.epochs += 1

    def _retire(self, now, r_of):
        still = []
        for j in self.active:
            if j.done < j.sweeps:
                still.append(j)
                continue
            self.backend.finish(j, r_of(j.L), self.keep_spins)
            self.bytes_in_use -= j.bytes
            j.finished_at = now()
            self.finished.append(j)
        self.active = still

    def run(self, jobs, realtime=True, r_of=workloads.r_sparse):
        """Serve jobs (arrival times in seconds from start); returns stats.
        With realtime=False every job is queued at once in arrival order."""
        pending = sorted(jobs, key=lambda j: j.arrival)
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        k = 0
        while k < len(pending) or self.queue or self.active:
            tnow = now()
            while k < len(pending) and (pending[k].arrival <= tnow or not realtime):
                self.submit(pending[k])
                k += 1
            self._admit(tnow)
            if self.active:
                self._run_epoch()
                self._retire(now, r_of)
            elif k < len(pending):
                time.sleep(max(0.0, pending[k].arrival - now()))
        wall = now()
        if hasattr(self.backend, "close"):
            self.backend.close()  # the last batch's device tables
        lat = np.array([j.finished_at - j.arrival for j in self.finished])
        return {"jobs": len(self.finished), "wall_s": wall, "jobs_per_s": len(self.finished) / wall,
                "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
                "epochs": self.epochs, "flips_per_ns": self.flips / wall / 1e9,
                "peak_active": self.peak_active, "peak_bytes": self.peak_bytes,
                "batches_built": getattr(self.backend, "batches_built", None)}
