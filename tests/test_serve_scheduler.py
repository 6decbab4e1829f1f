"""The serving scheduler's host logic on the CPU: the oracle stands in for
the device (lattices in host memory, one oracle sweep call per job and
epoch).  Checks admission by slots and memory budget, FIFO order, slot and
memory reuse, epoch lengths, completion of every job, and that each job's
result is its solo oracle run."""
import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads
from paper_2503_14688_amd.serve import Job, Server


class OracleBackend:
    def __init__(self):
        self.epoch_log = []

    def free_bytes(self):
        return 1 << 30

    def admit(self, job):
        job.state = oracle.init(job.model, job.L, job.seed)

    def epoch(self, jobs, n):
        self.epoch_log.append((n, sorted(j.id for j in jobs)))
        for j in jobs:
            oracle.sweep(j.model, j.state, j.seed, j.J, j.Delta, j.done, np.full(n, j.T))

    def finish(self, job, r, keep_spins):
        m = oracle.measure(job.state, r)
        job.result = m
        if keep_spins:
            job.spins = job.state.copy()
        job.state = None


def jobs(n=9):
    rng = np.random.default_rng(3)
    out = []
    for k in range(n):
        model = int(rng.integers(0, 2))
        L = int(rng.choice([64, 128]))
        out.append(Job(id=k, model=model, L=L, sweeps=int(rng.choice([8, 16, 24])),
                       seed=workloads.seed_for(k), T=2.2 if model == 0 else 1.7, arrival=0.0))
    return out


def test_slots_budget_and_results():
    be = OracleBackend()
    js = jobs()
    budget = 2 * 128 * 128 // 4  # room for two large BC lattices
    srv = Server(max_slots=3, mem_budget=budget, epoch=8, keep_spins=True, backend=be)
    stats = srv.run(js, realtime=False)
    assert stats["jobs"] == len(js)
    assert srv.peak_active <= 3 and srv.peak_bytes <= budget
    assert srv.bytes_in_use == 0 and not srv.active and not srv.queue
    # FIFO admission: admission order follows job order
    order = [j.id for j in sorted(srv.finished, key=lambda j: (j.admitted_at, j.id))]
    assert order == sorted(order)
    # every epoch length divides the remaining work of its jobs and is <= 8
    assert all(1 <= n <= 8 for n, _ in be.epoch_log)
    for j in js:
        s = oracle.init(j.model, j.L, j.seed)
        oracle.sweep(j.model, s, j.seed, 1.0, 0.0, 0, np.full(j.sweeps, j.T))
        assert np.array_equal(j.spins, s)
        assert j.result["bond"] == oracle.measure(s, [])["bond"]


def test_oversized_job_is_rejected_and_small_budget_queues():
    be = OracleBackend()
    srv = Server(max_slots=8, mem_budget=100, epoch=4, backend=be)
    with pytest.raises(MemoryError):
        srv.run([Job(id=0, model=0, L=64, sweeps=4, seed=1, T=2.0)], realtime=False)
    be = OracleBackend()
    one = 64 * 64 // 8
    srv = Server(max_slots=8, mem_budget=one, epoch=4, backend=be)
    js = [Job(id=k, model=0, L=64, sweeps=4, seed=k, T=2.0) for k in range(4)]
    srv.run(js, realtime=False)
    assert srv.peak_active == 1 and len(srv.finished) == 4
    assert [ids for _, ids in be.epoch_log] == [[0], [1], [2], [3]]
