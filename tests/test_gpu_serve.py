"""Continuous-batching server: a job's result is the same alone and in the
mix (bit-exact spins and integer sums), jobs that do not fit wait instead of
failing, and slots are reused."""
import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads

pytestmark = pytest.mark.gpu


def small_jobs(n=10):
    rng = np.random.default_rng(5)
    jobs = []
    for k in range(n):
        model = int(rng.integers(0, 2))
        jobs.append(dict(id=k, model=model, L=int(rng.choice([64, 128, 192, 256])),
                         sweeps=int(rng.choice([32, 64, 96, 160])), seed=workloads.seed_for(1000 + k),
                         T=workloads.TC_ISING if model == 0 else workloads.TC_BC, arrival=0.002 * k))
    return jobs


@pytest.mark.parametrize("max_slots,budget", [(3, None), (64, 40_000)])
def test_each_job_matches_its_solo_run(gpu, max_slots, budget):
    from paper_2503_14688_amd.serve import Job, Server
    specs = small_jobs()
    srv = Server(max_slots=max_slots, mem_budget=budget, epoch=32, keep_spins=True)
    stats = srv.run([Job(**d) for d in specs], realtime=True)
    assert stats["jobs"] == len(specs)
    assert stats["epochs"] > 3  # jobs joined and left at different epochs
    by_id = {j.id: j for j in srv.finished}
    for d in specs:
        j = by_id[d["id"]]
        solo = gpu.Lattice(d["model"], d["L"], d["seed"]).init_random()
        solo.sweep(np.full(d["sweeps"], d["T"]))
        assert np.array_equal(j.spins, solo.spins()), d
        m = solo.measure(workloads.r_sparse(d["L"]))
        assert j.result["bond"] == m["bond"] and j.result["sum_s"] == m["sum_s"]
        assert np.array_equal(j.result["Sx"], m["Sx"]) and np.array_equal(j.result["Sy"], m["Sy"])
        assert j.result["t"] == d["sweeps"]
        solo.close()
    # one job against the oracle as well
    d = specs[0]
    s = oracle.init(d["model"], d["L"], d["seed"])
    oracle.sweep(d["model"], s, d["seed"], 1.0, 0.0, 0, np.full(d["sweeps"], d["T"]))
    assert np.array_equal(by_id[0].spins, s)


def test_job_larger_than_budget_is_rejected(gpu):
    from paper_2503_14688_amd.serve import Job, Server
    srv = Server(max_slots=4, mem_budget=1000, epoch=16)
    with pytest.raises(MemoryError):
        srv.run([Job(id=0, model=0, L=256, sweeps=16, seed=1, T=2.0)])
