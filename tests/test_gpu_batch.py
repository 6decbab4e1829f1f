"""Batched replicas: every replica of a mixed batch (models, sizes, couplings
and schedules) must be bit-identical to the oracle and to the same replica
run alone, whatever the tile shape, with or without graph capture, and
whether the sweeps come in one run or several."""
import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads

pytestmark = pytest.mark.gpu


def mixed_replicas():
    reps = []
    sizes = [64, 128, 192, 256, 320]
    k = 0
    for model in (0, 1):
        for L in sizes:
            for Delta in ((0.0,) if model == 0 else (0.0, 0.6)):
                reps.append(dict(model=model, L=L, seed=workloads.seed_for(k), J=1.0 if k % 3 else 0.8,
                                 Delta=Delta, schedule=k % 3))
                k += 1
    return reps


def schedules(n_steps):
    tc = workloads.TC_ISING
    rows = [oracle.schedule(2, [2 * tc, 1.02 * tc, 8.0], 0, n_steps),
            oracle.schedule(1, [1.2, 5, 2.3], 0, n_steps),
            np.linspace(3.0, 0.5, n_steps)]
    T = np.stack(rows)
    if n_steps > 9:
        T[2, 4] = 0.0
        T[1, 9] = np.inf
    return T


def oracle_run(rep, T_row, n):
    s = oracle.init(rep["model"], rep["L"], rep["seed"])
    oracle.sweep(rep["model"], s, rep["seed"], rep["J"], rep["Delta"], 0, T_row[:n])
    return s


@pytest.mark.parametrize("flags", [0, 1 << 4, 2 << 4, 3 << 4, 4 << 4, 5 << 4, 1 | (3 << 4), 1 | (2 << 4)])
def test_batch_matches_oracle(gpu, flags):
    reps = mixed_replicas()
    n = 16
    T = schedules(n)
    b = gpu.Batch(reps, T).init_random()
    b.run(n, flags)
    b.sync()
    info = b.info()
    assert info["t"] == n and info["variant"] in range(gpu.BATCH_VARIANTS) and info["replicas"] == len(reps)
    for k, rep in enumerate(reps):
        assert np.array_equal(b.spins(k), oracle_run(rep, T[rep["schedule"]], n)), (k, rep)
    b.close()


def test_batch_chunks_and_solo_runs(gpu):
    reps = mixed_replicas()
    T = schedules(24)
    a = gpu.Batch(reps, T).init_random()
    a.run(24)
    c = gpu.Batch(reps, T).init_random()
    c.run(5)
    c.run(19, gpu.BATCH_DIRECT)
    a.sync()
    c.sync()
    for k, rep in enumerate(reps):
        solo = gpu.Lattice(rep["model"], rep["L"], rep["seed"], rep["J"], rep["Delta"]).init_random()
        solo.sweep(T[rep["schedule"]])
        want = solo.spins()
        assert np.array_equal(a.spins(k), want), k
        assert np.array_equal(c.spins(k), want), k
        ma, ms = a.measure(k, workloads.r_sparse(rep["L"])), solo.measure(workloads.r_sparse(rep["L"]))
        assert ma["bond"] == ms["bond"] and np.array_equal(ma["Sx"], ms["Sx"]) and ma["t"] == 24
        solo.close()
    with pytest.raises(gpu.SpinError):
        a.run(1)  # past the end of the schedule
    a.close()
    c.close()


def test_batch_rejects_bad_descriptors(gpu):
    reps = mixed_replicas()[:3]
    T = schedules(4)
    bad = [dict(r) for r in reps]
    bad[1]["schedule"] = 7
    with pytest.raises(gpu.SpinError):
        gpu.Batch(bad, T)
    T2 = T.copy()
    T2[0, 1] = -1.0
    with pytest.raises(gpu.SpinError):
        gpu.Batch(reps, T2)


def test_many_tiles_per_block_mixed_models(gpu):
    """Enough replicas that every block of the batched launch walks several
    tiles of different models and group counts (Ising, Blume-Capel at
    Delta = 0 and at Delta = 0.6).  Each wavefront's list storage must stay
    its own while neighbouring wavefronts are at other tiles: every forced
    strategy reproduces the solo runs."""
    reps = []
    for k in range(192):
        kind = k % 3
        reps.append(dict(model=0 if kind == 0 else 1, L=2048 if k % 2 else 1024, seed=workloads.seed_for(5000 + k),
                         J=1.0, Delta=0.6 if kind == 2 else 0.0, schedule=k % 3))
    n = 24
    T = schedules(n)
    T[0] = np.linspace(2.4, 2.2, n)   # keep every schedule finite and near the critical region
    T[1] = np.linspace(1.9, 1.6, n)
    T[2] = np.linspace(1.8, 1.5, n)
    want = []
    for rep in reps:
        solo = gpu.Lattice(rep["model"], rep["L"], rep["seed"], rep["J"], rep["Delta"]).init_random()
        solo.sweep(T[rep["schedule"]])
        want.append(solo.spins())
        solo.close()
    for v in (1, 2, 4, 5, 6, 7, 8):
        b = gpu.Batch(reps, T).init_random()
        b.run(n, gpu.BATCH_VARIANT(v))
        b.sync()
        bad = [k for k in range(len(reps)) if not np.array_equal(b.spins(k), want[k])]
        assert not bad, (v, bad[:10])
        b.close()


def test_batch_measure_all(gpu):
    """spin_batch_measure: every replica's integers equal its own spin_measure
    and, for a few replicas, the oracle's brute-force sums."""
    reps = mixed_replicas()
    T = schedules(12)
    b = gpu.Batch(reps, T).init_random()
    b.run(12)
    r = [1, 2, 3, 5, 8, 13, 21, 32, 63]
    got = b.measure_all(r)
    assert len(got) == len(reps)
    for k, rep in enumerate(reps):
        one = b.measure(k, r)
        for key in ("t", "sum_s", "sum_s2", "bond"):
            assert got[k][key] == one[key], (k, key)
        assert np.array_equal(got[k]["Sx"], one["Sx"]) and np.array_equal(got[k]["Sy"], one["Sy"])
        assert got[k]["t"] == 12
    for k in (0, len(reps) - 1):
        s = b.spins(k)
        want = oracle.measure(s, r)
        assert got[k]["bond"] == want["bond"] and np.array_equal(got[k]["Sx"], want["Sx"])
        assert np.array_equal(got[k]["Sy"], want["Sy"])
    with pytest.raises(gpu.SpinError):
        b.measure_all([64])  # not below L = 64 of the smallest replica
    b.close()


@pytest.mark.parametrize("model", [0, 1])
def test_single_model_batches(gpu, model):
    """A batch of one model runs the batched kernel specialised on that model
    (the Ising one keeps the single-lattice kernel's smaller LDS): every
    strategy reproduces the oracle."""
    reps = [rep for rep in mixed_replicas() if rep["model"] == model]
    n = 12
    T = schedules(n)
    want = [oracle_run(rep, T[rep["schedule"]], n) for rep in reps]
    for v in range(gpu.BATCH_VARIANTS):
        b = gpu.Batch(reps, T).init_random()
        b.run(n, gpu.BATCH_VARIANT(v))
        b.sync()
        for k in range(len(reps)):
            assert np.array_equal(b.spins(k), want[k]), (v, k)
        b.close()


def test_batch_measure_all_fast_kernels_and_reuse(gpu):
    """The sparse separation prefix takes the fast correlation kernels in the
    batched measurement too; a second call with fewer separations reuses the
    counter buffer (it must start from zero again)."""
    reps = mixed_replicas()
    T = schedules(8)
    b = gpu.Batch(reps, T).init_random()
    b.run(8)
    for r in (workloads.r_sparse(64), workloads.r_sparse(64)[:5], np.array([], dtype=np.uint32)):
        got = b.measure_all(r)
        for k in range(len(reps)):
            one = b.measure(k, r)
            assert got[k]["bond"] == one["bond"] and got[k]["sum_s"] == one["sum_s"]
            assert got[k]["xi"] == one["xi"] and got[k]["e"] == one["e"]
            assert np.array_equal(got[k]["Sx"], one["Sx"]) and np.array_equal(got[k]["Sy"], one["Sy"])
    b.close()


def test_batch_measure_all_large_rows(gpu):
    """The batched measurement launches (one per kernel kind for all
    replicas) on rows of whole 1024-word segments (L = 65536: the run-per-lane
    horizontal kernel) next to shorter rows, both models, with the sparse
    set up to r = 1024: every replica's sums equal its own spin_measure."""
    reps = [dict(model=m, L=L, seed=workloads.seed_for(7000 + 10 * m + k), J=1.0, Delta=0.0, schedule=m)
            for m in (0, 1) for k, L in enumerate((1 << 16, 4096, 2048))]
    n = 2
    T = np.stack([np.full(n, workloads.TC_ISING), np.full(n, workloads.TC_BC)])
    b = gpu.Batch(reps, T).init_random()
    b.run(n)
    r = workloads.r_sparse(2048)
    got = b.measure_all(r)
    for k in range(len(reps)):
        one = b.measure(k, r)
        for key in ("t", "sum_s", "sum_s2", "bond"):
            assert got[k][key] == one[key], (k, key)
        assert np.array_equal(got[k]["Sx"], one["Sx"]) and np.array_equal(got[k]["Sy"], one["Sy"]), k
    b.close()


def test_borrowed_handles_cannot_advance(gpu):
    """Only spin_batch_run advances a replica: sweeping, cluster-updating or
    re-timing a borrowed handle is refused, so no sweep index is reused."""
    reps = mixed_replicas()[:3]
    T = schedules(4)
    b = gpu.Batch(reps, T).init_random()
    b.run(2)
    h = b.replica(1)
    for call in (lambda: gpu.spin_sweep(h, [2.0]), lambda: gpu.spin_sw(h, [2.0]),
                 lambda: gpu.spin_set_t(h, 0)):
        with pytest.raises(gpu.SpinError) as ei:
            call()
        assert ei.value.code == -22
    assert gpu.spin_get_t(h) == 2
    b.run(2)
    s = b.spins(1)
    assert np.array_equal(s, oracle_run(reps[1], T[reps[1]["schedule"]], 4))
    b.close()


def test_graph_replays_match_direct_runs(gpu):
    """Runs of equal length replay one captured graph (its launches read the
    schedule step from the device counter).  Every replay, with eager work
    and synchronisations in between, must equal direct launches of the same
    steps, and the end state the oracle's."""
    reps = mixed_replicas()
    n, runs = 6, 4
    T = schedules(n * runs)
    g = gpu.Batch(reps, T).init_random()
    d = gpu.Batch(reps, T).init_random()
    for q in range(runs):
        g.run(n)
        d.run(n, gpu.BATCH_DIRECT | gpu.BATCH_VARIANT(g.info()["variant"]))
        g.measure_all([1, 2])  # eager kernels and a synchronisation between replays
        d.sync()
        for k in range(len(reps)):
            assert np.array_equal(g.spins(k), d.spins(k)), (q, k)
        assert g.info()["t"] == d.info()["t"] == n * (q + 1)
    for k, rep in enumerate(reps):
        assert np.array_equal(g.spins(k), oracle_run(rep, T[rep["schedule"]], n * runs)), k
    g.close()
    d.close()


def test_runs_of_any_length_replay_power_of_two_graphs(gpu):
    """A run of n sweeps replays the captured runs of 2^k sweeps (k <= 8)
    that n decomposes into, capturing only those not yet captured: runs of
    lengths 1, 3, 300 (256 + 32 + 8 + 4), 2 and 259 in a row, with eager
    measurements between them, equal direct launches of the same steps and,
    at the end, the oracle."""
    reps = [rep for rep in mixed_replicas() if rep["L"] <= 128]
    lengths = [1, 3, 300, 2, 259]
    total = sum(lengths)
    T = schedules(total)
    g = gpu.Batch(reps, T).init_random()
    d = gpu.Batch(reps, T).init_random()
    done = 0
    for n in lengths:
        g.run(n)
        d.run(n, gpu.BATCH_DIRECT | gpu.BATCH_VARIANT(g.info()["variant"]))
        g.measure_all([1, 2])
        d.sync()
        done += n
        for k in range(len(reps)):
            assert np.array_equal(g.spins(k), d.spins(k)), (n, k)
        assert g.info()["t"] == d.info()["t"] == done
    for k, rep in enumerate(reps):
        assert np.array_equal(g.spins(k), oracle_run(rep, T[rep["schedule"]], total)), k
    g.close()
    d.close()


def test_row_uniform_replicas_match_oracle(gpu):
    """Ising replicas whose rows are a multiple of 64 words (L = 4096) take
    the row-uniform Philox path of the batched kernel, next to Ising replicas
    whose rows are not (L = 192) and Blume-Capel replicas of both sizes in the
    same launch: every strategy gives the oracle's lattices."""
    reps = [dict(model=m, L=L, seed=workloads.seed_for(900 + 10 * m + k), J=1.0, Delta=0.0, schedule=m)
            for m in (0, 1) for k, L in enumerate((4096, 192))]
    n = 6
    T = np.stack([np.full(n, workloads.TC_ISING), np.full(n, workloads.TC_BC)])
    want = [oracle_run(rep, T[rep["schedule"]], n) for rep in reps]
    for v in range(gpu.BATCH_VARIANTS):
        b = gpu.Batch(reps, T).init_random()
        b.run(n, gpu.BATCH_VARIANT(v))
        b.sync()
        for k in range(len(reps)):
            assert np.array_equal(b.spins(k), want[k]), (v, k)
        b.close()
