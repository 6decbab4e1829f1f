"""Parity of the equilibrium kernels (paper App. B) with the CPU oracle,
through the C ABI: the Swendsen-Wang step restricted to s = +-1 and the
paper's elementary Monte Carlo step (Metropolis sweeps, then one
Swendsen-Wang step) give the oracle's configurations bit for bit; the row and
column sums are exact and the Fourier moments M(k_min) agree with the oracle's
plain double sum to rounding (1e-12 of L^2, the size of the largest term sum)."""
import math

import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads

pytestmark = pytest.mark.gpu

TC = {0: workloads.TC_ISING, 1: workloads.TC_BC}


def check_fourier(gpu, lat, s):
    L = s.shape[0]
    f = lat.fourier()
    assert np.array_equal(f["row"], s.sum(axis=1, dtype=np.int64))
    assert np.array_equal(f["col"], s.sum(axis=0, dtype=np.int64))
    want = oracle.fourier(s)
    sums = oracle.measure(s, [])
    assert f["sum_s"] == sums["sum_s"] == int(want["M0"])
    assert f["sum_s2"] == sums["sum_s2"] and f["bond"] == sums["bond"]
    tol = 1e-12 * L * L
    assert abs(f["k1"] - want["k1"]) <= tol and abs(f["k2"] - want["k2"]) <= tol


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("L", [64, 320])
@pytest.mark.parametrize("T", ["tc", 1.0, 5.0, 0.0, math.inf])
def test_swendsen_wang_step_matches_oracle(gpu, model, L, T):
    T = TC[model] if T == "tc" else T
    seed = 31 + L + model
    lat = gpu.Lattice(model, L, seed).init_random()
    s = oracle.init(model, L, seed)
    pre = np.full(3, TC[model])
    lat.sweep(pre)
    oracle.sweep(model, s, seed, 1.0, 0.0, 0, pre)
    for k in range(3):
        lat.sw([T])
        oracle.sw(model, s, seed, 1.0, 3 + k, [T])
        assert np.array_equal(lat.spins(), s), k
    assert lat.t == 6
    check_fourier(gpu, lat, s)
    lat.close()


@pytest.mark.parametrize("model,L", [(1, 256), (0, 256), (1, 1024)])
def test_elementary_monte_carlo_steps_match_oracle(gpu, model, L):
    """The paper's EMCS: 10 Metropolis sweeps, then one Swendsen-Wang step."""
    T = TC[model]
    seed = 4000 + L + model
    lat = gpu.Lattice(model, L, seed).init_random()
    s = oracle.init(model, L, seed)
    ten = np.full(10, T)
    t = 0
    for k in range(3):
        lat.sweep(ten)
        oracle.sweep(model, s, seed, 1.0, 0.0, t, ten)
        lat.sw([T])
        oracle.sw(model, s, seed, 1.0, t + 10, [T])
        t += 11
        assert np.array_equal(lat.spins(), s), k
        check_fourier(gpu, lat, s)
    lat.close()


def test_blume_capel_with_crystal_field(gpu):
    """Delta != 0 enters only the Metropolis sweeps; the cluster step keeps s^2."""
    L, seed, T, Delta = 128, 808, 1.4, 0.7
    lat = gpu.Lattice(1, L, seed, 1.0, Delta).init_random()
    s = oracle.init(1, L, seed)
    for k in range(4):
        lat.sweep([T, T])
        oracle.sweep(1, s, seed, 1.0, Delta, 3 * k, [T, T])
        before = s.copy()
        lat.sw([T])
        oracle.sw(1, s, seed, 1.0, 3 * k + 2, [T])
        assert np.array_equal(before != 0, s != 0)
        assert np.array_equal(lat.spins(), s)
    f = lat.fourier()
    want = oracle.derive(L, 1.0, Delta, oracle.measure(s, []), [])
    assert abs(f["e"] - want["e"]) <= 1e-12 * max(1.0, abs(want["e"]))
    lat.close()


def test_swendsen_wang_arguments(gpu):
    import torch
    lat = gpu.Lattice(0, 64, 1).init_random()
    with pytest.raises(gpu.SpinError):
        lat.sw([-1.0])
    with pytest.raises(gpu.SpinError):
        lat.sw([float("nan")])
    assert lat.t == 0
    lat.close()
    big = 32768 + 64  # beyond the 32-bit cluster forest
    buf = torch.empty(gpu.spin_lattice_bytes(0, big), dtype=torch.uint8, device="cuda")
    h = gpu.spin_create(0, big, 1, 1.0, 0.0, buf.data_ptr(), buf.numel(), 0)
    with pytest.raises(gpu.SpinError) as ei:
        gpu.spin_sw(h, [2.0])
    assert ei.value.code == -22
    gpu.spin_destroy(h)


def test_batched_elementary_steps_match_oracle_and_solo_runs(gpu):
    """spin_batch_sw and spin_batch_measure_fourier: a batch of both models
    and three sizes, with per-replica schedules and couplings, alternating
    runs of Metropolis sweeps with batched Swendsen-Wang steps, gives every
    replica the oracle's configuration after each step and the Fourier
    moments of its own spin_measure_fourier; equilibrium.emcs_batch gives the
    samples of emcs_run on the same lattices alone."""
    from paper_2503_14688_amd import equilibrium
    reps = [dict(model=m, L=L, seed=5100 + 10 * m + L, J=J, Delta=0.0, schedule=m)
            for m, L, J in ((0, 64, 1.0), (1, 128, 1.2), (1, 320, 1.0), (0, 192, 0.9))]
    n_metropolis, n_steps = 3, 4
    total = n_steps * (n_metropolis + 1)
    T = np.stack([np.linspace(3.0, TC[0], total), np.full(total, TC[1])])
    b = gpu.Batch(reps, T).init_random()
    states = [oracle.init(r["model"], r["L"], r["seed"]) for r in reps]
    t = 0
    for k in range(n_steps):
        b.run(n_metropolis)
        b.sw()
        for r, s in zip(reps, states):
            Tr = T[r["schedule"]]
            oracle.sweep(r["model"], s, r["seed"], r["J"], 0.0, t, Tr[t:t + n_metropolis])
            oracle.sw(r["model"], s, r["seed"], r["J"], t + n_metropolis, Tr[t + n_metropolis:t + n_metropolis + 1])
        t += n_metropolis + 1
        got = b.fourier_all()
        for q, (r, s) in enumerate(zip(reps, states)):
            assert np.array_equal(b.spins(q), s), (k, q)
            one = gpu.spin_measure_fourier(b.replica(q), r["L"])
            for key in ("t", "sum_s", "sum_s2", "bond", "e", "k1", "k2"):
                assert got[q][key] == one[key], (k, q, key)
            assert got[q]["t"] == t
    with pytest.raises(gpu.SpinError):
        b.sw()  # the schedule is used up
    b.close()
    seeds = [7001, 7002, 7003]
    batched = equilibrium.emcs_batch(1, 64, seeds, TC[1], 6, every=2, n_therm=2, n_metropolis=4)
    for seed, got in zip(seeds, batched):
        lat = gpu.Lattice(1, 64, seed).init_random()
        want = equilibrium.emcs_run(lat, TC[1], 6, every=2, n_therm=2, n_metropolis=4)
        lat.close()
        for key in ("H", "M0", "Mk2"):
            assert np.array_equal(got[key], want[key]), (seed, key)
