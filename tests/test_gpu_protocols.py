"""The thermal-protocol drivers on the GPU against the same drivers over the
CPU oracle: identical integer sums at every measurement, the same switch
times, and batched two-step runs identical to solo ones."""
import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import protocols, workloads

from test_protocols import OracleLattice

pytestmark = pytest.mark.gpu

REL = 1e-12


def same(got, want):
    assert [m["t"] for m in got] == [m["t"] for m in want]
    for a, b in zip(got, want):
        for k in ("e", "m", "xi"):
            assert abs(a[k] - b[k]) <= REL * max(1.0, abs(b[k])), (a["t"], k)


@pytest.mark.parametrize("model,T1,T2,L", [(0, 1.66, 2.2741, 128), (1, 1.24, 1.6966, 192)])
def test_two_step_series_matches_oracle(gpu, model, T1, T2, L):
    seed, t_switch = workloads.seed_for(300 + L), 37
    r = workloads.r_sparse(L)
    times = protocols.log_times(96, 4)
    lat = gpu.Lattice(model, L, seed).init_random()
    got = protocols.two_step_series(lat, T1, T2, t_switch, times, r, full=True)
    ref = OracleLattice(model, L, seed)
    want = protocols.two_step_series(ref, T1, T2, t_switch, times, r, full=True)
    for a, b in zip(got, want):
        assert a["t"] == b["t"] and a["bond"] == b["bond"] and a["sum_s"] == b["sum_s"]
        assert np.array_equal(a["Sx"], b["Sx"]) and np.array_equal(a["Sy"], b["Sy"])
    same(got, want)
    assert np.array_equal(lat.spins(), ref.s)
    lat.close()


def test_switch_times_match_oracle(gpu):
    L, seed = 256, workloads.seed_for(17)
    r = workloads.r_sparse(L)
    fs, xi_eq = (0.4, 0.6, 0.8), 15.0
    lat = gpu.Lattice(0, L, seed).init_random()
    t_gpu, c_gpu = protocols.switch_times(lat, 1.66, fs, xi_eq, r, t_limit=1024, per_octave=4)
    ref = OracleLattice(0, L, seed)
    t_cpu, c_cpu = protocols.switch_times(ref, 1.66, fs, xi_eq, r, t_limit=1024, per_octave=4)
    same(c_gpu, c_cpu)
    # the xi series are identical, so the crossings must be the same sweep
    for f in fs:
        assert t_gpu[f] is not None and t_gpu[f] == t_cpu[f], f
    lat.close()


def test_two_step_batch_matches_solo_runs(gpu):
    """One batch of replicas with different switch times (two share the seed,
    so they follow one trajectory up to the earlier switch) equals solo runs."""
    model, L, T1, T2 = 0, 256, 1.66, 2.27414861561203
    seeds = [workloads.seed_for(40), workloads.seed_for(40), workloads.seed_for(41)]
    t_switches = [13, 29, 29]
    r = workloads.r_sparse(L)
    times = protocols.log_times(80, 2)
    runs = protocols.two_step_batch(model, L, seeds, T1, T2, t_switches, times, r)
    assert len(runs) == 3
    for k in range(3):
        lat = gpu.Lattice(model, L, seeds[k]).init_random()
        solo = protocols.two_step_series(lat, T1, T2, t_switches[k], times, r)
        same(runs[k], solo)
        lat.close()
    # the shared prefix: identical until the first switch, apart after it
    assert runs[0][0]["e"] == runs[1][0]["e"]
    assert all(a["e"] == b["e"] for a, b in zip(runs[0], runs[1]) if a["t"] <= 13)
    assert any(a["e"] != b["e"] for a, b in zip(runs[0], runs[1]) if a["t"] > 13)
    with pytest.raises(ValueError):
        protocols.two_step_batch(model, L, seeds[:2], T1, T2, t_switches, times, r)


def test_quench_batch_matches_solo_runs(gpu):
    """The ensemble driver's per-replica sums equal solo runs of each seed,
    and the ensemble analysis runs on them."""
    from paper_2503_14688_amd import analysis
    L, T = 128, workloads.TC_ISING
    seeds = [workloads.seed_for(60 + k) for k in range(4)]
    r = workloads.r_sparse(L)
    times = [1, 2, 4, 8, 16, 32]
    data = protocols.quench_batch(0, L, seeds, T, times, r)
    assert [d["t"] for d in data] == times
    for k, s in enumerate(seeds):
        lat = gpu.Lattice(0, L, s).init_random()
        for d in data:
            lat.sweep(np.full(d["t"] - lat.t, T))
            m = lat.measure(r)
            assert np.array_equal(d["Sx"][k], m["Sx"]) and np.array_equal(d["Sy"][k], m["Sy"])
            assert d["sum_s2"][k] == m["sum_s2"] and d["e"][k] == m["e"]
        lat.close()
    C = (data[-1]["Sx"] + data[-1]["Sy"]) / (2.0 * L * L)
    xi, err, full, blocks = analysis.xi_ensemble(r, C, data[-1]["sum_s2"] / (L * L))
    assert xi > 0 and err >= 0 and blocks.shape == (4,)
