"""Exact (non-statistical) pins of the oracle.

* Z2: the Ising dynamics commutes with a global flip (dE is flip-invariant
  and the stream does not depend on the state), so a run from -s0 is -s(t).
* T = +inf: every Ising move is accepted, so each sweep negates the lattice.
* T = 0: no move with dE > 0 is accepted, so the energy never increases.
* Bookkeeping: the energy change of a half-sweep equals the summed dE of its
  accepted moves (sites of one colour are independent), which ties the dE of
  the sweep to the Hamiltonian evaluated by the measurement.
* Correlation sums against patterns whose C(r) is known in closed form, and
  the symmetries S(0) = sum s^2, S(r) = S(L - r), Sx(s) = Sy(s transposed).
* xi = I2 / I1 against the closed form of the trapezoid sums of e^(-r/a).
* The light-cone window evolution equals the full-lattice run inside.
* Initial-state statistics (fair coin for Ising, thirds for Blume-Capel).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))


def energy(s, J, Delta):
    m = oracle.measure(s, [])
    return -J * m["bond"] + Delta * m["sum_s2"]


def test_ising_z2_flip_symmetry_bit_exact():
    L, seed = 32, 42
    s = oracle.init(oracle.ISING, L, seed)
    sf = (-s).astype(np.int8)
    T = np.full(20, TC_ISING)
    oracle.sweep(oracle.ISING, s, seed, 1.0, 0.0, 0, T)
    oracle.sweep(oracle.ISING, sf, seed, 1.0, 0.0, 0, T)
    assert np.array_equal(sf, -s)
    r = np.arange(1, 17)
    a, b = oracle.measure(s, r), oracle.measure(sf, r)
    assert a["bond"] == b["bond"] and a["sum_s"] == -b["sum_s"]
    assert np.array_equal(a["Sx"], b["Sx"]) and np.array_equal(a["Sy"], b["Sy"])


def test_ising_infinite_temperature_negates():
    L, seed = 16, 3
    s = oracle.init(oracle.ISING, L, seed)
    s0 = s.copy()
    oracle.sweep(oracle.ISING, s, seed, 1.0, 0.0, 0, np.array([np.inf]))
    assert np.array_equal(s, -s0)
    oracle.sweep(oracle.ISING, s, seed, 1.0, 0.0, 1, np.array([np.inf, np.inf]))
    assert np.array_equal(s, -s0)


@pytest.mark.parametrize("model,Delta", [(oracle.ISING, 0.0), (oracle.BLUME_CAPEL, 0.0),
                                         (oracle.BLUME_CAPEL, 0.5)])
def test_zero_temperature_energy_never_increases(model, Delta):
    L, seed = 32, 9
    s = oracle.init(model, L, seed)
    e_prev = energy(s, 1.0, Delta)
    for t in range(30):
        oracle.sweep(model, s, seed, 1.0, Delta, t, np.array([0.0]))
        e = energy(s, 1.0, Delta)
        assert e <= e_prev
        e_prev = e


@pytest.mark.parametrize("model,J,Delta", [(oracle.ISING, 1.0, 0.0), (oracle.ISING, 0.7, 0.0),
                                           (oracle.BLUME_CAPEL, 1.0, 0.0),
                                           (oracle.BLUME_CAPEL, 1.3, 0.45),
                                           (oracle.BLUME_CAPEL, 1.0, -0.6)])
def test_energy_bookkeeping_per_half_sweep(model, J, Delta):
    L, seed = 24, 77
    s = oracle.init(model, L, seed)
    Ts = np.array([1.2, 2.0, 3.5, 1.69, 0.9, 5.0])
    e0 = energy(s, J, Delta)
    dE = oracle.sweep(model, s, seed, J, Delta, 0, Ts, with_dE=True)
    e1 = energy(s, J, Delta)
    assert abs((e1 - e0) - dE.sum()) < 1e-9
    # half-sweep by half-sweep via one sweep at a time
    s = oracle.init(model, L, seed)
    e = energy(s, J, Delta)
    for k, T in enumerate(Ts):
        d = oracle.sweep(model, s, seed, J, Delta, k, np.array([T]), with_dE=True)
        e_new = energy(s, J, Delta)
        assert abs((e_new - e) - d.sum()) < 1e-9
        e = e_new


def test_correlation_sums_closed_forms():
    L = 16
    r = np.arange(0, L, dtype=np.uint32)
    N = L * L
    up = np.ones((L, L), dtype=np.int8)
    m = oracle.measure(up, r)
    assert np.all(m["Sx"] == N) and np.all(m["Sy"] == N) and m["bond"] == 2 * N
    i, j = np.indices((L, L))
    neel = np.where((i + j) % 2 == 0, 1, -1).astype(np.int8)
    m = oracle.measure(neel, r)
    sign = np.where(r % 2 == 0, 1, -1)
    assert np.array_equal(m["Sx"], sign * N) and np.array_equal(m["Sy"], sign * N)
    assert m["bond"] == -2 * N and m["sum_s"] == 0
    stripes = np.where(i % 2 == 0, 1, -1).astype(np.int8)  # rows alternate
    m = oracle.measure(stripes, r)
    assert np.all(m["Sx"] == N) and np.array_equal(m["Sy"], sign * N)
    # one column of vacancies in an all-up BC lattice
    vac = np.ones((L, L), dtype=np.int8)
    vac[:, 3] = 0
    m = oracle.measure(vac, r)
    assert m["sum_s2"] == N - L
    assert np.all(m["Sy"][1:] == N - L)
    assert np.all(m["Sx"][1:] == N - 2 * L)  # pairs touching the empty column vanish
    assert m["Sx"][0] == N - L


@pytest.mark.parametrize("model", [oracle.ISING, oracle.BLUME_CAPEL])
def test_correlation_symmetries(model):
    L = 32
    s = oracle.init(model, L, 5)
    oracle.sweep(model, s, 5, 1.0, 0.0, 0, np.full(3, 2.0))
    r = np.arange(0, L, dtype=np.uint32)
    m = oracle.measure(s, r)
    assert m["Sx"][0] == m["sum_s2"] and m["Sy"][0] == m["sum_s2"]
    assert np.array_equal(m["Sx"][1:], m["Sx"][1:][::-1])
    assert np.array_equal(m["Sy"][1:], m["Sy"][1:][::-1])
    assert m["bond"] == m["Sx"][1] + m["Sy"][1]
    mt = oracle.measure(np.ascontiguousarray(s.T), r)
    assert np.array_equal(mt["Sx"], m["Sy"]) and np.array_equal(mt["Sy"], m["Sx"])


def test_xi_closed_form_exponential():
    # C(r) = x^r with x = e^{-1/a} on r = 0..R; the trapezoid sums are
    # sum_{r=0}^{R} r^n x^r minus half the end terms, with
    # sum r x^r = x (1 - (R+1) x^R + R x^{R+1}) / (1-x)^2 and
    # sum r^2 x^r = x (1 + x - (R+1)^2 x^R + (2R^2+2R-1) x^{R+1} - R^2 x^{R+2}) / (1-x)^3
    for a, R in [(3.0, 200), (17.5, 400), (1.2, 60)]:
        x = math.exp(-1.0 / a)
        r = np.arange(1, R + 1)
        C = x ** r
        S1 = x * (1 - (R + 1) * x**R + R * x ** (R + 1)) / (1 - x) ** 2
        S2 = x * (1 + x - (R + 1) ** 2 * x**R + (2 * R * R + 2 * R - 1) * x ** (R + 1)
                  - R * R * x ** (R + 2)) / (1 - x) ** 3
        I1 = S1 - 0.5 * R * x**R
        I2 = S2 - 0.5 * R * R * x**R
        xi = oracle.xi_second_moment_integral(r, C, 1.0)
        assert abs(xi - I2 / I1) <= 1e-12 * (I2 / I1)


def test_xi_cut_at_first_non_positive():
    r = np.array([1, 2, 4, 8, 16])
    C = np.array([0.5, 0.25, -0.01, 0.3, 0.2])
    # only (0,1), (1,.5), (2,.25) count
    I1 = 1 * (0 + 0.5) / 2 + 1 * (0.5 + 0.5) / 2
    I2 = 1 * (0 + 0.5) / 2 + 1 * (0.5 + 4 * 0.25) / 2
    assert abs(oracle.xi_second_moment_integral(r, C, 1.0) - I2 / I1) < 1e-15


@pytest.mark.parametrize("model", [oracle.ISING, oracle.BLUME_CAPEL])
def test_window_evolution_matches_full_run(model):
    L, seed, n = 64, 1234, 5
    T = np.array([2.1, 1.7, 2.4, 1.9, 2.0])
    s = oracle.init(model, L, seed)
    oracle.sweep(model, s, seed, 1.0, 0.0, 0, T)
    for (i0, j0, H, W) in [(0, 0, 30, 26), (50, 55, 29, 31), (7, 60, 24, 40)]:
        win = oracle.init_window(model, L, seed, i0, j0, H, W)
        full0 = oracle.init(model, L, seed)
        rows = (i0 + np.arange(H)) % L
        cols = (j0 + np.arange(W)) % L
        assert np.array_equal(win, full0[np.ix_(rows, cols)])
        oracle.window_sweep(model, win, L, seed, 1.0, 0.0, i0, j0, 0, T)
        k = 2 * n
        assert np.array_equal(win[k:H - k, k:W - k], s[np.ix_(rows, cols)][k:H - k, k:W - k])


def test_initial_state_statistics():
    L = 256
    s = oracle.init(oracle.ISING, L, 2503146880)
    assert set(np.unique(s).tolist()) == {-1, 1}
    n_up = int((s == 1).sum())
    assert abs(n_up - L * L / 2) < 5 * math.sqrt(L * L / 4)
    b = oracle.init(oracle.BLUME_CAPEL, L, 2503146880)
    counts = [int((b == v).sum()) for v in (-1, 0, 1)]
    assert stats.chisquare(counts).pvalue > 1e-3
    # magnetisation over seeds: Ising M / L ~ N(0, 1), BC M / L ~ N(0, 2/3)
    Ls = 32
    Mi = np.array([oracle.init(oracle.ISING, Ls, k).sum() / Ls for k in range(400)])
    Mb = np.array([oracle.init(oracle.BLUME_CAPEL, Ls, k).sum() / Ls for k in range(400)])
    assert stats.kstest(Mi, "norm", args=(0, 1)).pvalue > 1e-3
    assert stats.kstest(Mb, "norm", args=(0, math.sqrt(2 / 3))).pvalue > 1e-3


def test_schedules():
    assert np.all(oracle.schedule(0, [2.5], 0, 5) == 2.5)
    two = oracle.schedule(1, [1.66, 4, 2.27414861561203], 2, 5)  # t = 2..6, switch at 4
    assert two.tolist() == [1.66, 1.66, 2.27414861561203, 2.27414861561203, 2.27414861561203]
    Tc = TC_ISING
    ex = oracle.schedule(2, [2 * Tc, 1.02 * Tc, 64.0], 0, 129)
    assert ex[0] == 2 * Tc
    assert abs(ex[64] - (1.02 * Tc + 0.98 * Tc / math.e)) < 1e-14
    assert np.all(np.diff(ex) < 0)
