"""Pins of the equilibrium estimators of App. B (Binder cumulant, second-moment
correlation length, single-histogram reweighting, beta_{L,g} crossings) on
exact data, and of the whole EMCS recipe on oracle chains.

Exact data: every 4 x 4 Ising state (2^16) with its energy and Fourier
moments (numpy's FFT), weighted by an exact Boltzmann factor.  Closed forms:
at beta = 0 the spins are independent, so <M^2> = N and <M^4> = 3N^2 - 2N
(U4 = 3 - 2/N) and chi(k) = 1 for every k; at large beta only the two ground
states survive (U4 -> 1).  Reweighting the exact beta_0 ensemble to beta must
reproduce the exact beta ensemble to rounding.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2503_14688_amd import equilibrium

TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))


def all_4x4_ising():
    n = 16
    codes = np.arange(2 ** n, dtype=np.int64)
    s = (1 - 2 * ((codes[:, None] >> np.arange(n)) & 1)).reshape(-1, 4, 4).astype(np.float64)
    bond = (s * np.roll(s, -1, 1)).sum(axis=(1, 2)) + (s * np.roll(s, -1, 2)).sum(axis=(1, 2))
    F = np.fft.fft2(s)
    return {"H": -bond, "M0": s.sum(axis=(1, 2)), "Mk2": 0.5 * (np.abs(F[:, 1, 0]) ** 2 + np.abs(F[:, 0, 1]) ** 2)}


EXACT = all_4x4_ising()


def exact_average(beta, f):
    w = np.exp(-beta * (EXACT["H"] - EXACT["H"].min()))
    return float((w * f).sum() / w.sum())


def exact_U4(beta):
    return exact_average(beta, EXACT["M0"] ** 4) / exact_average(beta, EXACT["M0"] ** 2) ** 2


def test_infinite_temperature_closed_forms():
    o = equilibrium.observables(EXACT, 4, 0.0, w0=np.ones(EXACT["H"].shape[0]))
    N = 16
    assert abs(o["U4"] - (3.0 - 2.0 / N)) < 1e-12
    assert abs(o["chi0"] - 1.0) < 1e-12 and abs(o["chi_kmin"] - 1.0) < 1e-12


def test_ground_state_limit():
    beta = 6.0
    w0 = np.exp(-beta * (EXACT["H"] - EXACT["H"].min()))
    o = equilibrium.observables(EXACT, 4, beta, w0=w0)
    assert abs(o["U4"] - 1.0) < 1e-6
    assert o["chi_kmin"] < 1e-6 * o["chi0"]


@pytest.mark.parametrize("beta0,beta", [(0.3, 0.45), (0.44, 0.40), (0.5, 0.5), (0.2, 0.6)])
def test_reweighting_is_exact_on_exact_data(beta0, beta):
    w0 = np.exp(-beta0 * (EXACT["H"] - EXACT["H"].min()))
    o = equilibrium.observables(EXACT, 4, beta0, beta, w0=w0)
    M2 = exact_average(beta, EXACT["M0"] ** 2)
    Mk = exact_average(beta, EXACT["Mk2"])
    assert abs(o["U4"] - exact_U4(beta)) < 1e-11
    assert abs(o["chi0"] - M2 / 16) < 1e-11 * M2
    xi2 = math.sqrt(M2 / Mk - 1.0) / (2.0 * math.sin(math.pi / 4))
    assert abs(o["xi2"] - xi2) < 1e-10 * xi2


def test_crossing_on_exact_data():
    beta0 = 0.4
    w0 = np.exp(-beta0 * (EXACT["H"] - EXACT["H"].min()))
    target = 1.4
    want = brentq(lambda b: exact_U4(b) - target, 0.05, 1.5, xtol=1e-13)
    got = equilibrium.beta_crossing(EXACT, 4, beta0, "U4", target, 0.3, w0=w0)
    assert got is not None and abs(got - want) < 1e-9
    assert equilibrium.beta_crossing(EXACT, 4, beta0, "U4", 0.5, 0.3, w0=w0) is None  # U4 >= 1 always


class OracleChain:
    """The Lattice interface over the oracle, for the EMCS driver."""

    def __init__(self, model, L, seed, J=1.0, Delta=0.0):
        self.model, self.L, self.seed, self.J, self.Delta = model, L, seed, J, Delta
        self.s = oracle.init(model, L, seed)
        self.t = 0

    def sweep(self, T):
        oracle.sweep(self.model, self.s, self.seed, self.J, self.Delta, self.t, T)
        self.t += len(T)

    def sw(self, T):
        oracle.sw(self.model, self.s, self.seed, self.J, self.t, T)
        self.t += len(T)

    def fourier(self):
        f = oracle.fourier(self.s)
        m = oracle.measure(self.s, [])
        return {"sum_s": m["sum_s"], "sum_s2": m["sum_s2"], "bond": m["bond"], "k1": f["k1"], "k2": f["k2"]}


def test_ising_critical_point_from_emcs_chains():
    """2D Ising at L = 16: U4 and xi2/L at beta_c sit near the universal values
    (finite-size corrections of a few per cent), and the crossings land near
    beta_c = ln(1 + sqrt 2) / 2."""
    L, beta_c = 16, 1.0 / TC_ISING
    runs = []
    for k in range(6):
        lat = OracleChain(0, L, 9000 + k)
        runs.append(equilibrium.emcs_run(lat, TC_ISING, 300, every=1, n_therm=20, n_metropolis=2))
    c = equilibrium.crossings(runs, L, beta_c)
    assert abs(c["U4"] - equilibrium.U4_STAR) < 0.04, c
    assert abs(c["xi2_over_L"] - equilibrium.XI_OVER_L_STAR) < 0.05, c
    for key in ("beta_U", "beta_xi"):
        assert c[key] is not None and abs(c[key] - beta_c) < 0.02, c
        assert c[key + "_err"] is not None and 0 < c[key + "_err"] < 0.02, c
