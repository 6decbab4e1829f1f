"""Pins of oracle.derive, the FP64 observables taken from the integer sums.

derive turns the sums of oracle.measure into
  e     = (-J * bond + Delta * sum s^2) / L^2   (Eq. 3 read with the sign of
          the Hamiltonian of Eq. 1: the energy density H / L^2)
  m     = sum s / L^2
  C-hat = (Sx + Sy) / (2 L^2)                   (axis average of Eq. 2)
Each is checked here on constructed lattices whose energy density,
magnetisation and correlations follow from Eq. 1 and Eq. 2 by hand, with
J != 1 and Delta != 0 so that every factor shows.  The expected values are
written from the lattice, never from the formula being tested:

* all up:        every bond aligned, H / L^2 = -2J + Delta, m = 1, C(r) = 1;
* Neel:          every bond anti-aligned, H / L^2 = +2J + Delta, m = 0,
                 C(r) = (-1)^r;
* row stripes:   horizontal bonds aligned, vertical anti-aligned, H = Delta N,
                 C_x(r) = 1, C_y(r) = (-1)^r;
* vacancy column (Blume-Capel, all up but one column of zeros): per row
                 L - 2 aligned horizontal bonds (the two touching the empty
                 column vanish), L aligned vertical bonds in each of the
                 L - 1 occupied columns, N - L occupied sites;
* a single down spin in an all-up lattice: four bonds turn, H rises by 8J;
* the Onsager test of test_oracle_equilibrium reads e from derive as well.

check_derive collects the failures, and the planted-mistake test shows that
a sign slip, a dropped Delta term, a doubled C-hat and a wrong magnetisation
norm each fail it (the mistakes are planted in copies of derive on the CPU).
"""
import numpy as np
import pytest

import oracle


def _cases(L=16, J=0.7, Delta=0.45):
    N = float(L * L)
    r = np.arange(1, L, dtype=np.uint32)
    sign = np.where(r % 2 == 0, 1.0, -1.0)
    i, j = np.indices((L, L))
    up = np.ones((L, L), dtype=np.int8)
    neel = np.where((i + j) % 2 == 0, 1, -1).astype(np.int8)
    stripes = np.where(i % 2 == 0, 1, -1).astype(np.int8)
    vac = np.ones((L, L), dtype=np.int8)
    vac[:, 3] = 0
    one_down = np.ones((L, L), dtype=np.int8)
    one_down[5, 9] = -1
    occupied = N - L
    # vacancy column: horizontal pairs at distance r >= 1 with both ends
    # occupied: (L - 2) per row (the two pairs touching column 3 vanish);
    # vertical pairs: all L rows of the L - 1 occupied columns
    vac_cx = L * (L - 2) / N
    vac_cy = L * (L - 1) / N
    return [
        ("all_up", up, J, Delta, dict(e=-2.0 * J + Delta, m=1.0, C=np.ones(r.shape))),
        ("neel", neel, J, Delta, dict(e=2.0 * J + Delta, m=0.0, C=sign)),
        ("stripes", stripes, J, Delta, dict(e=Delta, m=0.0, C=(1.0 + sign) / 2.0)),
        ("vacancy_column", vac, J, Delta,
         dict(e=(-J * (L * (L - 2) + L * (L - 1)) + Delta * occupied) / N, m=occupied / N,
              C=np.full(r.shape, (vac_cx + vac_cy) / 2.0))),
        ("one_down", one_down, J, Delta,
         dict(e=(-2.0 * J * N + 8.0 * J) / N + Delta, m=(N - 2.0) / N, C=None)),
    ], r


def check_derive(derive):
    """Failures of a derive function on the constructed lattices (empty: all pass)."""
    bad = []
    cases, r = _cases()
    for name, s, J, Delta, want in cases:
        L = s.shape[0]
        got = derive(L, J, Delta, oracle.measure(s, r), r)
        if abs(got["e"] - want["e"]) > 1e-12:
            bad.append(f"{name}: e = {got['e']!r}, expected {want['e']!r}")
        if abs(got["m"] - want["m"]) > 1e-12:
            bad.append(f"{name}: m = {got['m']!r}, expected {want['m']!r}")
        if want["C"] is not None and not np.allclose(got["C_hat"], want["C"], rtol=0, atol=1e-12):
            bad.append(f"{name}: C-hat differs")
    return bad


def test_derive_on_constructed_lattices():
    assert check_derive(oracle.derive) == []


def test_ising_energy_density_at_delta_zero():
    # the Ising path: Delta = 0 and J = 1, all up and Neel give -2 and +2
    L = 8
    r = np.arange(1, L, dtype=np.uint32)
    up = np.ones((L, L), dtype=np.int8)
    i, j = np.indices((L, L))
    neel = np.where((i + j) % 2 == 0, 1, -1).astype(np.int8)
    assert oracle.derive(L, 1.0, 0.0, oracle.measure(up, r), r)["e"] == -2.0
    assert oracle.derive(L, 1.0, 0.0, oracle.measure(neel, r), r)["e"] == 2.0


def _planted(kind):
    def derive(L, J, Delta, sums, r):
        out = dict(oracle.derive(L, J, Delta, sums, r))
        N = float(L) * L
        if kind == "sign":
            out["e"] = (J * sums["bond"] + Delta * sums["sum_s2"]) / N
        elif kind == "no_delta":
            out["e"] = -J * sums["bond"] / N
        elif kind == "c_hat_sum":
            out["C_hat"] = (np.asarray(sums["Sx"], float) + np.asarray(sums["Sy"], float)) / N
        elif kind == "m_norm":
            out["m"] = sums["sum_s"] / float(L)
        return out
    return derive


@pytest.mark.parametrize("kind", ["sign", "no_delta", "c_hat_sum", "m_norm"])
def test_planted_mistakes_fail_the_pin(kind):
    assert check_derive(_planted(kind)) != []
