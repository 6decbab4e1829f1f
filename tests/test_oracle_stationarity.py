"""Exact stationarity of the checkerboard half-sweep (paper, Introduction:
Metropolis updates of one sublattice at a time) under the integer rule.

On a 4 x 4 periodic Ising lattice every state sigma and every colour c
define the half-sweep kernel K_c(sigma -> sigma'): each colour-c site flips
independently, with probability 1 when dE = 2 J s h <= 0 and p(dE) otherwise.
Enumerating all 2^16 states and the 2^8 flip patterns of each colour checks
(pi K_c)(sigma') = sum_sigma pi(sigma) K_c(sigma -> sigma') against the
Boltzmann weights pi(sigma'):

* with p = exp(-dE / T) the identity holds to FP64 rounding;
* with the oracle's integer rule, p = thr(dE, T) / 2^32 (u uniform on the
  2^32 integers, accept iff u < thr), every p is within 2^-32 of the exact
  value, so |(pi K_c)(sigma') - pi(sigma')| <= 8 * 2^-32 * sum of pi over the
  256 states that reach sigma'.

A wrong neighbour, sign, colour or threshold breaks the identity far beyond
these bounds (the planted-mistake test shows the check has that power).
"""
import numpy as np
import pytest

import oracle

L = 4
N = L * L
STATES = np.arange(1 << N, dtype=np.int64)


def spins_of(states):
    # bit k of the state: site k = 4 i + j is -1
    bits = (states[:, None] >> np.arange(N)) & 1
    return 1 - 2 * bits.astype(np.int64)


def neighbours(k):
    i, j = divmod(k, L)
    return [((i - 1) % L) * L + j, ((i + 1) % L) * L + j, i * L + (j - 1) % L, i * L + (j + 1) % L]


def boltzmann(s, J, T):
    bonds = sum(s[:, k] * s[:, n] for k in range(N) for n in neighbours(k)[1::2])  # down and right bonds
    E = -J * bonds
    w = np.exp(-(E - E.min()) / T)
    return w / w.sum()


def apply_kernel(s, pi, c, J, prob):
    """(pi K_c) and, for the error bound, the pi mass reaching each state.
    prob(dE) gives the flip probability of a move with dE > 0."""
    sites = [k for k in range(N) if (k // L + k % L) % 2 == c]
    p = np.empty((STATES.size, len(sites)))
    for a, k in enumerate(sites):
        h = sum(s[:, n] for n in neighbours(k))
        dE = 2.0 * J * s[:, k] * h
        pk = np.ones(STATES.size)
        for v in (4.0 * J, 8.0 * J):
            pk[dE == v] = prob(v)
        p[:, a] = pk
    out = np.zeros(STATES.size)
    mass = np.zeros(STATES.size)
    for m_idx in range(1 << len(sites)):
        m = sum(1 << sites[a] for a in range(len(sites)) if (m_idx >> a) & 1)
        sel = (m_idx >> np.arange(len(sites))) & 1
        np.add.at(out, STATES ^ m, pi * np.prod(np.where(sel[None, :] == 1, p, 1.0 - p), axis=1))
        np.add.at(mass, STATES ^ m, pi)
    return out, mass


def integer_prob(T):
    def prob(dE):
        always, thr = oracle.threshold(dE, T)
        assert not always
        return thr / 2.0 ** 32
    return prob


@pytest.mark.parametrize("T", [1.5, 2.269185314213022, 3.5])
@pytest.mark.parametrize("c", [0, 1])
def test_half_sweep_kernel_keeps_boltzmann(T, c):
    J = 1.0
    s = spins_of(STATES)
    pi = boltzmann(s, J, T)
    exact, _ = apply_kernel(s, pi, c, J, lambda dE: np.exp(-dE / T))
    assert np.max(np.abs(exact - pi) / pi) < 1e-12
    out, mass = apply_kernel(s, pi, c, J, integer_prob(T))
    assert np.all(np.abs(out - pi) <= 8 * 2.0 ** -32 * mass + 1e-15)


def test_stationarity_check_detects_a_wrong_rule():
    """Planted mistake in the rule: the thresholds of dE = 4J and 8J swapped."""
    T, J, c = 2.269185314213022, 1.0, 0
    s = spins_of(STATES)
    pi = boltzmann(s, J, T)
    right = integer_prob(T)
    out, mass = apply_kernel(s, pi, c, J, lambda dE: right(12.0 * J - dE))
    assert np.max(np.abs(out - pi) - 8 * 2.0 ** -32 * mass) > 1e-4
