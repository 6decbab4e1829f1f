"""Statistical pins of the oracle's dynamics against exact equilibrium results.

A correct Metropolis chain samples the Boltzmann weight of the Hamiltonian of
Eq. 1, so the long-run histograms of the oracle must match:

* brute-force enumeration of every 4 x 4 Ising state (2^16) and every 4 x 4
  Blume-Capel state (3^16, by rows), both with periodic boundaries;
* Onsager's exact internal energy of the infinite Ising lattice for L = 64
  off-critical, where finite-size corrections are far below the errors.

Errors are batch means over a fixed-seed run; the bar is 4.5 sigma per bin.
A wrong sign or factor in dE, a wrong neighbour, a wrong proposal or a wrong
threshold shifts these distributions by many sigma.
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle

TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))
TC_BC = 1.69355839821214427017  # paper Table I


def _row_tables(values, width=4):
    """All rows of `width` spins: intra-row periodic bond sums and sum s^2."""
    rows = np.array(np.meshgrid(*([values] * width), indexing="ij")).reshape(width, -1).T
    hb = (rows * np.roll(rows, -1, axis=1)).sum(axis=1)
    q = (rows * rows).sum(axis=1)
    vb = rows @ rows.T  # vertical bonds between two stacked rows
    return rows, hb, q, vb


def exact_joint_counts(values):
    """g[B + 32, Q]: number of 4 x 4 periodic states with bond sum B and sum s^2 = Q."""
    _, hb, q, vb = _row_tables(np.array(values))
    n = hb.shape[0]
    g = np.zeros((65, 17), dtype=np.int64)
    for r0 in range(n):
        # B and Q over (r1, r2, r3) with r0 fixed; rows stacked cyclically
        B = (hb[r0] + hb[:, None, None] + hb[None, :, None] + hb[None, None, :]
             + vb[r0][:, None, None] + vb[:, :, None] + vb[None, :, :] + vb[:, r0][None, None, :])
        Q = q[r0] + q[:, None, None] + q[None, :, None] + q[None, None, :]
        np.add.at(g, (B.ravel() + 32, Q.ravel()), 1)
    return g


def run_chain(model, L, seed, J, Delta, T, n_sweeps, start=None, energies=False):
    """Bond sums and sum s^2 after each sweep; with energies, also the energy
    density that oracle.derive gives for each state."""
    s = oracle.init(model, L, seed) if start is None else start.copy()
    Bs = np.zeros(n_sweeps, dtype=np.int64)
    Qs = np.zeros(n_sweeps, dtype=np.int64)
    Es = np.zeros(n_sweeps, dtype=np.float64)
    Tarr = np.array([T])
    for k in range(n_sweeps):
        oracle.sweep(model, s, seed, J, Delta, k, Tarr)
        m = oracle.measure(s, [])
        Bs[k] = m["bond"]
        Qs[k] = m["sum_s2"]
        if energies:
            Es[k] = oracle.derive(L, J, Delta, m, [])["e"]
    if energies:
        return Bs, Qs, Es
    return Bs, Qs


def compare_histogram(keys, exact_p, n_batches=40, nsig=4.5):
    """keys: integer bin per sample; exact_p: dict bin -> probability."""
    n = keys.shape[0]
    per = n // n_batches
    keys = keys[: per * n_batches].reshape(n_batches, per)
    worst = 0.0
    for b, p in exact_p.items():
        if p < 2e-3:
            continue
        bm = (keys == b).mean(axis=1)
        obs = bm.mean()
        sig = max(bm.std(ddof=1) / math.sqrt(n_batches), math.sqrt(p * (1 - p) / (per * n_batches)))
        z = abs(obs - p) / sig
        worst = max(worst, z)
        assert z < nsig, f"bin {b}: observed {obs:.5f} exact {p:.5f} ({z:.1f} sigma)"
    return worst


@pytest.mark.parametrize("T", [1.8, TC_ISING, 3.0])
def test_ising_4x4_energy_histogram(T):
    g = exact_joint_counts([-1, 1])[:, 16]  # Q = 16 always
    assert g.sum() == 2**16
    J = 1.0
    B = np.arange(-32, 33)
    w = g * np.exp(J * B / T - np.max(J * B[g > 0] / T))
    p = w / w.sum()
    Bs, _ = run_chain(oracle.ISING, 4, 11 + int(T * 100), J, 0.0, T, 60000)
    compare_histogram(Bs[1000:], {int(b): float(pb) for b, pb in zip(B, p)})


@pytest.mark.parametrize("T,Delta", [(TC_BC, 0.0), (1.2, 0.0), (2.5, 0.0), (1.5, 0.6), (1.5, -0.8)])
def test_blume_capel_4x4_joint_histogram(T, Delta):
    g = exact_joint_counts([-1, 0, 1])
    assert g.sum() == 3**16
    J = 1.0
    B = np.arange(-32, 33)[:, None]
    Q = np.arange(17)[None, :]
    logw = np.where(g > 0, -(-J * B + Delta * Q) / T, -np.inf)
    w = g * np.exp(logw - logw.max())
    p = w / w.sum()
    Bs, Qs = run_chain(oracle.BLUME_CAPEL, 4, 101 + int(T * 100), J, Delta, T, 60000)
    keys = (Bs + 32) * 17 + Qs
    exact = {int(b * 17 + q): float(p[b, q]) for b in range(65) for q in range(17)}
    compare_histogram(keys[1000:], exact)


def onsager_energy(T, J=1.0):
    """Energy per spin of the infinite square-lattice Ising model (Onsager 1944)."""
    K = J / T
    kappa = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    K1 = special.ellipk(kappa**2)
    return -J / math.tanh(2 * K) * (1.0 + 2.0 / math.pi * (2.0 * math.tanh(2 * K) ** 2 - 1.0) * K1)


def test_onsager_closed_form_at_tc():
    # the elliptic term vanishes at T_c, leaving -coth(2K_c) = -sqrt 2 (paper,
    # Results: E_eq(T_c) = -sqrt 2); K1 diverges only logarithmically there
    for eps in (1e-7, -1e-7):
        assert abs(onsager_energy(TC_ISING * (1 + eps)) + math.sqrt(2.0)) < 1e-5


@pytest.mark.parametrize("T", [1.5, 2.0, 3.0])
def test_ising_energy_matches_onsager(T):
    L = 64
    start = np.ones((L, L), dtype=np.int8) if T < TC_ISING else None
    _, _, es = run_chain(oracle.ISING, L, 5000 + int(T * 10), 1.0, 0.0, T, 3400, start, energies=True)
    e = es[400:]
    nb = 30
    per = e.shape[0] // nb
    bm = e[: per * nb].reshape(nb, per).mean(axis=1)
    mean = bm.mean()
    err = bm.std(ddof=1) / math.sqrt(nb)
    u = onsager_energy(T)
    assert abs(mean - u) < 4.5 * err + 1e-4, (mean, u, err)
