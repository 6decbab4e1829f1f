"""Pins of the oracle's Swendsen-Wang step and Fourier moments (paper App. B:
Swendsen-Wang restricted to s = +-1 combined with Metropolis, the Binder
cumulant and the second-moment correlation length from Fourier moments).

* T = 0 activates every bond between equal non-zero spins, so the clusters
  are the connected components of like non-zero spins of the periodic
  lattice: checked against scipy's graph routine.  T = inf activates none:
  every site is its own cluster.  At any T the clusters refine the T = 0
  components and carry their smallest site index as name.
* The chain samples the Boltzmann weight of Eq. 1: Swendsen-Wang alone on
  4 x 4 Ising, and Metropolis + Swendsen-Wang on 4 x 4 Blume-Capel, against
  exact enumeration; Swendsen-Wang alone on Blume-Capel keeps s^2 and samples
  the signs of the non-zero spins with the Ising weight of the diluted
  lattice, against enumeration of those signs.
* The Fourier moments equal numpy's FFT (M(k) is the complex conjugate of
  numpy's forward transform for a real field).
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from test_oracle_equilibrium import TC_BC, TC_ISING, compare_histogram, exact_joint_counts


def like_spin_components(s):
    """Smallest site index of each site's component of equal non-zero
    nearest neighbours (periodic), by scipy's connected components."""
    L = s.shape[0]
    N = L * L
    idx = np.arange(N).reshape(L, L)
    a, b = [], []
    for axis in (0, 1):
        nb = np.roll(s, -1, axis=axis)
        nbi = np.roll(idx, -1, axis=axis)
        mask = (s != 0) & (s == nb)
        a.append(idx[mask])
        b.append(nbi[mask])
    a, b = np.concatenate(a), np.concatenate(b)
    g = coo_matrix((np.ones(a.shape[0]), (a, b)), shape=(N, N))
    _, comp = connected_components(g, directed=False)
    first = np.full(comp.max() + 1, N, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(N))
    return first[comp].reshape(L, L)


@pytest.mark.parametrize("model,L,seed", [(0, 8, 1), (0, 16, 2), (1, 16, 3), (1, 6, 4), (1, 32, 5), (0, 10, 6)])
def test_zero_temperature_clusters_are_like_spin_components(model, L, seed):
    s = oracle.init(model, 64, seed)[:L, :L].copy()  # any disordered state
    want = like_spin_components(s)
    before = s.copy()
    lab = oracle.sw(model, s, seed, 1.0, 7, [0.0], with_labels=True)
    assert np.array_equal(lab.astype(np.int64), want)
    # every cluster flips as a whole, vacancies stay
    flipped = s != before
    assert np.array_equal(s == 0, before == 0)
    assert np.array_equal(s[before != 0], np.where(flipped, -before, before)[before != 0])
    for name in np.unique(want[before != 0]):
        members = flipped[(want == name) & (before != 0)]
        assert members.all() or not members.any()


@pytest.mark.parametrize("model", [0, 1])
def test_infinite_temperature_leaves_every_site_alone(model):
    L = 16
    s = oracle.init(model, 64, 9)[:L, :L].copy()
    lab = oracle.sw(model, s, 9, 1.0, 0, [math.inf], with_labels=True)
    assert np.array_equal(lab.ravel(), np.arange(L * L, dtype=np.uint64))


@pytest.mark.parametrize("model,T", [(0, 1.8), (0, TC_ISING), (1, TC_BC), (1, 1.0)])
def test_clusters_refine_like_spin_components(model, T):
    L = 24
    s = oracle.init(model, 64, 21)[:L, :L].copy()
    comp = like_spin_components(s)
    lab = oracle.sw(model, s.copy(), 21, 1.0, 3, [T], with_labels=True).astype(np.int64)
    flat = lab.ravel()
    assert (flat <= np.arange(L * L)).all()           # a name is one of the cluster's sites...
    assert np.array_equal(flat[flat], flat)             # ...and names itself
    for name in np.unique(flat):
        assert np.unique(comp.ravel()[flat == name]).shape[0] == 1
    n_clusters = np.unique(flat).shape[0]
    assert np.unique(comp).shape[0] <= n_clusters < L * L


def test_bond_threshold_limits():
    assert oracle.sw_threshold(1.0, 0.0) == (True, 0)
    assert oracle.sw_threshold(1.0, math.inf) == (False, 0)
    always, thr = oracle.sw_threshold(1.0, TC_ISING)
    # p = 1 - exp(-2 / T_c) = 1 - (sqrt 2 - 1) = 2 - sqrt 2 at the Ising T_c
    assert not always and abs(thr - (2.0 - math.sqrt(2.0)) * 2**32) <= 1.0


@pytest.mark.parametrize("T", [1.8, TC_ISING, 3.0])
def test_ising_4x4_swendsen_wang_alone_samples_boltzmann(T):
    g = exact_joint_counts([-1, 1])[:, 16]
    B = np.arange(-32, 33)
    w = g * np.exp(B / T - np.max(B[g > 0] / T))
    p = w / w.sum()
    seed = 300 + int(T * 10)
    s = oracle.init(0, 4, seed)
    n = 40000
    Bs = np.zeros(n, dtype=np.int64)
    for k in range(n):
        oracle.sw(0, s, seed, 1.0, k, [T])
        Bs[k] = oracle.measure(s, [])["bond"]
    compare_histogram(Bs[200:], {int(b): float(pb) for b, pb in zip(B, p)})


@pytest.mark.parametrize("T,Delta", [(TC_BC, 0.0), (1.2, 0.0), (1.5, 0.6)])
def test_blume_capel_4x4_metropolis_plus_swendsen_wang(T, Delta):
    g = exact_joint_counts([-1, 0, 1])
    B = np.arange(-32, 33)[:, None]
    Q = np.arange(17)[None, :]
    logw = np.where(g > 0, -(-B + Delta * Q) / T, -np.inf)
    w = g * np.exp(logw - logw.max())
    p = w / w.sum()
    seed = 700 + int(T * 100)
    s = oracle.init(1, 4, seed)
    n = 40000
    keys = np.zeros(n, dtype=np.int64)
    Tarr = np.array([T])
    for k in range(n):
        oracle.sweep(1, s, seed, 1.0, Delta, 2 * k, Tarr)
        oracle.sw(1, s, seed, 1.0, 2 * k + 1, Tarr)
        m = oracle.measure(s, [])
        keys[k] = (m["bond"] + 32) * 17 + m["sum_s2"]
    exact = {int(b * 17 + q): float(p[b, q]) for b in range(65) for q in range(17)}
    compare_histogram(keys[200:], exact)


@pytest.mark.parametrize("T", [1.2, TC_BC])
def test_blume_capel_swendsen_wang_alone_samples_diluted_ising(T):
    # a fixed vacancy pattern: s^2 never changes, and the signs of the twelve
    # non-zero spins follow exp(J/T sum s_x s_y) over the bonds between them
    s = np.array([[1, 0, -1, 1], [1, 1, 0, -1], [-1, 1, 1, 0], [0, -1, 1, 1]], dtype=np.int8)
    occ = s != 0
    sites = np.argwhere(occ)
    signs = np.array(np.meshgrid(*([[-1, 1]] * sites.shape[0]), indexing="ij")).reshape(sites.shape[0], -1).T
    Bexact = np.zeros(signs.shape[0], dtype=np.int64)
    for q, sg in enumerate(signs):
        f = np.zeros((4, 4), dtype=np.int64)
        f[occ] = sg
        Bexact[q] = (f * np.roll(f, -1, 0)).sum() + (f * np.roll(f, -1, 1)).sum()
    vals, counts = np.unique(Bexact, return_counts=True)
    w = counts * np.exp(vals / T - (vals / T).max())
    p = w / w.sum()
    n = 40000
    Bs = np.zeros(n, dtype=np.int64)
    for k in range(n):
        oracle.sw(1, s, 55, 1.0, k, [T])
        assert k % 5000 or np.array_equal(s != 0, occ)
        Bs[k] = oracle.measure(s, [])["bond"]
    assert np.array_equal(s != 0, occ)
    compare_histogram(Bs[200:], {int(v): float(pv) for v, pv in zip(vals, p)})


@pytest.mark.parametrize("model,L", [(0, 16), (1, 32), (1, 6)])
def test_fourier_moments_equal_fft(model, L):
    s = oracle.init(model, 64, 77)[:L, :L].copy()
    got = oracle.fourier(s)
    F = np.fft.fft2(s.astype(np.float64))
    tol = 1e-9 * L * L
    assert abs(got["M0"] - F[0, 0].real) <= tol
    assert abs(got["k1"] - np.conj(F[1, 0])) <= tol  # phase along the row index i
    assert abs(got["k2"] - np.conj(F[0, 1])) <= tol  # phase along the column index j
    assert got["M0"] == float(s.sum())
