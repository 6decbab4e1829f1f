"""Equilibrium finite-size scaling of the Blume-Capel critical temperature
(paper App. B), as a host driver over the library's sweep, Swendsen-Wang and
Fourier-moment calls plus FP64 estimators on the host.

Simulation (App. B): an elementary Monte Carlo step (EMCS) is ten Metropolis
sweeps followed by one Swendsen-Wang step restricted to the sites with
s = +-1; independent runs start from the T = infinity state, are thermalised
and then measured every few EMCS.  Each measurement records the total energy
H = -J sum s_x s_y + Delta sum s^2 (Eq. 1), M(0) and |M(k)|^2 for the two
smallest non-zero wave vectors.

Estimators (App. B):
  U4      = <M(0)^4> / <M(0)^2>^2                                  (Binder)
  chi(k)  = <|M(k)|^2> / L^2, chi_kmin the average over the two axes
  xi_2    = sqrt(chi(0) / chi_kmin - 1) / (2 sin(pi / L))
Single-histogram reweighting (Ferrenberg and Swendsen 1988) moves an average
from the simulated inverse temperature beta_0 to a nearby beta:
  <O>_beta = sum_n O_n w_n / sum_n w_n,  w_n = exp(-(beta - beta_0) H_n).
beta_{L,U} and beta_{L,xi2/L} solve U4(L, beta) = U4* and
xi_2(L, beta) / L = [xi_2/L]*, the universal values quoted in App. B
(Salas and Sokal); errors are jackknife over independent runs.
"""
import math

import numpy as np

from .analysis import jackknife_error

# Universal large-L values at criticality of the 2D Ising universality class,
# as quoted in App. B.
U4_STAR = 1.1679229
XI_OVER_L_STAR = 0.9050488292
EMCS_METROPOLIS = 10  # Metropolis sweeps per elementary Monte Carlo step (App. B)


def emcs_run(lat, T, n_emcs, every=1, n_therm=0, n_metropolis=EMCS_METROPOLIS):
    """Run n_therm + n_emcs elementary Monte Carlo steps at bath temperature T
    on lat (anything with sweep, sw, fourier and J / Delta / L attributes) and
    measure after every `every`-th step past thermalisation.

    Returns dict of arrays: H (total energy), M0, Mk2 (|M(k1)|^2 + |M(k2)|^2) / 2."""
    sweeps = np.full(n_metropolis, float(T))
    one = np.array([float(T)])
    H, M0, Mk2 = [], [], []
    for k in range(n_therm + n_emcs):
        lat.sweep(sweeps)
        lat.sw(one)
        if k >= n_therm and (k - n_therm + 1) % every == 0:
            f = lat.fourier()
            H.append(-lat.J * float(f["bond"]) + lat.Delta * float(f["sum_s2"]))
            M0.append(float(f["sum_s"]))
            Mk2.append(0.5 * (abs(f["k1"]) ** 2 + abs(f["k2"]) ** 2))
    return {"H": np.array(H), "M0": np.array(M0), "Mk2": np.array(Mk2)}


def emcs_runs(lats, T, n_emcs, every=1, n_therm=0, n_metropolis=EMCS_METROPOLIS):
    """emcs_run for several independent lattices, advanced step by step in
    turn so that lattices on different streams overlap on the device.
    Returns one sample dict per lattice."""
    sweeps = np.full(n_metropolis, float(T))
    one = np.array([float(T)])
    out = [{"H": [], "M0": [], "Mk2": []} for _ in lats]
    for k in range(n_therm + n_emcs):
        for lat in lats:
            lat.sweep(sweeps)
            lat.sw(one)
        if k >= n_therm and (k - n_therm + 1) % every == 0:
            for lat, o in zip(lats, out):
                f = lat.fourier()
                o["H"].append(-lat.J * float(f["bond"]) + lat.Delta * float(f["sum_s2"]))
                o["M0"].append(float(f["sum_s"]))
                o["Mk2"].append(0.5 * (abs(f["k1"]) ** 2 + abs(f["k2"]) ** 2))
    return [{k: np.array(v) for k, v in o.items()} for o in out]


def emcs_batch(model, L, seeds, T, n_emcs, every=1, n_therm=0, n_metropolis=EMCS_METROPOLIS, J=1.0, Delta=0.0):
    """emcs_run for independent lattices of one size (one per seed, from the
    T = infinity start) held in one batch: each elementary step is one batched
    run of n_metropolis sweeps and one batched Swendsen-Wang step, each
    measurement one batched Fourier call.  Lattice k draws the random numbers
    it would draw alone (seed k, sweep index from 0), so the samples equal
    emcs_run's on the same lattices.  Returns one sample dict per lattice."""
    from . import Batch
    n_steps = (n_therm + n_emcs) * (n_metropolis + 1)
    Ts = np.full((1, max(n_steps, 1)), float(T))
    reps = [dict(model=model, L=L, seed=int(s), J=J, Delta=Delta, schedule=0) for s in seeds]
    b = Batch(reps, Ts).init_random()
    out = [{"H": [], "M0": [], "Mk2": []} for _ in seeds]
    try:
        for k in range(n_therm + n_emcs):
            if n_metropolis > 0:
                b.run(n_metropolis)
            b.sw()
            if k >= n_therm and (k - n_therm + 1) % every == 0:
                for o, f in zip(out, b.fourier_all()):
                    o["H"].append(-J * float(f["bond"]) + Delta * float(f["sum_s2"]))
                    o["M0"].append(float(f["sum_s"]))
                    o["Mk2"].append(0.5 * (abs(f["k1"]) ** 2 + abs(f["k2"]) ** 2))
    finally:
        b.close()
    return [{k: np.array(v) for k, v in o.items()} for o in out]


def jackknife_observables(runs, L, beta0, beta=None):
    """U4 and xi_2 / L at beta (default beta0) with jackknife errors over runs."""
    full = observables(concat(runs), L, beta0, beta)
    out = {"U4": full["U4"], "xi2_over_L": full["xi2_over_L"]}
    if len(runs) > 1:
        loo = [observables(concat(runs[:k] + runs[k + 1:]), L, beta0, beta) for k in range(len(runs))]
        for key in ("U4", "xi2_over_L"):
            out[key + "_err"] = float(jackknife_error(np.array([o[key] for o in loo])))
    return out


def constant_fit(values, errors):
    """Weighted mean of estimates with errors (the paper's fit of beta_{L,g}
    to a constant over L): (mean, error, chi^2 / dof)."""
    v = np.asarray(values, dtype=np.float64)
    w = 1.0 / np.asarray(errors, dtype=np.float64) ** 2
    mean = float((w * v).sum() / w.sum())
    err = float(1.0 / math.sqrt(w.sum()))
    dof = v.shape[0] - 1
    chi2 = float((w * (v - mean) ** 2).sum())
    return mean, err, (chi2 / dof if dof > 0 else float("nan"))


def _weights(H, beta0, beta, w0=None):
    x = -(beta - beta0) * np.asarray(H, dtype=np.float64)
    w = np.exp(x - x.max())
    if w0 is not None:
        w = w * np.asarray(w0, dtype=np.float64)
    return w / w.sum()


def observables(sample, L, beta0, beta=None, w0=None):
    """U4, xi_2, xi_2 / L, chi(0) and chi_kmin of one sample (dict of arrays H,
    M0, Mk2, as emcs_run returns, or several runs concatenated), reweighted
    from beta0 to beta (default: no reweighting).  w0: optional prior weight
    of each entry (1 for Monte Carlo samples)."""
    beta = beta0 if beta is None else beta
    w = _weights(sample["H"], beta0, beta, w0)
    M0 = np.asarray(sample["M0"], dtype=np.float64)
    M2 = float((w * M0 ** 2).sum())
    M4 = float((w * M0 ** 4).sum())
    Mk2 = float((w * np.asarray(sample["Mk2"], dtype=np.float64)).sum())
    N = float(L) * float(L)
    chi0, chik = M2 / N, Mk2 / N
    ratio = chi0 / chik - 1.0 if chik > 0 else float("nan")
    xi2 = math.sqrt(ratio) / (2.0 * math.sin(math.pi / L)) if ratio >= 0 else float("nan")
    return {"U4": M4 / (M2 * M2), "xi2": xi2, "xi2_over_L": xi2 / L, "chi0": chi0, "chi_kmin": chik}


def reweight_window(sample, n_sigma=2.0):
    """Half-width in beta over which single-histogram reweighting is trusted:
    n_sigma / sigma(H), the shift that moves the mean energy by about n_sigma
    standard deviations."""
    s = float(np.std(np.asarray(sample["H"], dtype=np.float64)))
    return n_sigma / s if s > 0 else 0.0


def beta_crossing(sample, L, beta0, key, target, half_width, w0=None):
    """beta in [beta0 - half_width, beta0 + half_width] where the reweighted
    observable `key` ('U4' or 'xi2_over_L') equals target (Brent's method on
    a bracketing grid), or None when it does not cross there."""
    from scipy.optimize import brentq

    def f(b):
        return observables(sample, L, beta0, b, w0)[key] - target

    grid = np.linspace(beta0 - half_width, beta0 + half_width, 33)
    vals = [f(b) for b in grid]
    for a, b, fa, fb in zip(grid, grid[1:], vals, vals[1:]):
        if fa == 0.0:
            return float(a)
        if np.isfinite(fa) and np.isfinite(fb) and fa * fb < 0:
            return float(brentq(f, a, b, xtol=1e-12, rtol=1e-14))
    return None


def concat(runs):
    return {k: np.concatenate([r[k] for r in runs]) for k in ("H", "M0", "Mk2")}


def crossings(runs, L, beta0, half_width=None):
    """beta_{L,U} and beta_{L,xi2/L} from independent runs at beta0 with
    jackknife errors over runs (each leave-one-out sample reweighted again).
    Returns dict(beta_U, beta_U_err, beta_xi, beta_xi_err, U4, xi2_over_L,
    half_width)."""
    full = concat(runs)
    hw = reweight_window(full) if half_width is None else half_width
    out = {"half_width": hw}
    obs = observables(full, L, beta0)
    out["U4"], out["xi2_over_L"] = obs["U4"], obs["xi2_over_L"]
    for name, key, target in (("beta_U", "U4", U4_STAR), ("beta_xi", "xi2_over_L", XI_OVER_L_STAR)):
        b = beta_crossing(full, L, beta0, key, target, hw)
        out[name] = b
        out[name + "_err"] = None
        if b is None or len(runs) < 2:
            continue
        blocks = []
        for k in range(len(runs)):
            bk = beta_crossing(concat(runs[:k] + runs[k + 1:]), L, beta0, key, target, hw)
            if bk is None:
                blocks = None
                break
            blocks.append(bk)
        if blocks is not None:
            out[name + "_err"] = float(jackknife_error(np.array(blocks)))
    return out
