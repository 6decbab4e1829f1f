"""Seeded synthetic inputs shared by the library's users, the tests and the
benchmark: seeds, bath temperatures, separation sets and workload mixes.

Holds none of the dynamics' arithmetic (no thresholds, no schedules, no
observables); both the HIP path and the CPU oracle receive these inputs.
The paper's workloads are synthetic by construction (disordered T = infinity
starts, paper Thermal protocols), so nothing here stands in for a dataset.
"""
import math

import numpy as np

SEED_BASE = 2503146880

# Ising T_c = 2 / ln(1 + sqrt 2) (paper, Models); Blume-Capel (Delta = 0)
# T_c as simulated in Table I; the L = 2^18 Blume-Capel workload runs at
# T = 1.6937 as specified for it.
TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))
TC_BC = 1.69355839821214427017
T_BC_WORKLOAD = 1.6937


def seed_for(k: int) -> int:
    """Seed of replica or job k."""
    return SEED_BASE + int(k)


def r_sparse(L: int, r_max: int = 4096):
    """Sparse separations: r = 1..16 and round(16 * 2^(k/4)), k = 1..32,
    capped at min(r_max, L / 2) (the paper samples C(r) sparsely, App. C)."""
    cap = min(r_max, L // 2)
    rs = set(range(1, 17))
    for k in range(1, 33):
        rs.add(int(round(16.0 * 2.0 ** (k / 4.0))))
    return np.array(sorted(r for r in rs if r <= cap), dtype=np.uint32)


def r_dense(L: int):
    """Every separation 1..L/2."""
    return np.arange(1, L // 2 + 1, dtype=np.uint32)


def measure_times(n_sweeps: int):
    """Measurement points: after 0 sweeps and after 2^k sweeps."""
    ts = [0]
    k = 1
    while k <= n_sweeps:
        ts.append(k)
        k *= 2
    return ts


# Workloads (the sizes and parameters of the benchmark configurations).
ISING_SMALL = dict(name="ising_L64_tc", model=0, L=64, sweeps=1024, T=TC_ISING, seed=SEED_BASE)
ISING_LARGE = dict(name="ising_L1048576_tc", model=0, L=1 << 20, sweeps=64, T=TC_ISING, seed=SEED_BASE)
ISING_CHECK = dict(name="ising_L4096_tc", model=0, L=1 << 12, sweeps=64, T=TC_ISING, seed=SEED_BASE)
BC_LARGE = dict(name="bc_L262144_t16937", model=1, L=1 << 18, sweeps=256, T=T_BC_WORKLOAD, seed=SEED_BASE,
                J=1.0, Delta=0.0)
BC_CHECK = dict(name="bc_L4096_t16937", model=1, L=1 << 12, sweeps=256, T=T_BC_WORKLOAD, seed=SEED_BASE,
                J=1.0, Delta=0.0)


# The paper's second protocol for the Ising model (Thermal protocols;
# Table II): L = 2^16, disordered start at T1 = 1.66 (about 0.73 T_c), switch
# to T2 = 2.27414861561203, whose equilibrium coherence length the paper gives
# as 407(1) lattice spacings, when xi(t; T1) = f xi_eq(T2).  Table II lists the
# switch times 3746, 4467, 5312 (read as f = 0.54, 0.59, 0.64 in that order:
# a longer stay at T1 reaches a larger xi).  The benchmark follows each f to
# t_max = 8192 sweeps (the paper goes to 3,000,000).
# t_switch(f) comes from an ensemble of `replicas` quenches at T1 (the App. C
# estimator), measured on a grid of 8 times per octave up to t_limit.
PROTOCOL2_ISING = dict(name="protocol2_ising_L65536", model=0, L=1 << 16, T1=1.66, T2=2.27414861561203,
                       xi_eq=407.0, f=(0.54, 0.59, 0.64), t_switch_paper=(3746, 4467, 5312), t_max=8192,
                       t_limit=8192, replicas=4, seed=SEED_BASE)
# The same for Blume-Capel (Delta = 0; Table II): T1 = 1.24, T2 = 1.69661396797728
# with xi_eq(T2) = 405(2), switch times 34540, 41270, 48599 at L = 2^16.  Run
# here at L = 2^14 (L / xi_eq = 40) to keep the benchmark within minutes, and
# each two-step run followed to 4096 sweeps past the latest switch.
PROTOCOL2_BC = dict(name="protocol2_bc_L16384", model=1, L=1 << 14, T1=1.24, T2=1.69661396797728,
                    xi_eq=405.0, f=(0.54, 0.59, 0.64), t_switch_paper=(34540, 41270, 48599), t_max=None,
                    t_after=4096, t_limit=65536, replicas=4, seed=SEED_BASE + 7)


# Ensemble of direct quenches for the analysis of App. C and D: 128 Ising
# replicas of L = 4096 at T_c measured on a grid of two times per octave up to
# t = 8192 (xi = I2 / I1 grows to about 170, L / xi about 24), z fitted from
# t = 256 on.
ENSEMBLE_ISING = dict(name="ensemble_ising_L4096_tc", model=0, L=1 << 12, replicas=128, T=TC_ISING,
                      t_max=8192, per_octave=2, fit_from=256, seed0=1000)
# The same for Blume-Capel (Delta = 0) at its T_c (Table I): the paper's
# universality claim is one z for both models.
ENSEMBLE_BC = dict(name="ensemble_bc_L4096_tc", model=1, L=1 << 12, replicas=128, T=TC_BC,
                   t_max=8192, per_octave=2, fit_from=256, seed0=2000)


# Equilibrium finite-size study of the Blume-Capel critical temperature
# (App. B): Delta = 0, 16 independent runs per L from the T = infinity start
# at the paper's T_c, elementary Monte Carlo step = 10 Metropolis sweeps + one
# Swendsen-Wang step, 40 EMCS of thermalisation (the paper's equilibration
# time at L = 4096), then 2000 EMCS measured after every step (the paper: L up
# to 4096, 100 runs of 4 x 10^5 EMCS each).
EQUILIBRIUM_BC = dict(name="equilibrium_bc_tc", model=1, sizes=(64, 128, 256, 512, 1024, 2048, 4096), runs=16,
                      n_therm=40, n_emcs=2000, every=1, T=TC_BC, seed0=3000)


def batched_replicas(n=512, sizes=(256, 512, 1024, 2048), taus=(64.0, 256.0, 1024.0)):
    """Replica descriptors of the batched exponential-schedule workload:
    uniform mix of sizes, half Ising and half Blume-Capel (Delta = 0), tau
    round-robin, T0 = 2 T_c and T_f = 1.02 T_c with each model's own T_c."""
    reps = []
    for k in range(n):
        model = k % 2
        L = sizes[(k // 2) % len(sizes)]
        tau = taus[k % len(taus)]
        tc = TC_ISING if model == 0 else TC_BC
        reps.append(dict(id=k, model=model, L=L, seed=seed_for(k), J=1.0, Delta=0.0,
                         T0=2.0 * tc, Tf=1.02 * tc, tau=tau))
    return reps


def serving_jobs(n, rate_per_s, seed=SEED_BASE, log2_L=(8, 14), log2_sweeps=(10, 14)):
    """Poisson stream of quench jobs: arrival times (s), L = 2^U with U uniform
    in log2_L, model Bernoulli(1/2), sweeps 2^V with V uniform in
    log2_sweeps, each at its model's T_c."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for k in range(n):
        model = int(rng.integers(0, 2))
        L = 1 << int(rng.integers(log2_L[0], log2_L[1] + 1))
        sweeps = 1 << int(rng.integers(log2_sweeps[0], log2_sweeps[1] + 1))
        jobs.append(dict(id=k, arrival=float(arrivals[k]), model=model, L=L, sweeps=sweeps,
                         seed=seed_for(10_000_000 + k), J=1.0, Delta=0.0,
                         T=TC_ISING if model == 0 else TC_BC))
    return jobs
