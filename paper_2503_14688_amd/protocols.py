"""The paper's two thermal protocols (Thermal protocols; Table II) as host
drivers over the library's sweep, measure and batch calls.

Protocol 1, the direct quench: a disordered (T = infinity) start evolves in a
bath at T from t = 0, and E, M, C(r) and xi are measured at chosen sweep
counts.

Protocol 2, pre-cooling: the disordered start evolves at T1 < T_c until
t_switch and in a bath at T2 >= T_c afterwards.  The switch is characterised
by the fraction f of the equilibrium coherence length at T2 that the system
has reached at T1: xi(t_switch; T1) = f xi_eq(T2).  Every random number is
keyed by (seed, row, word, sweep index, colour), so runs with the same seed
follow one trajectory up to their switch: the T1 run that locates t_switch(f)
is the common prefix of the two-step runs for every f.

Every sweep and every sum runs in the HIP library; this module only chooses
temperatures and measurement times and reads the results.  A lattice argument
is anything with the Lattice interface (sweep(T array), measure(r), t).
"""
import math

import numpy as np

from . import SCHEDULE_TWO_STEP, Batch, spin_schedule_fill


def log_times(t_max, per_octave=4):
    """Measurement times: 0, the distinct round(2^(k / per_octave)) for k >= 0
    below t_max, and t_max."""
    if t_max < 0 or per_octave < 1:
        raise ValueError("need t_max >= 0 and per_octave >= 1")
    ts = {0, int(t_max)}
    k = 0
    while True:
        t = int(round(2.0 ** (k / per_octave)))
        if t >= t_max:
            break
        ts.add(t)
        k += 1
    return sorted(ts)


def crossing_time(times, values, target):
    """First sweep count at which a measured series reaches target.

    Between the last measurement below target and the first at or above it
    the series is interpolated linearly in (log t, log value) (in t when the
    earlier point is t = 0 or a value is not positive), and the crossing is
    rounded up to a whole sweep.  Returns None if the series never reaches
    target, times[0] if it starts there."""
    times = [int(t) for t in times]
    values = [float(v) for v in values]
    if len(times) != len(values) or not times:
        raise ValueError("times and values must be non-empty and of equal length")
    if any(b <= a for a, b in zip(times, times[1:])):
        raise ValueError("times must increase")
    if values[0] >= target:
        return times[0]
    for k in range(1, len(times)):
        if values[k] < target:
            continue
        t0, t1, v0, v1 = times[k - 1], times[k], values[k - 1], values[k]
        if t0 > 0 and v0 > 0.0 and target > 0.0:
            a = (math.log(target) - math.log(v0)) / (math.log(v1) - math.log(v0)) if v1 != v0 else 1.0
            t = math.exp(math.log(t0) + a * (math.log(t1) - math.log(t0)))
        else:
            a = (target - v0) / (v1 - v0) if v1 != v0 else 1.0
            t = t0 + a * (t1 - t0)
        return min(t1, max(t0 + 1, int(math.ceil(t - 1e-9))))
    return None


def _keep(m):
    return {"t": int(m["t"]), "e": float(m["e"]), "m": float(m["m"]), "xi": float(m["xi"])}


def series(lat, T_of_t, times, r, full=False):
    """Advance lat (at sweep lat.t) through the bath temperatures T_of_t
    (indexed by the absolute sweep index) and measure at every sweep count in
    times (each >= lat.t).  Returns one dict per time: t, e, m, xi (and the
    whole measurement when full)."""
    out = []
    for t in times:
        n = int(t) - lat.t
        if n < 0:
            raise ValueError(f"time {t} is before the lattice's sweep count {lat.t}")
        if n:
            lat.sweep(np.ascontiguousarray(T_of_t[lat.t:int(t)], dtype=np.float64), fuse_measure=True)
        m = lat.measure(r)
        out.append(m if full else _keep(m))
    return out


def switch_times(lat, T1, fs, xi_eq, r, t_limit, per_octave=8):
    """Protocol 1 at T1 on lat (normally the T = infinity start, t = 0),
    measuring xi on a log grid until xi >= max(fs) xi_eq or t_limit.

    Returns ({f: t_switch or None}, the measured series)."""
    target_max = max(fs) * xi_eq
    T = np.full(int(t_limit), float(T1))
    done = []
    for t in log_times(t_limit, per_octave):
        if t < lat.t:
            continue
        done += series(lat, T, [t], r)
        if done[-1]["xi"] >= target_max:
            break
    ts, xs = [m["t"] for m in done], [m["xi"] for m in done]
    return {f: crossing_time(ts, xs, f * xi_eq) for f in fs}, done


def ensemble_xi_series(data, r, L):
    """xi(t) by the App. C recipe with jackknife errors, from the per-time
    ensemble data of quench_batch.  window_ok reports whether the cut points
    satisfy r* < r_min < r_max < r_cut (the paper adds statistics where they
    do not)."""
    from . import analysis
    out = []
    for d in data:
        C = (np.asarray(d["Sx"], dtype=np.float64) + np.asarray(d["Sy"], dtype=np.float64)) / (2.0 * L * L)
        xi, err, full, _ = analysis.xi_ensemble(r, C, np.asarray(d["sum_s2"], dtype=np.float64) / (float(L) * L))
        out.append({"t": int(d["t"]), "xi": float(xi), "xi_err": float(err), "window_ok": bool(full["ok"]),
                    "r_cut": int(full["r_cut"])})
    return out


def switch_times_from_series(series, fs, xi_eq):
    """t_switch(f) = first crossing of f xi_eq by an ensemble series (points
    where xi is not defined are left out)."""
    pts = [(m["t"], m["xi"]) for m in series if m["t"] >= 1 and math.isfinite(m["xi"]) and m["xi"] > 0]
    ts, xs = [p[0] for p in pts], [p[1] for p in pts]
    return {f: crossing_time(ts, xs, f * xi_eq) if pts else None for f in fs}


def switch_times_ensemble(model, L, seeds, T1, fs, xi_eq, r, t_limit, per_octave=8, J=1.0, Delta=0.0):
    """t_switch(f) from an ensemble of protocol-1 runs at T1 (one replica per
    seed, one batch): xi(t) of the replica-averaged C(r) by the App. C
    recipe, whose cut-off r_cut follows the statistical errors, crossed with
    f xi_eq(T2) as in switch_times.  Returns ({f: t_switch or None}, series)."""
    times = [t for t in log_times(t_limit, per_octave) if t >= 1]
    data = quench_batch(model, L, seeds, T1, times, r, J, Delta)
    series = ensemble_xi_series(data, r, L)
    return switch_times_from_series(series, fs, xi_eq), series


def two_step_temperatures(T1, T2, t_switch, n):
    """T(t) of protocol 2 for t = 0 .. n - 1 (T1 before t_switch, then T2)."""
    return spin_schedule_fill(SCHEDULE_TWO_STEP, [T1, t_switch, T2], 0, n)


def two_step_series(lat, T1, T2, t_switch, times, r, full=False):
    """Protocol 2 on lat from its current sweep count (normally 0)."""
    return series(lat, two_step_temperatures(T1, T2, t_switch, int(max(times))), times, r, full)


def two_step_batch(model, L, seeds, T1, T2, t_switches, times, r, J=1.0, Delta=0.0):
    """Protocol 2 for every (seed, t_switch) pair as one batch of replicas
    (one launch per half-sweep covers them all).  Returns, per replica, the
    list of measurements (t, e, m, xi) at times."""
    if len(seeds) != len(t_switches):
        raise ValueError("one t_switch per seed")
    t_max = int(max(times))
    T = np.stack([two_step_temperatures(T1, T2, ts, t_max) for ts in t_switches])
    reps = [dict(model=model, L=L, seed=int(s), J=J, Delta=Delta, schedule=k) for k, s in enumerate(seeds)]
    b = Batch(reps, T).init_random()
    out = [[] for _ in reps]
    t_now = 0
    try:
        for t in times:
            if int(t) > t_now:
                b.run(int(t) - t_now)
                t_now = int(t)
            for k, m in enumerate(b.measure_all(r)):
                out[k].append(_keep(m))
    finally:
        b.close()
    return out


def quench_batch(model, L, seeds, T, times, r, J=1.0, Delta=0.0):
    """Protocol 1 for an ensemble of replicas (one per seed) as one batch.

    Returns, per measurement time, a dict with t and the per-replica arrays
    Sx, Sy (n_replicas, len(r)), sum_s2, e, m (n_replicas,): the input of the
    ensemble analysis (jackknife over replicas)."""
    t_max = int(max(times))
    Tm = np.full((1, max(t_max, 1)), float(T))
    reps = [dict(model=model, L=L, seed=int(s), J=J, Delta=Delta, schedule=0) for s in seeds]
    b = Batch(reps, Tm).init_random()
    out = []
    t_now = 0
    try:
        for t in times:
            if int(t) > t_now:
                b.run(int(t) - t_now)
                t_now = int(t)
            ms = b.measure_all(r)
            out.append({"t": t_now,
                        "Sx": np.stack([m["Sx"] for m in ms]), "Sy": np.stack([m["Sy"] for m in ms]),
                        "sum_s2": np.array([m["sum_s2"] for m in ms], dtype=np.float64),
                        "e": np.array([m["e"] for m in ms]), "m": np.array([m["m"] for m in ms])})
    finally:
        b.close()
    return out
