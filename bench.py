"""Benchmark of the checkerboard Metropolis hot path on one MI355X.

Workload (default): Ising, L = 2^20 (1.1e12 spins, 128 GiB packed), T = infinity
start, quench at T_c.  One step is one sweep at T_c; the timed region covers
`--steps` sweeps and, inside it, the measurements (energy, magnetisation and
C(r) on the sparse separation set up to r = 4096, both axes) at every sweep
count 2^k reached.  `--warmup` sweeps (and one measurement) run untimed
first.  Inputs are resident in HBM before timing starts.

Prints one JSON line: throughput in attempted spin flips per ns, the
roofline of the half-sweep kernel (algorithmic HBM bytes per launch over its
measured duration, against 8 TB/s), and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "attempted spin flips/ns @1 GPU + % HBM roofline; batched vs plain replica-sweeps/s"
HBM_PEAK_GBS = 8000.0


# HBM traffic of the half-sweep kernel per launch, from two rocprofv3 counter
# passes (FETCH_SIZE, WRITE_SIZE) scaled by a plain-copy calibration, recorded
# in profiles/k_sweep_traffic_ising_L1048576_bc_L262144.txt.  Valid only for
# the sweep sources it was taken with (their SHA-256 below, first 16 hex
# digits); any change to those sources makes the bench report null.
SWEEP_SOURCES = ["paper_2503_14688_amd/csrc/kernels.hip", "paper_2503_14688_amd/csrc/sweep_tiles.hpp",
                 "paper_2503_14688_amd/csrc/device.hpp", "paper_2503_14688_amd/csrc/kernels.hpp"]
MEASURED_TRAFFIC = {
    # (workload, sweep strategy): bytes per launch
    ("ising_L1048576_tc", 2): 225.22e9,
    ("bc_L262144_t16937", 0): 28.53e9,
    ("bc_L262144_t16937", 1): 27.25e9,
}
MEASURED_WITH = "cbe525478358cd34"
# (workload, sweep strategy): wave instructions per 64 words of a colour plane
# (SQ_INSTS_VALU, SQ_INSTS_SALU) and the clock (GHz, GRBM_GUI_ACTIVE over the
# dispatch) from the same counter pass
MEASURED_ISSUE = {
    ("ising_L1048576_tc", 2): (125.8, 84.9, 2.05),
    ("bc_L262144_t16937", 0): (248.3, 219.6, 2.23),
    ("bc_L262144_t16937", 1): (233.2, 170.8, 2.08),
}


def sweep_sources_hash():
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, strategy):
    if sweep_sources_hash() != MEASURED_WITH:
        return None
    return MEASURED_TRAFFIC.get((workload, strategy))


def issue_busy(workload, strategy, words_per_launch, launch_s):
    """Busy fractions of the vector and scalar issue of the sweep kernel:
    measured wave instructions per 64 words x words per launch over the
    launch's cycles (1024 SIMDs at one vector instruction per 4 cycles; 256
    scalar units at one instruction per cycle; clock as measured with the
    counters).  None unless the counters were taken on these sources."""
    if sweep_sources_hash() != MEASURED_WITH or (workload, strategy) not in MEASURED_ISSUE:
        return None
    valu, salu, ghz = MEASURED_ISSUE[(workload, strategy)]
    cycles = launch_s * ghz * 1e9
    waves = words_per_launch / 64.0
    return {"valu": round(valu * waves * 4 / (1024 * cycles), 3), "salu": round(salu * waves / (256 * cycles), 3),
            "clock_ghz": ghz, "source": "profiles/issue_rates_ising_L1048576_bc_L262144.txt",
            "note": "valu counts 4 cycles per vector instruction; two-operand forms issue in 2, so above 1 is possible"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_half_sweep(model, L):
    # read own colour plane + write it back + read the other colour plane
    plane = (L * L // 2) * (1 if model == 0 else 2) // 8
    return 3 * plane


def cpu_baseline(workload, budget_s=12.0):
    """The oracle as it stands, on the host's cores, on an L = 4096 sample."""
    import oracle
    L = 4096
    model = workload["model"]
    T = workload["T"]
    s = oracle.init(model, L, workload["seed"])
    threads = oracle.num_threads()
    done = 0
    t0 = time.perf_counter()
    while done < 4096:
        oracle.sweep(model, s, workload["seed"], workload.get("J", 1.0), workload.get("Delta", 0.0), done,
                     np.array([T]))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done * L * L / (dt * 1e9), "unit": "flips/ns", "cores": threads, "kind": "oracle",
            "sample": f"{workload['name'].split('_')[0]} L=4096 (2^24 spins), {done} sweeps at the workload's T "
                      f"from the T=inf start, sweeps only, {threads} OpenMP threads, {dt:.1f} s"}


def run_batched(args):
    """512 replicas (L in {256..2048}, half Ising half Blume-Capel, own
    exponential schedules): the batched engine over the full schedule, and
    batched vs the plain per-replica launch loop over the same first sweeps."""
    import torch
    import paper_2503_14688_amd as spin
    from paper_2503_14688_amd import workloads

    reps = workloads.batched_replicas(args.replicas)
    n_steps = args.batch_sweeps
    keys = sorted({(r["model"], r["tau"]) for r in reps})
    rows = []
    for (model, tau) in keys:
        tc = workloads.TC_ISING if model == 0 else workloads.TC_BC
        rows.append(spin.spin_schedule_fill(spin.SCHEDULE_EXPONENTIAL, [2.0 * tc, 1.02 * tc, tau], 0, n_steps))
    T = np.stack(rows)
    for r in reps:
        r["schedule"] = keys.index((r["model"], r["tau"]))
    flips_per_sweep = sum(r["L"] * r["L"] for r in reps)

    b = spin.Batch(reps, T).init_random()
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(n_steps)
    b.sync()
    full_s = time.perf_counter() - t0
    info = b.info()
    log(f"batched: {args.replicas} replicas x {n_steps} sweeps in {full_s:.3f} s (strategy {info['variant']})")
    b.close()

    cmp_sweeps = min(args.compare_sweeps, n_steps)
    b = spin.Batch(reps, T).init_random()
    b.run(1)  # tile-shape choice and graph warm-up outside the timed range
    b.sync()
    b.close()
    b = spin.Batch(reps, T).init_random()
    b.sync()
    t0 = time.perf_counter()
    b.run(cmp_sweeps, spin.BATCH_VARIANT(info["variant"]))
    b.sync()
    batched_s = time.perf_counter() - t0
    plain = [spin.Lattice(r["model"], r["L"], r["seed"], r["J"], r["Delta"]).init_random() for r in reps]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat, r in zip(plain, reps):
        lat.sweep(T[r["schedule"], :cmp_sweeps])
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    same = all(np.array_equal(b.spins(k), plain[k].spins()) for k in range(0, len(reps), max(1, len(reps) // 16)))
    log(f"plain loop: {cmp_sweeps} sweeps in {plain_s:.3f} s vs batched {batched_s:.3f} s; identical: {same}")
    for lat in plain:
        lat.close()
    b.close()
    n = len(reps)
    return {"workload": f"{n} replicas, L in {{256,512,1024,2048}}, half Ising half Blume-Capel, "
                        f"T(t) = Tf + (T0 - Tf) exp(-t/tau), tau in {{64,256,1024}}",
            "replica_sweeps_per_s": round(n * n_steps / full_s, 1), "sweeps": n_steps,
            "flips_per_ns": round(flips_per_sweep * n_steps / full_s / 1e9, 2), "strategy": info["variant"],
            "compare_sweeps": cmp_sweeps,
            "batched_replica_sweeps_per_s": round(n * cmp_sweeps / batched_s, 1),
            "plain_replica_sweeps_per_s": round(n * cmp_sweeps / plain_s, 1),
            "ratio": round(plain_s / batched_s, 2), "identical_results": bool(same)}


def run_serving(args, saturated_flips_per_ns):
    """Poisson stream of quench jobs through the continuous-batching server."""
    from paper_2503_14688_amd import workloads
    from paper_2503_14688_amd.serve import Job, Server

    mean_L2 = np.mean([4.0 ** u for u in range(8, 15)])
    mean_sweeps = np.mean([2.0 ** v for v in range(10, 15)])
    mean_job_s = mean_L2 * mean_sweeps / (saturated_flips_per_ns * 1e9)
    rate = 0.8 / mean_job_s  # arrivals that keep the device 80 % busy
    jobs = [Job(**d) for d in workloads.serving_jobs(args.jobs, rate)]
    srv = Server(epoch=64)
    stats = srv.run(jobs)
    log(f"serving: {stats['jobs']} jobs in {stats['wall_s']:.2f} s, p50 {stats['latency_p50_s']:.3f} s, "
        f"p99 {stats['latency_p99_s']:.3f} s")
    # capacity: the same jobs all queued at once (offered load above one), so
    # the device never waits for arrivals
    jobs = [Job(**dict(d, arrival=0.0)) for d in workloads.serving_jobs(args.jobs, rate)]
    cap = Server(epoch=64).run(jobs, realtime=False)
    log(f"serving at capacity: {cap['jobs']} jobs in {cap['wall_s']:.2f} s, {cap['flips_per_ns']:.0f} flips/ns")
    stats["capacity"] = {"jobs_per_s": round(cap["jobs_per_s"], 3), "flips_per_ns": round(cap["flips_per_ns"], 1),
                         "fraction_of_batched_engine": round(cap["flips_per_ns"] / saturated_flips_per_ns, 3),
                         "latency_p50_s": round(cap["latency_p50_s"], 3), "batches_built": cap["batches_built"],
                         "note": "all jobs queued at t = 0"}
    stats.update({"arrival_rate_per_s": round(rate, 3), "offered_load": 0.8,
                  "workload": "Poisson arrivals, L = 2^U (U uniform 8..14), sweeps 2^V (V uniform 10..14), "
                              "Ising or Blume-Capel at T_c, admitted by slots and 80% of free HBM"})
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}


def _protocol2(wl):
    """The paper's pre-cooling protocol for one model: an ensemble of quenches
    at T1 (one batch) locates t_switch(f) where the App. C coherence length
    reaches f xi_eq(T2); then the three two-step runs (one seed, so one
    trajectory up to each switch) run to t_max as one batch.  flips_per_ns:
    all attempted flips of both phases over the wall time."""
    import torch
    from paper_2503_14688_amd import protocols, workloads
    L, seed, T1, T2, fs = wl["L"], wl["seed"], wl["T1"], wl["T2"], wl["f"]
    r = workloads.r_sparse(L)
    seeds = [seed + k for k in range(wl["replicas"])]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_sw, series = protocols.switch_times_ensemble(wl["model"], L, seeds, T1, fs, wl["xi_eq"], r, wl["t_limit"])
    torch.cuda.synchronize()
    wall_a = time.perf_counter() - wall0
    sweeps_a = max(m["t"] for m in series)
    if any(t_sw[f] is None for f in fs):
        raise RuntimeError(f"xi did not reach f xi_eq within {wl['t_limit']} sweeps at T1: {t_sw}")
    tsw = [t_sw[f] for f in fs]
    t_max = wl["t_max"] if wl["t_max"] else max(tsw) + wl["t_after"]
    times = protocols.log_times(t_max, 4)
    runs = protocols.two_step_batch(wl["model"], L, [seed] * len(fs), T1, T2, tsw, times, r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    flips = float(L) * L * (len(seeds) * sweeps_a + len(fs) * t_max)
    log(f"protocol 2 {wl['name']}: t_switch {tsw} (paper {list(wl['t_switch_paper'])}), "
        f"{flips / wall / 1e9:.1f} flips/ns")
    pick = [m for m in series if m["t"] in (256, 1024, 4096, 16384, 32768)]
    return {"workload": wl["name"], "L": L, "T1": T1, "T2": T2, "xi_eq_T2": wl["xi_eq"], "f": list(fs),
            "t_switch": tsw, "t_switch_paper": list(wl["t_switch_paper"]),
            "t_switch_estimator": f"ensemble of {len(seeds)} quenches at T1, App. C xi with jackknife errors",
            "xi_at_T1": {str(m["t"]): [round(m["xi"], 3), round(m["xi_err"], 3)] for m in pick},
            "window_ok_fraction": round(float(np.mean([m["window_ok"] for m in series if m["t"] >= 16])), 3),
            "t_max": t_max, "sweeps_at_T1": sweeps_a, "wall_s": round(wall, 3),
            "wall_T1_ensemble_s": round(wall_a, 3), "measurements_at_T1": len(series),
            "flips_per_ns": round(flips / wall / 1e9, 2),
            "E_at_t_max": [round(run[-1]["e"], 6) for run in runs],
            "xi_at_t_max": [round(run[-1]["xi"], 2) for run in runs]}


def run_protocol2(args):
    from paper_2503_14688_amd import workloads
    out = _protocol2(workloads.PROTOCOL2_ISING)
    try:
        out["blume_capel"] = _protocol2(workloads.PROTOCOL2_BC)
    except Exception as exc:  # noqa: BLE001
        log(f"protocol 2 (Blume-Capel) failed: {exc!r}")
        out["blume_capel"] = {"error": repr(exc)}
    return out


def _fit_summary(fit, window):
    return {"z": round(fit["z"], 4), "z_err": round(fit["z_err"], 4) if fit["z_err"] is not None else None,
            "chi2_dof": round(fit["chi2_dof"], 3), "Q": round(fit["Q"], 3), "t_window": window}


def _ensemble_z(wl):
    """One model's ensemble of direct quenches (one batch) with xi(t) by the
    App. C recipe and z from Eq. for log t (with and without the b' xi^-omega
    correction) and, for Ising, from the excess energy (App. D); jackknife
    errors.  Also returns the data sets for the joint fit."""
    import torch
    from paper_2503_14688_amd import analysis, protocols, workloads
    L, n = wl["L"], wl["replicas"]
    r = workloads.r_sparse(L)
    times = [t for t in protocols.log_times(wl["t_max"], wl["per_octave"]) if t >= 1]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    data = protocols.quench_batch(wl["model"], L, [workloads.seed_for(wl["seed0"] + k) for k in range(n)],
                                  wl["T"], times, r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    series = protocols.ensemble_xi_series(data, r, L)
    blocks = []
    for d in data:
        C = (d["Sx"] + d["Sy"]) / (2.0 * L * L)
        blocks.append(analysis.xi_ensemble(r, C, d["sum_s2"] / (float(L) * L))[3])
    xi = np.array([m["xi"] for m in series])
    err = np.array([m["xi_err"] for m in series])
    blocks = np.array(blocks).T
    sel = np.array([t >= wl["fit_from"] for t in times])
    t_sel = np.array(times, dtype=np.float64)[sel]
    window = [wl["fit_from"], wl["t_max"]]
    fit = analysis.fit_z(t_sel, xi[sel], err[sel], blocks[:, sel])
    fit_plain = analysis.fit_z(t_sel, xi[sel], err[sel], blocks[:, sel], correction=False)
    flips = float(L) * L * n * wl["t_max"]
    out = {"workload": wl["name"], "replicas": n, "t_max": wl["t_max"], "wall_s": round(wall, 3),
           "flips_per_ns": round(flips / wall / 1e9, 2),
           "xi": {str(t): [round(float(a), 3), round(float(b), 3)] for t, a, b in zip(times, xi, err)
                  if t in (16, 64, 256, 1024, 4096, 8192)},
           "window_ok": {str(m["t"]): m["window_ok"] for m in series if m["t"] >= wl["fit_from"]},
           "z_fit": _fit_summary(fit, window), "z_fit_without_correction": _fit_summary(fit_plain, window)}
    group = wl["name"]
    sets = [dict(kind="xi", t=t_sel, y=xi[sel], err=err[sel], blocks=blocks[:, sel], group=group)]
    if wl["model"] == 0:
        # excess energy over E_eq(T_c) = -sqrt(2), known exactly for Ising only
        dE = np.array([d["e"] for d in data]).T + math.sqrt(2.0)  # (replicas, times)
        dE_mean, dE_err = dE.mean(axis=0)[sel], dE.std(axis=0, ddof=1)[sel] / math.sqrt(n)
        dE_blocks = analysis.jackknife_means(dE)[:, sel]
        fit_e = analysis.fit_z_energy(t_sel, dE_mean, dE_err, dE_blocks)
        out["z_fit_energy"] = _fit_summary(fit_e, window)
        out["z_fit_energy_without_correction"] = _fit_summary(
            analysis.fit_z_energy(t_sel, dE_mean, dE_err, dE_blocks, correction=False), window)
        sets.append(dict(kind="energy", t=t_sel, y=dE_mean, err=dE_err, blocks=dE_blocks, group=group))
    log(f"ensemble {wl['name']}: z = {fit['z']:.4f} +- {fit['z_err']:.4f} (xi, Q = {fit['Q']:.2f})"
        + (f", {out['z_fit_energy']['z']:.4f} +- {out['z_fit_energy']['z_err']:.4f} (energy)"
           if "z_fit_energy" in out else "") + f", {flips / wall / 1e9:.1f} flips/ns")
    return out, sets


def run_ensemble(args):
    """Ising and Blume-Capel ensembles at their critical temperatures: the
    paper's universality check, one z per model and the joint fit of Ising
    xi, Ising energy and Blume-Capel xi (its value: 2.1676(1))."""
    from paper_2503_14688_amd import analysis, workloads
    out, sets = _ensemble_z(workloads.ENSEMBLE_ISING)
    out["z_paper"] = 2.1676
    out["blume_capel"], bc_sets = _ensemble_z(workloads.ENSEMBLE_BC)
    joint = analysis.fit_z_joint(sets + bc_sets)
    out["z_joint"] = {"z": round(joint["z"], 4), "z_err": round(joint["z_err"], 4),
                      "chi2_dof": round(joint["chi2_dof"], 3), "Q": round(joint["Q"], 3),
                      "data_sets": "Ising xi + Ising energy + Blume-Capel xi"}
    plain = analysis.fit_z_joint(sets + bc_sets, correction=False)
    out["z_joint_without_correction"] = {"z": round(plain["z"], 4), "z_err": round(plain["z_err"], 4),
                                         "chi2_dof": round(plain["chi2_dof"], 3), "Q": round(plain["Q"], 3)}
    log(f"joint z = {joint['z']:.4f} +- {joint['z_err']:.4f} (Q = {joint['Q']:.2f})")
    return out


def single_lattice(wl, steps, warmup, variant=-1):
    """One lattice of workload wl: T = infinity start, `warmup` untimed sweeps
    and one measurement, then `steps` timed sweeps with E, M (fused) and C(r)
    at every sweep count 2^k.  HIP events on the library's stream time each
    sweep; the roofline entry is the half-sweep kernel's."""
    import torch
    import paper_2503_14688_amd as spin
    from paper_2503_14688_amd import workloads

    model, L, T, seed = wl["model"], wl["L"], wl["T"], wl["seed"]
    J, Delta = wl.get("J", 1.0), wl.get("Delta", 0.0)
    r = workloads.r_sparse(L)
    stream = torch.cuda.current_stream()
    lat = spin.Lattice(model, L, seed, J, Delta, stream=stream)
    strategy = lat.tune(T) if variant < 0 else variant
    lat.variant = strategy
    lat.init_random()
    log(f"allocated and initialised {wl['name']} ({lat.buf.numel() / 2**30:.1f} GiB), sweep strategy {strategy}")
    Tk = np.array([T])
    for _ in range(warmup):
        lat.sweep(Tk)
    lat.measure(r)  # loads every kernel once
    torch.cuda.synchronize()
    log(f"warmup done ({warmup} sweeps and one measurement)")

    t_start = lat.t
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    n_meas = 0
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(steps):
        t_after = t_start + k + 1
        measure_now = t_after & (t_after - 1) == 0
        ev[2 * k].record(stream)
        lat.sweep(Tk, fuse_measure=measure_now)
        ev[2 * k + 1].record(stream)
        if measure_now:
            lat.measure(r)
            n_meas += 1
            log(f"measured at t = {t_after}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sweep_ms = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps))
    half_sweep_s = sweep_ms / 1e3 / (2 * steps)
    flips = float(L) * L * steps
    bytes_launch = algorithmic_bytes_per_half_sweep(model, L)
    achieved = bytes_launch / half_sweep_s / 1e9
    traffic = measured_traffic(wl["name"], strategy)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return {
        "value": round(flips / (wall * 1e9), 3), "wall_s": wall, "steps": steps,
        "ms_per_step": round(wall * 1e3 / steps, 3),
        "config": {"workload": wl["name"], "model": "ising" if model == 0 else "blume-capel", "L": L,
                   "spins": L * L, "T": T, "J": J, "Delta": Delta, "seed": seed,
                   "measure": f"E, M, C(r) on {len(r)} separations <= {int(r[-1])} at sweeps 2^k",
                   "measurements_timed": n_meas, "sweep_strategy": strategy},
        "sweep_only_flips_per_ns": round(flips / (sweep_ms / 1e3) / 1e9, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "binding_unit": "valu",
                     "issue_busy": issue_busy(wl["name"], strategy, float(L) * L / 64, half_sweep_s),
                     "kernel": "k_sweep_ising" if model == 0 else "k_sweep_bc",
                     "avg_launch_ms": round(half_sweep_s * 1e3, 3),
                     "algorithmic_bytes_per_launch": bytes_launch},
    }


def run_equilibrium(args):
    """Equilibrium Blume-Capel at Delta = 0 (App. B): independent runs per L
    (one batch per L) of EMCS = 10 Metropolis sweeps + 1 Swendsen-Wang step at
    T_c^BC, U4 and xi_2/L from the Fourier moments, and the reweighted
    crossings beta_{L,U}, beta_{L,xi2/L} with jackknife errors."""
    import torch
    from paper_2503_14688_amd import equilibrium, workloads
    wl = dict(workloads.EQUILIBRIUM_BC)
    if getattr(args, "equilibrium_sizes", None):
        wl["sizes"] = tuple(int(x) for x in args.equilibrium_sizes.split(","))
    if getattr(args, "equilibrium_emcs", None):
        wl["n_emcs"] = args.equilibrium_emcs
    if getattr(args, "equilibrium_runs", None):
        wl["runs"] = args.equilibrium_runs
    T, beta0 = wl["T"], 1.0 / wl["T"]
    out = {"workload": wl["name"], "T_sim": T, "Delta": 0.0, "runs_per_L": wl["runs"], "n_therm": wl["n_therm"],
           "n_emcs": wl["n_emcs"], "emcs": "10 Metropolis sweeps + 1 Swendsen-Wang step",
           "U4_star": equilibrium.U4_STAR, "xi2_over_L_star": equilibrium.XI_OVER_L_STAR,
           "T_c_paper": "1.6935583(5)", "sizes": {}}
    est = {"beta_U": ([], []), "beta_xi": ([], [])}
    for L in wl["sizes"]:
        seeds = [workloads.seed_for(wl["seed0"] + 1000 * k + L) for k in range(wl["runs"])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = equilibrium.emcs_batch(wl["model"], L, seeds, T, wl["n_emcs"], wl["every"], wl["n_therm"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        c = equilibrium.crossings(runs, L, beta0)
        j = equilibrium.jackknife_observables(runs, L, beta0)
        n_emcs = wl["runs"] * (wl["n_therm"] + wl["n_emcs"])
        row = {"U4": [round(j["U4"], 5), round(j.get("U4_err", float("nan")), 5)],
               "xi2_over_L": [round(j["xi2_over_L"], 5), round(j.get("xi2_over_L_err", float("nan")), 5)],
               "wall_s": round(wall, 3), "emcs_per_s": round(n_emcs / wall, 1),
               "flips_per_ns": round(n_emcs * 10.0 * L * L / wall / 1e9, 3)}
        for key in ("beta_U", "beta_xi"):
            b, e = c[key], c[key + "_err"]
            row[key] = [round(b, 6), round(e, 6)] if b is not None and e is not None else None
            row["T" + key[4:]] = round(1.0 / b, 5) if b is not None else None
            if b is not None and e is not None:
                est[key][0].append(b)
                est[key][1].append(e)
        out["sizes"][str(L)] = row
        log(f"equilibrium BC L = {L}: U4 = {j['U4']:.4f}, xi2/L = {j['xi2_over_L']:.4f}, "
            f"beta_U = {c['beta_U']}, beta_xi = {c['beta_xi']} ({wall:.1f} s)")
    for key, (vals, errs) in est.items():
        if vals:
            m, e, chi = equilibrium.constant_fit(vals, errs)
            out[key + "_constant_fit"] = {"beta": round(m, 6), "err": round(e, 6), "T_c": round(1.0 / m, 5),
                                          "chi2_dof": round(chi, 3)}
    return out


def run_bc_large(args):
    """The Blume-Capel L = 2^18 workload (16 GiB, T = 1.6937, 256 sweeps with
    E, M and C(r) at sweeps 2^k), timed like the main line."""
    from paper_2503_14688_amd import workloads
    wl = workloads.BC_LARGE
    res = single_lattice(wl, args.bc_steps, 1)
    res["flips_per_ns"] = res.pop("value")
    res["wall_s"] = round(res["wall_s"], 3)
    log(f"{wl['name']}: {res['flips_per_ns']} flips/ns, half-sweep {res['roofline']['avg_launch_ms']} ms")
    return res


def run(args):
    import torch
    from paper_2503_14688_amd import workloads

    wl = {"ising_large": workloads.ISING_LARGE, "bc_large": workloads.BC_LARGE,
          "ising_check": workloads.ISING_CHECK}[args.workload]
    torch.cuda.init()
    res = single_lattice(wl, args.steps, args.warmup, args.variant)
    out = {
        "metric": METRIC, "value": res["value"], "unit": "flips/ns", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 bit-packed spins, u32 Philox4x32-10",
        "data": "synthetic", "config": res["config"],
        "sweep_only_flips_per_ns": res["sweep_only_flips_per_ns"], "roofline": res["roofline"],
    }
    log(f"timed region done: {res['value']:.1f} flips/ns")
    if not args.skip_batched:
        out["batched"] = run_batched(args)
    if not args.skip_serving:
        sat = out["batched"]["flips_per_ns"] if "batched" in out else out["sweep_only_flips_per_ns"]
        out["serving"] = run_serving(args, sat)
    # the extra sections report an error instead of losing the line
    for name, skip, fn in (("blume_capel_large", args.skip_bc or args.workload == "bc_large", run_bc_large),
                           ("protocol2", args.skip_protocol2, run_protocol2),
                           ("ensemble", args.skip_ensemble, run_ensemble),
                           ("equilibrium", args.skip_equilibrium, run_equilibrium)):
        if skip:
            continue
        try:
            out[name] = fn(args)
        except Exception as exc:  # noqa: BLE001
            log(f"{name} failed: {exc!r}")
            out[name] = {"error": repr(exc)}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    return out


def calibrate_copy(gib=8):
    """A plain device copy of known size (for scaling HBM traffic counters)."""
    import torch
    n = gib << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {gib} GiB three times")
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n}),
          flush=True)


SECTIONS = {"batched": run_batched, "blume_capel_large": run_bc_large, "protocol2": run_protocol2,
            "ensemble": run_ensemble, "equilibrium": run_equilibrium}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ising_large", choices=["ising_large", "bc_large", "ising_check"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--skip-protocol2", action="store_true")
    ap.add_argument("--skip-ensemble", action="store_true")
    ap.add_argument("--skip-bc", action="store_true")
    ap.add_argument("--skip-equilibrium", action="store_true")
    ap.add_argument("--bc-steps", type=int, default=256)
    ap.add_argument("--replicas", type=int, default=512)
    ap.add_argument("--batch-sweeps", type=int, default=4096)
    ap.add_argument("--compare-sweeps", type=int, default=256)
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--variant", type=int, default=-1, help="sweep strategy (default: tuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 8 GiB device copy (traffic-counter calibration)")
    ap.add_argument("--section", choices=sorted(SECTIONS),
                    help="run only this section and print its JSON (profiling runs; not the benchmark line)")
    ap.add_argument("--equilibrium-sizes", type=str, default=None,
                    help="comma-separated L of the equilibrium section (default: the workload's)")
    ap.add_argument("--equilibrium-emcs", type=int, default=None,
                    help="measured EMCS per run of the equilibrium section (default: the workload's)")
    ap.add_argument("--equilibrium-runs", type=int, default=None,
                    help="independent runs per L of the equilibrium section (default: the workload's)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.section:
        import torch
        torch.cuda.init()
        print(json.dumps({args.section: SECTIONS[args.section](args)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab decomposition "
              "is not implemented", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
