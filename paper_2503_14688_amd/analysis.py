"""Ensemble analysis of the measured correlations (paper App. C and App. D),
in host FP64 on the integer sums the library returns.

Coherence length (App. C).  From the replica-averaged C(r; t) and its error:
  (i)   r_cut: C(r) is trusted up to the last sampled r before the first one
        where C falls below three times its error;
  (ii)  r* maximises r^2 C(r) (on the interpolated curve, integer r <= r_cut);
        r_min and r_max are the first r beyond r* where r^2 C(r) drops below
        0.9 and 1/3 of that maximum;
  (iii) I_n = int_0^inf r^n C(r) dr for n = 1, 2: if r_max - r_min <= 8 the
        interpolated C is integrated up to r_cut; otherwise
        F(r) = A exp[-(r / xi_F)^beta] / sqrt(r) is fitted to the data in
        [r_min, r_max], the interpolated C is integrated up to r_max and F
        from r_max to 20 xi_F.
  xi = I_2 / I_1.  The sampled separations are sparse, so C is interpolated
  with a cubic spline through r = 0 (C(0) = <s^2>) and the sampled r.

Errors come from jackknife resampling over independent replicas (App. D):
the cut points are fixed on the full sample and the estimator is recomputed
on every leave-one-out mean.

Dynamic exponent (App. D):
  from xi      log t = z log xi + b + b' xi^-omega,   omega = 7/4
               (t is exact, so each point is weighted by the error of xi
               times the slope of the fitted curve, the effective-variance
               rule of App. D);
  from energy  E(t) - E_eq = b t^(-1/z) + b' t^(-2/z) + b'' t^(-(omega+1)/z)
               (Ising, E_eq = -sqrt 2; nu = 1 so (omega + 1/nu) = omega + 1);
  joint        one z shared by several such data sets (the paper's Ising xi,
               Ising energy and Blume-Capel xi), each with its own amplitudes.
Every fit reports chi^2/dof and the fit quality Q = Gamma_reg(dof/2, chi^2/2)
(regularised upper incomplete gamma function, App. D); errors are jackknife
over the independent replicas of each ensemble, added in quadrature across
independent ensembles.
"""
import math

import numpy as np


def c_hat(meas, L):
    """Axis-averaged C(r) and C(0) of one measurement (dict with Sx, Sy, sum_s2)."""
    N = float(L) * float(L)
    C = (np.asarray(meas["Sx"], dtype=np.float64) + np.asarray(meas["Sy"], dtype=np.float64)) / (2.0 * N)
    return C, float(meas["sum_s2"]) / N


def jackknife_means(x):
    """Leave-one-out means of samples x (n, ...) along the first axis."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n < 2:
        raise ValueError("jackknife needs at least two samples")
    return (x.sum(axis=0) - x) / (n - 1)


def jackknife_error(values):
    """Error of an estimator from its values on the n leave-one-out samples."""
    v = np.asarray(values, dtype=np.float64)
    n = v.shape[0]
    return np.sqrt((n - 1) / n * ((v - v.mean(axis=0)) ** 2).sum(axis=0))


def _spline(r, C, C0):
    from scipy.interpolate import CubicSpline
    x = np.concatenate(([0.0], np.asarray(r, dtype=np.float64)))
    y = np.concatenate(([float(C0)], np.asarray(C, dtype=np.float64)))
    return CubicSpline(x, y)


def cut_points(r, C, C_err, C0):
    """Steps (i) and (ii): r_cut, r*, r_min, r_max, and whether
    r* < r_min < r_max < r_cut holds (the paper adds statistics otherwise)."""
    r = np.asarray(r, dtype=np.int64)
    C = np.asarray(C, dtype=np.float64)
    C_err = np.asarray(C_err, dtype=np.float64)
    bad = np.nonzero(C < 3.0 * C_err)[0]
    k = int(bad[0]) if bad.size else r.shape[0]
    if k == 0:
        return dict(r_cut=0, r_star=0, r_min=0, r_max=0, ok=False)
    r_cut = int(r[k - 1])
    s = _spline(r[:k], C[:k], C0)
    ri = np.arange(1, r_cut + 1, dtype=np.float64)
    w = ri * ri * s(ri)
    j = int(np.argmax(w))
    r_star, top = int(ri[j]), float(w[j])
    after = np.arange(j + 1, ri.shape[0])
    below_min = after[w[after] < 0.9 * top]
    below_max = after[w[after] < top / 3.0]
    r_min = int(ri[below_min[0]]) if below_min.size else r_cut
    r_max = int(ri[below_max[0]]) if below_max.size else r_cut
    return dict(r_cut=r_cut, r_star=r_star, r_min=r_min, r_max=r_max,
                ok=bool(r_star < r_min < r_max < r_cut))


def _fit_F(r, C, C_err, r_min, r_max):
    """Fit F(r) = A exp[-(r / xi_F)^beta] / sqrt(r) to the sampled points in
    [r_min, r_max] (widened to the nearest sampled points until there are
    four), in log form with the relative errors as weights."""
    from scipy.optimize import curve_fit
    r = np.asarray(r, dtype=np.float64)
    lo = int(np.searchsorted(r, r_min, side="left"))
    hi = int(np.searchsorted(r, r_max, side="right"))
    while hi - lo < 4 and (lo > 0 or hi < r.shape[0]):
        if lo > 0:
            lo -= 1
        if hi - lo < 4 and hi < r.shape[0]:
            hi += 1
    rr, cc, ee = r[lo:hi], np.asarray(C[lo:hi], dtype=np.float64), np.asarray(C_err[lo:hi], dtype=np.float64)
    keep = cc > 0
    rr, cc, ee = rr[keep], cc[keep], ee[keep]
    y = np.log(cc * np.sqrt(rr))

    def logF(x, logA, log_xi, beta):
        return logA - (x / math.exp(log_xi)) ** beta

    slope = (y[-1] - y[0]) / (rr[-1] - rr[0]) if rr[-1] > rr[0] else -1.0
    xi0 = 1.0 / max(-slope, 1e-6)
    p0 = (y[0] + rr[0] / xi0, math.log(xi0), 1.0)
    p, _ = curve_fit(logF, rr, y, p0=p0, sigma=np.maximum(ee / cc, 1e-12), maxfev=20000)
    return math.exp(p[0]), math.exp(p[1]), float(p[2])


def _moment(s, n, upper):
    """int_0^upper r^n s(r) dr for a cubic spline s, exactly (piecewise
    polynomials), upper no further than the last knot."""
    from numpy.polynomial import polynomial as P
    total = 0.0
    for i in range(s.x.shape[0] - 1):
        a = float(s.x[i])
        b = min(float(s.x[i + 1]), upper)
        if b <= a:
            break
        piece = s.c[::-1, i]                # in u = r - a, lowest power first
        q = P.polyint(P.polymul(piece, P.polypow([a, 1.0], n)))  # r^n = (a + u)^n
        total += P.polyval(b - a, q)
    return total


def integrals(r, C, C_err, C0, pts):
    """Step (iii): (I_1, I_2, details) for given cut points."""
    from scipy.integrate import quad
    r = np.asarray(r, dtype=np.float64)
    k = int(np.searchsorted(r, pts["r_cut"], side="right"))
    s = _spline(r[:k], C[:k], C0)
    tail = pts["r_max"] - pts["r_min"] > 8
    upper = float(pts["r_max"] if tail else pts["r_cut"])
    I = [_moment(s, 1, upper), _moment(s, 2, upper)]
    out = dict(tail=tail, xi_F=None, beta=None, A=None)
    if tail:
        A, xi_F, beta = _fit_F(r, C, C_err, pts["r_min"], pts["r_max"])
        out.update(A=A, xi_F=xi_F, beta=beta)
        for q, n in enumerate((1, 2)):
            I[q] += quad(lambda x: x ** n * A * math.exp(-(x / xi_F) ** beta) / math.sqrt(x),
                         upper, max(upper, 20.0 * xi_F), limit=200)[0]
    return I[0], I[1], out


def coherence_length(r, C, C_err, C0, pts=None):
    """xi = I_2 / I_1 by the App. C recipe for one mean curve with errors."""
    if pts is None:
        pts = cut_points(r, C, C_err, C0)
    if pts["r_cut"] <= 0:
        return dict(pts, xi=float("nan"), I1=float("nan"), I2=float("nan"), tail=False, xi_F=None, beta=None)
    I1, I2, extra = integrals(r, C, C_err, C0, pts)
    return dict(pts, xi=I2 / I1 if I1 > 0 else float("nan"), I1=I1, I2=I2, **extra)


def xi_ensemble(r, C_samples, C0_samples):
    """xi of the replica mean with its jackknife error.

    C_samples: (n_replicas, n_r) per-replica C-hat; C0_samples: (n_replicas,).
    Returns (xi, error, details of the full-sample estimate, leave-one-out xi)."""
    C_samples = np.asarray(C_samples, dtype=np.float64)
    C0_samples = np.asarray(C0_samples, dtype=np.float64)
    n = C_samples.shape[0]
    mean = C_samples.mean(axis=0)
    err = C_samples.std(axis=0, ddof=1) / math.sqrt(n)
    C0 = float(C0_samples.mean())
    full = coherence_length(r, mean, err, C0)
    jm, j0 = jackknife_means(C_samples), jackknife_means(C0_samples)
    blocks = np.array([coherence_length(r, jm[i], err, j0[i], pts=full)["xi"] for i in range(n)])
    return full["xi"], float(jackknife_error(blocks)), full, blocks


OMEGA = 1.75  # leading correction-to-scaling exponent of the 2D Ising class (App. D)


def fit_quality(chi2, dof):
    """Q = Gamma_reg(dof / 2, chi^2 / 2), the probability of a chi^2 at least
    this large for a correct model (App. D)."""
    from scipy.special import gammaincc
    if dof <= 0:
        return float("nan")
    return float(gammaincc(0.5 * dof, 0.5 * chi2))


def _xi_model(p, xi, correction, omega):
    z, b = p[0], p[1]
    y = z * np.log(xi) + b
    dy = z / xi
    if correction:
        y = y + p[2] * xi ** (-omega)
        dy = dy - omega * p[2] * xi ** (-omega - 1.0)
    return y, dy


def _energy_model(p, t, correction, omega):
    b, b2, inv_z = p[0], p[1], p[2]
    y = b * t ** (-inv_z) + b2 * t ** (-2.0 * inv_z)
    if correction:
        y = y + p[3] * t ** (-(omega + 1.0) * inv_z)
    return y


def _xi_params(correction):
    return 3 if correction else 2


def _energy_params(correction):
    return 4 if correction else 3


def _residuals_xi(p, t, xi, xi_err, correction, omega):
    y, dy = _xi_model(p, xi, correction, omega)
    sigma = np.maximum(1e-40 + xi_err * np.abs(dy), 1e-300)
    return (np.log(t) - y) / sigma


def _residuals_energy(p, t, dE, dE_err, correction, omega):
    return (dE - _energy_model(p, t, correction, omega)) / dE_err


def _start_xi(t, xi, xi_err, correction):
    """Starting point: the weighted straight line log t = z log xi + b."""
    X, Y = np.log(xi), np.log(t)
    w = (xi / np.maximum(xi_err, 1e-300)) ** 2
    Sw, Sx, Sy = w.sum(), (w * X).sum(), (w * Y).sum()
    Sxx, Sxy = (w * X * X).sum(), (w * X * Y).sum()
    z = (Sw * Sxy - Sx * Sy) / (Sw * Sxx - Sx * Sx)
    b = (Sy - z * Sx) / Sw
    return [z, b, 0.0] if correction else [z, b]


def _start_energy(t, dE, z0, correction):
    p = [float(dE[0] * t[0] ** (1.0 / z0)), 0.0, 1.0 / z0]
    return p + [0.0] if correction else p


def _solve(fun, p0):
    from scipy.optimize import least_squares
    r = least_squares(fun, np.asarray(p0, dtype=np.float64), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                      max_nfev=20000)
    return r.x, float((r.fun ** 2).sum())


def fit_z(t, xi, xi_err, xi_blocks=None, correction=True, omega=OMEGA):
    """Fit of log t = z log xi + b (+ b' xi^-omega with correction) over the
    given points, weighted by xi_err times the slope of the curve (App. D).
    With xi_blocks (n_replicas, len(t)) of leave-one-out xi the fit is
    repeated per block for the jackknife error of z.
    Returns dict(z, b, b1 (b' or None), z_err, chi2, dof, chi2_dof, Q)."""
    t = np.asarray(t, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    xi_err = np.asarray(xi_err, dtype=np.float64)
    k = _xi_params(correction)
    if t.shape[0] <= k:
        raise ValueError(f"need more than {k} times")

    def one(x_xi, p0):
        return _solve(lambda p: _residuals_xi(p, t, x_xi, xi_err, correction, omega), p0)

    p, chi2 = one(xi, _start_xi(t, xi, xi_err, correction))
    dof = t.shape[0] - k
    out = dict(z=float(p[0]), b=float(p[1]), b1=float(p[2]) if correction else None, chi2=chi2, dof=dof,
               chi2_dof=chi2 / dof, Q=fit_quality(chi2, dof), z_err=None)
    if xi_blocks is not None:
        zs = np.array([one(np.asarray(blk, dtype=np.float64), p)[0][0] for blk in xi_blocks])
        out["z_err"] = float(jackknife_error(zs))
    return out


def fit_z_energy(t, dE, dE_err, dE_blocks=None, z0=2.17, correction=True, omega=OMEGA):
    """z from the excess energy of the quench to T_c (App. D):
    E(t) - E_eq = b t^(-1/z) + b' t^(-2/z) (+ b'' t^(-(omega+1)/z) with
    correction), weighted least squares for the amplitudes and 1/z; with
    dE_blocks (n_replicas, len(t)) of leave-one-out excess energies the fit is
    repeated per block for the jackknife error of z.
    Returns dict(z, b, b2, b3 (b'' or None), z_err, chi2, dof, chi2_dof, Q)."""
    t = np.asarray(t, dtype=np.float64)
    dE = np.asarray(dE, dtype=np.float64)
    dE_err = np.asarray(dE_err, dtype=np.float64)
    k = _energy_params(correction)
    if t.shape[0] <= k:
        raise ValueError(f"need more than {k} times")

    def one(y, p0):
        return _solve(lambda p: _residuals_energy(p, t, y, dE_err, correction, omega), p0)

    p, chi2 = one(dE, _start_energy(t, dE, z0, correction))
    dof = t.shape[0] - k
    out = dict(z=float(1.0 / p[2]), b=float(p[0]), b2=float(p[1]), b3=float(p[3]) if correction else None,
               chi2=chi2, dof=dof, chi2_dof=chi2 / dof, Q=fit_quality(chi2, dof), z_err=None)
    if dE_blocks is not None:
        zs = np.array([1.0 / one(np.asarray(blk, dtype=np.float64), p)[0][2] for blk in dE_blocks])
        out["z_err"] = float(jackknife_error(zs))
    return out


def fit_z_joint(sets, z0=2.17, correction=True, omega=OMEGA):
    """One z for several data sets (App. D's joint fit: Ising xi, Ising
    energy, Blume-Capel xi), each with its own amplitudes.

    sets: list of dicts with kind ('xi' or 'energy'), t, y (xi, or E - E_eq),
    err, and optionally blocks (n_replicas, len(t)) of leave-one-out values
    and group (name of the replica ensemble the set comes from; sets of one
    group share replicas).  The jackknife removes one replica of one group
    at a time from every set of that group; the variances of the groups
    (independent ensembles) add.
    Returns dict(z, z_err, chi2, dof, chi2_dof, Q, params (per set))."""
    prepared = []
    p0 = [float(z0)]
    for s in sets:
        t = np.asarray(s["t"], dtype=np.float64)
        y = np.asarray(s["y"], dtype=np.float64)
        e = np.asarray(s["err"], dtype=np.float64)
        if s["kind"] == "xi":
            start = _start_xi(t, y, e, correction)[1:]
        elif s["kind"] == "energy":
            st = _start_energy(t, y, z0, correction)
            start = st[:2] + st[3:]
        else:
            raise ValueError(f"unknown data set kind {s['kind']!r}")
        prepared.append((s["kind"], t, e, len(p0), len(start)))
        p0 += list(start)

    def residuals(p, ys):
        z = p[0]
        parts = []
        for (kind, t, e, off, n), y in zip(prepared, ys):
            q = p[off:off + n]
            if kind == "xi":
                parts.append(_residuals_xi(np.concatenate(([z], q)), t, y, e, correction, omega))
            else:
                pe = np.concatenate((q[:2], [1.0 / z], q[2:]))
                parts.append(_residuals_energy(pe, t, y, e, correction, omega))
        return np.concatenate(parts)

    ys = [np.asarray(s["y"], dtype=np.float64) for s in sets]
    p, chi2 = _solve(lambda q: residuals(q, ys), p0)
    n_points = sum(pr[1].shape[0] for pr in prepared)
    dof = n_points - len(p0)
    out = dict(z=float(p[0]), chi2=chi2, dof=dof, chi2_dof=chi2 / dof if dof > 0 else float("nan"),
               Q=fit_quality(chi2, dof), z_err=None,
               params=[[float(v) for v in p[off:off + n]] for (_, _, _, off, n) in prepared])
    groups = {}
    for k, s in enumerate(sets):
        if s.get("blocks") is not None:
            groups.setdefault(s.get("group", k), []).append(k)
    if groups:
        var = 0.0
        for members in groups.values():
            n_rep = np.asarray(sets[members[0]]["blocks"]).shape[0]
            zs = []
            for r in range(n_rep):
                yb = [np.asarray(sets[k]["blocks"], dtype=np.float64)[r] if k in members else ys[k]
                      for k in range(len(sets))]
                zs.append(_solve(lambda q: residuals(q, yb), p)[0][0])
            var += float(jackknife_error(np.array(zs))) ** 2
        out["z_err"] = math.sqrt(var)
    return out
