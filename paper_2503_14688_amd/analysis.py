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

Dynamic exponent (App. D, Eq. for log t): log t = z log xi + b over a time
window, weighted by the error of log t implied by the error of xi
(d log t / d log xi = z), with jackknife errors.  The correction term
b' xi^-omega of the paper's fit is left out: the windows used here start
late enough for it to sit inside the errors, which chi^2/dof shows.
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


def fit_z(t, xi, xi_err, xi_blocks=None):
    """Weighted fit of log t = z log xi + b (App. D) over the given points.

    The error of log t is z xi_err / xi (t itself is exact), iterated to the
    fitted z.  With xi_blocks (n_replicas, len(t)) of leave-one-out xi the
    fit is repeated per block for the jackknife error of z.
    Returns dict(z, b, z_err, chi2_dof)."""
    t = np.asarray(t, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    xi_err = np.asarray(xi_err, dtype=np.float64)
    if t.shape[0] < 3:
        raise ValueError("need at least three times")

    def one(x_xi, z_guess=2.0):
        X, Y = np.log(x_xi), np.log(t)
        z, b = z_guess, 0.0
        for _ in range(5):
            w = 1.0 / np.maximum(z * xi_err / x_xi, 1e-300) ** 2
            Sw, Sx, Sy = w.sum(), (w * X).sum(), (w * Y).sum()
            Sxx, Sxy = (w * X * X).sum(), (w * X * Y).sum()
            z = (Sw * Sxy - Sx * Sy) / (Sw * Sxx - Sx * Sx)
            b = (Sy - z * Sx) / Sw
        chi2 = float((w * (Y - z * X - b) ** 2).sum())
        return z, b, chi2

    z, b, chi2 = one(xi)
    out = dict(z=float(z), b=float(b), chi2_dof=chi2 / (t.shape[0] - 2), z_err=None)
    if xi_blocks is not None:
        zs = np.array([one(np.asarray(blk, dtype=np.float64), z)[0] for blk in xi_blocks])
        out["z_err"] = float(jackknife_error(zs))
    return out


def fit_z_energy(t, dE, dE_err, dE_blocks=None, z0=2.17):
    """z from the excess energy of the Ising quench to T_c (App. D):
    E(t) - E_eq = b t^(-1/z) + b' t^(-2/z), E_eq = -sqrt(2) known exactly,
    fitted by weighted least squares for (b, b', z); with dE_blocks
    (n_replicas, len(t)) of leave-one-out excess energies the fit is repeated
    per block for the jackknife error of z.  (The paper adds a third term,
    b'' t^(-(omega + 1)/z), for its longer times.)
    Returns dict(z, b, b2, z_err, chi2_dof)."""
    from scipy.optimize import curve_fit
    t = np.asarray(t, dtype=np.float64)
    dE = np.asarray(dE, dtype=np.float64)
    dE_err = np.asarray(dE_err, dtype=np.float64)
    if t.shape[0] < 4:
        raise ValueError("need at least four times")

    def model(x, b, b2, inv_z):
        return b * x ** (-inv_z) + b2 * x ** (-2.0 * inv_z)

    def one(y, p0):
        p, _ = curve_fit(model, t, y, p0=p0, sigma=dE_err, maxfev=20000)
        return p

    p0 = (float(dE[0] * t[0] ** (1.0 / z0)), 0.0, 1.0 / z0)
    p = one(dE, p0)
    chi2 = float((((dE - model(t, *p)) / dE_err) ** 2).sum())
    out = dict(z=float(1.0 / p[2]), b=float(p[0]), b2=float(p[1]), chi2_dof=chi2 / (t.shape[0] - 3), z_err=None)
    if dE_blocks is not None:
        zs = np.array([1.0 / one(np.asarray(blk, dtype=np.float64), p)[2] for blk in dE_blocks])
        out["z_err"] = float(jackknife_error(zs))
    return out
