"""The ensemble analysis (App. C coherence length, App. D jackknife and z
fit) on constructed correlation functions whose integrals are known."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2503_14688_amd import analysis, workloads

R = workloads.r_sparse(1 << 20).astype(np.float64)


def F(r, A, xi_F, beta):
    return A * np.exp(-(r / xi_F) ** beta) / np.sqrt(r)


@pytest.mark.parametrize("A,xi_F,beta", [(0.9, 30.0, 1.3), (0.7, 120.0, 0.9), (1.0, 16.0, 1.6)])
def test_tail_form_is_recovered(A, xi_F, beta):
    """C(r) = F(r) for r >= 1: the fit finds F's parameters, and xi equals the
    exact I2/I1 of F beyond r = 1 (plus the same spline piece on [0, 1])."""
    C = F(R, A, xi_F, beta)
    res = analysis.coherence_length(R, C, np.full_like(C, 1e-9), 1.0)
    assert res["ok"] and res["tail"]
    assert res["A"] == pytest.approx(A, rel=1e-6) and res["xi_F"] == pytest.approx(xi_F, rel=1e-6)
    assert res["beta"] == pytest.approx(beta, rel=1e-6)
    s = analysis._spline(R, C, 1.0)
    f = lambda x, n: x ** n * A * math.exp(-(x / xi_F) ** beta) / math.sqrt(x)
    I1 = analysis._moment(s, 1, 1.0) + quad(f, 1.0, 60 * xi_F, args=(1,), limit=500)[0]
    I2 = analysis._moment(s, 2, 1.0) + quad(f, 1.0, 60 * xi_F, args=(2,), limit=500)[0]
    assert res["xi"] == pytest.approx(I2 / I1, rel=1e-3)  # spline error between sparse r


@pytest.mark.parametrize("a", [1.5, 3.0, 10.0, 80.0])
def test_exponential_correlation(a):
    """C(r) = exp(-r/a): I2/I1 = 2a.  Short correlations take the plain
    integration branch (r_max - r_min <= 8); long ones the F tail, whose form
    differs from an exponential by a 1/sqrt(r) factor (bias under 0.5%)."""
    C = np.exp(-R / a)
    res = analysis.coherence_length(R, C, np.full_like(C, 1e-7), 1.0)
    assert res["ok"]
    assert res["tail"] == (a > 4)
    assert res["xi"] == pytest.approx(2 * a, rel=5e-3 if res["tail"] else 1e-3)


def test_cut_points_rule():
    C = np.exp(-R / 10.0)
    err = np.full_like(C, 1e-3)
    pts = analysis.cut_points(R, C, err, 1.0)
    first_bad = int(np.nonzero(C < 3e-3)[0][0])
    assert pts["r_cut"] == int(R[first_bad - 1])
    assert pts["r_star"] == 20  # argmax of r^2 exp(-r/10)
    w = lambda r: r * r * math.exp(-r / 10.0)
    # r_min / r_max: first integers past r* below 0.9 and 1/3 of the maximum
    # (on the spline, which follows the exponential closely on this grid)
    assert abs(pts["r_min"] - next(r for r in range(21, 200) if w(r) < 0.9 * w(20))) <= 1
    assert abs(pts["r_max"] - next(r for r in range(21, 200) if w(r) < w(20) / 3)) <= 1
    assert analysis.cut_points(R, C, np.full_like(C, 10.0), 1.0)["r_cut"] == 0


def test_jackknife_of_the_mean_is_the_standard_error():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(37, 5))
    err = analysis.jackknife_error(analysis.jackknife_means(x))
    assert np.allclose(err, x.std(axis=0, ddof=1) / math.sqrt(37), rtol=1e-12)
    with pytest.raises(ValueError):
        analysis.jackknife_means(x[:1])


def test_fit_z_power_law():
    t = np.array([64, 128, 256, 512, 1024, 2048, 4096], dtype=np.float64)
    z = 2.1676
    xi = 0.8 * t ** (1.0 / z)
    res = analysis.fit_z(t, xi, 0.01 * xi)
    assert res["z"] == pytest.approx(z, rel=1e-12) and res["chi2_dof"] < 1e-20
    # replicas with noise: the jackknife error follows the spread
    rng = np.random.default_rng(2)
    reps = xi * (1 + 0.05 * rng.normal(size=(40, t.shape[0])))
    mean = reps.mean(axis=0)
    err = reps.std(axis=0, ddof=1) / math.sqrt(40)
    res = analysis.fit_z(t, mean, err, analysis.jackknife_means(reps))
    assert abs(res["z"] - z) < 5 * res["z_err"] and 0 < res["z_err"] < 0.2


def test_xi_ensemble_jackknife():
    rng = np.random.default_rng(3)
    a = 12.0
    n = 32
    C = np.exp(-R / a)[None, :] * (1 + 0.02 * rng.normal(size=(n, R.shape[0])))
    C0 = np.ones(n)
    xi, err, full, blocks = analysis.xi_ensemble(R, C, C0)
    assert full["ok"] and blocks.shape == (n,)
    assert 0 < err < 0.05 * xi
    assert abs(xi - 2 * a) < 0.01 * 2 * a + 5 * err


def test_c_hat_definition():
    m = {"Sx": np.array([10, -4]), "Sy": np.array([6, 0]), "sum_s2": 12}
    C, C0 = analysis.c_hat(m, 4)
    assert np.array_equal(C, np.array([0.5, -0.125])) and C0 == 0.75


def test_fit_z_energy_two_terms():
    """E - E_eq = b t^(-1/z) + b' t^(-2/z): the fit returns z exactly on
    exact data and a jackknife error that covers it on noisy replicas."""
    z, b, b2 = 2.1676, 0.31, -0.12
    t = np.array([16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192], dtype=np.float64)
    dE = b * t ** (-1 / z) + b2 * t ** (-2 / z)
    res = analysis.fit_z_energy(t, dE, 1e-3 * dE)
    assert res["z"] == pytest.approx(z, rel=1e-8) and res["b"] == pytest.approx(b, rel=1e-6)
    rng = np.random.default_rng(4)
    reps = dE[None, :] + 0.002 * dE[None, :] * rng.normal(size=(48, t.shape[0]))
    mean = reps.mean(axis=0)
    err = reps.std(axis=0, ddof=1) / math.sqrt(48)
    res = analysis.fit_z_energy(t, mean, err, analysis.jackknife_means(reps))
    assert abs(res["z"] - z) < 5 * res["z_err"] and res["z_err"] < 0.1


def test_fit_quality_closed_forms():
    # Gamma_reg(1, x) = exp(-x) and Gamma_reg(2, x) = exp(-x) (1 + x)
    assert analysis.fit_quality(2.0, 2) == pytest.approx(math.exp(-1.0), rel=1e-14)
    assert analysis.fit_quality(3.0, 4) == pytest.approx(math.exp(-1.5) * 2.5, rel=1e-14)
    assert analysis.fit_quality(0.0, 7) == 1.0


def test_fit_z_with_the_correction_term():
    """log t = z log xi + b + b' xi^-omega: exact data give back (z, b, b')
    and a perfect fit; the plain straight line misses it."""
    z, b, b1, om = 2.1676, -0.4, 3.0, analysis.OMEGA
    xi = np.array([3.0, 4.5, 7.0, 11.0, 17.0, 26.0, 40.0, 62.0])
    t = np.exp(z * np.log(xi) + b + b1 * xi ** (-om))
    res = analysis.fit_z(t, xi, 0.01 * xi)
    assert res["z"] == pytest.approx(z, rel=1e-9) and res["b1"] == pytest.approx(b1, rel=1e-7)
    assert res["chi2_dof"] < 1e-16 and res["Q"] == pytest.approx(1.0, abs=1e-12) and res["dof"] == 5
    plain = analysis.fit_z(t, xi, 0.01 * xi, correction=False)
    assert abs(plain["z"] - z) > 1e-3 and plain["chi2_dof"] > 1.0 and plain["Q"] < 0.01


def test_fit_z_energy_three_terms():
    z, b, b2, b3 = 2.1676, 0.31, -0.12, 0.05
    t = np.array([16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192], dtype=np.float64)
    dE = b * t ** (-1 / z) + b2 * t ** (-2 / z) + b3 * t ** (-(analysis.OMEGA + 1) / z)
    res = analysis.fit_z_energy(t, dE, 1e-3 * dE)
    assert res["z"] == pytest.approx(z, rel=1e-8) and res["b3"] == pytest.approx(b3, rel=1e-5)
    assert res["dof"] == 6 and res["chi2_dof"] < 1e-16


def _joint_sets(rng=None, n_rep=(30, 24)):
    z, om = 2.1676, analysis.OMEGA
    xi_i = np.array([3.0, 4.5, 7.0, 11.0, 17.0, 26.0, 40.0, 62.0])
    t_i = np.exp(z * np.log(xi_i) + 0.2 + 1.5 * xi_i ** (-om))
    dE = 0.31 * t_i ** (-1 / z) - 0.12 * t_i ** (-2 / z) + 0.05 * t_i ** (-(om + 1) / z)
    xi_b = np.array([2.5, 4.0, 6.0, 9.5, 15.0, 23.0, 36.0])
    t_b = np.exp(z * np.log(xi_b) + 0.7 - 0.8 * xi_b ** (-om))
    exact = [("xi", t_i, xi_i, "ising"), ("energy", t_i, dE, "ising"), ("xi", t_b, xi_b, "bc")]
    sets = []
    reps = {}
    for kind, t, y, group in exact:
        s = dict(kind=kind, t=t, y=y, err=0.01 * np.abs(y), group=group)
        if rng is not None:
            n = n_rep[0] if group == "ising" else n_rep[1]
            noise = reps.setdefault(group, rng.normal(size=(n, 1)))  # one draw per replica and group
            r = y[None, :] * (1 + 0.02 * noise + 0.01 * rng.normal(size=(n, y.shape[0])))
            s.update(y=r.mean(axis=0), err=r.std(axis=0, ddof=1) / math.sqrt(n),
                     blocks=analysis.jackknife_means(r))
        sets.append(s)
    return z, sets


def test_joint_fit_shares_z():
    z, sets = _joint_sets()
    res = analysis.fit_z_joint(sets)
    assert res["z"] == pytest.approx(z, rel=1e-8) and res["chi2_dof"] < 1e-14
    assert res["dof"] == 8 + 8 + 7 - (1 + 2 + 3 + 2)
    z, sets = _joint_sets(np.random.default_rng(11))
    res = analysis.fit_z_joint(sets)
    assert 0 < res["z_err"] < 0.1 and abs(res["z"] - z) < 5 * res["z_err"]
    single = analysis.fit_z(sets[2]["t"], sets[2]["y"], sets[2]["err"], sets[2]["blocks"])
    assert res["z_err"] < single["z_err"]  # three data sets pin z better than one
