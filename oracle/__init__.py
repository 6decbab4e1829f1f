"""CPU oracle for the checkerboard Metropolis dynamics of arXiv:2503.14688.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP library.

The C part holds the dynamics, the random stream and the brute-force
correlation sums (spin_oracle.c), and the Swendsen-Wang cluster step and the
Fourier moments of the equilibrium study of App. B (equilibrium_oracle.c);
this module wraps it with ctypes and numpy and adds the FP64 observables
derived from the integer sums:

  energy density   e = (-J * B + Delta * sum s^2) / L^2, B = Sx(1) + Sy(1)
                   (paper Eq. 3 with the sign of the Hamiltonian, Eq. 1)
  magnetisation    m = sum s / L^2
  C-hat(r)         (Sx(r) + Sy(r)) / (2 L^2), the axis average of Eq. 2
  xi               I2 / I1 with I_n the integral of r^n C(r) (paper App. C),
                   taken here by the trapezoid rule over r = 0 and the
                   sampled r up to r_cut, the largest sampled r such that
                   C-hat is positive at every sampled r' <= r.

parity pins: see tests/test_oracle_*.py (Philox against rocRAND and the
Random123 known answers, Ising thresholds against closed forms, brute-force
Boltzmann histograms, Onsager's energy, Z2, T = 0 / T = inf limits, energy
bookkeeping, correlation-sum invariants, xi against a closed form, and the
energy density, magnetisation and C-hat of derive() on constructed lattices
whose values follow from Eq. 1 and Eq. 2 by hand; the Swendsen-Wang step
against connected components from scipy's graph routine at T = 0, isolated
sites at T = inf and exact Boltzmann histograms; the Fourier moments against
numpy's FFT).
"""
import ctypes
import os

import numpy as np

ISING = 0
BLUME_CAPEL = 1

PURPOSE_INIT = 0
PURPOSE_ACCEPT = 1
PURPOSE_PROPOSE = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i8p = ctypes.POINTER(ctypes.c_int8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_uniform.restype = ctypes.c_uint32
    lib.orc_threshold.argtypes = [ctypes.c_double, ctypes.c_double, u32p]
    lib.orc_threshold.restype = ctypes.c_int
    lib.orc_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, i8p]
    lib.orc_init.restype = ctypes.c_int
    lib.orc_init_window.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, i8p]
    lib.orc_init_window.restype = ctypes.c_int
    lib.orc_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                              ctypes.c_double, i8p, ctypes.c_uint32, ctypes.c_uint32, f64p, f64p]
    lib.orc_sweep.restype = ctypes.c_int
    lib.orc_window_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                     ctypes.c_double, i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, f64p]
    lib.orc_window_sweep.restype = ctypes.c_int
    lib.orc_measure.argtypes = [ctypes.c_int, i8p, u32p, ctypes.c_int, i64p, i64p, i64p]
    lib.orc_measure.restype = ctypes.c_int
    lib.orc_schedule.argtypes = [ctypes.c_int, f64p, ctypes.c_uint32, ctypes.c_uint32, f64p]
    lib.orc_schedule.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.orc_sw_threshold.argtypes = [ctypes.c_double, ctypes.c_double, u32p]
    lib.orc_sw_threshold.restype = ctypes.c_int
    lib.orc_sw.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_double, i8p,
                           ctypes.c_uint32, ctypes.c_uint32, f64p, u64p]
    lib.orc_sw.restype = ctypes.c_int
    lib.orc_fourier.argtypes = [ctypes.c_int, i8p, f64p]
    lib.orc_fourier.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def philox4x32_10(counter, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    lib = _load()
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                          _ptr(out, ctypes.c_uint32))
    return out


def uniform(seed, purpose, t, c, i, m):
    """The 32-bit bit-plane uniform of site (row i, colour c, m = j >> 1)."""
    return int(_load().orc_uniform(seed, purpose, t, c, i, m))


def threshold(dE, T):
    """(accept_always, thr): the integer Metropolis rule for one move."""
    thr = ctypes.c_uint32(0)
    always = _load().orc_threshold(float(dE), float(T), ctypes.byref(thr))
    return bool(always), int(thr.value)


def init(model, L, seed):
    """T = infinity start as an int8 L x L array."""
    s = np.zeros((L, L), dtype=np.int8)
    _check(_load().orc_init(model, L, seed, _ptr(s, ctypes.c_int8)), "init")
    return s


def init_window(model, L, seed, i0, j0, H, W):
    win = np.zeros((H, W), dtype=np.int8)
    _check(_load().orc_init_window(model, L, seed, i0, j0, H, W, _ptr(win, ctypes.c_int8)),
           "init_window")
    return win


def sweep(model, s, seed, J, Delta, t0, T, with_dE=False):
    """Run len(T) sweeps in place on s (int8, C-contiguous L x L).

    Sweep k uses bath temperature T[k] and stream sweep index t0 + k.
    With with_dE, returns the accepted energy change per half-sweep.
    """
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    T = np.ascontiguousarray(T, dtype=np.float64)
    n = T.shape[0]
    dE = np.zeros(2 * n, dtype=np.float64) if with_dE else None
    rc = _load().orc_sweep(model, s.shape[0], seed, J, Delta, _ptr(s, ctypes.c_int8), t0, n,
                           _ptr(T, ctypes.c_double),
                           _ptr(dE, ctypes.c_double) if with_dE else None)
    _check(rc, "sweep")
    return dE


def window_sweep(model, win, L, seed, J, Delta, i0, j0, t0, T):
    """Light-cone evolution of a window; the exact part is win[2n:-2n, 2n:-2n]."""
    assert win.dtype == np.int8 and win.flags.c_contiguous
    T = np.ascontiguousarray(T, dtype=np.float64)
    H, W = win.shape
    rc = _load().orc_window_sweep(model, L, seed, J, Delta, _ptr(win, ctypes.c_int8), i0, j0,
                                  H, W, t0, T.shape[0], _ptr(T, ctypes.c_double))
    _check(rc, "window_sweep")


def measure(s, r):
    """Integer sums: dict(sum_s, sum_s2, bond, Sx[len r], Sy[len r])."""
    assert s.dtype == np.int8 and s.flags.c_contiguous
    L = s.shape[0]
    r = np.ascontiguousarray(r, dtype=np.uint32)
    sums = np.zeros(3, dtype=np.int64)
    Sx = np.zeros(r.shape[0], dtype=np.int64)
    Sy = np.zeros(r.shape[0], dtype=np.int64)
    rc = _load().orc_measure(L, _ptr(s, ctypes.c_int8), _ptr(r, ctypes.c_uint32), r.shape[0],
                             _ptr(sums, ctypes.c_int64), _ptr(Sx, ctypes.c_int64),
                             _ptr(Sy, ctypes.c_int64))
    _check(rc, "measure")
    return {"sum_s": int(sums[0]), "sum_s2": int(sums[1]), "bond": int(sums[2]),
            "Sx": Sx, "Sy": Sy}


def schedule(kind, params, t0, n):
    """T(t) for t = t0 .. t0 + n - 1 (kind 0 constant, 1 two-step, 2 exponential)."""
    p = np.zeros(3, dtype=np.float64)
    p[:len(params)] = params
    out = np.zeros(n, dtype=np.float64)
    _check(_load().orc_schedule(kind, _ptr(p, ctypes.c_double), t0, n,
                                _ptr(out, ctypes.c_double)), "schedule")
    return out


def sw_threshold(J, T):
    """(always, thr): the integer Swendsen-Wang bond rule, p = 1 - exp(-2J/T)."""
    thr = ctypes.c_uint32(0)
    always = _load().orc_sw_threshold(float(J), float(T), ctypes.byref(thr))
    return bool(always), int(thr.value)


def sw(model, s, seed, J, t0, T, with_labels=False):
    """len(T) Swendsen-Wang steps (restricted to s = +-1) in place on s; step
    k uses bath temperature T[k] and sweep index t0 + k.  With with_labels,
    returns the cluster names (smallest site index) of the last step."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    T = np.ascontiguousarray(T, dtype=np.float64)
    lab = np.zeros(s.shape, dtype=np.uint64) if with_labels else None
    rc = _load().orc_sw(model, s.shape[0], seed, J, _ptr(s, ctypes.c_int8), t0, T.shape[0],
                        _ptr(T, ctypes.c_double), _ptr(lab, ctypes.c_uint64) if with_labels else None)
    _check(rc, "sw")
    return lab


def fourier(s):
    """Fourier moments by the plain double sum: dict(M0, k1, k2) with k1 =
    M(2 pi / L, 0) (phase along the row index i) and k2 = M(0, 2 pi / L)
    as complex numbers."""
    assert s.dtype == np.int8 and s.flags.c_contiguous
    out = np.zeros(5, dtype=np.float64)
    _check(_load().orc_fourier(s.shape[0], _ptr(s, ctypes.c_int8), _ptr(out, ctypes.c_double)), "fourier")
    return {"M0": out[0], "k1": complex(out[1], out[2]), "k2": complex(out[3], out[4])}


def num_threads():
    return int(_load().orc_num_threads())


def set_num_threads(n):
    _load().orc_set_num_threads(int(n))


def xi_second_moment_integral(r, C_hat, C0):
    """xi = I2 / I1 by the trapezoid rule over (0, C0) and the sampled (r, C-hat).

    r must be strictly increasing and positive.  The integration stops at
    r_cut, the last sampled r before the first non-positive C-hat.
    """
    r = np.asarray(r, dtype=np.float64)
    C = np.asarray(C_hat, dtype=np.float64)
    rr = [0.0]
    cc = [float(C0)]
    if C0 <= 0.0:
        return 0.0
    for q in range(r.shape[0]):
        if not (C[q] > 0.0):
            break
        rr.append(float(r[q]))
        cc.append(float(C[q]))
    if len(rr) < 2:
        return 0.0
    I1 = 0.0
    I2 = 0.0
    for a in range(len(rr) - 1):
        h = rr[a + 1] - rr[a]
        I1 += h * (rr[a] * cc[a] + rr[a + 1] * cc[a + 1]) / 2.0
        I2 += h * (rr[a] ** 2 * cc[a] + rr[a + 1] ** 2 * cc[a + 1]) / 2.0
    if I1 <= 0.0:
        return 0.0
    return I2 / I1


def derive(L, J, Delta, sums, r):
    """FP64 observables from the integer sums of measure()."""
    N = float(L) * float(L)
    Sx = np.asarray(sums["Sx"], dtype=np.float64)
    Sy = np.asarray(sums["Sy"], dtype=np.float64)
    C_hat = (Sx + Sy) / (2.0 * N)
    C0 = sums["sum_s2"] / N
    e = (-J * sums["bond"] + Delta * sums["sum_s2"]) / N
    m = sums["sum_s"] / N
    xi = xi_second_moment_integral(r, C_hat, C0)
    return {"e": e, "m": m, "C_hat": C_hat, "xi": xi}
