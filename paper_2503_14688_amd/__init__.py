"""Python binding of libspin.so (include/spin.h): argument marshalling only.

Checkerboard Metropolis dynamics of the 2D Ising and spin-1 Blume-Capel
models (arXiv:2503.14688) on MI355X (gfx950).  Every step of the dynamics,
the measurements and the derived observables runs inside the native library;
this module converts arguments, allocates the caller-owned device buffer
with torch and raises on error codes.  There is no fallback: if libspin.so
is missing or fails to load, every call raises.
"""
import ctypes
import os

import numpy as np

ISING = 0
BLUME_CAPEL = 1
FUSE_MEASURE = 1
SCHEDULE_CONSTANT = 0
SCHEDULE_TWO_STEP = 1
SCHEDULE_EXPONENTIAL = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspin.so")
_lib = None


class SpinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class spin_meas(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint64), ("sum_s", ctypes.c_int64), ("sum_s2", ctypes.c_int64),
                ("bond", ctypes.c_int64), ("e", ctypes.c_double), ("m", ctypes.c_double),
                ("xi", ctypes.c_double)]


class spin_fourier(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint64), ("sum_s", ctypes.c_int64), ("sum_s2", ctypes.c_int64),
                ("bond", ctypes.c_int64), ("e", ctypes.c_double), ("re_k1", ctypes.c_double),
                ("im_k1", ctypes.c_double), ("re_k2", ctypes.c_double), ("im_k2", ctypes.c_double)]


BATCH_DIRECT = 1


BATCH_VARIANTS = 9  # batched strategies: (Ising, Blume-Capel) sweep strategy pairs


def BATCH_VARIANT(v):
    """spin_batch_run flag forcing batched strategy v (0 <= v < BATCH_VARIANTS):
    sweep strategy v for both models for v < 5, else the (Ising, Blume-Capel)
    pair (2, 0), (2, 3), (1, 3) or (2, 1)."""
    if not 0 <= v < BATCH_VARIANTS:
        raise ValueError(f"batched strategy {v} outside 0..{BATCH_VARIANTS - 1}")
    return (v + 1) << 4



class spin_replica_desc(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("L", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("J", ctypes.c_double), ("Delta", ctypes.c_double), ("dev_buf", ctypes.c_void_p),
                ("buf_bytes", ctypes.c_size_t), ("schedule", ctypes.c_uint32), ("t0", ctypes.c_uint64)]


EXPORTS = ["spin_lattice_bytes", "spin_create", "spin_init_random", "spin_sweep", "spin_sweep_ex",
           "spin_measure", "spin_measure_noalloc", "spin_get_spins", "spin_get_window", "spin_set_spins", "spin_set_t",
           "spin_get_t", "spin_threshold_table", "spin_schedule_fill", "spin_destroy",
           "spin_set_variant", "spin_get_variant", "spin_tune", "spin_sw", "spin_measure_fourier",
           "spin_last_error", "spin_batch_create", "spin_batch_init_random", "spin_batch_run",
           "spin_batch_sync", "spin_batch_replica", "spin_batch_measure", "spin_batch_sw",
           "spin_batch_measure_fourier", "spin_batch_info", "spin_batch_destroy"]


def load_library():
    """Load libspin.so (built by paper_2503_14688_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_14688_amd/build.py "
                          "(no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    i8p = ctypes.POINTER(ctypes.c_int8)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    sig = {
        "spin_lattice_bytes": (ctypes.c_int64, [ctypes.c_int, ctypes.c_uint32]),
        "spin_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                       ctypes.c_double, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "spin_init_random": (ctypes.c_int, [vp]),
        "spin_sweep": (ctypes.c_int, [vp, ctypes.c_uint32, f64p]),
        "spin_sweep_ex": (ctypes.c_int, [vp, ctypes.c_uint32, f64p, ctypes.c_uint32]),
        "spin_measure": (ctypes.c_int, [vp, u32p, ctypes.c_uint32, ctypes.POINTER(spin_meas), i64p, i64p,
                                        f64p]),
        "spin_measure_noalloc": (ctypes.c_int, [vp, u32p, ctypes.c_uint32, ctypes.POINTER(spin_meas), i64p,
                                                i64p, f64p]),
        "spin_get_spins": (ctypes.c_int, [vp, i8p]),
        "spin_get_window": (ctypes.c_int, [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32, i8p]),
        "spin_set_spins": (ctypes.c_int, [vp, i8p]),
        "spin_set_t": (ctypes.c_int, [vp, ctypes.c_uint64]),
        "spin_get_t": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "spin_threshold_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, u32p, u8p, ctypes.c_int]),
        "spin_schedule_fill": (ctypes.c_int, [ctypes.c_int, f64p, ctypes.c_uint64, ctypes.c_uint32,
                                              f64p]),
        "spin_destroy": (ctypes.c_int, [vp]),
        "spin_set_variant": (ctypes.c_int, [vp, ctypes.c_int]),
        "spin_get_variant": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int)]),
        "spin_tune": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
        "spin_sw": (ctypes.c_int, [vp, ctypes.c_uint32, f64p]),
        "spin_measure_fourier": (ctypes.c_int, [vp, ctypes.POINTER(spin_fourier), i64p, i64p]),
        "spin_last_error": (ctypes.c_char_p, []),
        "spin_batch_create": (ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(spin_replica_desc), ctypes.c_uint32,
                                             ctypes.c_uint32, f64p, vp, ctypes.POINTER(vp)]),
        "spin_batch_init_random": (ctypes.c_int, [vp]),
        "spin_batch_run": (ctypes.c_int, [vp, ctypes.c_uint32, ctypes.c_uint32]),
        "spin_batch_sync": (ctypes.c_int, [vp]),
        "spin_batch_replica": (ctypes.c_int, [vp, ctypes.c_uint32, ctypes.POINTER(vp)]),
        "spin_batch_measure": (ctypes.c_int, [vp, u32p, ctypes.c_uint32, ctypes.POINTER(spin_meas), i64p, i64p]),
        "spin_batch_sw": (ctypes.c_int, [vp]),
        "spin_batch_measure_fourier": (ctypes.c_int, [vp, ctypes.POINTER(spin_fourier)]),
        "spin_batch_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint64)]),
        "spin_batch_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc):
    if rc < 0:
        raise SpinError(rc, load_library().spin_last_error().decode())
    return rc


# ---------------------------------------------------------------- C ABI --

def spin_lattice_bytes(model, L):
    return _check(load_library().spin_lattice_bytes(model, L))


def spin_create(model, L, seed, J, Delta, dev_ptr, buf_bytes, hip_stream):
    h = ctypes.c_void_p()
    _check(load_library().spin_create(model, L, seed, J, Delta, ctypes.c_void_p(dev_ptr), buf_bytes,
                                      ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h


def spin_init_random(h):
    _check(load_library().spin_init_random(h))


def spin_sweep(h, T):
    T = np.ascontiguousarray(T, dtype=np.float64)
    _check(load_library().spin_sweep(h, T.shape[0], _ptr(T, ctypes.c_double)))


def spin_sweep_ex(h, T, flags):
    T = np.ascontiguousarray(T, dtype=np.float64)
    _check(load_library().spin_sweep_ex(h, T.shape[0], _ptr(T, ctypes.c_double), flags))


def spin_measure(h, r=()):
    """Returns dict(t, sum_s, sum_s2, bond, e, m, xi, Sx, Sy, C_hat)."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    n = r.shape[0]
    Sx = np.zeros(n, dtype=np.int64)
    Sy = np.zeros(n, dtype=np.int64)
    C = np.zeros(n, dtype=np.float64)
    out = spin_meas()
    _check(load_library().spin_measure(h, _ptr(r, ctypes.c_uint32), n, ctypes.byref(out),
                                       _ptr(Sx, ctypes.c_int64), _ptr(Sy, ctypes.c_int64),
                                       _ptr(C, ctypes.c_double)))
    return {"t": out.t, "sum_s": out.sum_s, "sum_s2": out.sum_s2, "bond": out.bond, "e": out.e,
            "m": out.m, "xi": out.xi, "Sx": Sx, "Sy": Sy, "C_hat": C}


def spin_measure_noalloc(h, r=()):
    """spin_measure through the entry point that allocates no device memory."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    n = r.shape[0]
    Sx = np.zeros(n, dtype=np.int64)
    Sy = np.zeros(n, dtype=np.int64)
    C = np.zeros(n, dtype=np.float64)
    out = spin_meas()
    _check(load_library().spin_measure_noalloc(h, _ptr(r, ctypes.c_uint32), n, ctypes.byref(out),
                                               _ptr(Sx, ctypes.c_int64), _ptr(Sy, ctypes.c_int64),
                                               _ptr(C, ctypes.c_double)))
    return {"t": out.t, "sum_s": out.sum_s, "sum_s2": out.sum_s2, "bond": out.bond, "e": out.e,
            "m": out.m, "xi": out.xi, "Sx": Sx, "Sy": Sy, "C_hat": C}


def spin_get_spins(h, L):
    s = np.zeros((L, L), dtype=np.int8)
    _check(load_library().spin_get_spins(h, _ptr(s, ctypes.c_int8)))
    return s


def spin_get_window(h, i0, j0, rows, cols):
    w = np.zeros((rows, cols), dtype=np.int8)
    _check(load_library().spin_get_window(h, i0, j0, rows, cols, _ptr(w, ctypes.c_int8)))
    return w


def spin_set_spins(h, s):
    s = np.ascontiguousarray(s, dtype=np.int8)
    _check(load_library().spin_set_spins(h, _ptr(s, ctypes.c_int8)))


def spin_set_t(h, t):
    _check(load_library().spin_set_t(h, t))


def spin_get_t(h):
    t = ctypes.c_uint64()
    _check(load_library().spin_get_t(h, ctypes.byref(t)))
    return t.value


def spin_threshold_table(model, J, Delta, T):
    out = np.zeros(32, dtype=np.uint32)
    always = np.zeros(32, dtype=np.uint8)
    n = _check(load_library().spin_threshold_table(model, J, Delta, T, _ptr(out, ctypes.c_uint32),
                                                   _ptr(always, ctypes.c_uint8), 32))
    return out[:n].copy(), always[:n].astype(bool)


def spin_schedule_fill(kind, params, t0, n):
    p = np.zeros(3, dtype=np.float64)
    p[:len(params)] = params
    out = np.zeros(n, dtype=np.float64)
    _check(load_library().spin_schedule_fill(kind, _ptr(p, ctypes.c_double), t0, n,
                                             _ptr(out, ctypes.c_double)))
    return out


def spin_destroy(h):
    _check(load_library().spin_destroy(h))


def spin_set_variant(h, v):
    _check(load_library().spin_set_variant(h, v))


def spin_get_variant(h):
    v = ctypes.c_int()
    _check(load_library().spin_get_variant(h, ctypes.byref(v)))
    return v.value


def spin_tune(h, T):
    v = ctypes.c_int()
    _check(load_library().spin_tune(h, T, ctypes.byref(v)))
    return v.value


def spin_sw(h, T):
    """len(T) Swendsen-Wang steps restricted to the non-zero spins."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    _check(load_library().spin_sw(h, T.shape[0], _ptr(T, ctypes.c_double)))


def spin_measure_fourier(h, L):
    """dict(t, sum_s, sum_s2, bond, e, k1, k2 (complex), row, col)."""
    out = spin_fourier()
    row = np.zeros(L, dtype=np.int64)
    col = np.zeros(L, dtype=np.int64)
    _check(load_library().spin_measure_fourier(h, ctypes.byref(out), _ptr(row, ctypes.c_int64),
                                               _ptr(col, ctypes.c_int64)))
    return {"t": out.t, "sum_s": out.sum_s, "sum_s2": out.sum_s2, "bond": out.bond, "e": out.e,
            "k1": complex(out.re_k1, out.im_k1), "k2": complex(out.re_k2, out.im_k2), "row": row, "col": col}


def spin_last_error():
    return load_library().spin_last_error().decode()


def spin_batch_create(descs, T, hip_stream=0):
    """descs: list of spin_replica_desc; T: (n_sched, n_steps) float64."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    arr = (spin_replica_desc * len(descs))(*descs)
    b = ctypes.c_void_p()
    _check(load_library().spin_batch_create(len(descs), arr, T.shape[0], T.shape[1], _ptr(T, ctypes.c_double),
                                            ctypes.c_void_p(hip_stream), ctypes.byref(b)))
    return b


def spin_batch_init_random(b):
    _check(load_library().spin_batch_init_random(b))


def spin_batch_run(b, n, flags=0):
    _check(load_library().spin_batch_run(b, n, flags))


def spin_batch_sync(b):
    _check(load_library().spin_batch_sync(b))


def spin_batch_measure(b, n, r=()):
    """Per-replica measurements: list of dicts as spin_measure returns."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    nr = r.shape[0]
    out = (spin_meas * n)()
    Sx = np.zeros((n, nr), dtype=np.int64)
    Sy = np.zeros((n, nr), dtype=np.int64)
    _check(load_library().spin_batch_measure(b, _ptr(r, ctypes.c_uint32), nr, out, _ptr(Sx, ctypes.c_int64),
                                             _ptr(Sy, ctypes.c_int64)))
    return [{"t": o.t, "sum_s": o.sum_s, "sum_s2": o.sum_s2, "bond": o.bond, "e": o.e, "m": o.m, "xi": o.xi,
             "Sx": Sx[k], "Sy": Sy[k]} for k, o in enumerate(out)]


def spin_batch_sw(b):
    _check(load_library().spin_batch_sw(b))


def spin_batch_measure_fourier(b, n):
    """Per-replica Fourier moments: list of dicts as spin_measure_fourier
    returns, without the row and column sums."""
    out = (spin_fourier * n)()
    _check(load_library().spin_batch_measure_fourier(b, out))
    return [{"t": o.t, "sum_s": o.sum_s, "sum_s2": o.sum_s2, "bond": o.bond, "e": o.e,
             "k1": complex(o.re_k1, o.im_k1), "k2": complex(o.re_k2, o.im_k2)} for o in out]


def spin_batch_replica(b, k):
    h = ctypes.c_void_p()
    _check(load_library().spin_batch_replica(b, k, ctypes.byref(h)))
    return h


def spin_batch_info(b):
    n = ctypes.c_uint32()
    t = ctypes.c_uint64()
    variant = ctypes.c_int()
    tiles = ctypes.c_uint64()
    _check(load_library().spin_batch_info(b, ctypes.byref(n), ctypes.byref(t), ctypes.byref(variant),
                                          ctypes.byref(tiles)))
    return {"replicas": n.value, "t": t.value, "variant": variant.value, "tiles": tiles.value}


def spin_batch_destroy(b):
    _check(load_library().spin_batch_destroy(b))


# ------------------------------------------------- device-buffer holder --

class Lattice:
    """A lattice whose packed spins live in a torch uint8 tensor on the GPU.

    Holds the tensor (the caller-owned buffer of the C ABI) and the handle;
    methods forward to the C ABI on the handle's stream.
    """

    def __init__(self, model, L, seed, J=1.0, Delta=0.0, device="cuda", stream=None):
        import torch
        self.model, self.L, self.seed, self.J, self.Delta = model, L, seed, J, Delta
        nbytes = spin_lattice_bytes(model, L)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buf.device)
        self.h = spin_create(model, L, seed, J, Delta, self.buf.data_ptr(), nbytes,
                             self.stream.cuda_stream)

    def init_random(self):
        spin_init_random(self.h)
        return self

    def sweep(self, T, fuse_measure=False):
        spin_sweep_ex(self.h, T, FUSE_MEASURE if fuse_measure else 0)

    def measure(self, r=()):
        return spin_measure(self.h, r)

    def spins(self):
        return spin_get_spins(self.h, self.L)

    @property
    def variant(self):
        return spin_get_variant(self.h)

    @variant.setter
    def variant(self, v):
        spin_set_variant(self.h, v)

    def tune(self, T):
        return spin_tune(self.h, T)

    def sw(self, T):
        spin_sw(self.h, T)

    def fourier(self):
        return spin_measure_fourier(self.h, self.L)

    def window(self, i0, j0, rows, cols):
        return spin_get_window(self.h, i0, j0, rows, cols)

    def set_spins(self, s):
        spin_set_spins(self.h, s)

    @property
    def t(self):
        return spin_get_t(self.h)

    @t.setter
    def t(self, value):
        spin_set_t(self.h, value)

    def close(self):
        if self.h is not None:
            spin_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Replicas in torch uint8 device buffers, advanced together by the C ABI.

    reps: dicts with model, L, seed, J, Delta and schedule (row index of T).
    """

    def __init__(self, reps, T, device="cuda"):
        import torch
        self.reps = reps
        self.bufs = []
        descs = []
        for r in reps:
            nbytes = spin_lattice_bytes(r["model"], r["L"])
            buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
            self.bufs.append(buf)
            descs.append(spin_replica_desc(r["model"], r["L"], r["seed"], r.get("J", 1.0), r.get("Delta", 0.0),
                                           buf.data_ptr(), nbytes, r["schedule"], r.get("t0", 0)))
        self.b = spin_batch_create(descs, T)

    def init_random(self):
        spin_batch_init_random(self.b)
        return self

    def run(self, n, flags=0):
        spin_batch_run(self.b, n, flags)

    def sync(self):
        spin_batch_sync(self.b)

    def replica(self, k):
        return spin_batch_replica(self.b, k)

    def spins(self, k):
        return spin_get_spins(self.replica(k), self.reps[k]["L"])

    def measure(self, k, r=()):
        return spin_measure(self.replica(k), r)

    def measure_all(self, r=()):
        return spin_batch_measure(self.b, len(self.reps), r)

    def sw(self):
        """One Swendsen-Wang step on every replica (one schedule step)."""
        spin_batch_sw(self.b)

    def fourier_all(self):
        return spin_batch_measure_fourier(self.b, len(self.reps))

    def info(self):
        return spin_batch_info(self.b)

    def close(self):
        if self.b is not None:
            spin_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
