"""C ABI checks that need no GPU: the library loads, exports every symbol
include/spin.h declares, validates arguments, and its host-side arithmetic
(acceptance thresholds, schedules) equals the oracle's independently written
definition bit for bit."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2503_14688_amd as spin
from paper_2503_14688_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "spin.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spin_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_functions():
    names = declared_functions()
    assert "spin_sweep" in names and "spin_measure" in names
    assert sorted(spin.EXPORTS) == names


def test_batch_flags_match_header():
    text = open(os.path.join(ROOT, "include", "spin.h")).read()
    assert int(re.search(r"#define SPIN_BATCH_VARIANTS (\d+)", text).group(1)) == spin.BATCH_VARIANTS
    assert spin.BATCH_VARIANT(0) == 1 << 4 and spin.BATCH_VARIANT(spin.BATCH_VARIANTS - 1) == spin.BATCH_VARIANTS << 4
    for bad in (-1, spin.BATCH_VARIANTS):
        with pytest.raises(ValueError):
            spin.BATCH_VARIANT(bad)


def test_library_exports_every_declared_symbol():
    lib = spin.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_batch_calls_reject_null_batches():
    """The batch entry points check their arguments before any HIP call."""
    lib = spin.load_library()
    out = (spin.spin_fourier * 1)()
    assert lib.spin_batch_sw(None) == -22
    assert lib.spin_batch_measure_fourier(None, out) == -22
    assert lib.spin_batch_run(None, 1, 0) == -22
    assert lib.spin_batch_measure(None, None, 0, None, None, None) == -22
    assert "NULL" in spin.spin_last_error()


def test_lattice_bytes_and_validation():
    assert spin.spin_lattice_bytes(spin.ISING, 64) == 64 * 64 // 8
    assert spin.spin_lattice_bytes(spin.BLUME_CAPEL, 64) == 64 * 64 // 4
    assert spin.spin_lattice_bytes(spin.ISING, 1 << 20) == (1 << 40) // 8
    assert spin.spin_lattice_bytes(spin.BLUME_CAPEL, 1 << 22) == (1 << 44) // 4
    for model, L in [(spin.ISING, 32), (spin.ISING, 100), (spin.ISING, (1 << 22) + 64), (7, 64)]:
        with pytest.raises(spin.SpinError) as ei:
            spin.spin_lattice_bytes(model, L)
        assert ei.value.code == -22
    with pytest.raises(spin.SpinError):
        spin.spin_create(spin.ISING, 64, 1, 1.0, 0.5, 0, 0, 0)   # Ising with Delta != 0
    with pytest.raises(spin.SpinError):
        spin.spin_create(spin.ISING, 64, 1, -1.0, 0.0, 0, 0, 0)  # J <= 0
    with pytest.raises(spin.SpinError):
        spin.spin_create(spin.ISING, 64, 1, 1.0, 0.0, 0, 512, 0)  # NULL buffer
    host = np.zeros(512, dtype=np.uint8)
    with pytest.raises(spin.SpinError) as ei:  # host memory is rejected before any launch
        spin.spin_create(spin.ISING, 64, 1, 1.0, 0.0, host.ctypes.data, 512, 0)
    assert "device memory" in str(ei.value) or "aligned" in str(ei.value)


@pytest.mark.parametrize("T", [workloads.TC_ISING, 1.0, 2.0, 3.7, 0.3, 50.0, 0.0, float("inf")])
@pytest.mark.parametrize("J", [1.0, 0.37, 2.5])
def test_ising_thresholds_equal_oracle(T, J):
    thr, always = spin.spin_threshold_table(spin.ISING, J, 0.0, T)
    for q, dE in enumerate((4.0 * J, 8.0 * J)):
        a, t = oracle.threshold(dE, T)
        assert bool(always[q]) == a and (a or int(thr[q]) == t)


@pytest.mark.parametrize("T", [workloads.TC_BC, workloads.T_BC_WORKLOAD, 0.7, 2.9, 0.0, float("inf")])
@pytest.mark.parametrize("J,Delta", [(1.0, 0.0), (1.0, 0.5), (0.8, -1.3), (1.7, 2.0)])
def test_blume_capel_thresholds_equal_oracle(T, J, Delta):
    thr, always = spin.spin_threshold_table(spin.BLUME_CAPEL, J, Delta, T)
    assert thr.shape[0] == 27
    for f, (s, sp) in enumerate([(1, 0), (0, 1), (1, -1)]):
        for v in range(9):
            y = v - 4
            dE = -J * float((sp - s) * y) + Delta * float(sp * sp - s * s)
            a, t = oracle.threshold(dE, T)
            assert bool(always[9 * f + v]) == a
            if not a:
                assert int(thr[9 * f + v]) == t


def test_published_threshold_values():
    thr, always = spin.spin_threshold_table(spin.ISING, 1.0, 0.0, workloads.TC_ISING)
    assert thr.tolist() == [736899888, 126432032] and not always.any()


@pytest.mark.parametrize("kind,params", [(0, [2.269]), (1, [1.66, 5312, 2.27414861561203]),
                                         (2, [2 * workloads.TC_ISING, 1.02 * workloads.TC_ISING, 64.0]),
                                         (2, [2 * workloads.TC_BC, 1.02 * workloads.TC_BC, 1024.0])])
def test_schedules_equal_oracle(kind, params):
    for t0, n in [(0, 300), (5000, 700), (123456, 10)]:
        a = spin.spin_schedule_fill(kind, params, t0, n)
        b = oracle.schedule(kind, params, t0, n)
        assert np.array_equal(a, b)


def test_sparse_r_set():
    r = workloads.r_sparse(1 << 20)
    assert r[0] == 1 and r[15] == 16 and r[-1] == 4096 and len(r) == 48
    assert np.all(np.diff(r.astype(np.int64)) > 0)
    assert workloads.r_sparse(64).max() == 32
    assert math.isclose(workloads.TC_ISING, 2.26918531421302196814, rel_tol=1e-15)
