"""spin_measure_noalloc (the measurement entry point that allocates no device
memory) against spin_measure on the same states, through the C ABI: two
calls in a row on each model, the second on a smaller lattice with fewer
separations, and the oracle's sums as the common reference."""
import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads

pytestmark = pytest.mark.gpu


def check_same(gpu, lat, r):
    a = gpu.spin_measure(lat.h, r)
    b = gpu.spin_measure_noalloc(lat.h, r)
    for k in ("t", "sum_s", "sum_s2", "bond", "e", "m", "xi"):
        assert a[k] == b[k], k
    for k in ("Sx", "Sy", "C_hat"):
        assert np.array_equal(a[k], b[k]), k
    want = oracle.measure(lat.spins(), r)
    assert b["sum_s"] == want["sum_s"] and b["bond"] == want["bond"] and b["sum_s2"] == want["sum_s2"]
    assert np.array_equal(b["Sx"], want["Sx"]) and np.array_equal(b["Sy"], want["Sy"])


@pytest.mark.parametrize("model", [0, 1])
def test_noalloc_measure_matches_measure(gpu, model):
    T = workloads.TC_ISING if model == 0 else workloads.TC_BC
    # first call: L = 512 on the sparse separations (the fast kernels) plus
    # one off-set separation (the generic kernels)
    big = gpu.Lattice(model, 512, 4242).init_random()
    big.sweep(np.full(5, T), fuse_measure=True)
    check_same(gpu, big, workloads.r_sparse(512))
    check_same(gpu, big, np.append(workloads.r_sparse(512), np.uint32(257)))
    # second call: a smaller lattice and fewer separations; the counters
    # the first call left behind must not leak into it
    small = gpu.Lattice(model, 128, 99).init_random()
    small.sweep(np.full(3, T))
    check_same(gpu, small, np.array([1, 2, 5], dtype=np.uint32))
    check_same(gpu, small, np.array([], dtype=np.uint32))
    big.close()
    small.close()


def test_noalloc_measure_limits(gpu):
    lat = gpu.Lattice(0, 2048, 7).init_random()
    with pytest.raises(gpu.SpinError):
        gpu.spin_measure_noalloc(lat.h, np.arange(1, 1026, dtype=np.uint32))  # 1025 > 1024
    r = np.arange(1, 1025, dtype=np.uint32)  # exactly the limit
    a = gpu.spin_measure(lat.h, r)
    b = gpu.spin_measure_noalloc(lat.h, r)
    assert np.array_equal(a["Sx"], b["Sx"]) and np.array_equal(a["Sy"], b["Sy"]) and a["bond"] == b["bond"]
    lat.close()
