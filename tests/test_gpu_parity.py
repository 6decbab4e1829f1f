"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results -- spin configurations, sum s, sum s^2, the bond sum and the
correlation sums S_x(r), S_y(r) -- must be bit-exact.  The FP64 observables
(e, m, C-hat, xi) are derived from those integers by separate code on each
side; they must agree to 1e-12 relative (the same IEEE operations in the same
order give equal values; the bound only allows for a reordered sum).

Sizes: L = 64 .. 4096 full-lattice comparisons (several row groups and word
columns per thread block, L = 192 and 320 give word counts that are not
powers of two), and the full workload sizes (Ising L = 2^20, 128 GiB;
Blume-Capel L = 2^18, 16 GiB) on sampled windows that the oracle evolves by
light cone from the same initial state.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2503_14688_amd import workloads

pytestmark = pytest.mark.gpu

REL = 1e-12


def make(spin, model, L, seed, J=1.0, Delta=0.0):
    return spin.Lattice(model, L, seed, J, Delta).init_random()


def compare_measure(got, L, J, Delta, s, r):
    want = oracle.measure(s, r)
    for k in ("sum_s", "sum_s2", "bond"):
        assert got[k] == want[k], k
    assert np.array_equal(got["Sx"], want["Sx"])
    assert np.array_equal(got["Sy"], want["Sy"])
    d = oracle.derive(L, J, Delta, want, r)
    for k in ("e", "m", "xi"):
        assert abs(got[k] - d[k]) <= REL * max(1.0, abs(d[k])), k
    assert np.allclose(got["C_hat"], d["C_hat"], rtol=REL, atol=0)


@pytest.mark.parametrize("model", [oracle.ISING, oracle.BLUME_CAPEL])
@pytest.mark.parametrize("L", [64, 192, 256])
def test_initial_state(gpu, model, L):
    lat = make(gpu, model, L, 2503146880 + L)
    assert np.array_equal(lat.spins(), oracle.init(model, L, 2503146880 + L))
    lat.close()


def test_ising_L64_quench_at_tc(gpu):
    """The small Ising workload: L = 64, T_c, 1024 sweeps, measured at 0 and 2^k."""
    w = workloads.ISING_SMALL
    L, seed, T = w["L"], w["seed"], w["T"]
    r = workloads.r_dense(L)
    lat = make(gpu, 0, L, seed)
    s = oracle.init(0, L, seed)
    done = 0
    for t in workloads.measure_times(w["sweeps"]):
        n = t - done
        if n:
            lat.sweep(np.full(n, T), fuse_measure=True)
            oracle.sweep(0, s, seed, 1.0, 0.0, done, np.full(n, T))
            done = t
        assert np.array_equal(lat.spins(), s), t
        got = lat.measure(r)
        assert got["t"] == t
        compare_measure(got, L, 1.0, 0.0, s, r)
    lat.close()


@pytest.mark.parametrize("model,J,Delta,L", [(0, 1.0, 0.0, 128), (0, 0.6, 0.0, 320),
                                             (1, 1.0, 0.0, 128), (1, 1.0, 0.5, 192),
                                             (1, 1.4, -0.9, 320)])
def test_time_dependent_schedule(gpu, model, J, Delta, L):
    """Per-sweep bath temperatures, including T = 0 and T = inf sweeps."""
    seed = 777 + L
    rng = np.random.default_rng(seed)
    T = rng.uniform(0.5, 4.0, size=40) * J
    T[5] = 0.0
    T[17] = np.inf
    T[30:33] = 0.0
    r = workloads.r_dense(L)
    lat = make(gpu, model, L, seed, J, Delta)
    s = oracle.init(model, L, seed)
    for a in range(0, 40, 8):
        lat.sweep(T[a:a + 8])
        oracle.sweep(model, s, seed, J, Delta, a, T[a:a + 8])
        assert np.array_equal(lat.spins(), s), a
    compare_measure(lat.measure(r), L, J, Delta, s, r)
    lat.close()


@pytest.mark.parametrize("model", [0, 1])
def test_exponential_schedule_protocol(gpu, model):
    """T(t) = T_f + (T_0 - T_f) e^{-t/tau} from the library's own schedule helper."""
    L, seed = 256, 99
    tc = workloads.TC_ISING if model == 0 else workloads.TC_BC
    params = [2 * tc, 1.02 * tc, 64.0]
    Tg = gpu.spin_schedule_fill(gpu.SCHEDULE_EXPONENTIAL, params, 0, 48)
    To = oracle.schedule(2, params, 0, 48)
    lat = make(gpu, model, L, seed)
    lat.sweep(Tg)
    s = oracle.init(model, L, seed)
    oracle.sweep(model, s, seed, 1.0, 0.0, 0, To)
    assert np.array_equal(lat.spins(), s)
    lat.close()


@pytest.mark.parametrize("model", [0, 1])
def test_chunking_and_fused_measure(gpu, model):
    L, seed, T = 192, 5, 2.1
    a = make(gpu, model, L, seed)
    b = make(gpu, model, L, seed)
    a.sweep(np.full(10, T))
    b.sweep(np.full(3, T))
    b.sweep(np.full(7, T), fuse_measure=True)
    assert np.array_equal(a.spins(), b.spins())
    ma, mb = a.measure(), b.measure()  # standalone reduction vs fused pass
    for k in ("sum_s", "sum_s2", "bond", "t"):
        assert ma[k] == mb[k]
    gpu.spin_sweep_ex(a.h, np.zeros(0), gpu.FUSE_MEASURE)  # fused sums of the current state
    assert a.measure()["bond"] == ma["bond"]
    a.close()
    b.close()


@pytest.mark.parametrize("model", [0, 1])
def test_checkpoint_resume(gpu, model):
    L, seed = 128, 31
    T = np.linspace(1.2, 3.0, 20)
    ref = make(gpu, model, L, seed)
    ref.sweep(T)
    a = make(gpu, model, L, seed)
    a.sweep(T[:7])
    snap, t = a.spins(), a.t
    a.close()
    b = gpu.Lattice(model, L, seed)
    b.set_spins(snap)
    b.t = t
    b.sweep(T[7:])
    assert np.array_equal(b.spins(), ref.spins())
    ref.close()
    b.close()


def test_ising_z2_symmetry(gpu):
    L, seed = 256, 8
    a = make(gpu, 0, L, seed)
    b = gpu.Lattice(0, L, seed)
    b.set_spins(-a.spins())
    T = np.full(12, workloads.TC_ISING)
    a.sweep(T)
    b.sweep(T)
    assert np.array_equal(b.spins(), -a.spins())
    a.close()
    b.close()


@pytest.mark.parametrize("model", [0, 1])
def test_window_decoder(gpu, model):
    L = 192
    lat = make(gpu, model, L, 4)
    lat.sweep(np.full(3, 2.0))
    s = lat.spins()
    for (i0, j0, h, w) in [(0, 0, L, L), (150, 170, 60, 50), (5, 191, 7, 3)]:
        rows = (i0 + np.arange(h)) % L
        cols = (j0 + np.arange(w)) % L
        assert np.array_equal(lat.window(i0, j0, h, w), s[np.ix_(rows, cols)])
    lat.close()


def test_invalid_arguments(gpu):
    lat = make(gpu, 0, 64, 1)
    with pytest.raises(gpu.SpinError):
        lat.sweep(np.array([1.0, -0.5]))
    with pytest.raises(gpu.SpinError):
        lat.sweep(np.array([np.nan]))
    with pytest.raises(gpu.SpinError):
        lat.measure([3, 2])
    with pytest.raises(gpu.SpinError):
        lat.measure([64])
    bad = np.ones((64, 64), dtype=np.int8)
    bad[3, 3] = 0  # vacancy is not an Ising state
    with pytest.raises(gpu.SpinError):
        lat.set_spins(bad)
    with pytest.raises(gpu.SpinError):
        lat.window(64, 0, 2, 2)
    lat.close()


@pytest.mark.parametrize("model,L", [(0, 512), (1, 512), (0, 192), (1, 320)])
def test_sparse_and_generic_correlation_kernels_agree(gpu, model, L):
    """The sparse-set kernels (LDS tiles / LDS ring) against the generic ones
    (a list that is not a prefix of the sparse set) and the oracle."""
    lat = make(gpu, model, L, 13)
    lat.sweep(np.full(4, 2.2 if model == 0 else 1.6))
    r_fast = workloads.r_sparse(L)
    r_slow = np.append(r_fast, np.uint32(r_fast[-1] + 1))
    a, b = lat.measure(r_fast), lat.measure(r_slow)
    n = len(r_fast)
    assert np.array_equal(a["Sx"], b["Sx"][:n]) and np.array_equal(a["Sy"], b["Sy"][:n])
    compare_measure(a, L, 1.0, 0.0, lat.spins(), r_fast)
    lat.close()


@pytest.mark.parametrize("model,L", [(0, 65536), (0, 131072), (1, 65536)])
def test_whole_segment_correlation_kernel(gpu, model, L):
    """Rows of whole 1024-word segments take the run-per-lane horizontal
    kernel (one segment per row at L = 65536, where the halo wraps to the
    row start; two at L = 131072, where it runs into the next segment).  It
    must match the generic per-separation kernels on the full sparse set."""
    lat = make(gpu, model, L, 29)
    lat.sweep(np.full(2, 2.2 if model == 0 else 1.6))
    r_fast = workloads.r_sparse(L)
    r_slow = np.append(r_fast, np.uint32(r_fast[-1] + 1))
    a, b = lat.measure(r_fast), lat.measure(r_slow)
    n = len(r_fast)
    assert np.array_equal(a["Sx"], b["Sx"][:n]) and np.array_equal(a["Sy"], b["Sy"][:n])
    assert a["bond"] == b["bond"]
    lat.close()


@pytest.mark.parametrize("model", [0, 1])
def test_sweep_strategies_agree(gpu, model):
    """All sweep strategies (rows per thread, per-word or compacting lazy
    test, list size) give the oracle's trajectory; the tuner picks one."""
    L, seed = 512, 77
    T = np.full(6, 2.2 if model == 0 else 1.7)
    s = oracle.init(model, L, seed)
    oracle.sweep(model, s, seed, 1.0, 0.0, 0, T)
    bond = oracle.measure(s, [])["bond"]
    for v in range(5):
        lat = make(gpu, model, L, seed)
        lat.variant = v
        assert lat.variant == v
        lat.sweep(T, fuse_measure=True)
        assert np.array_equal(lat.spins(), s), v
        assert lat.measure()["bond"] == bond
        lat.close()
    lat = make(gpu, model, L, seed)
    assert lat.tune(float(T[0])) in range(5)
    lat.sweep(T)
    assert np.array_equal(lat.spins(), s)
    with pytest.raises(gpu.SpinError):
        lat.variant = 5
    lat.close()


def test_uniform_row_tiles_all_strategies(gpu):
    """L = 16384: a plane row is a whole number of 256-word tiles, so the Ising
    sweep takes its row-uniform path (the path of the L = 2^20 workload).
    Every strategy, including the 16-slot list whose overflow words finish in
    place, reproduces the oracle's trajectory and bond sum after 3 sweeps and
    after 64 sweeps at T_c (the depth of the timed workload, where the relaxed
    lattice sends more words to the work list than near the start)."""
    L, seed = 16384, 2024
    Tc = workloads.TC_ISING
    s3 = oracle.init(0, L, seed)
    oracle.sweep(0, s3, seed, 1.0, 0.0, 0, np.full(3, Tc))
    s64 = s3.copy()
    oracle.sweep(0, s64, seed, 1.0, 0.0, 3, np.full(61, Tc))
    bond3, bond64 = oracle.measure(s3, [])["bond"], oracle.measure(s64, [])["bond"]
    for v in range(5):
        print(f"strategy {v}", flush=True)
        lat = make(gpu, 0, L, seed)
        lat.variant = v
        lat.sweep(np.full(3, Tc), fuse_measure=True)
        assert lat.measure()["bond"] == bond3, v
        assert np.array_equal(lat.spins(), s3), v
        lat.sweep(np.full(61, Tc), fuse_measure=True)
        assert lat.measure()["bond"] == bond64, v
        assert np.array_equal(lat.spins(), s64), v
        lat.close()


def test_blume_capel_uniform_row_tiles_all_strategies(gpu):
    """Blume-Capel L = 4096 at Delta = 0: a plane row is 64 words, so every
    strategy takes the row-uniform form of its tile (Philox rounds started in
    scalar registers) with the select-free classification; each reproduces
    the oracle's trajectory and bond sum, with the E/M sums fused into the
    last sweep."""
    L, seed = 4096, 4242
    T = np.full(6, workloads.TC_BC)
    s = oracle.init(1, L, seed)
    oracle.sweep(1, s, seed, 1.0, 0.0, 0, T)
    bond = oracle.measure(s, [])["bond"]
    for v in range(5):
        print(f"strategy {v}", flush=True)
        lat = make(gpu, 1, L, seed)
        lat.variant = v
        lat.sweep(T, fuse_measure=True)
        assert lat.measure()["bond"] == bond, v
        assert np.array_equal(lat.spins(), s), v
        lat.close()


@pytest.mark.parametrize("J,Delta,T", [(1.0, 0.5, 1.5), (1.3, -0.9, 2.6)])
def test_blume_capel_general_delta_all_strategies(gpu, J, Delta, T):
    """Blume-Capel at Delta != 0 takes the 13-group test (no merged groups, no
    plane-pattern branch): every sweep strategy, with the fused measurement,
    gives the oracle's lattice and sums at L = 512 (rows of 8 words), and the
    tuned one does at L = 4096 (rows of 64 words) over 16 sweeps."""
    L, seed = 512, 4321
    Ts = np.full(6, T)
    s = oracle.init(1, L, seed)
    oracle.sweep(1, s, seed, J, Delta, 0, Ts)
    want = oracle.measure(s, [])
    for v in range(5):
        lat = make(gpu, 1, L, seed, J, Delta)
        lat.variant = v
        lat.sweep(Ts, fuse_measure=True)
        assert np.array_equal(lat.spins(), s), v
        got = lat.measure()
        assert (got["bond"], got["sum_s"], got["sum_s2"]) == (want["bond"], want["sum_s"], want["sum_s2"]), v
        lat.close()
    L = 4096
    r = workloads.r_sparse(L)
    Ts = np.full(16, T)
    lat = make(gpu, 1, L, seed, J, Delta)
    lat.variant = lat.tune(T)
    s = oracle.init(1, L, seed)
    lat.sweep(Ts, fuse_measure=True)
    oracle.sweep(1, s, seed, J, Delta, 0, Ts)
    assert np.array_equal(lat.spins(), s)
    compare_measure(lat.measure(r), L, J, Delta, s, r)
    lat.close()


@pytest.mark.parametrize("model", [0, 1])
def test_ragged_rows_all_strategies(gpu, model):
    """L = 4160: rows of 65 words (not a multiple of 64, so the general tile
    path with its bounds tests) and a last tile of 8-row groups that is only
    partly filled; every strategy gives the oracle's lattice after 4 sweeps
    at T_c, and the fused sums equal the oracle's."""
    L, seed = 4160, 2718
    T = np.full(4, workloads.TC_ISING if model == 0 else workloads.TC_BC)
    s = oracle.init(model, L, seed)
    oracle.sweep(model, s, seed, 1.0, 0.0, 0, T)
    want = oracle.measure(s, [])
    for v in range(5):
        lat = make(gpu, model, L, seed)
        lat.variant = v
        lat.sweep(T, fuse_measure=True)
        assert np.array_equal(lat.spins(), s), v
        got = lat.measure()
        assert (got["bond"], got["sum_s"], got["sum_s2"]) == (want["bond"], want["sum_s"], want["sum_s2"]), v
        lat.close()


def test_ising_L4096_check_run(gpu):
    """The bit-exact check lattice of the large Ising workload: 2^12 x 2^12, 64 sweeps."""
    w = workloads.ISING_CHECK
    L, seed, T = w["L"], w["seed"], w["T"]
    r = workloads.r_sparse(L)
    lat = make(gpu, 0, L, seed)
    s = oracle.init(0, L, seed)
    lat.sweep(np.full(w["sweeps"], T), fuse_measure=True)
    oracle.sweep(0, s, seed, 1.0, 0.0, 0, np.full(w["sweeps"], T))
    assert np.array_equal(lat.spins(), s)
    compare_measure(lat.measure(r), L, 1.0, 0.0, s, r)
    lat.close()


def test_blume_capel_L4096_check_run(gpu):
    """The Blume-Capel check lattice: 2^12 x 2^12 at T = 1.6937, 256 sweeps."""
    w = workloads.BC_CHECK
    L, seed, T = w["L"], w["seed"], w["T"]
    r = workloads.r_sparse(L)
    lat = make(gpu, 1, L, seed)
    s = oracle.init(1, L, seed)
    lat.sweep(np.full(w["sweeps"], T), fuse_measure=True)
    oracle.sweep(1, s, seed, 1.0, 0.0, 0, np.full(w["sweeps"], T))
    assert np.array_equal(lat.spins(), s)
    compare_measure(lat.measure(r), L, 1.0, 0.0, s, r)
    lat.close()


def sampled_full_size(gpu, model, L, T, n_sweeps, seed, windows, J=1.0, Delta=0.0):
    import torch
    lat = gpu.Lattice(model, L, seed, J, Delta)
    lat.variant = lat.tune(T)  # the launch configuration the benchmark times
    lat.init_random()
    lat.sweep(np.full(n_sweeps, T), fuse_measure=True)
    k = 2 * n_sweeps
    for (i0, j0, size) in windows:
        print(f"window ({i0}, {j0}) of {size} after {n_sweeps} sweeps", flush=True)
        win = oracle.init_window(model, L, seed, i0, j0, size, size)
        oracle.window_sweep(model, win, L, seed, J, Delta, i0, j0, 0, np.full(n_sweeps, T))
        got = lat.window(i0, j0, size, size)
        assert np.array_equal(got[k:size - k, k:size - k], win[k:size - k, k:size - k]), (i0, j0)
    # properties that hold at any size: fused and standalone sums agree,
    # S(0)-type identities, |sums| bounded by the pair counts
    fused = lat.measure([1])
    # a second handle over the same buffer has no fused sums: standalone reduction
    h2 = gpu.spin_create(model, L, seed, J, Delta, lat.buf.data_ptr(), lat.buf.numel(),
                         lat.stream.cuda_stream)
    again = gpu.spin_measure(h2, [1])
    gpu.spin_destroy(h2)
    assert fused["bond"] == again["bond"] == int(fused["Sx"][0] + fused["Sy"][0])
    assert fused["sum_s"] == again["sum_s"] and fused["sum_s2"] == again["sum_s2"]
    assert abs(fused["sum_s"]) <= fused["sum_s2"] <= L * L
    # C(r) on the full sparse set: the fast kernels against the generic ones
    r_fast = workloads.r_sparse(L)
    r_slow = np.append(r_fast, np.uint32(r_fast[-1] + 1))
    a, b = lat.measure(r_fast), lat.measure(r_slow)
    assert np.array_equal(a["Sx"], b["Sx"][:len(r_fast)]) and np.array_equal(a["Sy"], b["Sy"][:len(r_fast)])
    lat.close()
    del lat
    torch.cuda.empty_cache()


def test_full_size_ising_sampled(gpu):
    """Ising L = 2^20 (128 GiB packed), the timed workload's kernels, sampled windows."""
    import torch
    L = workloads.ISING_LARGE["L"]
    if torch.cuda.get_device_properties(0).total_memory < (L * L) // 8 + (8 << 30):
        pytest.skip("needs a GPU with more than 136 GiB")
    n = 64  # the timed workload's depth; the exact interior is 4 n sites narrower
    size = 4 * n + 32
    windows = [(0, 0, size), (L - 150, L - 170, size), (123457, 987651, size), (L // 2, 64 * 1000 - 3, size)]
    sampled_full_size(gpu, 0, L, workloads.TC_ISING, n, workloads.SEED_BASE, windows)


def test_full_size_blume_capel_sampled(gpu):
    """Blume-Capel L = 2^18 (16 GiB), sampled windows after 64 sweeps."""
    L = workloads.BC_LARGE["L"]
    n = 64
    size = 4 * n + 32
    windows = [(0, 0, size), (L - 121, 5, size), (77777, 131071, size)]
    sampled_full_size(gpu, 1, L, workloads.T_BC_WORKLOAD, n, workloads.SEED_BASE, windows)
