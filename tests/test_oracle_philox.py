"""Pins of the oracle's random stream.

* Philox4x32-10 against the published known-answer vectors (tests/golden)
  and against rocRAND's host-callable Philox engine on random blocks.
* The bit-plane uniform: every 32-bit value is what the definition assembles
  from the Philox planes (checked on a brute-force sample by a routine that
  reads the planes through the Philox pin, not through the oracle), and the
  uniforms are uniform and uncorrelated across purposes, colours and sweeps.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("rocrand") / "rocrand_philox"
    subprocess.run([hipcc, "-O1", "-o", str(out), os.path.join(HERE, "support", "rocrand_philox.cpp")],
                   check=True, capture_output=True)
    return str(out)


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(2503146880)
    blocks = rng.integers(0, 2**32, size=(256, 6), dtype=np.uint64)
    blocks[:8, :] = 0
    blocks[8:16, 0:4] = 0xFFFFFFFF
    text = "\n".join(" ".join(f"{int(x):08x}" for x in row) for row in blocks) + "\n"
    res = subprocess.run([rocrand_philox], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == blocks.shape[0]
    for row, line in zip(blocks, lines):
        want = [int(x, 16) for x in line.split()]
        got = oracle.philox4x32_10(row[0:4].astype(np.uint32), row[4:6].astype(np.uint32))
        assert [int(x) for x in got] == want


def test_uniform_is_the_bit_plane_assembly(rocrand_philox):
    # Site (i, m) of colour c, sweep t: plane k is word k & 3 of the Philox
    # block at counter (i, m >> 5, t, purpose << 16 | c << 8 | k >> 2); the
    # uniform has plane 0 as its most significant bit.  The planes are read
    # through rocRAND here, so the oracle's own Philox is not used.
    seed = 0x1234_5678_9ABC_DEF0
    key = (seed & 0xFFFFFFFF, seed >> 32)
    cases = [(p, t, c, i, m) for (p, t, c, i, m) in
             [(0, 0, 0, 0, 0), (1, 7, 1, 3, 31), (2, 1023, 0, 4095, 32), (1, 2**31, 1, 2**20 - 1, 2**19 - 1),
              (0, 0, 1, 17, 100), (1, 5, 0, 9, 33)]]
    lines = []
    for (p, t, c, i, m) in cases:
        for blk in range(8):
            lines.append(f"{i:08x} {m >> 5:08x} {t:08x} {(p << 16) | (c << 8) | blk:08x} "
                         f"{key[0]:08x} {key[1]:08x}")
    res = subprocess.run([rocrand_philox], input="\n".join(lines) + "\n",
                         capture_output=True, text=True, check=True)
    words = [[int(x, 16) for x in ln.split()] for ln in res.stdout.strip().split("\n")]
    for q, (p, t, c, i, m) in enumerate(cases):
        planes = [w for blk in range(8) for w in words[8 * q + blk]]
        b = m & 31
        u = 0
        for k in range(32):
            u |= ((planes[k] >> b) & 1) << (31 - k)
        assert oracle.uniform(seed, p, t, c, i, m) == u


def test_uniform_distribution_and_independence():
    seed = 2503146880
    n = 4000
    idx = np.arange(n)
    u_acc0 = np.array([oracle.uniform(seed, 1, 3, 0, int(k) // 64, int(k) % 64) for k in idx], dtype=np.float64)
    u_acc1 = np.array([oracle.uniform(seed, 1, 3, 1, int(k) // 64, int(k) % 64) for k in idx], dtype=np.float64)
    u_prop = np.array([oracle.uniform(seed, 2, 3, 0, int(k) // 64, int(k) % 64) for k in idx], dtype=np.float64)
    u_next = np.array([oracle.uniform(seed, 1, 4, 0, int(k) // 64, int(k) % 64) for k in idx], dtype=np.float64)
    for u in (u_acc0, u_acc1, u_prop, u_next):
        x = u / 2.0**32
        assert stats.kstest(x, "uniform").pvalue > 1e-3
        # every bit is a fair coin
        bits = ((u.astype(np.uint64)[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
        assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(n))
    for a, b in [(u_acc0, u_acc1), (u_acc0, u_prop), (u_acc0, u_next)]:
        rho = np.corrcoef(a, b)[0, 1]
        assert abs(rho) < 5 / np.sqrt(n)
    # neighbouring lanes and words are distinct streams
    assert len(set(u_acc0.tolist())) == n
