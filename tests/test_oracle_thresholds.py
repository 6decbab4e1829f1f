"""Pins of the integer Metropolis rule: accept iff dE <= 0 or u < thr with
thr = floor(2^32 exp(-dE / T)).

* Ising at T_c = 2 / ln(1 + sqrt 2) (paper, Models): exp(-4/T_c) = 3 - 2 sqrt 2
  and exp(-8/T_c) = 17 - 12 sqrt 2 exactly, so the two thresholds follow from
  50-digit arithmetic.
* For random (dE, T) the integer threshold brackets the exact probability:
  thr / 2^32 <= exp(-dE/T) < (thr + 1) / 2^32 up to the last bit of an FP64 exp.
* Limits: dE <= 0 and T = +inf accept without a draw; T = 0 never accepts.
"""
import math

import mpmath
import numpy as np

import oracle

mpmath.mp.dps = 50
TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))


def test_tc_constant_matches_paper_table():
    # Table I prints T_c = 2.26918531421302196814
    assert abs(TC_ISING - 2.26918531421302196814) < 4e-16
    exact = 2 / mpmath.log(1 + mpmath.sqrt(2))
    assert abs(mpmath.mpf(TC_ISING) - exact) < 1e-15


def test_ising_tc_thresholds_closed_form():
    two32 = mpmath.mpf(2) ** 32
    want4 = int(mpmath.floor(two32 * (3 - 2 * mpmath.sqrt(2))))
    want8 = int(mpmath.floor(two32 * (17 - 12 * mpmath.sqrt(2))))
    assert (want4, want8) == (736899888, 126432032)
    for J in (1.0, 0.5, 2.0):
        # dE = 4J and 8J at temperature J * T_c are the same ratios
        a4, t4 = oracle.threshold(4.0 * J, TC_ISING * J)
        a8, t8 = oracle.threshold(8.0 * J, TC_ISING * J)
        assert not a4 and not a8
        assert (t4, t8) == (want4, want8)


def test_threshold_brackets_exact_probability():
    rng = np.random.default_rng(7)
    two32 = mpmath.mpf(2) ** 32
    for _ in range(3000):
        dE = float(rng.choice([rng.uniform(1e-6, 20.0), float(rng.integers(1, 17))]))
        T = float(rng.uniform(0.05, 10.0))
        always, thr = oracle.threshold(dE, T)
        p = mpmath.exp(-mpmath.mpf(dE) / mpmath.mpf(T))
        x = p * two32
        if x >= two32 * (1 - mpmath.mpf(2) ** -50):
            continue
        assert not always
        assert thr <= x * (1 + mpmath.mpf(2) ** -50)
        assert x < thr + 1 + x * mpmath.mpf(2) ** -50


def test_threshold_limits():
    assert oracle.threshold(0.0, 1.0) == (True, 0)
    assert oracle.threshold(-3.0, 0.0) == (True, 0)
    assert oracle.threshold(4.0, float("inf")) == (True, 0)
    assert oracle.threshold(4.0, 0.0) == (False, 0)
    assert oracle.threshold(1e-300, 1.0) == (True, 0)  # rounds to probability 1


def test_blume_capel_detailed_balance_of_the_rule():
    # Each BC move s -> s' is proposed with probability 1/2 (uniform over the
    # other two states) and the reverse move has the opposite dE, so the
    # integer rule satisfies P(s->s') / P(s'->s) = exp(-dE/T) within 2^-32.
    T = 1.69355839821214427017
    for J, Delta in [(1.0, 0.0), (1.0, 0.7), (0.8, -0.3)]:
        for s in (-1, 0, 1):
            for sp in (-1, 0, 1):
                if sp == s:
                    continue
                for h in range(-4, 5):
                    dE = -J * (sp - s) * h + Delta * (sp * sp - s * s)
                    fwd = oracle.threshold(dE, T)
                    bwd = oracle.threshold(-dE, T)
                    pf = 1.0 if fwd[0] else fwd[1] / 2**32
                    pb = 1.0 if bwd[0] else bwd[1] / 2**32
                    # pf * min(1, e^{dE/T}) = pb * min(1, e^{-dE/T}) is the
                    # balance condition scaled so both sides stay <= 1
                    lhs = pf * min(1.0, math.exp(dE / T))
                    rhs = pb * min(1.0, math.exp(-dE / T))
                    assert abs(lhs - rhs) <= 2.0**-31
