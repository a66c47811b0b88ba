"""Pins of the heat-bath threshold table and of the integer decision rule.

The threshold Tm(beta, a) = round-half-down(2^32 q), q = 1/(1 + exp(2 beta a)),
is the minority probability of the p-bit law m = sgn(tanh(beta I) - u)
(paper Sec. 1.2.1, Eq. 2 read with tanh and beta).  It is checked against
scipy's logistic function and against the tanh form, and the decision the
oracle takes inside a sweep is checked against the literal sgn(tanh - u).
"""
import math

import numpy as np
import pytest
from scipy.special import expit

from oracle import oracle


def test_fair_coin_at_zero_field_and_zero_beta():
    for beta in (0.0, 0.05, 1.0, 5.0, 100.0):
        assert oracle.minority_threshold(beta, 0) == 2**31
    for a in range(0, 20):
        assert oracle.minority_threshold(0.0, a) == 2**31


@pytest.mark.parametrize("beta", [0.01, 0.05, 0.1, 0.35, 1.0, 2.0, 3.5, 5.0])
def test_threshold_matches_logistic_and_tanh(beta):
    for a in range(0, 64):
        T = oracle.minority_threshold(beta, a)
        q_expit = float(expit(-2.0 * beta * a))
        q_tanh = (1.0 - math.tanh(beta * a)) / 2.0
        # round-half-down of 2^32 q: within 1/2 of the exact value, up to the
        # last-bit differences between the two formulas of q
        tol = 0.5 + 2**32 * 4e-16 * max(q_expit, 1e-300) + 1e-6
        assert abs(T - q_expit * 2**32) <= tol, (beta, a)
        if q_tanh > 1e-6:  # 1 - tanh cancels badly once tanh is near 1
            assert abs(T - q_tanh * 2**32) <= 0.5 + 2**32 * 1e-15, (beta, a)


def test_threshold_monotone_and_zero_beyond_cut():
    betas = np.linspace(0.0, 6.0, 61)
    tab = oracle.threshold_table(betas, 40)
    assert np.all(np.diff(tab.astype(np.int64), axis=1) <= 0)  # non-increasing in a
    assert np.all(np.diff(tab.astype(np.int64), axis=0) <= 0)  # non-increasing in beta
    assert tab.max() == 2**31
    # q 2^32 < 1/2  <=>  2 beta a > ln(2^33 - 1)  <=>  beta a > 11.4366...
    cut = math.log(2.0**33 - 1.0) / 2.0
    for beta in (0.05, 0.5, 1.0, 2.0):
        a_hi = math.ceil(cut / beta + 1e-9)
        assert oracle.minority_threshold(beta, a_hi) == 0
        a_lo = math.floor(cut / beta - 1e-9)
        if a_lo >= 0 and beta * a_lo < cut - 1e-6:
            assert oracle.minority_threshold(beta, a_lo) >= 1


def _star(k, J, h_center):
    """Centre 0 (colour 0) joined to k leaves (colour 1) with couplings J."""
    bi = np.zeros(k, np.int32)
    bj = np.arange(1, k + 1, dtype=np.int32)
    h = np.zeros(k + 1, np.int8)
    h[0] = h_center
    colour = np.array([0] + [1] * k, np.uint8)
    return oracle.Graph(k + 1, bi, bj, np.asarray(J, np.int8), h, colour, 2)


@pytest.mark.parametrize("beta", [0.0, 0.07, 0.3, 0.9, 2.5])
def test_sweep_decision_is_literal_sgn_tanh_minus_u(beta):
    """After one sweep the centre spin must equal sgn(tanh(beta I) - u) with
    u = (w + 1/2)/2^31 - 1 and w the Philox word of (centre, sweep, replica)."""
    rng = np.random.default_rng(11)
    k = 8
    seed = 0x1234_5678_9ABC
    R = 2048
    for trial in range(3):
        J = np.where(rng.random(k) < 0.5, 1, -1).astype(np.int8)
        hc = int(rng.integers(-1, 2))
        g = _star(k, J, hc)
        init = np.where(rng.random((R, k + 1)) < 0.5, 1, -1).astype(np.int8)
        t0 = int(rng.integers(0, 1000))
        res = oracle.anneal(g, [beta], R, seed, sweep_offset=t0, init_spins=init)
        I = init[:, 1:].astype(np.int64) @ J.astype(np.int64) + hc
        mism = 0
        for r in range(R):
            w = int(oracle.philox4x32_10([0, t0, r >> 2, 0], [seed & 0xFFFFFFFF, seed >> 32])[r & 3])
            u = (w + 0.5) / 2**31 - 1.0
            d = math.tanh(beta * I[r]) - u
            if abs(d) < 1e-9:
                continue  # inside the rounding band of the threshold
            lit = 1 if d > 0 else -1
            mism += int(lit != res.spins[r, 0])
        assert mism == 0
