"""Stationarity of the sweep: at fixed beta the chain's law is exp(-beta E)/Z
(paper Sec. 1.2.1, the Boltzmann law for symmetric J, whatever the update
order).  Exact on the transition matrix of the threshold rule, and statistical
(chi-square) on the oracle's own sweeps."""
import numpy as np
import pytest
from scipy import stats

import synth
from oracle import oracle
from tests import refmath


def _halfsweep_matrix(Jf, hv, colour_mask, beta):
    """Transition matrix of one update-group pass built from the threshold rule:
    each member of the group turns to +1 with probability P+ = 1 - Tm/2^32 if
    its field is >= 0 and Tm/2^32 otherwise, independently."""
    N = Jf.shape[0]
    states = refmath.all_states(N).astype(np.int64)
    S = states.shape[0]
    P = np.zeros((S, S))
    members = np.flatnonzero(colour_mask)
    for k in range(S):
        m = states[k]
        I = Jf @ m + hv
        p_plus = np.empty(N)
        for i in members:
            T = oracle.minority_threshold(beta, abs(int(I[i]))) / 2**32
            p_plus[i] = 1.0 - T if I[i] >= 0 else T
        for k2 in range(S):
            m2 = states[k2]
            if np.any(m2[~colour_mask] != m[~colour_mask]):
                continue
            pr = 1.0
            for i in members:
                pr *= p_plus[i] if m2[i] > 0 else 1.0 - p_plus[i]
            P[k, k2] = pr
    return P


@pytest.mark.parametrize("beta", [0.3, 1.0])
def test_exact_stationarity_of_two_halfsweeps(beta):
    # K_{2,3} with fields: 5 spins, 32 states
    inst = synth.biclique_instance(2, seed=4, nb=3)
    Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    states = refmath.all_states(5)
    pi = refmath.boltzmann(refmath.dense_energy(Jf, hv, states).astype(np.float64), beta)
    side_a = np.array([1, 1, 0, 0, 0], bool)
    P = _halfsweep_matrix(Jf, hv, side_a, beta) @ _halfsweep_matrix(Jf, hv, ~side_a, beta)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    assert np.max(np.abs(pi @ P - pi)) < 1e-8  # 2^-32 threshold quantisation


def _chi2_pvalue(observed, expected_p, n):
    exp = expected_p * n
    keep = exp >= 5
    o = np.append(observed[keep], observed[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    return stats.chisquare(o, e).pvalue


@pytest.mark.parametrize("beta", [0.2, 0.5, 1.0])
def test_sampled_states_follow_boltzmann_ea(beta):
    dims = (2, 2, 2)
    inst = synth.ea_instance(dims, seed=7, field="uniform3")
    g = oracle.ea_graph(dims, inst["J"], inst["h"])
    Jf, hv = refmath.ea_dense(dims, inst["J"], inst["h"])
    R = 32768
    res = oracle.anneal(g, np.full(300, beta), R, seed=100 + int(beta * 10))
    states = refmath.all_states(8)
    pi = refmath.boltzmann(refmath.dense_energy(Jf, hv, states).astype(np.float64), beta)
    counts = np.bincount(refmath.state_index(res.spins), minlength=256)
    assert _chi2_pvalue(counts, pi, R) > 1e-4


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_sampled_states_follow_boltzmann_biclique(beta):
    inst = synth.biclique_instance(3, seed=8)
    g = oracle.biclique_graph(3, 3, inst["J"], inst["h"])
    Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    R = 32768
    res = oracle.anneal(g, np.full(150, beta), R, seed=200 + int(beta * 10))
    states = refmath.all_states(6)
    pi = refmath.boltzmann(refmath.dense_energy(Jf, hv, states).astype(np.float64), beta)
    counts = np.bincount(refmath.state_index(res.spins), minlength=64)
    assert _chi2_pvalue(counts, pi, R) > 1e-4


def test_beta_zero_gives_uniform_states():
    inst = synth.ea_instance((2, 2, 2), seed=1, field="uniform3")
    g = oracle.ea_graph((2, 2, 2), inst["J"], inst["h"])
    R = 16384
    res = oracle.anneal(g, np.zeros(3), R, seed=5)
    counts = np.bincount(refmath.state_index(res.spins), minlength=256)
    assert _chi2_pvalue(counts, np.full(256, 1 / 256), R) > 1e-4
    assert abs(res.spins.astype(np.float64).mean()) < 0.02


def test_random_start_is_fair():
    g = oracle.ea_graph((4, 4, 4), synth.ea_instance(4, seed=1)["J"])
    res = oracle.anneal(g, np.zeros(0), 256, seed=77)  # zero sweeps: the initial spins
    assert abs(res.spins.astype(np.float64).mean()) < 0.02
    assert np.array_equal(res.energies, oracle.energy(g, res.spins))
