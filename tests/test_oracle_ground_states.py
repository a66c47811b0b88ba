"""Ground states: the oracle's anneal against brute-force enumeration on tiny
graphs and against the closed-form ferromagnetic ground energies (paper
Sec. 1.3.1: annealing seeks the ground state of Eq. 1)."""
import numpy as np
import pytest

import synth
from oracle import oracle
from tests import refmath


def _brute_min(Jf, hv):
    states = refmath.all_states(Jf.shape[0])
    return int(refmath.dense_energy(Jf, hv, states).min())


@pytest.mark.parametrize("dims,seed,field", [((2, 2, 2), 1, "zero"), ((2, 2, 2), 2, "uniform3"),
                                             ((2, 2, 4), 3, "zero"), ((2, 2, 4), 4, "uniform3")])
def test_ea_anneal_reaches_brute_force_minimum(dims, seed, field):
    inst = synth.ea_instance(dims, seed=seed, field=field)
    Jf, hv = refmath.ea_dense(dims, inst["J"], inst["h"])
    e0 = _brute_min(Jf, hv)
    g = oracle.ea_graph(dims, inst["J"], inst["h"])
    res = oracle.anneal(g, synth.beta_linear(0.1, 4.0, 300), 64, seed=seed)
    assert res.energies.min() == e0
    assert np.all(res.energies >= e0)


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (8, 3)])
def test_biclique_anneal_reaches_brute_force_minimum(n, seed):
    inst = synth.biclique_instance(n, seed=seed)
    Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    e0 = _brute_min(Jf, hv)
    g = oracle.biclique_graph(n, n, inst["J"], inst["h"])
    res = oracle.anneal(g, synth.beta_linear(0.05, 3.0, 300), 64, seed=seed)
    assert res.energies.min() == e0
    assert np.all(res.energies >= e0)


@pytest.mark.parametrize("L", [2, 4, 6])
def test_ferromagnetic_cube_ground_energy_is_minus_3N(L):
    inst = synth.ferro_ea(L)
    g = oracle.ea_graph((L, L, L), inst["J"], inst["h"])
    res = oracle.anneal(g, synth.beta_linear(0.1, 3.0, 400), 8, seed=L)
    assert res.energies.min() == -3 * L**3


@pytest.mark.parametrize("n,field,expected", [(8, 0, -64), (16, 0, -256), (8, 1, -64 - 16)])
def test_ferromagnetic_biclique_ground_energy(n, field, expected):
    inst = synth.ferro_biclique(n, field)
    g = oracle.biclique_graph(n, n, inst["J"], inst["h"])
    res = oracle.anneal(g, synth.beta_linear(0.05, 2.0, 200), 8, seed=n)
    assert res.energies.min() == expected
