"""Pins of the oracle's energy and of its problem builders (paper Sec. 1.1.1
Eq. 1, Sec. 2 periodic cubic lattice, Sec. 3 biclique)."""
import numpy as np
import pytest

import synth
from oracle import oracle
from tests import refmath


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (2, 4, 6), (6, 6, 6)])
@pytest.mark.parametrize("field", ["zero", "uniform3"])
def test_ea_energy_matches_shifted_lattice_formula(dims, field):
    inst = synth.ea_instance(dims, seed=sum(dims), field=field)
    g = oracle.ea_graph(dims, inst["J"], inst["h"])
    spins = synth.random_spins(16, g.n, seed=3)
    e = oracle.energy(g, spins)
    assert np.array_equal(e, refmath.ea_energy_roll(dims, inst["J"], inst["h"], spins))
    Jf, hv = refmath.ea_dense(dims, inst["J"], inst["h"])
    assert np.array_equal(e, refmath.dense_energy(Jf, hv, spins))


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 5), (16, 16), (64, 33)])
def test_biclique_energy_matches_dense_formula(na, nb):
    inst = synth.biclique_instance(na, seed=na * 100 + nb, nb=nb)
    g = oracle.biclique_graph(na, nb, inst["J"], inst["h"])
    spins = synth.random_spins(8, g.n, seed=5)
    e = oracle.energy(g, spins)
    mA = spins[:, :na].astype(np.int64)
    mB = spins[:, na:].astype(np.int64)
    direct = -np.einsum("ra,ab,rb->r", mA, inst["J"].astype(np.int64), mB) - spins.astype(np.int64) @ inst["h"].astype(np.int64)
    assert np.array_equal(e, direct)


def test_gauge_invariance():
    dims = (4, 4, 2)
    inst = synth.ea_instance(dims, seed=9, field="uniform3")
    N = 32
    g = oracle.ea_graph(dims, inst["J"], inst["h"])
    spins = synth.random_spins(4, N, seed=1)
    gauge = synth.random_spins(1, N, seed=2)[0].astype(np.int64)
    # J_ij -> s_i s_j J_ij on every bond, h_i -> s_i h_i, m_i -> s_i m_i
    g2 = oracle.Graph(N, g.bi, g.bj, (g.bJ * gauge[g.bi] * gauge[g.bj]).astype(np.int8),
                      (inst["h"] * gauge).astype(np.int8), g.colour, 2)
    assert np.array_equal(oracle.energy(g, spins), oracle.energy(g2, (spins * gauge).astype(np.int8)))


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 6, 8)])
def test_ea_bond_geometry(dims):
    Lx, Ly, Lz = dims
    N = Lx * Ly * Lz
    g = oracle.ea_graph(dims, np.ones((3, N), np.int8))
    assert g.n_bonds == 3 * N
    deg = np.bincount(np.concatenate([g.bi, g.bj]), minlength=N)
    assert np.all(deg == 6)
    xi, yi, zi = g.bi % Lx, (g.bi // Lx) % Ly, g.bi // (Lx * Ly)
    xj, yj, zj = g.bj % Lx, (g.bj // Lx) % Ly, g.bj // (Lx * Ly)
    steps = np.stack([(xj - xi) % Lx, (yj - yi) % Ly, (zj - zi) % Lz], axis=1)
    assert np.all(steps.sum(axis=1) == 1)  # exactly one +1 step in one axis
    assert np.all(g.colour[g.bi] != g.colour[g.bj])  # proper checkerboard
    assert g.colour.sum() == N // 2


def test_biclique_colouring_is_the_two_sides():
    g = oracle.biclique_graph(5, 7, np.ones((5, 7), np.int8))
    assert g.n_bonds == 35
    assert list(g.colour) == [0] * 5 + [1] * 7
    assert np.all(g.colour[g.bi] == 0) and np.all(g.colour[g.bj] == 1)
