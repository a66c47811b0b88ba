"""General sparse graphs on the CPU: the greedy colouring (paper Sec. 1.2.2)
of the oracle and of the library, pinned by the properties that define it,
and the oracle's sweep over more than two update groups, pinned by exact
stationarity of the Boltzmann law and by the cube's two-colour sweep."""
import itertools

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import pbit
from tests import refmath
from tests.test_oracle_boltzmann import _chi2_pvalue, _halfsweep_matrix


def _neighbours(n, bi, bj):
    nb = [set() for _ in range(n)]
    for a, b in zip(bi.tolist(), bj.tolist()):
        nb[a].add(b)
        nb[b].add(a)
    return nb


def _is_greedy(n, bi, bj, colour):
    """Proper, and every colour below a vertex's own is held by one of its
    earlier neighbours: together these fix the greedy colouring uniquely."""
    nb = _neighbours(n, bi, bj)
    for v in range(n):
        if any(colour[u] == colour[v] for u in nb[v]):
            return False
        earlier = {int(colour[u]) for u in nb[v] if u < v}
        if any(c not in earlier for c in range(int(colour[v]))):
            return False
    return True


def _graphs():
    yield "cube4", synth.ea_bond_list(synth.ea_instance(4, seed=1))
    yield "cube3", synth.ea_bond_list(synth.ea_instance(3, seed=2))
    yield "cube345", synth.ea_bond_list(synth.ea_instance((3, 4, 5), seed=3))
    yield "cube5", synth.ea_bond_list(synth.ea_instance(5, seed=4))
    for k, (n, d) in enumerate([(50, 4), (300, 6), (1000, 12), (200, 40)]):
        yield "random%d" % k, synth.random_sparse_graph(n, d, seed=k)
    for L in (3, 7):
        yield "dimer%d" % L, synth.dimerized_cube(L, seed=L)


@pytest.mark.parametrize("name,g", list(_graphs()))
def test_greedy_colouring_is_greedy_and_library_agrees(name, g):
    col, nc = oracle.greedy_colouring(g["n"], g["bond_i"], g["bond_j"])
    assert _is_greedy(g["n"], g["bond_i"], g["bond_j"], col)
    assert nc == int(col.max()) + 1
    deg = np.bincount(np.concatenate([g["bond_i"], g["bond_j"]]), minlength=g["n"])
    assert nc <= deg.max() + 1  # Brooks-type greedy bound
    lcol, lnc = pbit.pbit_greedy_colouring(g["n"], g["bond_i"], g["bond_j"])
    assert lnc == nc and np.array_equal(lcol, col)


@pytest.mark.parametrize("dims", [(4, 4, 4), (6, 4, 2), (8, 2, 6)])
def test_greedy_colouring_of_an_even_cube_is_the_checkerboard(dims):
    g = synth.ea_bond_list(synth.ea_instance(dims, seed=5))
    col, nc = oracle.greedy_colouring(g["n"], g["bond_i"], g["bond_j"])
    i = np.arange(g["n"])
    x, y, z = i % dims[0], (i // dims[0]) % dims[1], i // (dims[0] * dims[1])
    assert nc == 2 and np.array_equal(col, (x + y + z) % 2)


def test_greedy_colouring_special_graphs():
    # complete graph K_n: vertex i takes colour i
    n = 9
    pairs = np.array(list(itertools.combinations(range(n), 2)), np.int32)
    col, nc = oracle.greedy_colouring(n, pairs[:, 0], pairs[:, 1])
    assert nc == n and np.array_equal(col, np.arange(n))
    assert np.array_equal(pbit.pbit_greedy_colouring(n, pairs[:, 0], pairs[:, 1])[0], col)
    # K_{na,nb} with side A first: two colours, A = 0, B = 1
    g = oracle.biclique_graph(3, 4, np.ones((3, 4), np.int8))
    col, nc = oracle.greedy_colouring(g.n, g.bi, g.bj)
    assert nc == 2 and np.array_equal(col, g.colour)
    # odd cycle: three colours; no bonds: one colour
    c5 = np.arange(5, dtype=np.int32)
    assert oracle.greedy_colouring(5, c5, (c5 + 1) % 5)[1] == 3
    col, nc = pbit.pbit_greedy_colouring(6, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert nc == 1 and not col.any()
    # a crown graph in an interleaved order makes greedy use n/2 colours
    k = 5
    bi, bj = [], []
    for a in range(k):
        for b in range(k):
            if a != b:
                bi.append(2 * a)
                bj.append(2 * b + 1)
    col, nc = oracle.greedy_colouring(2 * k, np.array(bi), np.array(bj))
    assert nc == k and np.array_equal(pbit.pbit_greedy_colouring(2 * k, bi, bj)[0], col)


def test_greedy_colouring_rejects_bad_bonds():
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_greedy_colouring(4, [0, 1], [1, 4])
    assert ei.value.code == pbit.PBIT_E_ARG
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_greedy_colouring(4, [2], [2])
    assert ei.value.code == pbit.PBIT_E_ARG


def _small_graph():
    """Triangle 0-1-2 with a pendant 3 on vertex 2 and a 4-cycle 3-4-5-6:
    greedy needs three groups; fields on every vertex."""
    bi = np.array([0, 1, 0, 2, 3, 4, 5, 6], np.int32)
    bj = np.array([1, 2, 2, 3, 4, 5, 6, 3], np.int32)
    bJ = np.array([1, -1, 1, -1, 1, 1, -1, 1], np.int8)
    h = np.array([1, 0, -1, 1, 0, -1, 1], np.int8)
    return 7, bi, bj, bJ, h


def _dense(n, bi, bj, bJ):
    Jf = np.zeros((n, n), np.int64)
    for a, b, j in zip(bi, bj, bJ):
        Jf[a, b] += j
        Jf[b, a] += j
    return Jf


@pytest.mark.parametrize("beta", [0.4, 1.2])
def test_exact_stationarity_of_a_three_group_sweep(beta):
    n, bi, bj, bJ, h = _small_graph()
    col, nc = oracle.greedy_colouring(n, bi, bj)
    assert nc == 3
    Jf, hv = _dense(n, bi, bj, bJ), h.astype(np.int64)
    pi = refmath.boltzmann(refmath.dense_energy(Jf, hv, refmath.all_states(n)).astype(np.float64), beta)
    P = np.eye(2 ** n)
    for c in range(nc):
        P = P @ _halfsweep_matrix(Jf, hv, col == c, beta)
    assert np.max(np.abs(pi @ P - pi)) < 1e-8


@pytest.mark.parametrize("beta", [0.3, 0.9])
def test_oracle_samples_follow_boltzmann_on_a_three_group_graph(beta):
    n, bi, bj, bJ, h = _small_graph()
    g = oracle.graph_from_bonds(n, bi, bj, bJ, h)
    assert g.n_colours == 3
    R = 16384
    res = oracle.anneal(g, np.full(200, beta), R, seed=int(beta * 100))
    pi = refmath.boltzmann(refmath.dense_energy(_dense(n, bi, bj, bJ), h.astype(np.int64),
                                                refmath.all_states(n)).astype(np.float64), beta)
    counts = np.bincount(refmath.state_index(res.spins), minlength=2 ** n)
    assert _chi2_pvalue(counts, pi, R) > 1e-4
    assert np.array_equal(res.energies, refmath.dense_energy(_dense(n, bi, bj, bJ), h.astype(np.int64), res.spins))


def test_even_cube_as_a_graph_sweeps_like_the_cube():
    """The bond-list form of an even cube gets the checkerboard by greedy
    colouring, so its sweep is the cube's sweep, replica for replica."""
    inst = synth.ea_instance((4, 4, 2), seed=9, field="uniform3")
    gb = synth.ea_bond_list(inst)
    g1 = oracle.graph_from_bonds(gb["n"], gb["bond_i"], gb["bond_j"], gb["bond_J"], gb["h"])
    g2 = oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    beta = synth.beta_linear(0.1, 2.0, 25)
    r1 = oracle.anneal(g1, beta, 9, seed=3, trace_every=5)
    r2 = oracle.anneal(g2, beta, 9, seed=3, trace_every=5)
    assert np.array_equal(r1.spins, r2.spins) and np.array_equal(r1.energy_trace, r2.energy_trace)


@pytest.mark.parametrize("L", [7, 8, 9, 10, 14])
def test_dimerized_cubes_need_more_than_two_groups(L):
    """The stand-ins for the paper's hardware-embedded lattices (Sec. 2.2, which
    needed four or five update groups): 2 L^3 spins, every pair bonded
    ferromagnetically, a simple graph (no self-bonds or repeats), and a greedy
    colouring with five groups that stays within the degree bound."""
    g = synth.dimerized_cube(L, seed=L)
    n, bi, bj, bJ = g["n"], g["bond_i"], g["bond_j"], g["bond_J"]
    assert n == 2 * L ** 3
    assert np.all(bi != bj)
    pairs = set(zip(np.minimum(bi, bj).tolist(), np.maximum(bi, bj).tolist()))
    assert len(pairs) == bi.size
    dimer = (bi // 2 == bj // 2)
    assert int(dimer.sum()) == L ** 3 and np.all(bJ[dimer] == 1)
    assert set(np.unique(bJ[~dimer]).tolist()) <= {-1, 1}
    col, nc = pbit.pbit_greedy_colouring(n, bi, bj)
    deg = np.bincount(np.concatenate([bi, bj]), minlength=n)
    assert nc == 5 and nc <= deg.max() + 1
    assert np.all(col[bi] != col[bj])
