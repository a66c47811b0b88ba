"""Sweep mechanics of the oracle: update-group order independence (paper
Sec. 1.2.2: members of a group are independent, and Sec. 1.2.1: the law holds
whatever the order), resume / replica-slice / prefix identities of the
counter-based randomness, and the zero-temperature limit."""
import numpy as np
import pytest

import synth
from oracle import oracle


def _ea(L=4, seed=3, field="uniform3"):
    inst = synth.ea_instance(L, seed=seed, field=field)
    return oracle.ea_graph(inst["dims"], inst["J"], inst["h"])


def _bq(n=12, seed=5):
    inst = synth.biclique_instance(n, seed=seed)
    return oracle.biclique_graph(n, n, inst["J"], inst["h"])


@pytest.mark.parametrize("make", [_ea, _bq])
def test_order_within_groups_does_not_matter(make):
    g = make()
    beta = synth.beta_linear(0.1, 2.0, 40)
    base = oracle.anneal(g, beta, 8, seed=9)
    rev = oracle.anneal(g, beta, 8, seed=9, order=np.arange(g.n)[::-1].copy())
    shuf = oracle.anneal(g, beta, 8, seed=9, order=np.random.default_rng(1).permutation(g.n))
    for other in (rev, shuf):
        assert np.array_equal(base.spins, other.spins)
        assert np.array_equal(base.energies, other.energies)


@pytest.mark.parametrize("make", [_ea, _bq])
def test_resume_split_is_identical(make):
    g = make()
    beta = synth.beta_geometric(0.1, 5.0, 50)
    full = oracle.anneal(g, beta, 6, seed=21)
    first = oracle.anneal(g, beta[:17], 6, seed=21)
    second = oracle.anneal(g, beta[17:], 6, seed=21, sweep_offset=17, init_spins=first.spins)
    assert np.array_equal(full.spins, second.spins)
    assert np.array_equal(full.energies, second.energies)


@pytest.mark.parametrize("make", [_ea, _bq])
def test_replica_slices_are_identical(make):
    g = make()
    beta = synth.beta_linear(0.2, 3.0, 20)
    full = oracle.anneal(g, beta, 11, seed=4)
    for off, cnt in ((0, 3), (3, 5), (8, 3), (5, 1)):
        part = oracle.anneal(g, beta, cnt, seed=4, replica_offset=off)
        assert np.array_equal(full.spins[off:off + cnt], part.spins)


def test_prefix_property_and_traces():
    g = _ea()
    beta = synth.beta_linear(0.1, 3.0, 30)
    full = oracle.anneal(g, beta, 5, seed=8, trace_every=10, trace_spins=True)
    for k in (1, 2, 3):
        pre = oracle.anneal(g, beta[:10 * k], 5, seed=8)
        assert np.array_equal(full.spin_trace[k - 1], pre.spins)
        assert np.array_equal(full.energy_trace[k - 1], pre.energies)
        assert np.array_equal(full.energy_trace[k - 1], oracle.energy(g, full.spin_trace[k - 1]))


def test_seed_changes_the_run():
    g = _ea()
    beta = synth.beta_linear(0.1, 3.0, 5)
    a = oracle.anneal(g, beta, 4, seed=1).spins
    b = oracle.anneal(g, beta, 4, seed=2).spins
    c = oracle.anneal(g, beta, 4, seed=1 + (1 << 32)).spins  # high key word matters
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


@pytest.mark.parametrize("make,beta", [(lambda: _ea(field="zero"), 6.0), (_bq, 12.0)])
def test_zero_temperature_energy_never_rises(make, beta):
    # beta * min|I != 0| above the cut makes every non-zero-field minority
    # threshold 0: each half-sweep can only lower the energy or keep it.
    g = make()
    res = oracle.anneal(g, np.full(30, beta), 16, seed=13, trace_every=1)
    tr = res.energy_trace
    assert np.all(np.diff(tr, axis=0) <= 0)


def test_improper_colouring_is_rejected():
    g = _ea(L=2)
    bad = oracle.Graph(g.n, g.bi, g.bj, g.bJ, g.h, np.zeros(g.n, np.uint8), 2)
    with pytest.raises(RuntimeError, match="-2"):
        oracle.anneal(bad, [1.0], 1, seed=1)


def test_energy_drift_check_is_live():
    # the oracle checks its incremental energy at every traced sweep; a long
    # traced run on a frustrated instance with fields exercises that check
    g = _ea(L=6, seed=12)
    res = oracle.anneal(g, synth.beta_linear(0.1, 3.0, 100), 4, seed=3, trace_every=1)
    assert res.energy_trace.shape == (100, 4)
