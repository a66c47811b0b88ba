"""Algorithm 1 on the GPU (paper Sec. 1.3.3): the library's windowed search
over pbit_anneal / pbit_anneal_batch returns the budget the paper's loop
finds on the oracle, on closed-form, brute-force and oracle-best ground
truths, for cubes, bicliques and a general graph."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import alg1, pbit
from tests import refmath

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = pbit.Context(0)
    yield c.ctx
    c.close()


def _g(inst):
    if inst["kind"] == "ea3d":
        return oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    if inst["kind"] == "graph":
        return oracle.graph_from_bonds(inst["n"], inst["bond_i"], inst["bond_j"], inst["bond_J"], inst.get("h"))
    return oracle.biclique_graph(*inst["dims"], inst["J"], inst["h"])


def _brute_force_min(inst):
    if inst["kind"] == "ea3d":
        Jf, hv = refmath.ea_dense(inst["dims"], inst["J"], inst["h"])
    else:
        Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    return int(refmath.dense_energy(Jf, hv, refmath.all_states(Jf.shape[0])).min())


def _oracle_best(inst, sweeps=2000, R=128):
    return int(oracle.anneal(_g(inst), synth.beta_linear(0.35, 3.5, sweeps), R, seed=1).energies.min())


def _cases():
    ea2 = synth.ea_instance(2, seed=5, field="uniform3")
    k44 = synth.biclique_instance(4, seed=6)
    ea4 = synth.ea_instance(4, seed=3, field="uniform3")
    odd = synth.ea_bond_list(synth.ea_instance(3, seed=4, field="uniform3"))
    return [("ferro cube L=6", synth.ferro_ea(6), lambda i: -648, 0.9),
            ("ferro K_{32,32}", synth.ferro_biclique(32), lambda i: -1024, 0.95),
            ("EA 2x2x2 with fields", ea2, _brute_force_min, 0.99),
            ("K_{4,4} with fields", k44, _brute_force_min, 0.99),
            ("EA L=4 with fields", ea4, _oracle_best, 0.97),
            ("odd cube 3^3 as a graph", odd, _oracle_best, 0.97)]


@pytest.mark.parametrize("name,inst,truth,p", _cases())
@pytest.mark.parametrize("window", [1, 6])
def test_i_min_matches_the_paper_loop_on_the_oracle(ctx, name, inst, truth, p, window):
    G = truth(inst)
    seed = 11
    t, p_succ = 20, 0.9
    prob = pbit.load_instance(ctx, inst)
    _say("alg1 %s G=%d p=%.2f window=%d" % (name, G, p, window))
    res = alg1.i_min(ctx, prob, G, i_start=1, i_step=1, t=t, p=p, p_succ=p_succ, seed=seed, window=window,
                     i_max=400)
    pbit.pbit_unload_problem(ctx, prob)
    i_or, hist = oracle.alg1_minimal_budget(oracle.alg1_trial(_g(inst), lambda i: alg1.budget_seed(seed, i)), G, 1, 1,
                                            t, p, p_succ, 0.35, 3.5, 400)
    assert i_or is not None and res.i_min == i_or, (res.i_min, i_or)
    seen = dict(res.history)
    for i, m, _ in hist:
        assert (seen[i] <= res.m_max) == (m <= res.m_max), i


def test_i_min_series_chains_the_start(ctx):
    insts = [synth.ferro_ea(L) for L in (2, 4, 6)]
    probs = [pbit.load_instance(ctx, x) for x in insts]
    G = [-3 * int(np.prod(x["dims"])) for x in insts]
    out = alg1.i_min_series(ctx, list(zip(probs, G)), t=20, p=0.9, seed=3, window=4, i_max=400)
    assert all(r.i_min is not None for r in out)
    for prev, cur in zip(out, out[1:]):
        assert cur.history[0][0] == prev.i_min  # each search starts where the last one ended
    for pr in probs:
        pbit.pbit_unload_problem(ctx, pr)
