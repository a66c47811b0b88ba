"""Algorithm 1 (paper Sec. 1.3.3) and the quality metrics of Sec. 2.1-2.2 on
the CPU.  The oracle's Algorithm 1 follows the paper's loop, trial by trial
with the early exit; it is pinned by scripted solvers whose answer is worked
out by hand, by the paper's own settings (20 trials at 90 % give m_max = 2),
and by closed-form and brute-force ground truths.  The library's windowed
search is then checked against it."""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import alg1
from tests import refmath

GOLDEN = json.loads((Path(__file__).parent / "golden" / "paper_constants.json").read_text())


def _seed_of(i):
    return (7 + i * 0x9E3779B97F4A7C15) % 2 ** 64


def _scripted(fails_by_budget, t, good=-100, bad=-50):
    """A solver whose trial j at budget i fails iff j is listed for i."""
    def pc(i, beta, j):
        return bad if j in fails_by_budget.get(i, ()) else good
    return pc


def test_paper_settings_give_two_allowed_fails():
    t = GOLDEN["alg1_trials"]["value"]
    s = GOLDEN["alg1_success_target"]["value"]
    assert alg1.max_fails(t, s) == GOLDEN["alg1_max_fails"]["value"] == 2
    # the oracle's loop: 2 fails of 20 pass, 3 do not
    pc = _scripted({1: (0, 5), 2: (3, 4, 9)}, t)
    i, hist = oracle.alg1_minimal_budget(pc, -100.0, 1, 1, t, 0.9, s, 0.35, 3.5, 10)
    assert i == 1 and hist == [(1, 2, 20)]
    i, hist = oracle.alg1_minimal_budget(pc, -100.0, 2, 1, t, 0.9, s, 0.35, 3.5, 10)
    assert i == 3 and hist[0] == (2, 3, 10)  # trial loop left at the third fail (trial 9)


def test_oracle_loop_scripted():
    # budget 4: every trial fails (exit after m_max + 1 = 3 trials); 6: 3 fails; 8: 1 fail
    fails = {4: tuple(range(20)), 6: (0, 1, 2), 8: (19,)}
    i, hist = oracle.alg1_minimal_budget(_scripted(fails, 20), -100.0, 4, 2, 20, 0.9, 0.9, 0.35, 3.5, 100)
    assert i == 8
    assert hist == [(4, 3, 3), (6, 3, 3), (8, 1, 20)]
    # nothing passes before i_max
    i, hist = oracle.alg1_minimal_budget(_scripted({k: (0, 1, 2) for k in range(50)}, 20), -100.0, 1, 1, 20, 0.9,
                                         0.9, 0.35, 3.5, 5)
    assert i is None and len(hist) == 5


def test_threshold_is_p_times_G():
    # G = -100, p = 0.9: theta = -90.  v = -90 passes (not above), v = -89 fails
    seen = []

    def pc(i, beta, j):
        seen.append(beta)
        return -89 if (i == 1 and j < 3) else -90
    i, _ = oracle.alg1_minimal_budget(pc, -100.0, 1, 1, 20, 0.9, 0.9, 0.35, 3.5, 10)
    assert i == 2
    # the schedule: starts at beta_i, step delta_beta = (beta_f - beta_i) / i
    assert np.array_equal(seen[-1], np.array([0.35, 0.35 + 3.15 / 2]))
    assert np.array_equal(alg1.linear_schedule(0.35, 3.5, 2), seen[-1])
    assert np.array_equal(alg1.linear_schedule(0.35, 3.5, 1), [0.35])


@pytest.mark.parametrize("i", [1, 2, 3, 7, 100, 1000])
def test_schedule_takes_the_algorithms_step(i):
    """Algorithm 1 steps beta by (beta_f - beta_i) / i per iteration from beta_i:
    i values, the first beta_i, equal steps, the last one step short of beta_f."""
    b = alg1.linear_schedule(0.35, 3.5, i)
    step = (3.5 - 0.35) / i
    assert b.shape == (i,) and b[0] == 0.35
    assert np.allclose(np.diff(b), step, rtol=0, atol=1e-12)
    assert b[-1] == pytest.approx(3.5 - step, abs=1e-12)


@pytest.mark.parametrize("window", [1, 2, 3, 8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_windowed_search_equals_the_paper_loop_on_scripted_solvers(window, seed):
    rng = np.random.default_rng(seed)
    t, p_succ = 10, 0.8
    m_max = alg1.max_fails(t, p_succ)
    fail_p = {i: float(v) for i, v in zip(range(1, 200), np.linspace(0.9, 0.0, 199))}
    table = {i: rng.random(t) < fail_p[i] for i in range(1, 200)}
    energies = {i: np.where(table[i], -50, -100) for i in table}

    def pc(i, beta, j):
        return int(energies[i][j])

    i_or, hist_or = oracle.alg1_minimal_budget(pc, -100.0, 3, 2, t, 0.9, p_succ, 0.35, 3.5, 199)
    res = alg1.search(lambda bs: [energies[b] for b in bs], -100.0, 3, 2, t, 0.9, p_succ, window=window, i_max=199)
    assert res.i_min == i_or and res.m_max == m_max
    evaluated = dict(res.history)
    for i, m, _ in hist_or:
        assert (evaluated[i] <= m_max) == (m <= m_max)
        if m <= m_max:
            assert evaluated[i] == m


def _g(inst):
    if inst["kind"] == "ea3d":
        return oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    return oracle.biclique_graph(*inst["dims"], inst["J"], inst["h"])


def _brute_force_min(inst):
    if inst["kind"] == "ea3d":
        Jf, hv = refmath.ea_dense(inst["dims"], inst["J"], inst["h"])
    else:
        Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    return int(refmath.dense_energy(Jf, hv, refmath.all_states(Jf.shape[0])).min())


def _cases():
    ea2 = synth.ea_instance(2, seed=5, field="uniform3")
    k44 = synth.biclique_instance(4, seed=6)
    return [("ferro cube L=6", synth.ferro_ea(6), -648, 0.9),       # closed form -3N
            ("ferro K_{32,32}", synth.ferro_biclique(32), -1024, 0.95),  # closed form -n^2
            ("EA 2x2x2 with fields", ea2, _brute_force_min(ea2), 0.99),
            ("K_{4,4} with fields", k44, _brute_force_min(k44), 0.99)]


@pytest.mark.parametrize("name,inst,G,p", _cases())
def test_windowed_search_equals_the_paper_loop_on_oracle_anneals(name, inst, G, p):
    g = _g(inst)
    t, p_succ = 20, 0.9
    i_or, hist = oracle.alg1_minimal_budget(oracle.alg1_trial(g, _seed_of), G, 1, 1, t, p, p_succ, 0.35, 3.5, 400)
    assert i_or is not None, name
    run = lambda bs: [oracle.anneal(g, alg1.linear_schedule(0.35, 3.5, b), t, _seed_of(b)).energies for b in bs]
    for window in (1, 5):
        res = alg1.search(run, G, 1, 1, t, p, p_succ, window=window, i_max=400)
        assert res.i_min == i_or, (name, window)
    # minimality: every smaller budget failed
    assert all(m > 2 for i, m, _ in hist[:-1]) and hist[-1][0] == i_or


def test_budget_seed_convention():
    assert all(alg1.budget_seed(7, i) == _seed_of(i) for i in (1, 2, 1000, 2 ** 20))


def test_ground_truths_are_minimal():
    """The closed forms are the brute-force minima on boxes small enough to
    enumerate, and long oracle anneals reach them on larger ones."""
    for inst, E0 in ((synth.ferro_ea((2, 2, 2)), -24), (synth.ferro_biclique(4), -16)):
        assert _brute_force_min(inst) == E0
    for inst, E0 in ((synth.ferro_ea(4), -192), (synth.ferro_biclique(8), -64)):
        r = oracle.anneal(_g(inst), synth.beta_linear(0.35, 3.5, 300), 16, seed=2)
        assert r.energies.min() == E0


# ---------------------------------------------------------------- metrics

def test_b_eff_and_cooled_b():
    assert alg1.b_eff(64, -180, -192) == pytest.approx(64 / 12)
    assert math.isinf(float(alg1.b_eff(64, -192, -192)))
    assert np.allclose(alg1.b_eff(100, np.array([-90, -95]), -100), [10.0, 20.0])
    # b = (2 log 2)(|E0| / N) b_eff, with |E0| / N = 3 here
    assert alg1.b_cooled(64, -180, -192) == pytest.approx(2 * math.log(2) * 3.0 * 64 / 12)


def test_residual_and_success_rate():
    E0 = -1000
    E = np.array([-1000, -995, -990, -989, -900])
    assert np.allclose(alg1.residual(E, E0), [0.0, 0.005, 0.01, 0.011, 0.1])
    assert alg1.success_rate(E, E0, 0.99) == pytest.approx(3 / 5)
    # for a negative ground truth: E <= p E0  <=>  residual <= 1 - p (off the boundary)
    rng = np.random.default_rng(0)
    for _ in range(200):
        E0 = -int(rng.integers(100, 10000))
        p = float(rng.uniform(0.5, 0.999))
        e = int(rng.integers(E0, 0))
        if abs(e - p * E0) < 1e-6:
            continue
        assert (e <= p * E0) == (alg1.residual(e, E0) <= 1 - p)
