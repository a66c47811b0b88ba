"""Benchmark harness of the paper's Sec. 1.3.3 (Algorithm 1) and the solution
quality metrics of Sec. 2.1-2.2, run on the GPU through the C ABI.

Algorithm 1 looks for the smallest iteration budget i at which at most
m_max = round(t (1 - p_succ)) of t trials end above the threshold p G, where G
is the ground-truth energy, growing i by a fixed step from i_start.  Here

* a trial is one replica of an anneal: the t trials of one budget are the t
  replicas of a single anneal with the same linear schedule;
* the budget counts sweeps (every update group once, beta constant within a
  sweep); the paper's iterations are sweeps times the number of groups;
* the linear schedule over i sweeps starts at beta_i and grows by the
  algorithm's step delta_beta = (beta_f - beta_i) / i after every sweep;
* candidate budgets are tried ``window`` at a time in one batched launch; the
  answer is still the smallest passing budget in ascending order, so it does
  not depend on the window, and each budget's anneal uses a seed that depends
  on the budget only.

The fail test compares energies with the literal threshold p G: for a negative
ground truth and p < 1 a trial passes when its energy is at most p G, that is
when its residual (E - E0) / |E0| is at most 1 - p.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import pbit

_GOLDEN = 0x9E3779B97F4A7C15


def max_fails(t: int, p_succ: float) -> int:
    """m_max = round(t (1 - p_succ)), halves rounded up."""
    return int(math.floor(t * (1.0 - p_succ) + 0.5))


def linear_schedule(beta_i: float, beta_f: float, sweeps: int) -> np.ndarray:
    """beta for sweeps k = 0..sweeps-1: beta_i + k delta_beta with Algorithm 1's
    step delta_beta = (beta_f - beta_i) / sweeps."""
    if sweeps < 1:
        raise ValueError("a schedule needs at least one sweep")
    delta_beta = (beta_f - beta_i) / sweeps
    return np.array([beta_i + k * delta_beta for k in range(sweeps)], np.float64)


def budget_seed(seed: int, budget: int) -> int:
    """Seed of the anneal that evaluates one budget: distinct budgets draw
    unrelated random streams, and a budget's result does not depend on which
    other budgets share its launch."""
    return (int(seed) + int(budget) * _GOLDEN) % (1 << 64)


@dataclass
class SearchResult:
    i_min: int | None                                  # smallest passing budget (sweeps), None if none up to i_max
    history: list = field(default_factory=list)        # (budget, fails) in the order evaluated
    m_max: int = 0
    threshold: float = 0.0


def search(run_window, G: float, i_start: int, i_step: int, t: int, p: float, p_succ: float,
           window: int = 1, i_max: int | None = None) -> SearchResult:
    """Algorithm 1 over a runner.  ``run_window(budgets)`` returns, for each
    budget in the list, the final energies of its t trials."""
    if i_start < 1 or i_step < 1 or t < 1 or window < 1:
        raise ValueError("i_start, i_step, t and window must be positive")
    theta = p * G
    m_max = max_fails(t, p_succ)
    res = SearchResult(None, [], m_max, theta)
    i = int(i_start)
    while i_max is None or i <= i_max:
        cands = [i + k * i_step for k in range(window) if i_max is None or i + k * i_step <= i_max]
        outs = run_window(cands)
        for b, e in zip(cands, outs):
            e = np.asarray(e).reshape(-1)
            if e.size != t:
                raise ValueError("runner returned %d energies for %d trials" % (e.size, t))
            m = int(np.count_nonzero(e > theta))
            res.history.append((b, m))
            if m <= m_max:
                res.i_min = b
                return res
        i = cands[-1] + i_step
    return res


def gpu_runner(ctx, problem: int, beta_i: float, beta_f: float, t: int, seed: int):
    """Runner for ``search`` that anneals t replicas per budget on the GPU;
    the budgets of one window go to the batched persistent kernels when the
    problem kind allows, else to one pbit_anneal call each."""
    batched = [True]

    def run(budgets):
        jobs = [dict(problem=problem, beta=linear_schedule(beta_i, beta_f, b), n_replicas=t,
                     seed=budget_seed(seed, b)) for b in budgets]
        if batched[0] and len(jobs) > 1:
            try:
                return [o.energies for o in pbit.pbit_anneal_batch(ctx, jobs, want_spins=False)]
            except pbit.PbitError as e:
                if e.code != pbit.PBIT_E_UNSUPPORTED:
                    raise
                batched[0] = False
        return [pbit.pbit_anneal(ctx, problem, j["beta"], t, j["seed"], want_spins=False).energies for j in jobs]

    return run


def i_min(ctx, problem: int, G: float, *, i_start: int = 1, i_step: int = 1, t: int = 20, p: float = 0.99,
          p_succ: float = 0.9, beta_i: float = 0.35, beta_f: float = 3.5, seed: int = 1, window: int = 8,
          i_max: int | None = None) -> SearchResult:
    """Smallest sweep budget at which a linear anneal reaches p G in at least
    p_succ of t trials (defaults: 20 trials at 90 %, 1 % residual, the
    paper's 0.35 -> 3.5 schedule)."""
    return search(gpu_runner(ctx, problem, beta_i, beta_f, t, seed), G, i_start, i_step, t, p, p_succ,
                  window, i_max)


def i_min_series(ctx, problems_and_G, **kw) -> list:
    """Algorithm 1 chained over instances of growing size: each search starts
    at the budget the previous one found."""
    out = []
    start = kw.pop("i_start", 1)
    for problem, G in problems_and_G:
        r = i_min(ctx, problem, G, i_start=start, **kw)
        out.append(r)
        if r.i_min is not None:
            start = r.i_min
    return out


# ---------------------------------------------------------------- quality metrics

def residual(E, E0):
    """(E - E0) / |E0|: 0 at the ground truth, 0.01 at 99 % quality."""
    return (np.asarray(E, np.float64) - E0) / abs(E0)


def success_rate(E, G: float, p: float) -> float:
    """Fraction of runs that pass the Algorithm 1 test (energy not above p G)."""
    e = np.asarray(E).reshape(-1)
    return float(np.count_nonzero(e <= p * G)) / max(e.size, 1)


def b_eff(N: int, E, E0):
    """Inverse residual energy per site, N / (E - E0) (Eq. 5); inf at E0."""
    d = np.asarray(E, np.float64) - E0
    with np.errstate(divide="ignore"):
        return np.where(d == 0, np.inf, N / np.where(d == 0, 1.0, d))


def b_cooled(N: int, E, E0):
    """Inverse temperature reachable by digital cooling from b_eff (Sec. 2.2):
    (2 log 2)(|E0| / N) b_eff."""
    return 2.0 * math.log(2.0) * abs(E0) / N * b_eff(N, E, E0)
