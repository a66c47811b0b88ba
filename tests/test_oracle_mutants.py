"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of the oracle's C source (on the CPU only), builds it, and
checks that at least one of the pins used elsewhere in this suite fails on it.
"""
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

import synth
from oracle import oracle
from tests import refmath
from tests.test_oracle_boltzmann import _chi2_pvalue

SRC = Path(oracle.__file__).resolve().parent / "pbit_oracle.c"
HELPER = Path(__file__).resolve().parent / "helpers" / "rocrand_philox.cpp"

MUTANTS = {
    "decision_sign": ("return (x < row[a]) ? (int8_t)-s : s;", "return (x < row[a]) ? s : (int8_t)-s;"),
    "dropped_field": ("int32_t I = h ? h[i] : 0;", "int32_t I = 0;"),
    "field_sign": ("I += nJ[q] * m[nb[q]];", "I -= nJ[q] * m[nb[q]];"),
    "missing_factor_2": ("exp((2.0 * beta) * (double)a)", "exp(beta * (double)a)"),
    "philox_9_rounds": ("for (int round = 0; round < 10; ++round)", "for (int round = 0; round < 9; ++round)"),
    "philox_swapped_words": ("uint32_t y1 = lo1;", "uint32_t y1 = lo0;"),
    "replica_word": ("return out[replica & 3u];", "return out[(replica >> 2) & 3u];"),
    "energy_update_sign": ("e -= (int64_t)(mn - m[i]) * I;", "e += (int64_t)(mn - m[i]) * I;"),
    "energy_bond_sign": ("e -= (int64_t)bJ[b] * m[bi[b]] * m[bj[b]];", "e += (int64_t)bJ[b] * m[bi[b]] * m[bj[b]];"),
    "threshold_rounding": ("ceil(ldexp(q, 32) - 0.5)", "floor(ldexp(q, 31))"),
    "init_comparison": ("draw(seed, (uint32_t)i, 0u, rg, 1u) < 0x80000000u ? 1 : -1",
                        "draw(seed, (uint32_t)i, 0u, rg, 1u) >= 0x80000000u ? 1 : -1"),
    "init_domain": ("draw(seed, (uint32_t)i, 0u, rg, 1u) < 0x80000000u", "draw(seed, (uint32_t)i, 0u, rg, 0u) < 0x80000000u"),
}


def _build_mutant(tmpdir, name):
    old, new = MUTANTS[name]
    text = SRC.read_text()
    assert text.count(old) == 1, name
    src = tmpdir / ("%s.c" % name)
    src.write_text(text.replace(old, new))
    so = tmpdir / ("lib%s.so" % name)
    subprocess.run(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), str(src), "-lm"],
                   check=True)
    return oracle.load(so)


# ---- the pins, each returning True when it passes --------------------------

def pin_philox_rocrand(exe):
    rng = np.random.default_rng(3)
    cases = [(int(rng.integers(0, 2**63)), *[int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)])
             for _ in range(8)]
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        got = oracle.philox4x32_10(c[1:], [c[0] & 0xFFFFFFFF, c[0] >> 32])
        if tuple(int(v) for v in got) != tuple(int(v) for v in line.split()):
            return False
    return True


def pin_random_start_rocrand(exe):
    # the random start: +1 where word r & 3 of rocRAND's block (i, 0, r >> 2, 1) is below 2^31
    g = oracle.biclique_graph(3, 2, np.ones((3, 2), np.int8), None)
    got = oracle.anneal(g, np.zeros(0), 8, 77).spins
    cases = [(77, i, 0, r >> 2, 1) for r in range(8) for i in range(5)]
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (_, i, _, _, _), line, r in zip(cases, out, [r for r in range(8) for _ in range(5)]):
        if got[r, i] != (1 if int(line.split()[r & 3]) < 2**31 else -1):
            return False
    return True


def pin_threshold_closed_form():
    from scipy.special import expit
    for beta in (0.1, 1.0):
        for a in range(8):
            if abs(oracle.minority_threshold(beta, a) - expit(-2 * beta * a) * 2**32) > 0.5 + 1e-3:
                return False
    return True


def pin_energy_dense():
    inst = synth.ea_instance((2, 4, 4), seed=2, field="uniform3")
    g = oracle.ea_graph((2, 4, 4), inst["J"], inst["h"])
    sp = synth.random_spins(4, 32, seed=1)
    Jf, hv = refmath.ea_dense((2, 4, 4), inst["J"], inst["h"])
    return np.array_equal(oracle.energy(g, sp), refmath.dense_energy(Jf, hv, sp))


def pin_ferro_ground():
    inst = synth.ferro_biclique(8, 1)
    g = oracle.biclique_graph(8, 8, inst["J"], inst["h"])
    try:
        res = oracle.anneal(g, synth.beta_linear(0.05, 2.0, 100), 4, seed=8)
    except RuntimeError:
        return False
    return res.energies.min() == -80 and np.array_equal(res.energies, oracle.energy(g, res.spins))


def pin_boltzmann():
    inst = synth.biclique_instance(3, seed=8)
    g = oracle.biclique_graph(3, 3, inst["J"], inst["h"])
    Jf, hv = refmath.biclique_dense(inst["J"], inst["h"])
    try:
        res = oracle.anneal(g, np.full(40, 0.5), 8192, seed=5)
    except RuntimeError:
        return False
    pi = refmath.boltzmann(refmath.dense_energy(Jf, hv, refmath.all_states(6)).astype(float), 0.5)
    return _chi2_pvalue(np.bincount(refmath.state_index(res.spins), minlength=64), pi, 8192) > 1e-4


def pin_literal_decision():
    # one sweep of a star: the centre must follow sgn(tanh(beta I) - u)
    k, R, seed, beta = 6, 512, 99, 0.4
    J = np.array([1, -1, 1, 1, -1, 1], np.int8)
    g = oracle.Graph(k + 1, np.zeros(k, np.int32), np.arange(1, k + 1, dtype=np.int32), J,
                     np.array([1] + [0] * k, np.int8), np.array([0] + [1] * k, np.uint8), 2)
    init = synth.random_spins(R, k + 1, seed=4)
    try:
        res = oracle.anneal(g, [beta], R, seed, init_spins=init)
    except RuntimeError:
        return False
    I = init[:, 1:].astype(np.int64) @ J.astype(np.int64) + 1
    return _literal_ok(res, I, R, seed, beta)


def _literal_ok(res, I, R, seed, beta):
    import math
    # words from the rocRAND-pinned mapping: (spin 0, sweep 0, r >> 2, domain 0), word r & 3
    for r in range(R):
        w = int(oracle.philox4x32_10([0, 0, r >> 2, 0], [seed, 0])[r & 3])
        d = math.tanh(beta * I[r]) - ((w + 0.5) / 2**31 - 1.0)
        if abs(d) > 1e-9 and (1 if d > 0 else -1) != res.spins[r, 0]:
            return False
    return True


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    exe = tmp_path_factory.mktemp("rocrand_m") / "philox"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    subprocess.run([hipcc, "-O1", "-o", str(exe), str(HELPER)], check=True)
    return exe


def _all_pins(exe):
    return {
        "philox_rocrand": pin_philox_rocrand(exe),
        "random_start_rocrand": pin_random_start_rocrand(exe),
        "threshold_closed_form": pin_threshold_closed_form(),
        "energy_dense": pin_energy_dense(),
        "ferro_ground": pin_ferro_ground(),
        "boltzmann": pin_boltzmann(),
        "literal_decision": pin_literal_decision(),
    }


def test_pins_pass_on_the_real_oracle(rocrand_exe):
    assert all(_all_pins(rocrand_exe).values())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_fails_a_pin(name, rocrand_exe, tmp_path, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", _build_mutant(tmp_path, name))
    results = _all_pins(rocrand_exe)
    assert not all(results.values()), (name, results)
