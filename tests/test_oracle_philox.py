"""Pin the oracle's Philox4x32-10 to rocRAND's engine (an implementation it shares
no code with), called on the host from a small program built with hipcc."""
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

from oracle import oracle

HELPER = Path(__file__).resolve().parent / "helpers" / "rocrand_philox.cpp"


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(hipcc).exists():
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("rocrand") / "philox"
    subprocess.run([hipcc, "-O1", "-o", str(exe), str(HELPER)], check=True)
    return exe


def _cases():
    rng = np.random.default_rng(2510)
    edge = [0, 1, 2, 3, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF]
    cases = []
    for a in edge:
        cases.append((a | (edge[-1 - edge.index(a)] << 32), a, a, a, a))
    for _ in range(300):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        cases.append((seed, *ctr))
    # the counters the sweep actually uses: (spin, sweep, replica >> 2, domain)
    for spin, sweep, rq, dom in [(0, 0, 0, 0), (215, 999, 15, 0), (32767, 9999, 1023, 0), (5, 0, 3, 1)]:
        cases.append((1, spin, sweep, rq, dom))
    return cases


def test_philox_matches_rocrand(rocrand_exe):
    cases = _cases()
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([str(rocrand_exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        seed = c[0]
        got = oracle.philox4x32_10(c[1:], [seed & 0xFFFFFFFF, seed >> 32])
        assert tuple(int(v) for v in got) == r, c


def test_philox_words_look_uniform():
    # 4096 blocks -> 16384 words: mean of the top bit and of the word near 1/2
    words = np.concatenate([oracle.philox4x32_10([i, 7, 3, 0], [1, 0]) for i in range(4096)])
    assert abs((words >> 31).mean() - 0.5) < 0.02
    assert abs(words.astype(np.float64).mean() / 2**32 - 0.5) < 0.01


@pytest.mark.parametrize("kind", ["cube", "biclique"])
def test_random_start_is_the_domain_one_word_of_rocrand(rocrand_exe, kind):
    """The oracle's random start, spin by spin, against rocRAND's Philox4x32-10:
    replica r at spin i is +1 exactly when word r mod 4 of the block at counter
    (i, 0, global replica >> 2, 1) is below 2^31.  A swapped comparison, a wrong
    domain or sweep word, or a wrong word index fails here."""
    g = (oracle.ea_graph((4, 2, 2), np.ones((3, 16), np.int8), None) if kind == "cube"
         else oracle.biclique_graph(5, 3, np.ones((5, 3), np.int8), None))
    seed, R, off = 0x123456789AB, 11, 8
    got = oracle.anneal(g, np.zeros(0), R, seed, replica_offset=off).spins
    cases = [(seed, i, 0, (off + r) >> 2, 1) for r in range(R) for i in range(g.n)]
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([str(rocrand_exe)], input=inp, capture_output=True, text=True, check=True).stdout
    words = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    k = 0
    for r in range(R):
        for i in range(g.n):
            w = words[k][(off + r) & 3]
            assert got[r, i] == (1 if w < 2**31 else -1), (r, i)
            k += 1
