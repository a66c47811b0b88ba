"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every entry point include/pbit.h declares, the host-built threshold
table equals the oracle's entry by entry, and argument errors are reported."""
import re
from pathlib import Path

import numpy as np
import pytest

from oracle import oracle
from paper_2510_23419_amd import pbit

HEADER = Path(__file__).resolve().parent.parent / "include" / "pbit.h"


def _declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbit_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = pbit.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pbit.EXPORTS)


def test_version_string():
    assert "gfx950" in pbit.pbit_version()


@pytest.mark.parametrize("beta", [np.linspace(0.0, 6.0, 25), np.geomspace(0.01, 20.0, 30),
                                  np.array([0.05, 0.35, 3.5, 11.44, 11.4366, 1e-9])])
def test_threshold_table_equals_oracle_entry_by_entry(beta):
    A = 64
    lib_tab = pbit.pbit_threshold_table(beta, A)
    ref = oracle.threshold_table(beta, A)
    assert lib_tab.dtype == np.uint32 and lib_tab.shape == ref.shape
    assert np.array_equal(lib_tab, ref)


def test_large_threshold_table_split_over_threads_equals_oracle():
    """A biclique-sized table (2000 sweeps x 256 field values: built by several
    host threads, each a band of rows) equals the oracle entry by entry."""
    beta = np.geomspace(0.05, 2.0, 2000)
    A = 255
    lib_tab = pbit.pbit_threshold_table(beta, A)
    ref = oracle.threshold_table(beta, A)
    assert np.array_equal(lib_tab, ref)


def test_threshold_table_rejects_bad_beta():
    for bad in (np.nan, -0.1, np.inf):
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_threshold_table(np.array([0.5, bad]), 4)
        assert ei.value.code == pbit.PBIT_E_RANGE
        assert "beta[1]" in str(ei.value)


def test_null_context_is_an_argument_error():
    L = pbit.lib()
    assert L.pbit_load_problem(None, None, None) == pbit.PBIT_E_ARG
    assert L.pbit_anneal(None, 0, None, None) == pbit.PBIT_E_ARG
    assert L.pbit_submit(None, 0, None, None) == pbit.PBIT_E_ARG
    assert b"NULL" in L.pbit_last_error()
    L.pbit_destroy(None)  # ignored
