"""The ceiling probes (pbit_probe): each reports the work its launches do by the
formula the C interface documents, takes a positive time, and refuses bad
arguments without touching the device."""
import sys

import pytest

from paper_2510_23419_amd import pbit

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_probes_report_their_work():
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    with pbit.Context(0) as c:
        _say("probe copy, philox, mfma")
        ms, work = pbit.pbit_probe(c.ctx, pbit.PBIT_PROBE_COPY, 3 << 20, 3)
        assert ms > 0 and work == 2 * (3 << 20)  # bytes read plus bytes written
        ms, work = pbit.pbit_probe(c.ctx, pbit.PBIT_PROBE_COPY, 1000, 2)  # rounded up to 16 bytes
        assert ms > 0 and work == 2 * 1008
        ms, work = pbit.pbit_probe(c.ctx, pbit.PBIT_PROBE_PHILOX, 3, 2)
        assert ms > 0 and work == 4 * 3 * 8 * cus * 256  # words: 4 per block, 8 workgroups of 256 per CU
        ms, work = pbit.pbit_probe(c.ctx, pbit.PBIT_PROBE_MFMA, 5, 2)
        assert ms > 0 and work == 4 * 65536 * 5 * 2 * cus * 4  # int8 ops: 4 chains, 2 workgroups of 4 waves per CU


@pytest.mark.parametrize("probe,size,reps", [(9, 64, 1), (pbit.PBIT_PROBE_COPY, 0, 1), (pbit.PBIT_PROBE_COPY, 64, 0),
                                             (pbit.PBIT_PROBE_COPY, (1 << 36) + 16, 1),
                                             (pbit.PBIT_PROBE_PHILOX, (1 << 24) + 1, 1),
                                             (pbit.PBIT_PROBE_MFMA, (1 << 24) + 1, 1)])
def test_probe_errors(probe, size, reps):
    with pbit.Context(0) as c:
        with pytest.raises(pbit.PbitError) as err:
            pbit.pbit_probe(c.ctx, probe, size, reps)
        assert err.value.code == pbit.PBIT_E_ARG
