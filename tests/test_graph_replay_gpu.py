"""pbit_anneal_dev with its sweep launches captured into a HIP graph
(PBIT_GRAPH=1): every replay equals the eager run, with the program's own
eager work and synchronisations between replays; a changed schedule captures a
new graph."""
import os
import sys

import numpy as np
import pytest

import synth
from paper_2510_23419_amd import pbit

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _context(**env):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return pbit.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("name,make,R,S,env", [
    ("cube in LDS", lambda: synth.ea_instance(8, seed=3), 64, 40, {}),
    ("streaming cube", lambda: synth.ea_instance(8, seed=3, field="uniform3"), 48, 25, {"PBIT_EA_STREAM": "1"}),
    ("matrix-core cube", lambda: synth.ea_instance(8, seed=3, field="uniform3"), 130, 25, {"PBIT_EA_MFMA": "1"}),
    ("biclique bits", lambda: synth.biclique_instance(512, seed=5), 256, 12, {}),
    ("small biclique", lambda: synth.biclique_instance(40, seed=5, nb=70), 33, 30, {}),
    ("graph", lambda: synth.dimerized_cube(4, seed=2), 40, 20, {})])
def test_graph_replays_equal_the_eager_run(name, make, R, S, env):
    import torch

    inst = make()
    beta = synth.beta_linear(0.1, 3.0, S)
    beta2 = synth.beta_geometric(0.2, 2.5, S)
    env = {"PBIT_EA_STREAM": "0", "PBIT_EA_MFMA": "-1", **env}
    eager = _context(PBIT_GRAPH="0", **env)
    graph = _context(PBIT_GRAPH="1", **env)
    try:
        pe, pg = pbit.load_instance(eager.ctx, inst), pbit.load_instance(graph.ctx, inst)
        N = pbit.pbit_problem_spins(eager.ctx, pe)
        ref_s = torch.empty((R, N), dtype=torch.int8, device="cuda:0")
        ref_e = torch.empty(R, dtype=torch.int64, device="cuda:0")
        pbit.pbit_anneal_dev(eager.ctx, pe, beta, R, 11, ref_s, d_energies=ref_e)
        ref = (ref_s.cpu().numpy(), ref_e.cpu().numpy())
        _say("graph replay: %s R=%d S=%d" % (name, R, S))
        for k in range(3):
            s = torch.full((R, N), 3, dtype=torch.int8, device="cuda:0")
            e = torch.zeros(R, dtype=torch.int64, device="cuda:0")
            pbit.pbit_anneal_dev(graph.ctx, pg, beta, R, 11, s, d_energies=e)
            assert np.array_equal(s.cpu().numpy(), ref[0]), (name, k)
            assert np.array_equal(e.cpu().numpy(), ref[1]), (name, k)
            # the program's own eager work between replays
            x = torch.randn(1 << 16, device="cuda:0")
            assert float((x * 0).sum().item()) == 0.0
            torch.cuda.synchronize()
        assert pbit.pbit_profile_graph(graph.ctx) == (1, 3)
        # another schedule: a new capture, equal to its eager run
        pbit.pbit_anneal_dev(eager.ctx, pe, beta2, R, 11, ref_s, d_energies=ref_e)
        s = torch.empty((R, N), dtype=torch.int8, device="cuda:0")
        pbit.pbit_anneal_dev(graph.ctx, pg, beta2, R, 11, s)
        assert np.array_equal(s.cpu().numpy(), ref_s.cpu().numpy())
        assert pbit.pbit_profile_graph(graph.ctx) == (2, 4)
    finally:
        eager.close()
        graph.close()
