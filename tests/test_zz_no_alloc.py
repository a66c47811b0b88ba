"""pbit_anneal_dev_noalloc against pbit_anneal_dev: bit-identical spins and
energies for the same request, on two calls in a row with the second smaller
than the first (the static array keeps the first call's contents), for every
problem kind and kernel path; no device memory is allocated by the calls;
requests beyond the static array are refused before any work."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import pbit

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _graph_of(inst):
    if inst["kind"] == "ea3d":
        return oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    if inst["kind"] == "graph":
        return oracle.graph_from_bonds(inst["n"], inst["bond_i"], inst["bond_j"], inst["bond_J"], inst["h"])
    return oracle.biclique_graph(*inst["dims"], inst["J"], inst["h"])


def _pair(ctx, inst, beta, R, seed, path=None):
    """The same anneal through both entry points; returns the no-alloc result
    after checking it against the allocating one.  The no-alloc call comes first
    and must not change the context's device memory."""
    import torch

    prob = pbit.load_instance(ctx, inst)
    N = pbit.pbit_problem_spins(ctx, prob)
    held = pbit.pbit_bytes_in_use(ctx)
    a_s = torch.full((R, N), 7, dtype=torch.int8, device="cuda:0")
    a_e = torch.full((R,), 7, dtype=torch.int64, device="cuda:0")
    _say("noalloc %s dims=%s R=%d S=%d" % (inst["kind"], inst.get("dims", inst.get("n")), R, len(beta)))
    pbit.pbit_anneal_dev(ctx, prob, beta, R, seed, a_s, d_energies=a_e, noalloc=True)
    assert pbit.pbit_bytes_in_use(ctx) == held  # nothing allocated by the call
    if path is not None:
        assert pbit.pbit_profile_ea_path(ctx) == path
    b_s = torch.zeros((R, N), dtype=torch.int8, device="cuda:0")
    b_e = torch.zeros((R,), dtype=torch.int64, device="cuda:0")
    pbit.pbit_anneal_dev(ctx, prob, beta, R, seed, b_s, d_energies=b_e)
    got_s, got_e = a_s.cpu().numpy(), a_e.cpu().numpy()
    assert np.array_equal(got_s, b_s.cpu().numpy())
    assert np.array_equal(got_e, b_e.cpu().numpy())
    # and the first replica group against the oracle
    ref = oracle.anneal(_graph_of(inst), beta, min(4, R), seed)
    assert np.array_equal(got_s[:4], ref.spins) and np.array_equal(got_e[:4], ref.energies)
    pbit.pbit_unload_problem(ctx, prob)
    return got_s


@pytest.fixture(scope="module")
def ctx():
    c = pbit.Context(0)
    yield c.ctx
    c.close()


def test_cube_lds_resident_then_smaller(ctx):
    _pair(ctx, synth.ea_instance(16, seed=16), synth.beta_geometric(0.1, 5.0, 300), 1024, 1)
    _pair(ctx, synth.ea_instance((8, 6, 4), seed=5, field="uniform3"), synth.beta_linear(0.1, 3.0, 40), 37, 3)


def test_cube_matrix_cores_then_smaller(ctx):
    # without allocation (no timing), 24^3 and 32 x 16 x 20 at up to 1024 replicas take
    # the matrix-core half-sweep; 22^3 (5324 sites per colour, not a multiple of 32)
    # the streaming one
    _pair(ctx, synth.ea_instance(24, seed=24), synth.beta_geometric(0.1, 5.0, 20), 1024, 2, path=3)
    _pair(ctx, synth.ea_instance((32, 16, 20), seed=3, field="uniform3"), synth.beta_linear(0.1, 3.0, 12), 100, 3,
          path=3)
    _pair(ctx, synth.ea_instance(22, seed=22, field="uniform3"), synth.beta_geometric(0.1, 5.0, 15), 100, 4, path=1)


def test_biclique_kernels_then_smaller(ctx):
    # bit tiles (sides padded to 128, replicas to 256), then the same shape class
    # smaller (stale bits in the array), then small sides (64 x 64 tiles)
    _pair(ctx, synth.biclique_instance(1024, seed=1024), synth.beta_linear(0.05, 2.0, 12), 512, 5)
    _pair(ctx, synth.biclique_instance(600, seed=6, nb=520), synth.beta_linear(0.05, 2.0, 9), 200, 6)
    _pair(ctx, synth.biclique_instance(40, seed=40), synth.beta_linear(0.05, 2.0, 20), 70, 7)
    # at 128 replicas the bit tile is not available: the DMA tile
    _pair(ctx, synth.biclique_instance(512, seed=512), synth.beta_linear(0.05, 2.0, 6), 128, 8)


def test_graph_then_smaller(ctx):
    _pair(ctx, synth.dimerized_cube(8, seed=8), synth.beta_geometric(0.1, 5.0, 25), 512, 9)
    _pair(ctx, synth.dimerized_cube(5, seed=5), synth.beta_geometric(0.1, 5.0, 10), 20, 10)


def test_resume_from_device_spins(ctx):
    import torch

    inst = synth.ea_instance(10, seed=10)
    prob = pbit.load_instance(ctx, inst)
    beta = synth.beta_linear(0.1, 3.0, 30)
    R, N = 64, 1000
    s = torch.empty((R, N), dtype=torch.int8, device="cuda:0")
    pbit.pbit_anneal_dev(ctx, prob, beta[:12], R, 11, s, noalloc=True)
    pbit.pbit_anneal_dev(ctx, prob, beta[12:], R, 11, s, spins_in=True, sweep_offset=12, noalloc=True)
    full = pbit.pbit_anneal(ctx, prob, beta, R, 11)
    assert np.array_equal(s.cpu().numpy(), full.spins)
    pbit.pbit_unload_problem(ctx, prob)


def test_too_large_is_refused_before_any_work(ctx):
    import torch

    inst = synth.ea_instance(32, seed=32)
    prob = pbit.load_instance(ctx, inst)
    R, N = 4096, 32768  # 128 MiB of spins in the kernels' layout
    s = torch.full((R, N), 5, dtype=torch.int8, device="cuda:0")
    held = pbit.pbit_bytes_in_use(ctx)
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal_dev(ctx, prob, synth.beta_linear(0.1, 1.0, 3), R, 1, s, noalloc=True)
    assert ei.value.code == pbit.PBIT_E_UNSUPPORTED
    assert "static array" in str(ei.value)
    torch.cuda.synchronize()
    assert int((s != 5).sum().item()) == 0  # the caller's buffer is untouched
    assert pbit.pbit_bytes_in_use(ctx) == held
    pbit.pbit_unload_problem(ctx, prob)
