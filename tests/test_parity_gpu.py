"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
spins and energies, every replica after every sweep on the small cases, and
sampled replicas at several sweep counts at the full benchmark sizes."""
import os
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


def graph_of(inst):
    if inst["kind"] == "ea3d":
        return oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    return oracle.biclique_graph(*inst["dims"], inst["J"], inst["h"])


@pytest.fixture(scope="module")
def ctx():
    c = pbit.Context(0)
    yield c.ctx
    c.close()


@pytest.fixture(scope="module", params=["lds", "stream", "mfma"])
def ectx(request):
    """A context per cube path: the default (small cubes held in LDS for runs of
    sweeps, larger ones on the matrix cores where their tiles are built), every
    cube on the streaming stencil (PBIT_EA_STREAM=1), or every cube on the
    matrix cores where its tiles are built (PBIT_EA_MFMA=1)."""
    env = {"lds": {"PBIT_EA_STREAM": "0"}, "stream": {"PBIT_EA_STREAM": "1"},
           "mfma": {"PBIT_EA_STREAM": "0", "PBIT_EA_MFMA": "1"}}[request.param]
    old = {k: os.environ.get(k) for k in ("PBIT_EA_STREAM", "PBIT_EA_MFMA")}
    os.environ.update(env)
    try:
        c = pbit.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    c.mode = request.param
    yield c
    c.close()


def _mfma_tiles(dims):
    """The matrix-core path's tiles are built when a colour class splits into tiles of
    32 sites (every shape tested here then needs at most 8 neighbour blocks per tile)."""
    return (int(np.prod(dims)) // 2) % 32 == 0


def _check_path(c, inst):
    """The cube path the latest anneal took is the one the context asks for."""
    small = int(np.prod(inst["dims"])) <= 8192
    tiles = _mfma_tiles(inst["dims"])
    # by default a large cube takes whichever of the stencil and the matrix cores ran
    # faster when timed
    want = {"lds": {2} if small else ({1, 3} if tiles else {1}), "stream": {1},
            "mfma": {3} if tiles else ({2} if small else {1})}[c.mode]
    assert pbit.pbit_profile_ea_path(c.ctx) in want


def _ea_with_zeros(dims, seed):
    inst = synth.ea_instance(dims, seed=seed, field="uniform3")
    rng = np.random.default_rng(seed + 1)
    inst["J"] = (inst["J"] * (rng.random(inst["J"].shape) < 0.8)).astype(np.int8)  # some J = 0
    return inst


# ---------------------------------------------------------------- energies

@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 6, 2), (6, 6, 6), (10, 8, 6)])
@pytest.mark.parametrize("R", [1, 17, 64])
def test_ea_energy_matches_oracle(ctx, dims, R):
    inst = _ea_with_zeros(dims, seed=sum(dims) + R)
    prob = pbit.load_instance(ctx, inst)
    spins = synth.random_spins(R, int(np.prod(dims)), seed=R)
    _say("ea energy %s R=%d" % (dims, R))
    assert np.array_equal(pbit.pbit_energy(ctx, prob, spins), oracle.energy(graph_of(inst), spins))
    pbit.pbit_unload_problem(ctx, prob)


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 5), (64, 64), (65, 63), (7, 130), (200, 129)])
@pytest.mark.parametrize("R", [1, 63, 65, 130])
def test_biclique_energy_matches_oracle(ctx, na, nb, R):
    inst = synth.biclique_instance(na, seed=na * 7 + nb, nb=nb)
    if R % 2:  # couplings in {-1, 0, +1} for the odd replica counts
        keep = np.random.default_rng(na + nb).random(inst["J"].shape) < 0.65
        inst["J"] = (inst["J"] * keep).astype(np.int8)
    prob = pbit.load_instance(ctx, inst)
    spins = synth.random_spins(R, na + nb, seed=R + na)
    _say("biclique energy %dx%d R=%d" % (na, nb, R))
    assert np.array_equal(pbit.pbit_energy(ctx, prob, spins), oracle.energy(graph_of(inst), spins))
    pbit.pbit_unload_problem(ctx, prob)


# ---------------------------------------------------------------- every sweep

def _every_sweep(ctx, inst, beta, R, seed, init=None, sweep_offset=0, replica_offset=0):
    prob = pbit.load_instance(ctx, inst)
    off = dict(sweep_offset=sweep_offset, replica_offset=replica_offset)
    got = pbit.pbit_anneal(ctx, prob, beta, R, seed, init_spins=init, trace_every=1, trace_spins=True, **off)
    ref = oracle.anneal(graph_of(inst), beta, R, seed, init_spins=init, trace_every=1, trace_spins=True, **off)
    pbit.pbit_unload_problem(ctx, prob)
    assert got.spin_trace.shape == ref.spin_trace.shape
    for s in range(len(beta)):
        if not np.array_equal(got.spin_trace[s], ref.spin_trace[s]):
            bad = np.argwhere(got.spin_trace[s] != ref.spin_trace[s])
            raise AssertionError("first mismatch after sweep %d at (replica, site) %s" % (s + 1, bad[0]))
    assert np.array_equal(got.energy_trace, ref.energy_trace)
    assert np.array_equal(got.spins, ref.spins)
    assert np.array_equal(got.energies, ref.energies)
    assert got.best_energy == ref.energies.min()
    assert got.best_replica == int(np.argmin(ref.energies))
    return got


# schedules at the ends of the threshold table: beta = 0 (every update a fair coin, rows
# as wide as the largest field), large beta only (rows of two entries: every |I| >= 1
# clamps to the last, zero, threshold) and the two interleaved
EXTREME_BETAS = {"zero": [0.0, 0.0, 0.0], "cold": [25.0, 30.0, 40.0, 25.0],
                 "mixed": [0.0, 30.0, 0.4, 0.0, 50.0]}


@pytest.mark.parametrize("sched", sorted(EXTREME_BETAS))
@pytest.mark.parametrize("dims,R", [((8, 8, 8), 37), ((6, 4, 2), 5)])
def test_ea_extreme_betas(ectx, sched, dims, R):
    """Every replica after every sweep at the ends of the schedule range, on each cube
    path, with fields and zero couplings."""
    inst = _ea_with_zeros(dims, seed=5 * R + sum(dims))
    _say("ea %s R=%d beta %s (%s)" % (dims, R, sched, ectx.mode))
    _every_sweep(ectx.ctx, inst, np.array(EXTREME_BETAS[sched]), R, seed=41)
    _check_path(ectx, inst)


# Philox counter words past 31 bits: absolute sweeps from 2^31 - 3 (the index crosses 2^31
# during a run) and global replicas from 2^31 - 64
HIGH_SWEEP, HIGH_REPLICA = 2**31 - 3, 2**31 - 64


@pytest.mark.parametrize("dims,R", [((8, 8, 8), 37), ((6, 4, 2), 5)])
def test_ea_counters_past_31_bits(ectx, dims, R):
    """Every replica after every sweep with the sweep and replica counters near the top
    of their 32-bit range, on each cube path."""
    inst = _ea_with_zeros(dims, seed=97 + R)
    _say("ea %s R=%d counters past 31 bits (%s)" % (dims, R, ectx.mode))
    _every_sweep(ectx.ctx, inst, synth.beta_linear(0.1, 3.0, 6), R, seed=11, sweep_offset=HIGH_SWEEP,
                 replica_offset=HIGH_REPLICA)
    _check_path(ectx, inst)


def test_ea_L6_every_replica_every_sweep(ectx):
    """EA L=6 (216 spins), +-1 couplings, h = 0, 64 replicas from random starts,
    beta linear 0.1 -> 3.0 over 1000 sweeps, seed 1."""
    inst = synth.ea_instance(6, seed=1)
    _say("ea L=6 R=64 S=1000 every sweep (%s)" % ectx.mode)
    _every_sweep(ectx.ctx, inst, synth.beta_linear(0.1, 3.0, 1000), 64, seed=1)
    _check_path(ectx, inst)


@pytest.mark.parametrize("dims,R", [((2, 2, 2), 5), ((4, 6, 2), 33), ((10, 8, 6), 20), ((8, 8, 8), 130),
                                    ((16, 4, 6), 33), ((12, 10, 8), 7), ((32, 2, 4), 129), ((24, 4, 2), 64),
                                    ((4, 4, 4), 20), ((32, 2, 2), 9)])
def test_ea_ragged_with_fields_and_zero_couplings(ectx, dims, R):
    inst = _ea_with_zeros(dims, seed=3 * R)
    _say("ea ragged %s R=%d (%s)" % (dims, R, ectx.mode))
    _every_sweep(ectx.ctx, inst, synth.beta_geometric(0.1, 5.0, 40), R, seed=0xDEADBEEFCAFE)
    _check_path(ectx, inst)


@pytest.mark.parametrize("dims,R,S", [((2, 2, 2), 5, 2500), ((4, 6, 2), 33, 1500), ((20, 20, 20), 40, 30),
                                      ((10, 8, 6), 4096, 300)])
def test_ea_runs_of_sweeps(ectx, dims, R, S):
    """Runs longer than one launch of the LDS-resident kernel, the largest cube it
    takes, and a cube split over 256 workgroups; fields and zero couplings."""
    inst = _ea_with_zeros(dims, seed=7 * R + S)
    prob = pbit.load_instance(ectx.ctx, inst)
    beta = synth.beta_geometric(0.1, 5.0, S)
    _say("ea runs %s R=%d S=%d (%s)" % (dims, R, S, ectx.mode))
    got = pbit.pbit_anneal(ectx.ctx, prob, beta, R, seed=21)
    _check_path(ectx, inst)
    g = graph_of(inst)
    groups = range((R + 3) // 4) if R <= 64 else (0, 511, 1023)
    for gi in groups:
        ref = oracle.anneal(g, beta, min(4, R - 4 * gi), 21, replica_offset=4 * gi)
        assert np.array_equal(got.spins[4 * gi:4 * gi + 4], ref.spins), gi
        assert np.array_equal(got.energies[4 * gi:4 * gi + 4], ref.energies), gi
    pbit.pbit_unload_problem(ectx.ctx, prob)


@pytest.mark.parametrize("na,nb,R", [(40, 40, 70), (7, 130, 3), (130, 66, 129), (1, 1, 1)])
def test_biclique_every_replica_every_sweep(ctx, na, nb, R):
    inst = synth.biclique_instance(na, seed=na + nb, nb=nb)
    _say("biclique %dx%d R=%d every sweep" % (na, nb, R))
    _every_sweep(ctx, inst, synth.beta_linear(0.05, 2.0, 30), R, seed=5)


@pytest.mark.parametrize("na,nb,R", [(600, 520, 200), (512, 1024, 130)])
def test_biclique_large_tiles_ragged(ctx, na, nb, R):
    """Sides of 512 or more sites take the 128 x 128 LDS-tiled kernel; ragged
    sites and replicas exercise its padding."""
    inst = synth.biclique_instance(na, seed=na + 3 * nb, nb=nb)
    _say("biclique large tiles %dx%d R=%d" % (na, nb, R))
    _every_sweep(ctx, inst, synth.beta_linear(0.05, 2.0, 8), R, seed=12)


def test_given_initial_spins(ctx):
    inst = synth.ea_instance(4, seed=2, field="uniform3")
    init = synth.random_spins(9, 64, seed=9)
    _every_sweep(ctx, inst, synth.beta_linear(0.5, 1.0, 10), 9, seed=2, init=init)
    binst = synth.biclique_instance(20, seed=3)
    _every_sweep(ctx, binst, synth.beta_linear(0.5, 1.0, 10), 9, seed=2, init=synth.random_spins(9, 40, seed=1))


def test_given_spins_and_resume_each_cube_path(ectx):
    """Given initial spins, and a run split in two (the second half resumed from the first
    half's spins at its sweep offset), on each cube path: every sweep equals the oracle."""
    inst = _ea_with_zeros((8, 8, 8), seed=101)
    N, R = 512, 37
    beta = synth.beta_linear(0.2, 2.0, 12)
    init = synth.random_spins(R, N, seed=5)
    _say("ea 8^3 given spins and resume (%s)" % ectx.mode)
    _every_sweep(ectx.ctx, inst, beta, R, seed=17, init=init)
    _check_path(ectx, inst)
    prob = pbit.load_instance(ectx.ctx, inst)
    first = pbit.pbit_anneal(ectx.ctx, prob, beta[:5], R, seed=17)
    second = pbit.pbit_anneal(ectx.ctx, prob, beta[5:], R, seed=17, sweep_offset=5, init_spins=first.spins)
    whole = oracle.anneal(graph_of(inst), beta, R, seed=17)
    pbit.pbit_unload_problem(ectx.ctx, prob)
    assert np.array_equal(second.spins, whole.spins) and np.array_equal(second.energies, whole.energies)


def test_zero_sweeps_returns_the_random_start(ctx):
    for inst in (synth.ea_instance(4, seed=5), synth.biclique_instance(33, seed=5)):
        prob = pbit.load_instance(ctx, inst)
        got = pbit.pbit_anneal(ctx, prob, np.zeros(0), 12, seed=77)
        ref = oracle.anneal(graph_of(inst), np.zeros(0), 12, seed=77)
        assert np.array_equal(got.spins, ref.spins) and np.array_equal(got.energies, ref.energies)
        pbit.pbit_unload_problem(ctx, prob)


# ---------------------------------------------------------------- mechanics

@pytest.mark.parametrize("make", [lambda: synth.ea_instance(8, seed=4, field="uniform3"),
                                  lambda: synth.biclique_instance(100, seed=4)])
def test_resume_split_and_replica_slices(ctx, make):
    inst = make()
    prob = pbit.load_instance(ctx, inst)
    beta = synth.beta_linear(0.1, 3.0, 60)
    full = pbit.pbit_anneal(ctx, prob, beta, 24, seed=3)
    a = pbit.pbit_anneal(ctx, prob, beta[:25], 24, seed=3)
    b = pbit.pbit_anneal(ctx, prob, beta[25:], 24, seed=3, sweep_offset=25, init_spins=a.spins)
    assert np.array_equal(full.spins, b.spins) and np.array_equal(full.energies, b.energies)
    for off, cnt in ((0, 4), (8, 12), (20, 4), (4, 1)):
        part = pbit.pbit_anneal(ctx, prob, beta, cnt, seed=3, replica_offset=off)
        assert np.array_equal(full.spins[off:off + cnt], part.spins)
    ref = oracle.anneal(graph_of(inst), beta, 24, seed=3)
    assert np.array_equal(full.spins, ref.spins)
    pbit.pbit_unload_problem(ctx, prob)


def test_two_runs_are_identical(ectx):
    ctx = ectx.ctx
    inst = synth.ea_instance(16, seed=16)
    prob = pbit.load_instance(ctx, inst)
    beta = synth.beta_geometric(0.1, 5.0, 50)
    a = pbit.pbit_anneal(ctx, prob, beta, 256, seed=1)
    b = pbit.pbit_anneal(ctx, prob, beta, 256, seed=1)
    assert np.array_equal(a.spins, b.spins)
    _check_path(ectx, inst)
    pbit.pbit_unload_problem(ctx, prob)


def test_target_stops_at_first_reaching_sweep(ectx):
    ctx = ectx.ctx
    inst = synth.ea_instance(6, seed=11)
    beta = synth.beta_linear(0.1, 3.0, 300)
    ref = oracle.anneal(graph_of(inst), beta, 16, seed=4, trace_every=1)
    mins = ref.energy_trace.min(axis=1)
    target = int(mins[150])
    first = int(np.argmax(mins <= target)) + 1
    prob = pbit.load_instance(ctx, inst)
    got = pbit.pbit_anneal(ctx, prob, beta, 16, seed=4, target=target)
    _check_path(ectx, inst)
    assert got.sweeps_done == first
    assert got.best_energy <= target
    pre = oracle.anneal(graph_of(inst), beta[:first], 16, seed=4)
    assert np.array_equal(got.spins, pre.spins)
    pbit.pbit_unload_problem(ctx, prob)


@pytest.mark.parametrize("make,R,S,k", [
    (lambda: synth.biclique_instance(512, seed=9), 256, 120, 70),        # bit tiles; hit inside a chunk
    (lambda: synth.biclique_instance(40, seed=9, nb=33), 12, 100, 31),   # 64 x 64 tiles; hit on a chunk edge
    (lambda: synth.dimerized_cube(4, seed=4), 16, 90, 40),               # general graph, greedy groups
    (lambda: synth.ea_instance(24, seed=2), 8, 70, 65)])                 # matrix-core cube
def test_target_checked_on_the_device(ctx, make, R, S, k):
    """With a target and no trace the library checks the target on the device
    after every sweep and reads the result once per chunk of sweeps: the run
    still stops after the first sweep that meets the target, with the spins of
    that sweep; a target never met runs every sweep."""
    inst = make()
    g = graph_of(inst) if inst["kind"] != "graph" else oracle.graph_from_bonds(
        inst["n"], inst["bond_i"], inst["bond_j"], inst["bond_J"], inst["h"])
    beta = synth.beta_linear(0.05, 3.0, S)
    ref = oracle.anneal(g, beta, R, seed=6, trace_every=1)
    mins = ref.energy_trace.min(axis=1)
    target = int(mins[k - 1])
    first = int(np.argmax(mins <= target)) + 1
    prob = pbit.load_instance(ctx, inst)
    _say("device target check %s R=%d S=%d first=%d" % (inst["kind"], R, S, first))
    got = pbit.pbit_anneal(ctx, prob, beta, R, seed=6, target=target)
    assert got.sweeps_done == first
    pre = oracle.anneal(g, beta[:first], R, seed=6)
    assert np.array_equal(got.spins, pre.spins) and np.array_equal(got.energies, pre.energies)
    never = pbit.pbit_anneal(ctx, prob, beta, R, seed=6, target=int(mins.min()) - 1)
    assert never.sweeps_done == S and np.array_equal(never.spins, ref.spins)
    pbit.pbit_unload_problem(ctx, prob)


def test_anneal_dev_matches_blocking(ectx):
    import torch

    ctx = ectx.ctx
    for inst in (synth.ea_instance(8, seed=6), synth.biclique_instance(96, seed=6)):
        prob = pbit.load_instance(ctx, inst)
        N = pbit.pbit_problem_spins(ctx, prob)
        beta = synth.beta_linear(0.1, 2.0, 20)
        ref = pbit.pbit_anneal(ctx, prob, beta, 40, seed=9)
        d_spins = torch.zeros((40, N), dtype=torch.int8, device="cuda:0")
        d_e = torch.zeros(40, dtype=torch.int64, device="cuda:0")
        pbit.pbit_anneal_dev(ctx, prob, beta, 40, 9, d_spins, d_energies=d_e)
        assert np.array_equal(d_spins.cpu().numpy(), ref.spins)
        assert np.array_equal(d_e.cpu().numpy(), ref.energies)
        # spins_in: continue from the device spins
        beta2 = synth.beta_linear(2.0, 3.0, 5)
        pbit.pbit_anneal_dev(ctx, prob, beta2, 40, 9, d_spins, spins_in=True, d_energies=d_e, sweep_offset=20)
        ref2 = pbit.pbit_anneal(ctx, prob, beta2, 40, 9, sweep_offset=20, init_spins=ref.spins)
        assert np.array_equal(d_spins.cpu().numpy(), ref2.spins)
        pbit.pbit_unload_problem(ctx, prob)


# ---------------------------------------------------------------- errors

def test_errors_leave_state_untouched(ctx):
    with pytest.raises(pbit.PbitError) as ei:
        pbit.load_instance(ctx, synth.ea_instance((5, 4, 4), seed=1))
    assert ei.value.code == pbit.PBIT_E_COLOURING
    bad = synth.ea_instance(4, seed=1)
    bad["J"][1, 3] = 2
    with pytest.raises(pbit.PbitError) as ei:
        pbit.load_instance(ctx, bad)
    assert ei.value.code == pbit.PBIT_E_RANGE
    prob = pbit.load_instance(ctx, synth.ea_instance(4, seed=1))
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal(ctx, prob, [0.5, np.nan], 4, seed=1)
    assert ei.value.code == pbit.PBIT_E_RANGE
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal(ctx, prob, [0.5], 4, seed=1, replica_offset=2)
    assert ei.value.code == pbit.PBIT_E_ARG
    bad_init = synth.random_spins(2, 64, seed=1)
    bad_init[1, 5] = 0
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal(ctx, prob, [0.5], 2, seed=1, init_spins=bad_init)
    assert ei.value.code == pbit.PBIT_E_RANGE
    pbit.pbit_unload_problem(ctx, prob)
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal(ctx, prob, [0.5], 4, seed=1)
    assert ei.value.code == pbit.PBIT_E_HANDLE
    # a spin matrix beyond the kernels' 32-bit offsets is refused before anything is allocated
    big = pbit.load_instance(ctx, synth.ferro_ea(102))  # 1,061,208 spins
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal(ctx, big, [0.5], 4096, seed=1)
    assert ei.value.code == pbit.PBIT_E_UNSUPPORTED
    pbit.pbit_unload_problem(ctx, big)
    # the context still works
    prob = pbit.load_instance(ctx, synth.ea_instance(4, seed=1))
    assert pbit.pbit_anneal(ctx, prob, [0.5], 4, seed=1).spins.shape == (4, 64)
    pbit.pbit_unload_problem(ctx, prob)


def test_budget_is_enforced():
    with pbit.Context(0, hbm_budget_bytes=200_000) as c:
        prob = pbit.load_instance(c.ctx, synth.ea_instance(8, seed=1))  # ~3.6 KB of couplings
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_anneal(c.ctx, prob, [0.5], 4096, seed=1)  # 2 MB of spins
        assert ei.value.code == pbit.PBIT_E_NOMEM
        assert pbit.pbit_anneal(c.ctx, prob, [0.5], 16, seed=1).spins.shape == (16, 512)
        assert pbit.pbit_bytes_in_use(c.ctx) <= 200_000


# ---------------------------------------------------------------- full sizes, sampled

def _sample_groups(R, rng, extra=2):
    groups = {0, R // 4 - 1}
    while len(groups) < 2 + extra:
        groups.add(int(rng.integers(0, R // 4)))
    return sorted(groups)


def _check_sampled(ctx, inst, beta, R, seed, prefixes, full_groups, rng):
    prob = pbit.load_instance(ctx, inst)
    g = graph_of(inst)
    for S in prefixes:
        _say("  %s dims=%s R=%d prefix S=%d" % (inst["kind"], inst["dims"], R, S))
        got = pbit.pbit_anneal(ctx, prob, beta[:S], R, seed)
        groups = _sample_groups(R, rng) if S < len(beta) else full_groups
        for gidx in groups:
            ref = oracle.anneal(g, beta[:S], 4, seed, replica_offset=4 * gidx)
            assert np.array_equal(got.spins[4 * gidx:4 * gidx + 4], ref.spins), (S, gidx)
            assert np.array_equal(got.energies[4 * gidx:4 * gidx + 4], ref.energies), (S, gidx)
    pbit.pbit_unload_problem(ctx, prob)


def test_ea_L16_full_size_sampled(ectx):
    """L=16 cube, 4096 replicas, beta geometric 0.1 -> 5.0 over 10^4 sweeps."""
    inst = synth.ea_instance(16, seed=16)
    beta = synth.beta_geometric(0.1, 5.0, 10_000)
    rng = np.random.default_rng(16)
    _check_sampled(ectx.ctx, inst, beta, 4096, 1, [1, 2, 10, 100, 1000, 10_000], [1023], rng)
    _check_path(ectx, inst)


def test_ea_L32_full_size_sampled(ectx):
    """L=32 cube, 4096 replicas, beta geometric 0.1 -> 5.0 over 10^4 sweeps."""
    inst = synth.ea_instance(32, seed=32)
    beta = synth.beta_geometric(0.1, 5.0, 10_000)
    rng = np.random.default_rng(32)
    _check_sampled(ectx.ctx, inst, beta, 4096, 1, [1, 2, 10, 100], [], rng)
    _check_path(ectx, inst)


@pytest.mark.parametrize("n,prefixes", [(512, [1, 2, 10, 100, 2000]), (1024, [1, 2, 10, 100]),
                                        (2048, [1, 2, 10]), (4096, [1, 2])])
def test_biclique_full_size_sampled(ctx, n, prefixes):
    """K_{n,n}, 1024 replicas, beta linear 0.05 -> 2.0 over 2000 sweeps."""
    inst = synth.biclique_instance(n, seed=n)
    beta = synth.beta_linear(0.05, 2.0, 2000)
    rng = np.random.default_rng(n)
    _check_sampled(ctx, inst, beta, 1024, 1, prefixes, [0], rng)
