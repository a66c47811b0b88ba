"""General sparse graphs with k update groups (paper Sec. 1.2.2): the HIP
path through the C ABI against the oracle, bit-exact, on odd cubes (which a
checkerboard cannot colour), random sparse graphs with fields and zero
couplings, caller-given colourings, and the degree limits.  Every test runs on
both per-instance paths: graphs that fit LDS held there for runs of sweeps (the
default tile width, and tiles of 16 and 8 replicas forced through
PBIT_GRAPH_SLAB) and one launch per colour class (PBIT_GRAPH_SLAB=0)."""
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


SLAB = {}  # context -> graphs that fit LDS run there


@pytest.fixture(scope="module", params=["1", "16", "8", "0"], ids=["slab", "slab_rs16", "slab_rs8", "per_class"])
def ctx(request):
    old = os.environ.get("PBIT_GRAPH_SLAB")
    os.environ["PBIT_GRAPH_SLAB"] = request.param
    try:
        c = pbit.Context(0)
    finally:
        if old is None:
            del os.environ["PBIT_GRAPH_SLAB"]
        else:
            os.environ["PBIT_GRAPH_SLAB"] = old
    SLAB[c.ctx.value] = request.param != "0"
    yield c.ctx
    c.close()


def _oracle_graph(g, colour=None, n_colours=None):
    return oracle.graph_from_bonds(g["n"], g["bond_i"], g["bond_j"], g["bond_J"], g.get("h"), colour, n_colours)


def _with_zeros(g, frac, seed):
    rng = np.random.default_rng(seed)
    g["bond_J"] = (g["bond_J"] * (rng.random(g["bond_J"].size) >= frac)).astype(np.int8)
    return g


def _every_sweep(ctx, g, beta, R, seed, colour=None, n_colours=None, sweep_offset=0, replica_offset=0):
    prob = pbit.pbit_load_graph(ctx, g["n"], g["bond_i"], g["bond_j"], g["bond_J"], g.get("h"), colour,
                                n_colours or 0)
    off = dict(sweep_offset=sweep_offset, replica_offset=replica_offset)
    got = pbit.pbit_anneal(ctx, prob, beta, R, seed, trace_every=1, trace_spins=True, **off)
    ref = oracle.anneal(_oracle_graph(g, colour, n_colours), beta, R, seed, trace_every=1, trace_spins=True, **off)
    pbit.pbit_unload_problem(ctx, prob)
    for s in range(len(beta)):
        if not np.array_equal(got.spin_trace[s], ref.spin_trace[s]):
            bad = np.argwhere(got.spin_trace[s] != ref.spin_trace[s])
            raise AssertionError("first mismatch after sweep %d at (replica, site) %s" % (s + 1, bad[0]))
    assert np.array_equal(got.energy_trace, ref.energy_trace)
    assert np.array_equal(got.energies, ref.energies)
    return got


@pytest.mark.parametrize("dims,R", [((3, 3, 3), 1), ((5, 5, 5), 17), ((7, 5, 3), 70), ((3, 4, 6), 33)])
def test_odd_cube_every_replica_every_sweep(ctx, dims, R):
    inst = synth.ea_instance(dims, seed=sum(dims) + R, field="uniform3")
    g = _with_zeros(synth.ea_bond_list(inst), 0.15, seed=R)
    _say("odd cube %s R=%d every sweep" % (dims, R))
    _every_sweep(ctx, g, synth.beta_geometric(0.1, 5.0, 40), R, seed=0xDEADBEEFCAFE)


@pytest.mark.parametrize("n,deg,R", [(50, 4, 5), (700, 6, 40), (2000, 12, 130), (300, 60, 16)])
def test_random_sparse_graph_every_sweep(ctx, n, deg, R):
    g = _with_zeros(synth.random_sparse_graph(n, deg, seed=n + deg), 0.1, seed=n)
    _say("random graph n=%d deg=%d R=%d every sweep" % (n, deg, R))
    _every_sweep(ctx, g, synth.beta_linear(0.05, 3.0, 30), R, seed=7)


@pytest.mark.parametrize("sched", ["zero", "cold", "mixed"])
def test_graph_extreme_betas(ctx, sched):
    """The group sweep at the ends of the schedule range (beta = 0 only, large beta
    only, both interleaved)."""
    from tests.test_parity_gpu import EXTREME_BETAS
    g = _with_zeros(synth.random_sparse_graph(300, 8, seed=31), 0.1, seed=3)
    _say("random graph n=300 beta %s every sweep" % sched)
    _every_sweep(ctx, g, np.array(EXTREME_BETAS[sched]), 21, seed=53)


def test_graph_counters_past_31_bits(ctx):
    """The group sweep with its sweep and replica counters near the top of their
    32-bit range."""
    from tests.test_parity_gpu import HIGH_REPLICA, HIGH_SWEEP
    inst = synth.ea_instance((5, 5, 5), seed=8, field="uniform3")
    g = _with_zeros(synth.ea_bond_list(inst), 0.15, seed=8)
    _say("odd cube 5^3 counters past 31 bits")
    _every_sweep(ctx, g, synth.beta_linear(0.1, 3.0, 6), 19, seed=67, sweep_offset=HIGH_SWEEP,
                 replica_offset=HIGH_REPLICA)


@pytest.mark.parametrize("L,R,field", [(3, 5, "uniform3"), (7, 50, "zero"), (7, 33, "uniform3")])
def test_dimerized_cube_every_sweep(ctx, L, R, field):
    """The five-group stand-in for the paper's hardware-embedded lattices."""
    g = synth.dimerized_cube(L, seed=L + R, field=field)
    _say("dimerized cube L=%d R=%d %s every sweep" % (L, R, field))
    assert pbit.pbit_greedy_colouring(g["n"], g["bond_i"], g["bond_j"])[1] == (5 if L == 7 else 4)
    _every_sweep(ctx, g, synth.beta_geometric(0.1, 5.0, 30), R, seed=5)


def test_dimerized_cube_benchmark_size_sampled(ctx):
    """The benchmark's graph workload (L = 14: 5,488 spins, 4,096 replicas, the
    first 12 sweeps of its schedule) in the launch configuration the benchmark
    times; replica slices recomputed by the oracle through replica_offset."""
    g = synth.dimerized_cube(14, seed=14)
    prob = pbit.load_instance(ctx, g)
    beta = synth.beta_geometric(0.1, 5.0, 2000)[:12]
    _say("dimerized cube L=14 R=4096 S=12")
    got = pbit.pbit_anneal(ctx, prob, beta, 4096, seed=1)
    assert pbit.pbit_profile_graph_path(ctx) == (2 if SLAB[ctx.value] else 1)
    og = _oracle_graph(g)
    for off in (0, 1360, 4092):
        ref = oracle.anneal(og, beta, 4, seed=1, replica_offset=off)
        assert np.array_equal(got.spins[off:off + 4], ref.spins), off
        assert np.array_equal(got.energies[off:off + 4], ref.energies), off
    pbit.pbit_unload_problem(ctx, prob)


def test_profile_windows_count_group_launches(ctx):
    """pbit_profile_read keeps the half-sweep launches of each problem kind
    apart: k launches per sweep for a graph of k groups, 2 for a cube."""
    g = synth.dimerized_cube(3, seed=3)
    gp = pbit.load_instance(ctx, g)
    k = pbit.pbit_problem_colouring(ctx, gp)[1]
    cp = pbit.load_instance(ctx, synth.ea_instance(4, seed=1))
    pbit.pbit_profile_enable(ctx, 1)
    for kind in (pbit.PBIT_EA3D, pbit.PBIT_BICLIQUE, pbit.PBIT_GRAPH):
        pbit.pbit_profile_read(ctx, kind, reset=True)
    _say("profile windows: graph of %d groups, cube" % k)
    pbit.pbit_anneal(ctx, gp, synth.beta_linear(0.1, 1.0, 6), 16, seed=1)
    pbit.pbit_anneal(ctx, cp, synth.beta_linear(0.1, 1.0, 5), 16, seed=1)
    pbit.pbit_profile_enable(ctx, 0)
    ms_g, n_g = pbit.pbit_profile_read(ctx, pbit.PBIT_GRAPH, reset=True)
    ms_c, n_c = pbit.pbit_profile_read(ctx, pbit.PBIT_EA3D, reset=True)
    ms_b, n_b = pbit.pbit_profile_read(ctx, pbit.PBIT_BICLIQUE, reset=True)
    assert (n_g, n_c, n_b) == (6 * k, 10, 0)
    assert ms_g > 0 and ms_c > 0 and ms_b == 0
    pbit.pbit_unload_problem(ctx, gp)
    pbit.pbit_unload_problem(ctx, cp)


def test_caller_colouring_one_vertex_per_group(ctx):
    """Every vertex its own group: the sequential (Gibbs-order) sweep."""
    g = synth.random_sparse_graph(60, 5, seed=1)
    _every_sweep(ctx, g, synth.beta_linear(0.2, 2.0, 20), 9, seed=3, colour=np.arange(60, dtype=np.uint8),
                 n_colours=60)


def test_caller_colouring_with_an_empty_group(ctx):
    g = synth.ea_bond_list(synth.ea_instance((4, 4, 2), seed=2, field="uniform3"))
    i = np.arange(g["n"])
    col = (((i % 4) + (i // 4) % 4 + i // 16) % 2 * 2).astype(np.uint8)  # groups 0 and 2, group 1 empty
    _every_sweep(ctx, g, synth.beta_linear(0.2, 2.0, 15), 20, seed=4, colour=col, n_colours=3)


def test_even_cube_as_graph_equals_the_cube_path(ctx):
    inst = synth.ea_instance(8, seed=6, field="uniform3")
    g = synth.ea_bond_list(inst)
    pg = pbit.load_instance(ctx, g)
    pc = pbit.load_instance(ctx, inst)
    assert pbit.pbit_problem_colouring(ctx, pg)[1] == 2
    beta = synth.beta_linear(0.1, 3.0, 100)
    a = pbit.pbit_anneal(ctx, pg, beta, 64, seed=9)
    b = pbit.pbit_anneal(ctx, pc, beta, 64, seed=9)
    assert np.array_equal(a.spins, b.spins) and np.array_equal(a.energies, b.energies)
    pbit.pbit_unload_problem(ctx, pg)
    pbit.pbit_unload_problem(ctx, pc)


def test_fields_only_and_star_at_the_degree_limit(ctx):
    # no bonds at all: independent spins in their fields
    h = np.array([1, -1, 0, 1, 0, -1, 1, 1], np.int8)
    g = {"kind": "graph", "n": 8, "bond_i": np.zeros(0, np.int32), "bond_j": np.zeros(0, np.int32),
         "bond_J": np.zeros(0, np.int8), "h": h}
    _every_sweep(ctx, g, synth.beta_linear(0.1, 2.0, 10), 21, seed=1)
    # a hub with 127 ferromagnetic bonds and h = +1: |I| reaches 128
    k = 127
    g = {"kind": "graph", "n": k + 1, "bond_i": np.zeros(k, np.int32), "bond_j": np.arange(1, k + 1, dtype=np.int32),
         "bond_J": np.ones(k, np.int8), "h": np.ones(k + 1, np.int8)}
    _every_sweep(ctx, g, synth.beta_linear(0.01, 0.2, 12), 32, seed=2)


def test_graph_energy_and_resume(ctx):
    g = synth.random_sparse_graph(500, 8, seed=5)
    prob = pbit.load_instance(ctx, g)
    og = _oracle_graph(g)
    spins = synth.random_spins(37, 500, seed=3)
    assert np.array_equal(pbit.pbit_energy(ctx, prob, spins), oracle.energy(og, spins))
    beta = synth.beta_linear(0.1, 3.0, 40)
    full = pbit.pbit_anneal(ctx, prob, beta, 24, seed=3)
    a = pbit.pbit_anneal(ctx, prob, beta[:15], 24, seed=3)
    b = pbit.pbit_anneal(ctx, prob, beta[15:], 24, seed=3, sweep_offset=15, init_spins=a.spins)
    assert np.array_equal(full.spins, b.spins)
    part = pbit.pbit_anneal(ctx, prob, beta, 8, seed=3, replica_offset=12)
    assert np.array_equal(full.spins[12:20], part.spins)
    ref = oracle.anneal(og, beta, 24, seed=3)
    assert np.array_equal(full.spins, ref.spins) and np.array_equal(full.energies, ref.energies)
    pbit.pbit_unload_problem(ctx, prob)


def test_large_graph_sampled_replicas(ctx):
    """100k vertices of mean degree ~12, 512 replicas, 20 sweeps on the GPU;
    the oracle recomputes replica slices through replica_offset."""
    g = synth.random_sparse_graph(100_000, 12, seed=11)
    prob = pbit.load_instance(ctx, g)
    beta = synth.beta_linear(0.1, 2.0, 20)
    _say("graph n=100000 R=512 S=20")
    got = pbit.pbit_anneal(ctx, prob, beta, 512, seed=21)
    assert pbit.pbit_profile_graph_path(ctx) == 1  # 100k spins do not fit LDS
    og = _oracle_graph(g)
    for off in (0, 252, 508):
        ref = oracle.anneal(og, beta, 4, seed=21, replica_offset=off)
        assert np.array_equal(got.spins[off:off + 4], ref.spins), off
        assert np.array_equal(got.energies[off:off + 4], ref.energies), off
    pbit.pbit_unload_problem(ctx, prob)


def test_graph_errors(ctx):
    bi, bj = np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32)
    J = np.ones(3, np.int8)
    with pytest.raises(pbit.PbitError) as ei:  # improper: bond 0-1 inside group 0
        pbit.pbit_load_graph(ctx, 3, bi, bj, J, colour=np.array([0, 0, 1], np.uint8), n_colours=2)
    assert ei.value.code == pbit.PBIT_E_COLOURING
    with pytest.raises(pbit.PbitError) as ei:  # colour beyond n_colours
        pbit.pbit_load_graph(ctx, 3, bi, bj, J, colour=np.array([0, 1, 2], np.uint8), n_colours=2)
    assert ei.value.code == pbit.PBIT_E_COLOURING
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_load_graph(ctx, 3, bi, bj, np.array([1, 2, 1], np.int8))
    assert ei.value.code == pbit.PBIT_E_RANGE
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_load_graph(ctx, 3, bi, np.array([1, 3, 0], np.int32), J)
    assert ei.value.code == pbit.PBIT_E_ARG
    with pytest.raises(pbit.PbitError) as ei:  # 128 bonds on one vertex
        pbit.pbit_load_graph(ctx, 129, np.zeros(128, np.int32), np.arange(1, 129, dtype=np.int32),
                             np.ones(128, np.int8))
    assert ei.value.code == pbit.PBIT_E_UNSUPPORTED
    prob = pbit.pbit_load_graph(ctx, 3, bi, bj, J)
    assert pbit.pbit_problem_colouring(ctx, prob)[1] == 3
    pbit.pbit_unload_problem(ctx, prob)
    # a graph whose 4-replica tile does not fit the LDS is refused by the batched engine
    n = 41000
    ring_i = np.arange(n, dtype=np.int32)
    big = pbit.pbit_load_graph(ctx, n, ring_i, (ring_i + 1) % n, np.ones(n, np.int8))
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_anneal_batch(ctx, [dict(problem=big, beta=[1.0], n_replicas=4, seed=1)])
    assert ei.value.code == pbit.PBIT_E_UNSUPPORTED
    pbit.pbit_unload_problem(ctx, big)


def _batched_graphs():
    """Odd cubes (three or four groups), a dimerized cube (five groups), random
    graphs with zero couplings and fields, and a caller colouring."""
    rng = np.random.default_rng(12)
    jobs = []
    for k, (dims, R) in enumerate([((3, 3, 3), 5), ((5, 5, 5), 17), ((7, 5, 3), 40), ((3, 4, 6), 16)]):
        inst = synth.ea_instance(dims, seed=30 + k, field="uniform3")
        jobs.append(dict(g=_with_zeros(synth.ea_bond_list(inst), 0.15, seed=k), R=R, seed=70 + k,
                         beta=synth.beta_geometric(0.1, 5.0, int(rng.integers(8, 30)))))
    jobs.append(dict(g=synth.dimerized_cube(5, seed=5), R=33, seed=80, beta=synth.beta_geometric(0.1, 5.0, 25)))
    g = synth.random_sparse_graph(300, degree=7, seed=3)
    jobs.append(dict(g=_with_zeros(g, 0.2, seed=9), R=9, seed=81, beta=synth.beta_linear(0.1, 3.0, 20)))
    # a caller colouring: the greedy one with the colour ids reversed (groups swept in another order)
    g = synth.random_sparse_graph(120, degree=5, seed=4, field="zero")
    colour, nc = pbit.pbit_greedy_colouring(120, g["bond_i"], g["bond_j"])
    jobs.append(dict(g=g, R=64, seed=82, beta=synth.beta_linear(0.1, 3.0, 12),
                     colour=(nc - 1 - colour).astype(np.uint8), n_colours=nc))
    return jobs


def test_graphs_in_the_batched_tiles_match_the_oracle(ctx):
    jobs = _batched_graphs()
    probs = [pbit.pbit_load_graph(ctx, j["g"]["n"], j["g"]["bond_i"], j["g"]["bond_j"], j["g"]["bond_J"],
                                  j["g"].get("h"), j.get("colour"), j.get("n_colours", 0)) for j in jobs]
    # mixed with a cube and a biclique in the same call
    cube, bq = synth.ea_instance(6, seed=2), synth.biclique_instance(50, seed=2)
    pc, pq = pbit.load_instance(ctx, cube), pbit.load_instance(ctx, bq)
    beta = synth.beta_linear(0.1, 3.0, 15)
    _say("batched graphs: %d jobs with a cube and a biclique" % len(jobs))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
                                        for p, j in zip(probs, jobs)] +
                                  [dict(problem=pc, beta=beta, n_replicas=20, seed=3),
                                   dict(problem=pq, beta=beta, n_replicas=40, seed=4)])
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(_oracle_graph(j["g"], j.get("colour"), j.get("n_colours")), j["beta"], j["R"], j["seed"])
        assert np.array_equal(o.spins, ref.spins), j["g"]["n"]
        assert np.array_equal(o.energies, ref.energies), j["g"]["n"]
        assert o.sweeps_done == len(j["beta"])
        pbit.pbit_unload_problem(ctx, p)
    refc = oracle.anneal(oracle.ea_graph(cube["dims"], cube["J"], cube["h"]), beta, 20, 3)
    refq = oracle.anneal(oracle.biclique_graph(*bq["dims"], bq["J"], bq["h"]), beta, 40, 4)
    assert np.array_equal(outs[-2].spins, refc.spins) and np.array_equal(outs[-1].spins, refq.spins)
    pbit.pbit_unload_problem(ctx, pc)
    pbit.pbit_unload_problem(ctx, pq)


def test_graph_tiles_offsets_given_spins_traces_and_target(ctx):
    g = synth.dimerized_cube(4, seed=7)
    prob = pbit.load_instance(ctx, g)
    og = _oracle_graph(g)
    beta = synth.beta_linear(0.2, 3.0, 300)
    init = synth.random_spins(11, g["n"], seed=5)
    ref = oracle.anneal(og, beta, 11, 9, sweep_offset=7, replica_offset=12, init_spins=init, trace_every=50)
    out = pbit.pbit_anneal_batch(ctx, [dict(problem=prob, beta=beta, n_replicas=11, seed=9, sweep_offset=7,
                                             replica_offset=12, init_spins=init, trace_every=50)])[0]
    assert np.array_equal(out.spins, ref.spins) and np.array_equal(out.energy_trace, ref.energy_trace)
    # a target stops the job after the first checked sweep (every PBIT_CHECK_SWEEPS) that meets it
    full = oracle.anneal(og, beta, 16, 4, trace_every=pbit.PBIT_CHECK_SWEEPS)
    mins = full.energy_trace.min(axis=1)
    target = int(mins[1])
    first = (int(np.argmax(mins <= target)) + 1) * pbit.PBIT_CHECK_SWEEPS
    out = pbit.pbit_anneal_batch(ctx, [dict(problem=prob, beta=beta, n_replicas=16, seed=4, target=target)])[0]
    assert out.sweeps_done == first
    pre = oracle.anneal(og, beta[:first], 16, 4)
    assert np.array_equal(out.spins, pre.spins)
    pbit.pbit_unload_problem(ctx, prob)


def test_graph_job_served_alone_and_in_a_mix_is_the_same():
    jobs = _batched_graphs()[:5]
    with pbit.Context(0) as c:
        probs = [pbit.load_instance(c.ctx, dict(j["g"], kind="graph")) for j in jobs]
        pbit.pbit_serve_config(c.ctx, round_sweeps=5)
        res_alone, res_mix = {}, {}
        for k, (p, j) in enumerate(zip(probs, jobs)):
            jid = pbit.pbit_submit(c.ctx, p, j["beta"], j["R"], j["seed"])
            while (o := pbit.pbit_poll(c.ctx, jid, j["R"], j["g"]["n"], len(j["beta"]))) is None:
                pass
            res_alone[k] = o
        ids = {k: pbit.pbit_submit(c.ctx, p, j["beta"], j["R"], j["seed"]) for k, (p, j) in enumerate(zip(probs, jobs))}
        while ids:
            for k in list(ids):
                o = pbit.pbit_poll(c.ctx, ids[k], jobs[k]["R"], jobs[k]["g"]["n"], len(jobs[k]["beta"]))
                if o is not None:
                    res_mix[k] = o
                    del ids[k]
        for k, j in enumerate(jobs):
            ref = oracle.anneal(_oracle_graph(j["g"]), j["beta"], j["R"], j["seed"])
            assert np.array_equal(res_alone[k].spins, ref.spins)
            assert np.array_equal(res_mix[k].spins, ref.spins) and np.array_equal(res_mix[k].energies,
                                                                                   ref.energies)
