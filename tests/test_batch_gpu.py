"""Batched persistent kernels and the serving scheduler: every job's result is
bit-exact against the oracle (or against the same job run alone through
pbit_anneal), whatever it is batched with, in whatever order jobs arrive, and
under a device budget that forces queued admission."""
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


def _small_mix(seed=0):
    """Cubes and bicliques with ragged replica counts, fields and zero couplings."""
    rng = np.random.default_rng(seed)
    jobs = []
    for k, dims in enumerate([(4, 4, 4), (6, 4, 2), (8, 8, 8), (2, 2, 2), (10, 6, 4)]):
        inst = synth.ea_instance(dims, seed=10 + k, field="uniform3")
        inst["J"] = (inst["J"] * (rng.random(inst["J"].shape) < 0.9)).astype(np.int8)
        jobs.append(dict(inst=inst, beta=synth.beta_geometric(0.1, 5.0, int(rng.integers(5, 40))),
                         R=int(rng.integers(1, 23)), seed=100 + k))
    for k, (na, nb) in enumerate([(20, 20), (7, 130), (64, 64), (100, 37), (130, 129)]):
        inst = synth.biclique_instance(na, seed=20 + k, nb=nb)
        jobs.append(dict(inst=inst, beta=synth.beta_linear(0.05, 2.0, int(rng.integers(3, 20))),
                         R=int(rng.choice([5, 33, 64, 70, 130])), seed=200 + k))
    return jobs


def test_batch_matches_oracle(ctx):
    jobs = _small_mix()
    probs = [pbit.load_instance(ctx, j["inst"]) for j in jobs]
    _say("batch of %d small jobs" % len(jobs))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
                                        for p, j in zip(probs, jobs)])
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"])
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        assert o.sweeps_done == len(j["beta"])
        pbit.pbit_unload_problem(ctx, p)


@pytest.mark.parametrize("sched", ["zero", "cold", "mixed"])
def test_batch_extreme_betas(ctx, sched):
    """The small mix at the ends of the schedule range (beta = 0 only, large beta only,
    both interleaved): each tile kind builds its decision words from rows of every
    width."""
    from tests.test_parity_gpu import EXTREME_BETAS
    beta = np.array(EXTREME_BETAS[sched])
    jobs = _small_mix(seed=3)
    probs = [pbit.load_instance(ctx, j["inst"]) for j in jobs]
    _say("batch of %d small jobs, beta %s" % (len(jobs), sched))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=beta, n_replicas=j["R"], seed=j["seed"])
                                        for p, j in zip(probs, jobs)])
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), beta, j["R"], j["seed"])
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        pbit.pbit_unload_problem(ctx, p)


def test_batch_counters_past_31_bits(ctx):
    """The small mix with sweep and replica counters near the top of their 32-bit range
    (the absolute sweep index crosses 2^31 during the run)."""
    from tests.test_parity_gpu import HIGH_REPLICA, HIGH_SWEEP
    jobs = _small_mix(seed=4)
    probs = [pbit.load_instance(ctx, j["inst"]) for j in jobs]
    _say("batch of %d small jobs, counters past 31 bits" % len(jobs))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"],
                                             sweep_offset=HIGH_SWEEP - 2, replica_offset=HIGH_REPLICA)
                                        for p, j in zip(probs, jobs)])
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"], sweep_offset=HIGH_SWEEP - 2,
                            replica_offset=HIGH_REPLICA)
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        pbit.pbit_unload_problem(ctx, p)


def _oracle_groups(inst, beta, R, seed, got, groups):
    """Replica groups of a result against the oracle run on those replicas alone
    (replica_offset): the counters use the global replica index, so a slice of
    four replicas equals the same rows of the whole run."""
    g = graph_of(inst)
    for gi in groups:
        cnt = min(4, R - 4 * gi)
        ref = oracle.anneal(g, beta, cnt, seed, replica_offset=4 * gi)
        assert np.array_equal(got.spins[4 * gi:4 * gi + cnt], ref.spins), (inst["dims"], gi)
        assert np.array_equal(got.energies[4 * gi:4 * gi + cnt], ref.energies), (inst["dims"], gi)


def test_batch_equals_single_runs_at_mixed_bag_sizes(ctx):
    """A slice of the mixed bag (cubes L in 8..24, bicliques n in 64..1024,
    uneven replica and sweep counts), shortened to 60..200 sweeps: each job's
    batched result equals the same job through the per-instance path, and its
    first and last replica groups equal the oracle."""
    bag = synth.mixed_bag(seed=3, n_instances=12, replica_range=(32, 200), sweep_range=(60, 200))
    probs = [pbit.load_instance(ctx, j["instance"]) for j in bag]
    _say("mixed-bag slice of %d jobs" % len(bag))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"], seed=j["seed"])
                                        for p, j in zip(probs, bag)])
    for p, j, o in zip(probs, bag, outs):
        single = pbit.pbit_anneal(ctx, p, j["beta"], j["replicas"], j["seed"])
        assert np.array_equal(o.spins, single.spins), j["instance"]["dims"]
        assert np.array_equal(o.energies, single.energies)
        R = j["replicas"]
        _oracle_groups(j["instance"], j["beta"], R, j["seed"], o, sorted({0, (R - 1) // 4}))
        pbit.pbit_unload_problem(ctx, p)


def test_batch_cube_tile_widths(ctx):
    """Cube jobs of every tile width: 16-replica tiles (lattices up to 8192 sites
    with at least 16 replicas), 8-replica tiles (where 16 do not fit the LDS or the
    job has 8..15 replicas) and 4-replica tiles, each with a ragged last tile, dense
    and diluted couplings, with and without fields, and non-cubic sides; tiles of more
    and of less than 80 KiB of LDS rows (two cube launches of a round, 1024 and 512
    threads per workgroup) in one call: batched results equal the per-instance path,
    and the first replica group and the ragged last one equal the oracle."""
    rng = np.random.default_rng(7)
    cases = [((20, 20, 20), 20, "zero", 1.0), ((22, 22, 22), 12, "uniform3", 0.9), ((24, 24, 24), 8, "zero", 1.0),
             ((20, 22, 16), 17, "uniform3", 1.0), ((6, 6, 6), 16, "zero", 0.8), ((20, 20, 20), 5, "uniform3", 0.9),
             ((2, 2, 2), 33, "uniform3", 1.0), ((26, 26, 26), 9, "zero", 1.0), ((28, 28, 28), 16, "zero", 1.0),
             ((32, 32, 32), 6, "uniform3", 0.9)]
    jobs = []
    for k, (dims, R, field, keep) in enumerate(cases):
        inst = synth.ea_instance(dims, seed=40 + k, field=field)
        if keep < 1.0:
            inst["J"] = (inst["J"] * (rng.random(inst["J"].shape) < keep)).astype(np.int8)
        jobs.append(dict(inst=inst, R=R, seed=300 + k, beta=synth.beta_geometric(0.2, 3.0, int(rng.integers(20, 45)))))
    probs = [pbit.load_instance(ctx, j["inst"]) for j in jobs]
    _say("cube tile widths: %d jobs" % len(jobs))
    outs = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
                                        for p, j in zip(probs, jobs)])
    for p, j, o in zip(probs, jobs, outs):
        single = pbit.pbit_anneal(ctx, p, j["beta"], j["R"], j["seed"])
        assert np.array_equal(o.spins, single.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, single.energies), j["inst"]["dims"]
        assert o.sweeps_done == len(j["beta"])
        _oracle_groups(j["inst"], j["beta"], j["R"], j["seed"], o, sorted({0, (j["R"] - 1) // 4}))
        pbit.pbit_unload_problem(ctx, p)


def test_batch_given_spins_offsets_and_traces(ctx):
    inst = synth.ea_instance(6, seed=8, field="uniform3")
    binst = synth.biclique_instance(40, seed=8)
    p1, p2 = pbit.load_instance(ctx, inst), pbit.load_instance(ctx, binst)
    init1 = synth.random_spins(9, 216, seed=1)
    init2 = synth.random_spins(66, 80, seed=2)
    beta = synth.beta_linear(0.2, 2.5, 250)
    outs = pbit.pbit_anneal_batch(ctx, [
        dict(problem=p1, beta=beta, n_replicas=9, seed=5, sweep_offset=17, replica_offset=8, init_spins=init1,
             trace_every=50),
        dict(problem=p2, beta=beta, n_replicas=66, seed=6, sweep_offset=3, replica_offset=4, init_spins=init2,
             trace_every=125)])
    r1 = oracle.anneal(graph_of(inst), beta, 9, 5, sweep_offset=17, replica_offset=8, init_spins=init1, trace_every=50)
    r2 = oracle.anneal(graph_of(binst), beta, 66, 6, sweep_offset=3, replica_offset=4, init_spins=init2,
                       trace_every=125)
    assert np.array_equal(outs[0].spins, r1.spins) and np.array_equal(outs[0].energy_trace, r1.energy_trace)
    assert np.array_equal(outs[1].spins, r2.spins) and np.array_equal(outs[1].energy_trace, r2.energy_trace)
    pbit.pbit_unload_problem(ctx, p1)
    pbit.pbit_unload_problem(ctx, p2)


def test_batch_target_stops_at_first_checked_sweep(ctx):
    inst = synth.ea_instance(8, seed=21)
    beta = synth.beta_linear(0.1, 3.0, 1000)
    R = 12
    ref = oracle.anneal(graph_of(inst), beta, R, 4, trace_every=pbit.PBIT_CHECK_SWEEPS)
    mins = ref.energy_trace.min(axis=1)
    target = int(mins[4])
    first = (int(np.argmax(mins <= target)) + 1) * pbit.PBIT_CHECK_SWEEPS
    p = pbit.load_instance(ctx, inst)
    out = pbit.pbit_anneal_batch(ctx, [dict(problem=p, beta=beta, n_replicas=R, seed=4, target=target)])[0]
    assert out.sweeps_done == first
    pre = oracle.anneal(graph_of(inst), beta[:first], R, 4)
    assert np.array_equal(out.spins, pre.spins) and np.array_equal(out.energies, pre.energies)
    pbit.pbit_unload_problem(ctx, p)


def _serve_all(c, arrivals, budget_jobs=None):
    """Submit jobs in arrival waves, driving the scheduler between waves, and
    collect every result."""
    ids = {}
    results = {}
    for wave in arrivals:
        for key, (prob, j) in wave:
            ids[key] = (pbit.pbit_submit(c, prob, j["beta"], j["R"], j["seed"], target=j.get("target")), j)
        pbit.pbit_progress(c)
    pending = dict(ids)
    spins_n = {}
    while pending:
        for key in list(pending):
            jid, j = pending[key]
            out = pbit.pbit_poll(c, jid, j["R"], j["N"], len(j["beta"]))
            if out is not None:
                results[key] = out
                del pending[key]
    return results


def test_serving_results_are_the_same_alone_and_in_the_mix():
    jobs = _small_mix(seed=5)
    with pbit.Context(0) as c:
        probs = [pbit.load_instance(c.ctx, j["inst"]) for j in jobs]
        for p, j in zip(probs, jobs):
            j["N"] = pbit.pbit_problem_spins(c.ctx, p)
        pbit.pbit_serve_config(c.ctx, round_sweeps=7)  # short rounds: later jobs join running ones
        alone = {}
        for k, (p, j) in enumerate(zip(probs, jobs)):
            alone.update(_serve_all(c.ctx, [[(k, (p, j))]]))
        _say("serving: %d jobs alone done" % len(jobs))
        waves = [[(k, (probs[k], jobs[k])) for k in range(0, 4)],
                 [(k, (probs[k], jobs[k])) for k in range(4, 7)],
                 [(k, (probs[k], jobs[k])) for k in range(7, len(jobs))]]
        mixed = _serve_all(c.ctx, waves)
        for k, j in enumerate(jobs):
            ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"])
            assert np.array_equal(alone[k].spins, ref.spins)
            assert np.array_equal(mixed[k].spins, alone[k].spins)
            assert np.array_equal(mixed[k].energies, alone[k].energies)


def test_serving_admits_by_budget_and_keeps_results():
    jobs = _small_mix(seed=9)
    # enough for the problems and one or two jobs at a time
    with pbit.Context(0, hbm_budget_bytes=3_000_000) as c:
        probs = [pbit.load_instance(c.ctx, j["inst"]) for j in jobs]
        for p, j in zip(probs, jobs):
            j["N"] = pbit.pbit_problem_spins(c.ctx, p)
        pbit.pbit_serve_config(c.ctx, round_sweeps=5)
        res = _serve_all(c.ctx, [[(k, (p, j)) for k, (p, j) in enumerate(zip(probs, jobs))]])
        assert pbit.pbit_bytes_in_use(c.ctx) <= 3_000_000
        for k, j in enumerate(jobs):
            ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"])
            assert np.array_equal(res[k].spins, ref.spins)


def test_serving_errors(ctx):
    inst = synth.ea_instance(4, seed=1)
    p = pbit.load_instance(ctx, inst)
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_poll(ctx, 12345, 4, 64)
    assert ei.value.code == pbit.PBIT_E_HANDLE
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_submit(ctx, p, [np.nan], 4, 1)
    assert ei.value.code == pbit.PBIT_E_RANGE
    jid = pbit.pbit_submit(ctx, p, synth.beta_linear(0.1, 1.0, 30), 4, 1)
    with pytest.raises(pbit.PbitError) as ei:
        pbit.pbit_unload_problem(ctx, p)  # a queued job still holds the problem
    assert ei.value.code == pbit.PBIT_E_BUSY
    while pbit.pbit_poll(ctx, jid, 4, 64, 30) is None:
        pass
    pbit.pbit_unload_problem(ctx, p)
    with pbit.Context(0, hbm_budget_bytes=400_000) as c2:
        big = pbit.load_instance(c2.ctx, synth.ea_instance(16, seed=1))
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_submit(c2.ctx, big, synth.beta_linear(0.1, 1.0, 10), 256, 1)
        assert ei.value.code == pbit.PBIT_E_NOMEM
        pbit.pbit_serve_config(c2.ctx, max_queue=1, max_running=1)
        small = pbit.load_instance(c2.ctx, synth.ea_instance(2, seed=1))
        # a runs (4 rounds of 500 sweeps), b waits in the queue, c finds it full
        a = pbit.pbit_submit(c2.ctx, small, synth.beta_linear(0.1, 1.0, 2000), 4, 1)
        b = pbit.pbit_submit(c2.ctx, small, synth.beta_linear(0.1, 1.0, 2000), 4, 2)
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_submit(c2.ctx, small, synth.beta_linear(0.1, 1.0, 10), 4, 3)
        assert ei.value.code == pbit.PBIT_E_BUSY
        for jid in (a, b):
            while pbit.pbit_poll(c2.ctx, jid, 4, 8, 2000) is None:
                pass


def test_job_that_cannot_fit_fails_instead_of_waiting():
    """Under a budget that is tight after loading problems and running one
    pbit_anneal (whose scratch the context keeps), a job that fits the budget by
    itself but not beside what is already held fails with E_NOMEM, in a batch
    call and through submit/poll, instead of waiting for ever; the context keeps
    working afterwards."""
    budget = 3_000_000
    with pbit.Context(0, hbm_budget_bytes=budget) as c:
        inst = synth.ea_instance(20, seed=3)  # 8000 sites
        p = pbit.load_instance(c.ctx, inst)
        pbit.pbit_anneal(c.ctx, p, synth.beta_linear(0.1, 1.0, 3), 128, seed=1)  # ~2 MB of kept scratch
        held = pbit.pbit_bytes_in_use(c.ctx)
        R = 128  # 16-replica tiles: 8 x 128,000 bytes of tile state
        assert held + 8000 * R > budget and 8000 * R + 200_000 < budget, held
        beta = synth.beta_linear(0.1, 1.0, 20)
        _say("budget stall: %d bytes held of %d" % (held, budget))
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_anneal_batch(c.ctx, [dict(problem=p, beta=beta, n_replicas=R, seed=2)])
        assert ei.value.code == pbit.PBIT_E_NOMEM
        jid = pbit.pbit_submit(c.ctx, p, beta, R, 2)
        with pytest.raises(pbit.PbitError) as ei:
            for _ in range(10_000):
                if pbit.pbit_poll(c.ctx, jid, R, 8000, len(beta)) is not None:
                    break
        assert ei.value.code == pbit.PBIT_E_NOMEM
        with pytest.raises(pbit.PbitError) as ei:
            pbit.pbit_poll(c.ctx, jid, R, 8000, len(beta))  # the failed job is retired
        assert ei.value.code == pbit.PBIT_E_HANDLE
        # a job that fits still runs, bit-exact, and the problem can be unloaded
        out = pbit.pbit_anneal_batch(c.ctx, [dict(problem=p, beta=beta, n_replicas=16, seed=2)])[0]
        ref = oracle.anneal(graph_of(inst), beta, 4, 2)
        assert np.array_equal(out.spins[:4], ref.spins)
        pbit.pbit_unload_problem(c.ctx, p)


def test_tuned_and_fixed_tile_sizes_give_the_same_results():
    """The tile autotuner times the tile sizes a job's shape can take and caches
    the choice; whatever it picks, every job equals the fixed rule's result (and
    the oracle on sampled replicas), and a second batch of the same shapes
    reuses the cache."""
    import os

    bag = synth.mixed_bag(seed=8, n_instances=10, replica_range=(20, 300), sweep_range=(20, 60))
    old = os.environ.get("PBIT_TILE_TUNE")
    os.environ["PBIT_TILE_TUNE"] = "0"
    try:
        fixed = pbit.Context(0)
    finally:
        if old is None:
            del os.environ["PBIT_TILE_TUNE"]
        else:
            os.environ["PBIT_TILE_TUNE"] = old
    tuned = pbit.Context(0)
    try:
        outs = {}
        for name, c in (("fixed", fixed), ("tuned", tuned)):
            probs = [pbit.load_instance(c.ctx, j["instance"]) for j in bag]
            _say("tile sizes: %s" % name)
            outs[name] = pbit.pbit_anneal_batch(c.ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"],
                                                             seed=j["seed"]) for p, j in zip(probs, bag)])
            if name == "tuned":
                tunings, shapes = pbit.pbit_profile_tiles(c.ctx)
                assert tunings >= 1 and shapes == tunings
                again = pbit.pbit_anneal_batch(c.ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"],
                                                            seed=j["seed"]) for p, j in zip(probs, bag)])
                assert pbit.pbit_profile_tiles(c.ctx) == (tunings, shapes)
                for a, b in zip(again, outs[name]):
                    assert np.array_equal(a.spins, b.spins)
            else:
                assert pbit.pbit_profile_tiles(c.ctx) == (0, 0)
            for p in probs:
                pbit.pbit_unload_problem(c.ctx, p)
        for j, a, b in zip(bag, outs["fixed"], outs["tuned"]):
            assert np.array_equal(a.spins, b.spins), j["instance"]["dims"]
            assert np.array_equal(a.energies, b.energies)
        j = bag[0]
        _oracle_groups(j["instance"], j["beta"], j["replicas"], j["seed"], outs["tuned"][0], [0])
    finally:
        fixed.close()
        tuned.close()
