"""Every biclique half-sweep kernel the library can pick, forced through
PBIT_BQ_VARIANT and checked bit-exactly against the oracle, as the tuned
default is:

* 1: 64 x 64 tiles straight from global memory (any padding; the choice for
  sides below 512, forced here on large sides too);
* 2: 128 x 128 int8 tiles staged by the global-to-LDS DMA (sides padded to 128);
* 3: spins held as bits, widened to bytes for the int8 MFMA; the field is the
  site's field plus its coupling sum minus twice the product (sides padded to
  128; a forced bit kernel pads the replicas to 256), in tiles of 256, 128 or 64
  replicas (each forced through PBIT_BQ_BITS_RT too).  The batched engine's bit
  tiles run under this variant too;
* 4: sides of at most 512 sites held in LDS with their couplings (two-bit codes of
  J + 1 in both orientations) for runs of sweeps in one launch, 16 or 8 replicas
  per workgroup (each forced through PBIT_BQ_SLAB_RS), on the int8 MFMA 16 x 16 x 64.

Each kernel is checked on every replica after every sweep on ragged sides, on
sampled replicas at full size (n = 1024 and 4096, 1024 replicas), and at 128
replicas or fewer, where the tuner leaves the bit kernel out (its tiles hold
256 replicas)."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import pbit
from tests.test_parity_gpu import EXTREME_BETAS, HIGH_REPLICA, HIGH_SWEEP, _check_sampled, _every_sweep, graph_of

pytestmark = pytest.mark.gpu

_FORCED = {}  # context -> forced variant


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _forced_context(variant):
    old = os.environ.get("PBIT_BQ_VARIANT")
    os.environ["PBIT_BQ_VARIANT"] = variant
    try:
        c = pbit.Context(0)
        _FORCED[c.ctx.value] = int(variant)
    finally:
        if old is None:
            del os.environ["PBIT_BQ_VARIANT"]
        else:
            os.environ["PBIT_BQ_VARIANT"] = old
    return c


def _biclique_with_zeros(na, nb, seed, field="uniform3"):
    """Couplings in {-1, 0, +1}, about a third of them zero (the diluted form the
    problem statement allows), and fields in {-1, 0, +1} or none: the zero
    coupling, a code of its own in the two-bit forms, occurs only here."""
    inst = synth.biclique_instance(na, seed=seed, nb=nb, field=field)
    rng = np.random.default_rng(seed + 1)
    inst["J"] = (inst["J"] * (rng.random(inst["J"].shape) < 0.65)).astype(np.int8)
    assert (inst["J"] == 0).any() and (inst["J"] == 1).any() and (inst["J"] == -1).any()
    return inst


@pytest.fixture(scope="module", params=["1", "2", "3"], ids=["small", "int8dma", "bits"])
def vctx(request):
    """A context whose biclique kernels run the forced variant (read when the
    context is created)."""
    c = _forced_context(request.param)
    yield c.ctx
    c.close()


@pytest.fixture(scope="module")
def bits_ctx():
    c = _forced_context("3")
    yield c.ctx
    c.close()


@pytest.mark.parametrize("na,nb,R", [(600, 520, 200), (512, 1024, 130), (640, 512, 100), (520, 600, 3),
                                     (40, 40, 70)])
def test_variant_every_replica_every_sweep(vctx, na, nb, R):
    """Sides padded to 128 take the forced kernel; small sides keep the tuned one (the
    64 x 64 tile or the LDS-resident form)."""
    inst = synth.biclique_instance(na, seed=na + 3 * nb, nb=nb)
    _say("forced variant %d biclique %dx%d R=%d every sweep" % (_FORCED[vctx.value], na, nb, R))
    _every_sweep(vctx, inst, synth.beta_linear(0.05, 2.0, 8), R, seed=12)
    # the library reports the kernel that ran on large sides: the forced one
    if min(na, nb) >= 512:
        assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]
    else:
        assert pbit.pbit_profile_variant(vctx) in (1, 4)


@pytest.mark.parametrize("na,nb,R,field", [(600, 520, 70, "uniform3"), (512, 640, 40, "zero")])
def test_variant_zero_couplings_every_sweep(vctx, na, nb, R, field):
    """Diluted couplings through the forced kernel, with fields and without (h = NULL):
    every replica after every sweep."""
    inst = _biclique_with_zeros(na, nb, seed=na + 11 * nb + R, field=field)
    _say("forced variant %d diluted biclique %dx%d R=%d every sweep" % (_FORCED[vctx.value], na, nb, R))
    _every_sweep(vctx, inst, synth.beta_linear(0.05, 2.0, 8), R, seed=19)
    assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]


@pytest.mark.parametrize("sched", sorted(EXTREME_BETAS))
def test_variant_extreme_betas(vctx, sched):
    """beta = 0 only (threshold rows as wide as the largest field), large beta only
    (rows of two entries) and both interleaved, through the forced kernel."""
    inst = _biclique_with_zeros(520, 600, seed=77)
    _say("forced variant %d biclique 520x600 beta %s" % (_FORCED[vctx.value], sched))
    _every_sweep(vctx, inst, np.array(EXTREME_BETAS[sched]), 40, seed=43)
    assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]


def test_variant_given_spins_and_resume(vctx):
    """Given initial spins, and a run split in two (resumed from the first half's spins
    at its sweep offset), through the forced kernel."""
    inst = _biclique_with_zeros(520, 600, seed=81)
    R = 40
    beta = synth.beta_linear(0.05, 2.0, 8)
    _say("forced variant %d biclique 520x600 given spins and resume" % _FORCED[vctx.value])
    _every_sweep(vctx, inst, beta, R, seed=71, init=synth.random_spins(R, 1120, seed=6))
    prob = pbit.load_instance(vctx, inst)
    first = pbit.pbit_anneal(vctx, prob, beta[:3], R, seed=71)
    second = pbit.pbit_anneal(vctx, prob, beta[3:], R, seed=71, sweep_offset=3, init_spins=first.spins)
    assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]
    pbit.pbit_unload_problem(vctx, prob)
    whole = oracle.anneal(graph_of(inst), beta, R, seed=71)
    assert np.array_equal(second.spins, whole.spins) and np.array_equal(second.energies, whole.energies)


def test_variant_counters_past_31_bits(vctx):
    """Sweep and replica counters near the top of their 32-bit range through the forced
    kernel."""
    inst = _biclique_with_zeros(520, 600, seed=79)
    _say("forced variant %d biclique 520x600 counters past 31 bits" % _FORCED[vctx.value])
    _every_sweep(vctx, inst, synth.beta_linear(0.05, 2.0, 6), 40, seed=59, sweep_offset=HIGH_SWEEP,
                 replica_offset=HIGH_REPLICA)
    assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]


@pytest.mark.parametrize("n,R,prefixes", [(1024, 1024, [1, 2, 10]), (4096, 1024, [1, 2]), (1024, 128, [1, 2, 10]),
                                          (2048, 96, [1, 3]), (2048, 1024, [1, 2])])
def test_variant_full_size_sampled(vctx, n, R, prefixes):
    """K_{n,n}, beta linear 0.05 -> 2.0 over 2000 sweeps."""
    inst = synth.biclique_instance(n, seed=n)
    beta = synth.beta_linear(0.05, 2.0, 2000)
    _say("forced variant %d K_%d R=%d sampled" % (_FORCED[vctx.value], n, R))
    _check_sampled(vctx, inst, beta, R, 1, prefixes, [0], np.random.default_rng(n + R))
    assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]


@pytest.fixture(scope="module", params=["64", "128", "256"], ids=["rt64", "rt128", "rt256"])
def rt_ctx(request):
    """The bit kernel forced, with its replica tile forced too (PBIT_BQ_BITS_RT)."""
    old = os.environ.get("PBIT_BQ_BITS_RT")
    os.environ["PBIT_BQ_BITS_RT"] = request.param
    try:
        c = _forced_context("3")
    finally:
        if old is None:
            del os.environ["PBIT_BQ_BITS_RT"]
        else:
            os.environ["PBIT_BQ_BITS_RT"] = old
    yield c.ctx, int(request.param)
    c.close()


@pytest.mark.parametrize("na,nb,R", [(600, 520, 200), (512, 1024, 300), (640, 512, 70), (768, 896, 300)])
def test_bit_tile_widths_every_replica_every_sweep(rt_ctx, na, nb, R):
    """The bit kernel in each of its replica tiles (256 replicas on eight waves, 128 on
    four, 64 on two), with stages of 256 K where a side is a multiple of 256 and 128
    elsewhere, several replica tiles per launch: every replica after every sweep."""
    ctx, rt = rt_ctx
    inst = synth.biclique_instance(na, seed=na + 7 * nb + R, nb=nb)
    _say("bit kernel, %d-replica tiles, biclique %dx%d R=%d every sweep" % (rt, na, nb, R))
    _every_sweep(ctx, inst, synth.beta_linear(0.05, 2.0, 6), R, seed=23)
    assert pbit.pbit_profile_variant(ctx) == 3


@pytest.mark.parametrize("na,nb,R", [(512, 512, 128), (640, 768, 100), (1024, 1024, 64)])
def test_tuned_choice_without_the_bit_kernel(na, nb, R):
    """At 128 replicas or fewer the tuner leaves the bit kernel out (and times the
    LDS-resident form where the sides are at most 512); whichever it keeps is
    bit-exact every sweep."""
    with pbit.Context(0) as c:
        inst = synth.biclique_instance(na, seed=na + nb + R, nb=nb)
        _say("tuned biclique %dx%d R=%d every sweep" % (na, nb, R))
        _every_sweep(c.ctx, inst, synth.beta_linear(0.05, 2.0, 6), R, seed=31)
        assert pbit.pbit_profile_variant(c.ctx) in ((1, 2, 4) if max(na, nb) <= 512 else (1, 2))


def test_bit_tiles_batched_match_oracle(bits_ctx):
    """Bicliques with ragged sides and replica counts in 32-, 64- and
    128-replica bit tiles, started from random and from given spins."""
    rng = np.random.default_rng(4)
    jobs = []
    for k, (na, nb, R) in enumerate([(20, 20, 5), (7, 130, 33), (64, 64, 70), (100, 37, 130), (130, 129, 64),
                                     (260, 200, 129)]):
        inst = synth.biclique_instance(na, seed=40 + k, nb=nb)
        init = synth.random_spins(R, na + nb, seed=k) if k % 2 else None
        jobs.append(dict(inst=inst, beta=synth.beta_linear(0.05, 2.0, int(rng.integers(3, 20))), R=R,
                         seed=400 + k, init=init))
    probs = [pbit.load_instance(bits_ctx, j["inst"]) for j in jobs]
    _say("bit tiles: batch of %d bicliques" % len(jobs))
    descs = []
    for p, j in zip(probs, jobs):
        d = dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
        if j["init"] is not None:
            d["init_spins"] = j["init"]
        descs.append(d)
    outs = pbit.pbit_anneal_batch(bits_ctx, descs)
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"], init_spins=j["init"])
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        pbit.pbit_unload_problem(bits_ctx, p)


def test_bit_tiles_and_default_tiles_agree(bits_ctx):
    """A slice of the mixed bag through the bit tiles and the default int8 tiles:
    identical results."""
    bag = [j for j in synth.mixed_bag(seed=5, n_instances=16, replica_range=(32, 200), sweep_range=(40, 120))
           if j["instance"]["kind"] == "biclique"]
    assert bag
    with pbit.Context(0) as c8:
        outs8 = []
        for j in bag:
            p = pbit.load_instance(c8.ctx, j["instance"])
            outs8.append(pbit.pbit_anneal_batch(c8.ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"],
                                                               seed=j["seed"])])[0])
            pbit.pbit_unload_problem(c8.ctx, p)
    probs = [pbit.load_instance(bits_ctx, j["instance"]) for j in bag]
    _say("bit tiles vs default on %d bag bicliques" % len(bag))
    outs_v = pbit.pbit_anneal_batch(bits_ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"],
                                                    seed=j["seed"]) for p, j in zip(probs, bag)])
    for j, a, b in zip(bag, outs_v, outs8):
        assert np.array_equal(a.spins, b.spins), j["instance"]["dims"]
        assert np.array_equal(a.energies, b.energies)
    for p in probs:
        pbit.pbit_unload_problem(bits_ctx, p)


@pytest.fixture(scope="module", params=["16", "8"], ids=["rs16", "rs8"])
def slab_ctx(request):
    """The LDS-resident kernel forced, in slices of 16 replicas (the MFMA's 16 rows) or
    of 8 (two site blocks' rows merged in one epilogue), forced through PBIT_BQ_SLAB_RS."""
    old = os.environ.get("PBIT_BQ_SLAB_RS")
    os.environ["PBIT_BQ_SLAB_RS"] = request.param
    try:
        c = _forced_context("4")
    finally:
        if old is None:
            del os.environ["PBIT_BQ_SLAB_RS"]
        else:
            os.environ["PBIT_BQ_SLAB_RS"] = old
    yield c.ctx
    c.close()


@pytest.mark.parametrize("na,nb,R", [(40, 40, 70), (130, 70, 33), (512, 512, 130), (300, 500, 17), (64, 448, 5),
                                     (7, 130, 129), (600, 40, 20)])
def test_slab_every_replica_every_sweep(slab_ctx, na, nb, R):
    """The LDS-resident form on ragged sides with fields, every replica after every
    sweep (one launch per sweep here, as the trace asks for energies after each);
    sides beyond 512 fall back to the tuned kernel."""
    inst = synth.biclique_instance(na, seed=na + 5 * nb + R, nb=nb)
    _say("slab biclique %dx%d R=%d every sweep" % (na, nb, R))
    _every_sweep(slab_ctx, inst, synth.beta_linear(0.05, 2.0, 10), R, seed=17)
    assert (pbit.pbit_profile_variant(slab_ctx) == 4) == (max(na, nb) <= 512)


@pytest.mark.parametrize("na,nb,R,field", [(300, 200, 40, "uniform3"), (512, 512, 33, "uniform3"),
                                           (70, 130, 17, "zero")])
def test_slab_zero_couplings_every_sweep(slab_ctx, na, nb, R, field):
    """Diluted couplings (code 1 of the two-bit codes) in the LDS-resident form, with
    fields and without."""
    inst = _biclique_with_zeros(na, nb, seed=na + 13 * nb + R, field=field)
    _say("slab diluted biclique %dx%d R=%d every sweep" % (na, nb, R))
    _every_sweep(slab_ctx, inst, synth.beta_linear(0.05, 2.0, 10), R, seed=29)
    assert pbit.pbit_profile_variant(slab_ctx) == 4


@pytest.mark.parametrize("sched", sorted(EXTREME_BETAS))
def test_slab_extreme_betas(slab_ctx, sched):
    """The LDS-resident form at the ends of the schedule range (its decision words are
    built from each sweep's threshold row in LDS)."""
    inst = _biclique_with_zeros(130, 70, seed=78)
    _say("slab biclique 130x70 beta %s" % sched)
    _every_sweep(slab_ctx, inst, np.array(EXTREME_BETAS[sched]), 21, seed=47)
    assert pbit.pbit_profile_variant(slab_ctx) == 4


def test_slab_counters_past_31_bits(slab_ctx):
    """The LDS-resident form (runs of sweeps in one launch) with its counters past 31 bits."""
    inst = _biclique_with_zeros(130, 70, seed=80)
    _say("slab biclique 130x70 counters past 31 bits")
    _every_sweep(slab_ctx, inst, synth.beta_linear(0.05, 2.0, 6), 21, seed=61, sweep_offset=HIGH_SWEEP,
                 replica_offset=HIGH_REPLICA)
    assert pbit.pbit_profile_variant(slab_ctx) == 4


@pytest.mark.parametrize("mode", ["3", None], ids=["bit_tiles", "int8_tiles"])
def test_batched_tiles_zero_couplings(mode):
    """Diluted bicliques through the batched tiles, with the spins as bits (forced) and
    as int8 rows with two-bit coupling codes (default): every job equals the oracle."""
    c = _forced_context(mode) if mode else pbit.Context(0)
    try:
        jobs = []
        for k, (na, nb, R) in enumerate([(40, 40, 9), (130, 70, 33), (200, 260, 64), (520, 300, 40)]):
            inst = _biclique_with_zeros(na, nb, seed=60 + k, field="zero" if k == 1 else "uniform3")
            jobs.append(dict(inst=inst, beta=synth.beta_linear(0.05, 2.0, 12 + k), R=R, seed=500 + k))
        probs = [pbit.load_instance(c.ctx, j["inst"]) for j in jobs]
        _say("batched tiles (%s), %d diluted bicliques" % ("bits" if mode else "int8", len(jobs)))
        outs = pbit.pbit_anneal_batch(c.ctx, [dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
                                              for p, j in zip(probs, jobs)])
        for p, j, o in zip(probs, jobs, outs):
            ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"])
            assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
            assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
            pbit.pbit_unload_problem(c.ctx, p)
    finally:
        c.close()


@pytest.mark.parametrize("n,R,prefixes", [(512, 1024, [1, 2, 10, 1500]), (256, 96, [3, 1200]), (448, 2000, [2, 40])])
def test_slab_runs_of_sweeps_sampled(slab_ctx, n, R, prefixes):
    """K_{n,n}, beta linear 0.05 -> 2.0 over 2000 sweeps: runs of up to 1000 sweeps per
    launch (1500 and 1200 take two launches), sampled replica groups against the oracle."""
    inst = synth.biclique_instance(n, seed=n + R)
    beta = synth.beta_linear(0.05, 2.0, 2000)
    _say("slab K_%d R=%d sampled" % (n, R))
    _check_sampled(slab_ctx, inst, beta, R, 1, prefixes, [0, R // 4 - 1], np.random.default_rng(n))
    assert pbit.pbit_profile_variant(slab_ctx) == 4


def test_slab_offsets_resume_and_given_spins(slab_ctx):
    """Replica slices, a split run resumed from its spins, and given initial spins on
    the LDS-resident form equal the oracle."""
    inst = synth.biclique_instance(200, seed=8, nb=136)
    g = graph_of(inst)
    beta = synth.beta_linear(0.1, 2.5, 60)
    prob = pbit.load_instance(slab_ctx, inst)
    full = pbit.pbit_anneal(slab_ctx, prob, beta, 40, seed=5)
    assert pbit.pbit_profile_variant(slab_ctx) == 4
    ref = oracle.anneal(g, beta, 40, seed=5)
    assert np.array_equal(full.spins, ref.spins) and np.array_equal(full.energies, ref.energies)
    a = pbit.pbit_anneal(slab_ctx, prob, beta[:23], 40, seed=5)
    b = pbit.pbit_anneal(slab_ctx, prob, beta[23:], 40, seed=5, sweep_offset=23, init_spins=a.spins)
    assert np.array_equal(b.spins, full.spins)
    part = pbit.pbit_anneal(slab_ctx, prob, beta, 12, seed=5, replica_offset=16)
    assert np.array_equal(part.spins, full.spins[16:28])
    init = synth.random_spins(40, 336, seed=3)
    got = pbit.pbit_anneal(slab_ctx, prob, beta, 40, seed=9, init_spins=init)
    ref = oracle.anneal(g, beta, 40, seed=9, init_spins=init)
    assert np.array_equal(got.spins, ref.spins)
    pbit.pbit_unload_problem(slab_ctx, prob)
