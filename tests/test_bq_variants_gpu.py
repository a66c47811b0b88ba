"""Biclique kernel variants forced through PBIT_BQ_VARIANT, each bit-exact
against the oracle like the tuned default:

* 7: packed 4-bit float operands, per instance and in the batched tiles.  Every
  spin, coupling and field value is -1, 0 or +1 and every partial sum an
  integer far below 2^24, so the fp4 products with fp32 sums give the same
  fields as int8 products with int32 sums.
* 8: spins held as bits, widened to bytes for the int8 MFMA; the field is the
  site's field plus its coupling sum minus twice the product, per instance and
  in the batched tiles.
* 6: the int8 DMA tile per instance (the batched tiles keep their default int8
  rows)."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import pbit
from tests.test_parity_gpu import _check_sampled, _every_sweep, graph_of

pytestmark = pytest.mark.gpu

_FORCED = {}  # context -> forced variant


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["6", "7", "8"], ids=["int8dma", "fp4", "bits"])
def vctx(request):
    """A context whose biclique kernels run the forced variant (read when the
    context is created)."""
    old = os.environ.get("PBIT_BQ_VARIANT")
    os.environ["PBIT_BQ_VARIANT"] = request.param
    try:
        c = pbit.Context(0)
        _FORCED[c.ctx.value] = int(request.param)
    finally:
        if old is None:
            del os.environ["PBIT_BQ_VARIANT"]
        else:
            os.environ["PBIT_BQ_VARIANT"] = old
    yield c.ctx
    c.close()


@pytest.mark.parametrize("na,nb,R", [(600, 520, 200), (512, 1024, 130), (40, 40, 70)])
def test_variant_every_replica_every_sweep(vctx, na, nb, R):
    """Sides padded to 128 take the forced kernel; small sides keep the tuned one."""
    inst = synth.biclique_instance(na, seed=na + 3 * nb, nb=nb)
    _say("forced variant biclique %dx%d R=%d every sweep" % (na, nb, R))
    _every_sweep(vctx, inst, synth.beta_linear(0.05, 2.0, 8), R, seed=12)
    # the library reports the kernel that ran on large sides: the forced one
    if min(na, nb) >= 512:
        assert pbit.pbit_profile_variant(vctx) == _FORCED[vctx.value]


@pytest.mark.parametrize("n,prefixes", [(1024, [1, 2, 10]), (4096, [1, 2])])
def test_variant_full_size_sampled(vctx, n, prefixes):
    """K_{n,n}, 1024 replicas, beta linear 0.05 -> 2.0 over 2000 sweeps."""
    inst = synth.biclique_instance(n, seed=n)
    beta = synth.beta_linear(0.05, 2.0, 2000)
    _check_sampled(vctx, inst, beta, 1024, 1, prefixes, [0], np.random.default_rng(n))


def test_variant_batched_tiles_match_oracle(vctx):
    """Bicliques with ragged sides and replica counts in 32-, 64- and
    128-replica tiles, started from random and from given spins."""
    rng = np.random.default_rng(4)
    jobs = []
    for k, (na, nb, R) in enumerate([(20, 20, 5), (7, 130, 33), (64, 64, 70), (100, 37, 130), (130, 129, 64),
                                     (260, 200, 129)]):
        inst = synth.biclique_instance(na, seed=40 + k, nb=nb)
        init = synth.random_spins(R, na + nb, seed=k) if k % 2 else None
        jobs.append(dict(inst=inst, beta=synth.beta_linear(0.05, 2.0, int(rng.integers(3, 20))), R=R,
                         seed=400 + k, init=init))
    probs = [pbit.load_instance(vctx, j["inst"]) for j in jobs]
    _say("forced variant: batch of %d bicliques" % len(jobs))
    descs = []
    for p, j in zip(probs, jobs):
        d = dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
        if j["init"] is not None:
            d["init_spins"] = j["init"]
        descs.append(d)
    outs = pbit.pbit_anneal_batch(vctx, descs)
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"], init_spins=j["init"])
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        pbit.pbit_unload_problem(vctx, p)


def test_variant_and_default_batches_agree(vctx):
    """A slice of the mixed bag through the forced and the default kernels:
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
    probs = [pbit.load_instance(vctx, j["instance"]) for j in bag]
    _say("forced variant vs default on %d bag bicliques" % len(bag))
    outs_v = pbit.pbit_anneal_batch(vctx, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"], seed=j["seed"])
                                          for p, j in zip(probs, bag)])
    for j, a, b in zip(bag, outs_v, outs8):
        assert np.array_equal(a.spins, b.spins), j["instance"]["dims"]
        assert np.array_equal(a.energies, b.energies)
    for p in probs:
        pbit.pbit_unload_problem(vctx, p)
