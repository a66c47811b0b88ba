"""The biclique half-sweep on packed 4-bit float operands (PBIT_BQ_VARIANT=7),
per instance and in the batched tiles.  Every spin, coupling and field value
is -1, 0 or +1 and every partial sum an integer far below 2^24, so the fp4
products with fp32 sums give the same fields as the default int8 products
with int32 sums: the results are bit-exact against the oracle, like the
default path's."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import oracle
from paper_2510_23419_amd import pbit
from tests.test_parity_gpu import _check_sampled, _every_sweep, graph_of

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx4():
    """A context whose biclique kernels run on fp4 operands (the variant is
    read when the context is created)."""
    old = os.environ.get("PBIT_BQ_VARIANT")
    os.environ["PBIT_BQ_VARIANT"] = "7"
    try:
        c = pbit.Context(0)
    finally:
        if old is None:
            del os.environ["PBIT_BQ_VARIANT"]
        else:
            os.environ["PBIT_BQ_VARIANT"] = old
    yield c.ctx
    c.close()


@pytest.mark.parametrize("na,nb,R", [(600, 520, 200), (512, 1024, 130), (40, 40, 70)])
def test_fp4_every_replica_every_sweep(ctx4, na, nb, R):
    """Sides padded to 128 take the fp4 kernel; small sides keep the int8 one."""
    inst = synth.biclique_instance(na, seed=na + 3 * nb, nb=nb)
    _say("fp4 biclique %dx%d R=%d every sweep" % (na, nb, R))
    _every_sweep(ctx4, inst, synth.beta_linear(0.05, 2.0, 8), R, seed=12)


@pytest.mark.parametrize("n,prefixes", [(1024, [1, 2, 10]), (4096, [1, 2])])
def test_fp4_full_size_sampled(ctx4, n, prefixes):
    """K_{n,n}, 1024 replicas, beta linear 0.05 -> 2.0 over 2000 sweeps."""
    inst = synth.biclique_instance(n, seed=n)
    beta = synth.beta_linear(0.05, 2.0, 2000)
    _check_sampled(ctx4, inst, beta, 1024, 1, prefixes, [0], np.random.default_rng(n))


def test_fp4_batched_tiles_match_oracle(ctx4):
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
    probs = [pbit.load_instance(ctx4, j["inst"]) for j in jobs]
    _say("fp4 batch of %d bicliques" % len(jobs))
    descs = []
    for p, j in zip(probs, jobs):
        d = dict(problem=p, beta=j["beta"], n_replicas=j["R"], seed=j["seed"])
        if j["init"] is not None:
            d["init_spins"] = j["init"]
        descs.append(d)
    outs = pbit.pbit_anneal_batch(ctx4, descs)
    for p, j, o in zip(probs, jobs, outs):
        ref = oracle.anneal(graph_of(j["inst"]), j["beta"], j["R"], j["seed"], init_spins=j["init"])
        assert np.array_equal(o.spins, ref.spins), j["inst"]["dims"]
        assert np.array_equal(o.energies, ref.energies), j["inst"]["dims"]
        pbit.pbit_unload_problem(ctx4, p)


def test_fp4_and_int8_batches_agree(ctx4):
    """A slice of the mixed bag through both operand types: identical results."""
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
    probs = [pbit.load_instance(ctx4, j["instance"]) for j in bag]
    _say("fp4 vs int8 on %d bag bicliques" % len(bag))
    outs4 = pbit.pbit_anneal_batch(ctx4, [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"], seed=j["seed"])
                                          for p, j in zip(probs, bag)])
    for j, a, b in zip(bag, outs4, outs8):
        assert np.array_equal(a.spins, b.spins), j["instance"]["dims"]
        assert np.array_equal(a.energies, b.energies)
    for p in probs:
        pbit.pbit_unload_problem(ctx4, p)
