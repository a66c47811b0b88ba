#!/usr/bin/env python3
"""Benchmark of the p-bit sweep on one MI355X.

One step is one whole anneal of the workload: threshold table (host, FP64),
random start, every half-sweep of the beta schedule, final energies, all on
device buffers that are resident before the timed region starts.

Default workload: 3D Edwards-Anderson periodic cube L=32 (32,768 spins),
J iid +-1, h = 0, 4,096 replicas, beta geometric 0.1 -> 5.0 over 10,000 sweeps,
seed 1.  Other workloads (``--workload``) are the smaller cube and the biclique
sizes, printed in the same format.

Prints one JSON line with the throughput in p-bit updates per second (one
update = one spin of one replica in one sweep), the roofline of the dominant
kernel (its algorithmic bytes or int8 ops per launch over its mean launch time,
measured with HIP events on the stream the kernels run on), and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
INT8_MFMA_PEAK_TOPS = 5000.0   # MI355X dense int8 MFMA, published (TOP/s)
# biclique half-sweep kernels by variant number (pbit_profile_variant)
BQ_KERNELS = {1: "k_bq_halfsweep", 2: "k_bq_halfsweep_dma", 3: "k_bq_halfsweep_bits", 4: "k_bq_slab"}
VALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 32-bit vector lane-ops/s: CUs x SIMDs x lanes x clock

WORKLOADS = {
    "ea32": dict(kind="ea3d", L=32, R=4096, S=10_000, b0=0.1, b1=5.0, sched="geometric", inst_seed=32),
    "ea16": dict(kind="ea3d", L=16, R=4096, S=10_000, b0=0.1, b1=5.0, sched="geometric", inst_seed=16),
    "bq512": dict(kind="biclique", n=512, R=1024, S=2000, b0=0.05, b1=2.0, sched="linear", inst_seed=512),
    "bq1024": dict(kind="biclique", n=1024, R=1024, S=2000, b0=0.05, b1=2.0, sched="linear", inst_seed=1024),
    "bq2048": dict(kind="biclique", n=2048, R=1024, S=2000, b0=0.05, b1=2.0, sched="linear", inst_seed=2048),
    "bq4096": dict(kind="biclique", n=4096, R=1024, S=2000, b0=0.05, b1=2.0, sched="linear", inst_seed=4096),
    # general graph with k update groups: the dimerized, rewired cube that stands in for
    # the paper's hardware-embedded literature lattices (5,488 spins, 5 greedy groups)
    "dimer14": dict(kind="graph", L=14, R=4096, S=2000, b0=0.1, b1=5.0, sched="geometric", inst_seed=14),
}


def describe(w):
    if w["kind"] == "graph":
        return ("dimerized periodic cube L=%d (%d spins in ferromagnetic pairs, cube bonds J iid +-1 between random "
                "pair members, 10%% rewired), h=0, greedy update groups, %d replicas, beta %s %.2g->%.2g over %d "
                "sweeps, seed 1" % (w["L"], 2 * w["L"] ** 3, w["R"], w["sched"], w["b0"], w["b1"], w["S"]))
    if w["kind"] == "ea3d":
        return ("3D Edwards-Anderson periodic cube L=%d (%d spins), J iid +-1, h=0, checkerboard, %d replicas, "
                "beta %s %.2g->%.2g over %d sweeps, seed 1" % (w["L"], w["L"] ** 3, w["R"], w["sched"], w["b0"],
                                                               w["b1"], w["S"]))
    return ("biclique K_{%d,%d}, J iid +-1, h uniform {-1,0,1}, %d replicas, beta %s %.2g->%.2g over %d sweeps, "
            "seed 1" % (w["n"], w["n"], w["R"], w["sched"], w["b0"], w["b1"], w["S"]))


def make_instance(w):
    import synth
    if w["kind"] == "ea3d":
        inst = synth.ea_instance(w["L"], seed=w["inst_seed"])
    elif w["kind"] == "graph":
        inst = synth.dimerized_cube(w["L"], seed=w["inst_seed"])
    else:
        inst = synth.biclique_instance(w["n"], seed=w["inst_seed"])
    if w["sched"] == "geometric":
        beta = synth.beta_geometric(w["b0"], w["b1"], w["S"])
    else:
        beta = synth.beta_linear(w["b0"], w["b1"], w["S"])
    return inst, beta


def cpu_model():
    """The host CPU's model name and logical CPU count, as the kernel reports them."""
    name = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count() or 1


def host_threads():
    """Host threads for the oracle's all-core leg: the cores this process may run
    on, at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, inst, beta, budget_s):
    """The oracle as it stands on a bounded sample: the first sweeps of the same
    schedule for 8 replicas, sized to ~budget_s on one core; then the same sample
    on every host thread at once, thread t taking replicas 8t .. 8t + 7 (replicas
    are independent and drawn from their global index, so the slices are the
    corresponding part of one run).  The oracle is a C library called through
    ctypes, which releases the interpreter lock for the call."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle
    if w["kind"] == "ea3d":
        g = oracle.ea_graph(inst["dims"], inst["J"], inst["h"])
    elif w["kind"] == "graph":
        g = oracle.graph_from_bonds(inst["n"], inst["bond_i"], inst["bond_j"], inst["bond_J"], inst["h"])
    else:
        g = oracle.biclique_graph(*inst["dims"], inst["J"], inst["h"])
    N = g.n
    # calibrate on a tiny run, then size the sample
    t0 = time.perf_counter()
    oracle.anneal(g, beta[:2], 4, seed=1)
    rate = 2 * 4 * N / max(time.perf_counter() - t0, 1e-6)
    R = 8
    S = int(max(2, min(len(beta), budget_s * rate / (R * N))))
    t0 = time.perf_counter()
    oracle.anneal(g, beta[:S], R, seed=1)
    dt1 = time.perf_counter() - t0
    T = host_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=T) as pool:
        list(pool.map(lambda t: oracle.anneal(g, beta[:S], R, seed=1, replica_offset=R * t), range(T)))
    dtT = time.perf_counter() - t0
    model, nproc = cpu_model()
    return {"value": T * R * N * S / dtT, "unit": "p-bit updates/s", "cores": T, "kind": "oracle",
            "one_core_value": R * N * S / dt1, "cpu_model": model, "host_nproc": nproc,
            "sample": "first %d of %d sweeps of the same schedule, replicas 0-%d of %d on one core (%.1f s), then "
                      "replicas 0-%d on %d threads at once (%.1f s); C oracle on %s (%d logical CPUs, %d used)"
                      % (S, len(beta), R - 1, w["R"], dt1, T * R - 1, T, dtT, model, nproc, T)}


def graph_launch_bytes(ctx, prob, inst, R):
    """Algorithmic bytes per group launch of a general graph, averaged over the
    groups of one sweep: a group writes its own spin rows (1 byte per update),
    reads the rows of its sites' neighbours once each (1 byte per replica per
    distinct neighbour: rows shared by several sites of the group are fetched
    once when they stay in cache), and reads its adjacency (4-byte neighbour id
    and 1-byte code per bond end, CSR start, field base and class entry)."""
    import numpy as np
    from paper_2510_23419_amd import pbit
    colour, k = pbit.pbit_problem_colouring(ctx, prob)
    n = inst["n"]
    bi = np.asarray(inst["bond_i"], np.int64)
    bj = np.asarray(inst["bond_j"], np.int64)
    deg = np.bincount(np.concatenate([bi, bj]), minlength=n)
    total = 0
    for c in range(k):
        in_c = colour == c
        nbr = np.zeros(n, bool)
        nbr[bj[in_c[bi]]] = True
        nbr[bi[in_c[bj]]] = True
        sites = int(in_c.sum())
        total += sites * R + int(nbr.sum()) * R + 5 * int(deg[in_c].sum()) + 14 * sites
    return total / k, k


def profile_record(workload, kernel=None):
    """The committed rocprofv3 counter summary of the dominant kernel for this
    workload (profiles/traffic.json), or None if the kernel sources changed
    since the counters were taken or the record is of another kernel than
    `kernel`."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    recs = json.load(open(path))
    # a workload's records: one per kernel that runs it (the cube's matrix-core
    # half-sweep under "<workload>_mfma", the graph's launch per colour class under
    # "<workload>_class")
    for rec in (recs.get(workload), recs.get(workload + "_mfma"), recs.get(workload + "_class")):
        if not rec or (kernel and kernel not in rec["kernel"]):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["sha256"]:
            return rec
    return None


def measured_traffic(workload, kernel=None):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each scaled by what the
    counter reads for a plain copy), or None."""
    rec = profile_record(workload, kernel)
    return None if rec is None else float(rec["traffic_bytes_per_launch"])


def _bag_dtype():
    """Arithmetic of the batched tiles: int8 spins and couplings, biclique fields as
    int8 MFMA products with int32 sums."""
    return "int8"


def mixed_bag_bench(args, pbit, torch):
    """Mixed bag: 256 jobs (128 cubes, L in {8..24}; 128 bicliques, n in
    [64, 1024]; 32..512 replicas; 1000..5000 sweeps) in the persistent batched
    kernels, against the plain per-instance sweep (one job after another)."""
    import synth
    bag = synth.mixed_bag(seed=args.bag_seed, n_instances=args.bag_size)
    ctx = pbit.Context(0)
    probs = [pbit.load_instance(ctx.ctx, j["instance"]) for j in bag]
    jobs = [dict(problem=p, beta=j["beta"], n_replicas=j["replicas"], seed=j["seed"]) for p, j in zip(probs, bag)]
    updates = sum(pbit.pbit_problem_spins(ctx.ctx, p) * j["replicas"] * len(j["beta"]) for p, j in zip(probs, bag))
    # batched: one call, all jobs.  The warm-up runs every job for two sweeps: it loads
    # the code objects and lets the tile autotuner time the shapes it has not seen (the
    # choice is cached per shape, so the timed call reuses it); its time is reported
    t0 = time.perf_counter()
    pbit.pbit_anneal_batch(ctx.ctx, [dict(jb, beta=jb["beta"][:2]) for jb in jobs], want_spins=False)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    tunings, shapes = pbit.pbit_profile_tiles(ctx.ctx)
    t0 = time.perf_counter()
    outs = pbit.pbit_anneal_batch(ctx.ctx, jobs, want_spins=False)
    t_batch = time.perf_counter() - t0
    # plain per-instance sweep on the same jobs (device buffers, one job at a time)
    plain_idx = list(range(0, len(bag), max(1, len(bag) // args.plain_jobs)))[:args.plain_jobs]
    t_plain = 0.0
    plain_best = {}
    for k in plain_idx:
        j = bag[k]
        N = pbit.pbit_problem_spins(ctx.ctx, probs[k])
        d = torch.empty((j["replicas"], N), dtype=torch.int8, device="cuda:0")
        e = torch.empty(j["replicas"], dtype=torch.int64, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pbit.pbit_anneal_dev(ctx.ctx, probs[k], j["beta"], j["replicas"], j["seed"], d, d_energies=e)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        plain_best[k] = int(e.min().item())
    same = all(plain_best[k] == outs[k].best_energy for k in plain_idx)
    plain_per_job = t_plain / len(plain_idx)
    res = {
        "metric": "anneals/s (mixed bag, batched persistent kernels)",
        "value": len(bag) / t_batch,
        "unit": "anneals/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": t_batch * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": _bag_dtype(), "data": "synthetic",
        "config": {"workload": "mixed bag of %d jobs: 128 EA cubes L in {8,...,24}, 128 bicliques n in [64,1024], "
                               "replicas 32..512, sweeps 1000..5000, bag seed %d" % (len(bag), args.bag_seed),
                   "updates_per_s": updates / t_batch,
                   "plain_per_instance_anneals_per_s": 1.0 / plain_per_job,
                   "plain_jobs_timed": len(plain_idx),
                   "speedup_vs_plain": plain_per_job * len(bag) / t_batch,
                   "tile_tuning": {"shapes_timed": tunings, "shapes_cached": shapes,
                                   "warmup_s_two_sweeps_per_job": t_warm,
                                   "enabled": os.environ.get("PBIT_TILE_TUNE", "1") != "0"},
                   "plain_and_batched_best_energies_equal": same},
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def serve_pool(n, seed):
    """Serving instances: as the mixed bag, widened to cubes L <= 32 and bicliques n <= 2048."""
    import synth
    return synth.mixed_bag(seed=seed, n_instances=n, ea_sides=tuple(range(8, 33, 2)), n_range=(64, 2048))


def serve_bench(args, pbit, torch):
    """Poisson arrivals of anneal jobs with a target energy (the best of 64
    replicas of the same schedule plus 1 %), served by continuous batching."""
    import numpy as np
    import synth
    pool = serve_pool(args.pool, seed=11)
    ctx = pbit.Context(0)
    probs = [pbit.load_instance(ctx.ctx, j["instance"]) for j in pool]
    Ns = [pbit.pbit_problem_spins(ctx.ctx, p) for p in probs]
    # reference: best of 64 replicas on the GPU path (bit-identical to the oracle)
    refs = pbit.pbit_anneal_batch(ctx.ctx, [dict(problem=p, beta=j["beta"], n_replicas=64, seed=7777)
                                            for p, j in zip(probs, pool)], want_spins=False)
    e_ref = [r.best_energy for r in refs]
    targets = [e + int(abs(e) * 0.01) for e in e_ref]
    arrivals = synth.poisson_arrivals(args.rate, args.duration, seed=int(args.rate))
    rng = np.random.default_rng(int(args.rate) + 1)
    which = rng.integers(0, len(pool), size=len(arrivals))
    pending = {}
    lat, residual, reached = [], [], 0
    rejected = 0
    t0 = time.perf_counter()
    k = 0
    next_note = 10.0
    while k < len(arrivals) or pending:
        now = time.perf_counter() - t0
        if now >= next_note:  # progress on stderr (stdout carries the one result line)
            print("serve: %.0f s, %d offered, %d done, %d pending, %d rejected" % (now, k, len(lat), len(pending),
                                                                                 rejected), file=sys.stderr, flush=True)
            next_note += 10.0
        while k < len(arrivals) and arrivals[k] <= now:
            q = int(which[k])
            j = pool[q]
            try:
                jid = pbit.pbit_submit(ctx.ctx, probs[q], j["beta"], j["replicas"], seed=k + 1, target=targets[q])
                pending[jid] = (arrivals[k], q, j)
            except pbit.PbitError as e:
                if e.code != pbit.PBIT_E_BUSY:
                    raise
                rejected += 1
            k += 1
        for jid in list(pending):
            t_arr, q, j = pending[jid]
            out = pbit.pbit_poll(ctx.ctx, jid, j["replicas"], Ns[q], len(j["beta"]), want_spins=False)
            if out is not None:
                lat.append(time.perf_counter() - t0 - t_arr)
                residual.append((out.best_energy - e_ref[q]) / abs(e_ref[q]))
                reached += int(out.best_energy <= targets[q])
                del pending[jid]
        if not pending and k < len(arrivals):
            time.sleep(max(0.0, min(arrivals[k] - (time.perf_counter() - t0), 0.01)))
    makespan = time.perf_counter() - t0
    lat_ms = np.asarray(lat) * 1e3
    res = {
        "metric": "anneals/s at <= 1% residual energy (Poisson serving, continuous batching)",
        "value": len(lat) / makespan,
        "unit": "anneals/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": makespan * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": _bag_dtype(), "data": "synthetic",
        "config": {"workload": "Poisson arrivals at %.0f jobs/s for %.0f s; jobs from a pool of %d instances "
                               "(EA cubes L <= 32, bicliques n <= 2048, 32..512 replicas, 1000..5000 sweeps); "
                               "target = best of 64 replicas + 1 %%" % (args.rate, args.duration, len(pool)),
                   "offered": int(len(arrivals)), "rejected_busy": rejected, "completed": len(lat),
                   "reached_target": reached,
                   "p50_latency_ms": float(np.percentile(lat_ms, 50)) if len(lat) else None,
                   "p99_latency_ms": float(np.percentile(lat_ms, 99)) if len(lat) else None,
                   "mean_residual": float(np.mean(residual)) if residual else None},
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def alg1_bench(args, pbit, torch):
    """Algorithm 1 (Sec. 1.3.3) on the paper's ladder of cubic lattices N = 2^3 ... 10^3
    (J iid +-1, h = 0, periodic; odd sides run as general graphs with greedy groups):
    for each quality p, the smallest sweep budget of a linear 0.35 -> 3.5 schedule at
    which 18 of 20 trials end at or below p G, each size starting its search at the
    budget the previous size needed.  G is the best energy of 4096 replicas annealed
    over 10^4 sweeps (geometric 0.1 -> 5.0)."""
    import numpy as np
    import synth
    from paper_2510_23419_amd import alg1
    ctx = pbit.Context(0)
    t0 = time.perf_counter()
    ladder = []
    for L in range(2, 11):
        inst = synth.ea_instance(L, seed=L)
        prob = pbit.load_instance(ctx.ctx, inst if L % 2 == 0 else synth.ea_bond_list(inst))
        ref = pbit.pbit_anneal(ctx.ctx, prob, synth.beta_geometric(0.1, 5.0, 10_000), 4096, seed=99, want_spins=False)
        ladder.append((L, prob, ref.best_energy, pbit.pbit_problem_colouring(ctx.ctx, prob)[1]))
    t_ref = time.perf_counter() - t0
    results, updates = [], 0
    t1 = time.perf_counter()
    for p in args.alg1_qualities:
        start = 1
        for L, prob, G, groups in ladder:
            r = alg1.i_min(ctx.ctx, prob, G, i_start=start, i_step=1, t=20, p=p, p_succ=0.9, seed=1, window=16,
                           i_max=args.alg1_max)
            updates += sum(b for b, _ in r.history) * 20 * L ** 3
            print("alg1: p=%.2f L=%d i_min=%s (%d budgets, %.1f s)" % (p, L, r.i_min, len(r.history),
                                                                     time.perf_counter() - t1),
                  file=sys.stderr, flush=True)
            results.append({"L": L, "N": L ** 3, "groups": groups, "G": G, "p": p, "i_min_sweeps": r.i_min,
                            "i_min_iterations": None if r.i_min is None else r.i_min * groups,
                            "budgets_tried": len(r.history)})
            if r.i_min is not None:
                start = r.i_min
    wall = time.perf_counter() - t1
    for _, prob, _, _ in ladder:
        pbit.pbit_unload_problem(ctx.ctx, prob)
    res = {
        "metric": "p-bit updates/s inside Algorithm 1 searches (minimum iteration budgets, Sec. 1.3.3)",
        "value": updates / wall, "unit": "p-bit updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8", "data": "synthetic",
        "config": {"workload": "Algorithm 1 on random +-1 cubes L = 2..10 (seed L, h = 0), 20 trials at 90 %% "
                               "success, qualities %s, linear 0.35 -> 3.5, search window 16 budgets"
                               % ",".join("%.2f" % q for q in args.alg1_qualities),
                   "reference_seconds": t_ref, "i_min": results},
    }
    print(json.dumps(res), flush=True)
    ctx.close()


PROBES = {
    # name: (probe id, size, reps, metric, unit, peak, unit scale)
    "philox": (1, 64, 50, "Philox4x32-10 words/s (the sweep's counter layout, no other work)", "words/s", None),
    "copy": (2, 1 << 30, 20, "device copy bandwidth (bytes read + written per second, 1 GiB each way)", "GB/s",
             HBM_PEAK_GBS),
    # the spins of the EA L = 32, R = 4096 workload: 64 MiB per colour, each half-sweep reads
    # one colour and writes the other (the pair fits the 256 MB last-level cache)
    "copy64m": (2, 64 << 20, 50, "device copy bandwidth at the cube workload's size (64 MiB each way, "
                "alternating direction)", "GB/s", HBM_PEAK_GBS),
    "mfma": (3, 64, 10, "int8 MFMA throughput (v_mfma_i32_32x32x32_i8 chains, operands in registers)", "TOP/s",
             INT8_MFMA_PEAK_TOPS),
}


def probe_bench(args, pbit, name):
    """One of the ceilings the sweep kernels are measured against, timed on its own."""
    probe, size, reps, metric, unit, peak = PROBES[name]
    ctx = pbit.Context(0)
    ms, work = pbit.pbit_probe(ctx.ctx, probe, size, reps)
    rate = work / (ms * 1e-3)
    value = rate / 1e9 if unit == "GB/s" else (rate / 1e12 if unit == "TOP/s" else rate)
    extra = {}
    if name == "philox":
        # what the rate caps: one word per p-bit update, 2 algorithmic bytes per stencil update
        extra = {"updates_per_s_cap": rate, "stencil_hbm_cap_GBs": 2 * rate / 1e9,
                 "stencil_hbm_cap_frac": 2 * rate / 1e9 / HBM_PEAK_GBS,
                 "valu_lane_ops_per_word_at_peak": VALU_PEAK_TLANEOPS * 1e12 / rate}
    res = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": reps, "warmup": 1,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"philox": "u32", "copy": "u8", "copy64m": "u8", "mfma": "int8"}[name], "data": "synthetic",
           "config": dict({"workload": "ceiling probe %s, size %d, %d launches" % (name, size, reps),
                           "work_per_launch": work}, **extra),
           "roofline": {"bound": {"philox": "alu", "copy": "hbm", "copy64m": "hbm", "mfma": "mfma"}[name], "achieved": value,
                        "peak": peak if peak else VALU_PEAK_TLANEOPS * 1e12 / 10,
                        "unit": unit if peak else "words/s (10 lane-ops per word)",
                        "frac": value / peak if peak else rate / (VALU_PEAK_TLANEOPS * 1e12 / 10),
                        "traffic": None}}
    print(json.dumps(res), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ea32",
                    choices=sorted(WORKLOADS) + ["mixed", "serve", "alg1"] + sorted(PROBES))
    ap.add_argument("--alg1-qualities", type=float, nargs="+", default=[0.90, 0.95, 0.98],
                    help="alg1: solution qualities p (pass when E <= p G)")
    ap.add_argument("--alg1-max", type=int, default=20000, help="alg1: largest sweep budget tried")
    ap.add_argument("--bag-size", type=int, default=256)
    ap.add_argument("--bag-seed", type=int, default=0)
    ap.add_argument("--plain-jobs", type=int, default=32, help="jobs of the bag timed through the per-instance path")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate (jobs/s)")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: arrival window (s)")
    ap.add_argument("--pool", type=int, default=64, help="serve: distinct instances jobs are drawn from")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle sample budget (0 = skip)")
    ap.add_argument("--profile-every", type=int, default=32,
                    help="time a window of 8 consecutive half-sweeps with HIP events every k launches (0 = off)")
    ap.add_argument("--sweeps", type=int, default=0, help="run only the first k sweeps of the schedule (profiling)")
    ap.add_argument("--trace-points", type=int, default=100,
                    help="points of the residual-against-sweeps trace, from one untimed anneal (0 = off)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized int8 tensor 5 times (reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: measures one GPU only; run it with --gpus 1 (the path would shard replicas "
              "across GPUs with no exchange, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_23419_amd import pbit

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes, dtype=torch.int8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 5}))
        return

    if args.workload == "mixed":
        mixed_bag_bench(args, pbit, torch)
        return
    if args.workload == "serve":
        serve_bench(args, pbit, torch)
        return
    if args.workload == "alg1":
        alg1_bench(args, pbit, torch)
        return
    if args.workload in PROBES:
        probe_bench(args, pbit, args.workload)
        return

    w = WORKLOADS[args.workload]
    inst, beta = make_instance(w)
    if args.sweeps > 0:
        beta = beta[:args.sweeps]
    R = w["R"]
    dev = torch.device("cuda:0")
    ctx = pbit.Context(0)
    prob = pbit.load_instance(ctx.ctx, inst)
    N = pbit.pbit_problem_spins(ctx.ctx, prob)
    d_spins = torch.empty((R, N), dtype=torch.int8, device=dev)
    d_energy = torch.empty(R, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        pbit.pbit_anneal_dev(ctx.ctx, prob, beta, R, 1, d_spins, d_energies=d_energy, stream=stream)
    torch.cuda.synchronize()

    kind = {"ea3d": pbit.PBIT_EA3D, "graph": pbit.PBIT_GRAPH}.get(w["kind"], pbit.PBIT_BICLIQUE)
    pbit.pbit_profile_enable(ctx.ctx, args.profile_every)
    pbit.pbit_profile_read(ctx.ctx, kind, reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        pbit.pbit_anneal_dev(ctx.ctx, prob, beta, R, 1, d_spins, d_energies=d_energy, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    kern_ms, launches = pbit.pbit_profile_read(ctx.ctx, kind, reset=True)
    pbit.pbit_profile_enable(ctx.ctx, 0)
    best = int(d_energy.min().item())

    S = len(beta)
    updates = N * R * S * args.steps
    ms_per_step = wall * 1e3 / args.steps
    value = updates / wall

    # roofline of the half-sweep kernel
    avg_ms = kern_ms / launches if launches else float("inf")
    ea_path = pbit.pbit_profile_ea_path(ctx.ctx) if w["kind"] == "ea3d" else 0
    if ea_path == 2:
        # the cube held in LDS for runs of sweeps: no HBM traffic per half-sweep, so the
        # vector ALU is the roof; lane-ops per update from the committed counter run
        rec = profile_record(args.workload, "k_ea_slab")
        lops = None
        if rec and rec.get("valu_insts_per_dispatch"):
            # the counter run's one launch holds all of its sweeps
            sweeps = rec.get("sweeps_per_dispatch") or rec["pmc_sweeps"]
            lops = float(rec["valu_insts_per_dispatch"]) * 64 / (N * R * sweeps)
        upd_per_s = (N * R / 2) / (avg_ms * 1e-3)  # updates per second inside the kernel
        roof = {"bound": "alu", "achieved": None if lops is None else upd_per_s * lops / 1e12,
                "peak": VALU_PEAK_TLANEOPS, "unit": "Tlane-op/s", "traffic": None, "kernel": "k_ea_slab",
                "lane_ops_per_update": lops, "updates_per_s_in_kernel": upd_per_s,
                "avg_halfsweep_us": avg_ms * 1e3, "halfsweeps_timed": launches}
    elif w["kind"] == "ea3d":
        # per launch: N/2 x R updates, each reads its share of the other colour's
        # spins once (1 B) and writes its own spin (1 B); couplings ~0 B at R=4096.
        # The same algorithmic bytes for both one-launch-per-half-sweep paths: the
        # streaming stencil (path 1) and the fields on the matrix cores (path 3)
        alg_bytes = N * R + 4 * (N // 2)
        roof = {"bound": "hbm", "achieved": alg_bytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "traffic": None, "kernel": "k_eam_halfsweep" if ea_path == 3 else "k_ea_halfsweep",
                "ea_path": ea_path,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_us": avg_ms * 1e3, "launches_timed": launches}
    elif w["kind"] == "graph" and pbit.pbit_profile_graph_path(ctx.ctx) == 2:
        # the graph held in LDS for runs of sweeps (a tile of replicas per workgroup): the
        # vector ALU is the roof, as for the cube in LDS; the window counts one launch per
        # colour class and sweep, so a "launch" is one class update on average
        groups = pbit.pbit_problem_colouring(ctx.ctx, prob)[1]
        rec = profile_record(args.workload, "k_graph_slab")
        lops = None
        if rec and rec.get("valu_insts_per_dispatch"):
            sweeps = rec.get("sweeps_per_dispatch") or rec["pmc_sweeps"]
            lops = float(rec["valu_insts_per_dispatch"]) * 64 / (N * R * sweeps)
        upd_per_s = (N * R / groups) / (avg_ms * 1e-3)  # updates per second inside the kernel
        roof = {"bound": "alu", "achieved": None if lops is None else upd_per_s * lops / 1e12,
                "peak": VALU_PEAK_TLANEOPS, "unit": "Tlane-op/s", "traffic": None, "kernel": "k_graph_slab",
                "groups": groups, "lane_ops_per_update": lops, "updates_per_s_in_kernel": upd_per_s,
                "avg_class_update_us": avg_ms * 1e3, "class_updates_timed": launches}
    elif w["kind"] == "graph":
        alg_bytes, groups = graph_launch_bytes(ctx.ctx, prob, inst, R)
        roof = {"bound": "hbm", "achieved": alg_bytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "traffic": None, "kernel": "k_graph_halfsweep", "groups": groups,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_us": avg_ms * 1e3, "launches_timed": launches}
    else:
        n = w["n"]
        alg_ops = 2 * n * n * R  # one side's fields: n x n couplings times n x R spins
        # the kernel the library ran (autotuned unless PBIT_BQ_VARIANT forces one)
        variant = pbit.pbit_profile_variant(ctx.ctx)
        roof = {"bound": "mfma", "achieved": alg_ops / (avg_ms * 1e-3) / 1e12,
                "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s", "traffic": None,
                "kernel": BQ_KERNELS.get(variant, "k_bq_halfsweep"), "variant": variant, "operands": "int8",
                "alg_ops_per_launch": alg_ops, "avg_launch_us": avg_ms * 1e3, "launches_timed": launches}
    if launches == 0:  # launch timing switched off (--profile-every 0)
        roof["achieved"] = None
    roof["frac"] = None if roof["achieved"] is None else roof["achieved"] / roof["peak"]
    lds_resident = roof["bound"] == "alu"  # a cube or graph held in LDS: no per-launch HBM traffic
    if not lds_resident:
        roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    rec = profile_record(args.workload, roof["kernel"])
    if not lds_resident and rec and rec.get("valu_insts_per_dispatch") and launches:
        # vector ALU issue: wave instructions x 64 lanes per launch over the measured
        # launch time, against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
        lane_ops = float(rec["valu_insts_per_dispatch"]) * 64
        achieved = lane_ops / (avg_ms * 1e-3) / 1e12
        roof["valu"] = {"lane_ops_per_launch": lane_ops, "achieved": achieved, "peak": VALU_PEAK_TLANEOPS,
                        "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_TLANEOPS}
        if w["kind"] == "ea3d":
            roof["valu"]["lane_ops_per_update"] = lane_ops / (N * R / 2)  # a half-sweep updates N/2 sites
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"

    # residual energy against sweeps: one more anneal, outside the timed region, with every
    # replica's energy recorded every S/100 sweeps; residual of the best and of the mean
    # replica against an independent reference: the best of 64 replicas annealed over the
    # same schedule with another seed (bit-identical to the oracle's 64 runs by parity)
    trace = None
    if args.trace_points > 0:
        every = max(1, S // args.trace_points)
        t0 = time.perf_counter()
        tr = pbit.pbit_anneal(ctx.ctx, prob, beta, R, 1, trace_every=every, want_spins=False)
        traced_ms = (time.perf_counter() - t0) * 1e3
        et = tr.energy_trace.astype(float)
        ref = float(pbit.pbit_anneal(ctx.ctx, prob, beta, 64, 7777, want_spins=False).best_energy)
        trace = {"every_sweeps": every, "reference_energy": ref,
                 "reference": "best of 64 replicas, same schedule, seed 7777",
                 "final_best_energy": float(tr.best_energy), "traced_anneal_ms": traced_ms,
                 "sweeps": [every * (k + 1) for k in range(et.shape[0])],
                 "residual_best": [round((float(r.min()) - ref) / abs(ref), 6) for r in et],
                 "residual_mean": [round((float(r.mean()) - ref) / abs(ref), 6) for r in et]}

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(w, inst, beta, args.cpu_seconds)

    out = {
        "metric": "p-bit updates/s/GPU",
        "value": value,
        "unit": "p-bit updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": roof.get("operands", "int8"),
        "data": "synthetic",
        "config": {"workload": describe(w), "spins": N, "replicas": R, "sweeps": S,
                   "anneals_per_s": args.steps / wall, "device_ms_per_step": dev_ms / args.steps,
                   "best_energy": best, "residual_vs_sweeps": trace},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    pbit.pbit_unload_problem(ctx.ctx, prob)
    ctx.close()


if __name__ == "__main__":
    main()
