"""Seeded synthetic inputs for the p-bit sweep: instances, beta schedules, job streams.

This module only draws inputs.  It holds none of the sweep's arithmetic, so the
oracle and the HIP library can both be fed from it without sharing any code.
All draws use numpy's PCG64 (``numpy.random.default_rng(seed)``).

The paper's own instances (31 random cubes and bicliques, the literature
lattices, the MQLib ground truths; Sec. 2, Sec. 3) are not available, so these
generators stand in for them at the shapes the benchmarks use: iid +-1
couplings, fields in {-1, 0, +1}, even periodic cubes, square bicliques.
"""
from __future__ import annotations

import numpy as np


def ea_instance(L, seed: int, p_plus: float = 0.5, field: str = "zero"):
    """3D Edwards-Anderson periodic cube.

    ``L`` is an int (cube) or a (Lx, Ly, Lz) triple.  Couplings ``J[3][N]`` are
    iid +1 with probability ``p_plus`` and -1 otherwise; ``J[d][i]`` is the bond
    (i, i + e_d).  ``field`` is "zero" (h = 0, returned as None) or "uniform3"
    (h iid uniform on {-1, 0, +1}).
    """
    dims = (int(L),) * 3 if np.isscalar(L) else tuple(int(v) for v in L)
    N = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed)
    J = np.where(rng.random((3, N)) < p_plus, 1, -1).astype(np.int8)
    h = None
    if field == "uniform3":
        h = rng.integers(-1, 2, size=N).astype(np.int8)
    elif field != "zero":
        raise ValueError(field)
    return {"kind": "ea3d", "dims": dims, "J": J, "h": h}


def biclique_instance(n, seed: int, field: str = "uniform3", nb=None):
    """Biclique K_{n,nb}: J[n][nb] iid +-1 (p = 1/2); h on all n + nb spins."""
    na = int(n)
    nb = na if nb is None else int(nb)
    rng = np.random.default_rng(seed)
    J = np.where(rng.random((na, nb)) < 0.5, 1, -1).astype(np.int8)
    h = None
    if field == "uniform3":
        h = rng.integers(-1, 2, size=na + nb).astype(np.int8)
    elif field != "zero":
        raise ValueError(field)
    return {"kind": "biclique", "dims": (na, nb), "J": J, "h": h}


def ferro_ea(L, field: int = 0):
    """All-ferromagnetic periodic cube (J = +1), optional uniform field."""
    dims = (int(L),) * 3 if np.isscalar(L) else tuple(int(v) for v in L)
    N = dims[0] * dims[1] * dims[2]
    h = None if field == 0 else np.full(N, field, dtype=np.int8)
    return {"kind": "ea3d", "dims": dims, "J": np.ones((3, N), np.int8), "h": h}


def ferro_biclique(n, field: int = 0):
    h = None if field == 0 else np.full(2 * n, field, dtype=np.int8)
    return {"kind": "biclique", "dims": (n, n), "J": np.ones((n, n), np.int8), "h": h}


def beta_linear(b0: float, b1: float, S: int) -> np.ndarray:
    """beta_t = b0 + (b1 - b0) t / (S - 1), t = 0..S-1 (both ends included)."""
    if S == 1:
        return np.array([b0], dtype=np.float64)
    t = np.arange(S, dtype=np.float64)
    return b0 + (b1 - b0) * t / (S - 1)


def beta_geometric(b0: float, b1: float, S: int) -> np.ndarray:
    """beta_t = b0 (b1 / b0)^(t / (S - 1)), t = 0..S-1 (both ends included)."""
    if S == 1:
        return np.array([b0], dtype=np.float64)
    t = np.arange(S, dtype=np.float64)
    return b0 * (b1 / b0) ** (t / (S - 1))


def random_spins(R: int, N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.where(rng.random((R, N)) < 0.5, 1, -1).astype(np.int8)


def mixed_bag(seed: int = 0, n_instances: int = 256, ea_sides=tuple(range(8, 25, 2)),
              n_range=(64, 1024), replica_range=(32, 512), sweep_range=(1000, 5000)):
    """Mixed batch of EA cubes and bicliques (half each), as a list of job dicts.

    Each job: instance (ea_instance / biclique_instance with its own seed),
    beta schedule (geometric 0.1 -> 5.0 for cubes, linear 0.05 -> 2.0 for
    bicliques), replica count, sweep count and anneal seed.
    """
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n_instances):
        R = int(rng.integers(replica_range[0], replica_range[1] + 1))
        S = int(rng.integers(sweep_range[0], sweep_range[1] + 1))
        if k < n_instances // 2:
            L = int(rng.choice(ea_sides))
            inst = ea_instance(L, seed=1000 + k)
            beta = beta_geometric(0.1, 5.0, S)
        else:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            inst = biclique_instance(n, seed=1000 + k)
            beta = beta_linear(0.05, 2.0, S)
        jobs.append({"instance": inst, "beta": beta, "replicas": R, "seed": 1 + k})
    return jobs


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.default_rng(seed)
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    return np.asarray(times, dtype=np.float64)


def ea_bond_list(inst):
    """The cube as a general bond list: bond (i, i + e_d) with J[d][i], in the
    order d-major over sites (the graph form of ea_instance; works for odd sides)."""
    Lx, Ly, Lz = inst["dims"]
    N = Lx * Ly * Lz
    i = np.arange(N)
    x, y, z = i % Lx, (i // Lx) % Ly, i // (Lx * Ly)
    nbrs = [((x + 1) % Lx) + Lx * (y + Ly * z), x + Lx * (((y + 1) % Ly) + Ly * z), x + Lx * (y + Ly * ((z + 1) % Lz))]
    bi = np.concatenate([i, i, i]).astype(np.int32)
    bj = np.concatenate(nbrs).astype(np.int32)
    bJ = np.asarray(inst["J"], np.int8).reshape(3, N).reshape(-1)
    return {"kind": "graph", "n": N, "bond_i": bi, "bond_j": bj, "bond_J": bJ, "h": inst.get("h")}


def random_sparse_graph(n: int, degree: int, seed: int, field: str = "uniform3", zero_frac: float = 0.0):
    """Random simple graph of mean degree about `degree`: each vertex draws
    `degree // 2` uniform partners (repeats and self-pairs dropped), couplings
    iid +-1 (a fraction `zero_frac` set to 0), fields uniform in {-1, 0, +1}."""
    rng = np.random.default_rng(seed)
    pairs = set()
    for i in range(n):
        for _ in range(max(1, degree // 2)):
            j = int(rng.integers(0, n))
            if j != i:
                pairs.add((min(i, j), max(i, j)))
    pairs = sorted(pairs)
    bi = np.array([p[0] for p in pairs], np.int32)
    bj = np.array([p[1] for p in pairs], np.int32)
    bJ = np.where(rng.random(len(pairs)) < 0.5, 1, -1).astype(np.int8)
    if zero_frac > 0:
        bJ[rng.random(len(pairs)) < zero_frac] = 0
    h = rng.integers(-1, 2, size=n).astype(np.int8) if field == "uniform3" else None
    return {"kind": "graph", "n": n, "bond_i": bi, "bond_j": bj, "bond_J": bJ, "h": h}


def dimerized_cube(L: int, seed: int, rewire: float = 0.1, field: str = "zero"):
    """Stand-in for the paper's literature lattices (Sec. 2.2: cubic lattices
    dimerized at every site and rewired to a hardware graph, which needed four
    or five update groups): a periodic L^3 cube with iid +-1 bonds whose sites
    are split into ferromagnetic pairs (spins 2 i and 2 i + 1, J = +1); each cube
    bond joins a uniformly drawn member of each pair, and a fraction `rewire` of
    them has its far end moved to a uniformly drawn spin (a self-pair or a repeat
    is dropped).  N = 2 L^3: 686, 1024, 1458, 2000, 5488 for L = 7, 8, 9, 10, 14,
    near the paper's 678 ... 5627.  The library's greedy colouring gives five
    groups on these."""
    rng = np.random.default_rng(seed)
    N = L ** 3
    i = np.arange(N)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    far = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z), x + L * (y + L * ((z + 1) % L))]
    ci = np.concatenate([i, i, i])
    cj = np.concatenate(far)
    a = 2 * ci + rng.integers(0, 2, ci.size)
    b = 2 * cj + rng.integers(0, 2, ci.size)
    moved = rng.random(ci.size) < rewire
    b[moved] = rng.integers(0, 2 * N, int(moved.sum()))
    J = np.where(rng.random(ci.size) < 0.5, 1, -1)
    bonds = {}
    for k in range(N):
        bonds[(2 * k, 2 * k + 1)] = 1
    for p, q, j in zip(a.tolist(), b.tolist(), J.tolist()):
        key = (min(p, q), max(p, q))
        if p // 2 != q // 2 and key not in bonds:
            bonds[key] = j
    keys = sorted(bonds)
    bi = np.array([k[0] for k in keys], np.int32)
    bj = np.array([k[1] for k in keys], np.int32)
    bJ = np.array([bonds[k] for k in keys], np.int8)
    h = np.random.default_rng(seed + 1).integers(-1, 2, size=2 * N).astype(np.int8) if field == "uniform3" else None
    return {"kind": "graph", "n": 2 * N, "bond_i": bi, "bond_j": bj, "bond_J": bJ, "h": h}
