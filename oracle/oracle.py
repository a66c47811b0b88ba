"""Python front end of the CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The HIP library never does, and the two
share no code: the oracle's arithmetic lives in ``pbit_oracle.c`` (built with
gcc) and in this file's graph builders.

Problem conventions (paper, Sec. 1.1.1 Eq. 1, Sec. 1.2.2, Sec. 2, Sec. 3):

* 3D Edwards-Anderson cube with periodic boundaries: site id
  ``i = x + Lx*(y + Ly*z)``; couplings ``J[d][i]`` (d = 0, 1, 2 for x, y, z)
  join site ``i`` to ``i + e_d`` (periodic), so there are ``3N`` bonds; with
  ``L = 2`` the two bonds between a pair stay distinct.  Colour
  ``(x + y + z) mod 2`` (the checkerboard; needs every side even).
* Biclique K_{na,nb}: side A is sites ``0..na-1``, side B is ``na..na+nb-1``;
  ``J[a][b]`` joins ``a`` and ``na + b``.  Side A has colour 0, side B colour 1.
* Spins are +-1 int8 in ``[replica][site]`` order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "pbit_oracle.c"
_LIB = _HERE / "liboracle.so"

ORACLE_OK = 0
ORACLE_E_ARG = -1
ORACLE_E_COLOURING = -2
ORACLE_E_NOMEM = -4
ORACLE_E_ENERGY_DRIFT = -100


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc: single-threaded, -O2, no fast-math, no FMA contraction."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wextra", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load(path) -> ctypes.CDLL:
    """Open a built oracle library and declare its entry points."""
    L = ctypes.CDLL(str(path))
    P = ctypes.c_void_p
    i32, u32, u64, dbl = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    L.oracle_philox4x32_10.argtypes = [P, P, P]
    L.oracle_philox4x32_10.restype = None
    L.oracle_minority_threshold.argtypes = [dbl, i32]
    L.oracle_minority_threshold.restype = u32
    L.oracle_energy.argtypes = [i32, i32, P, P, P, P, P, i32, P]
    L.oracle_energy.restype = ctypes.c_int
    L.oracle_anneal.argtypes = [i32, i32, P, P, P, P, P, i32,
                                P, i32, i32, i32, i32, u64,
                                P, P, P, P, i32, P, P]
    L.oracle_anneal.restype = ctypes.c_int
    return L


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        _lib = load(_LIB)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- primitives

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 uint32 counter words, 2 uint32 key words -> 4 uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def minority_threshold(beta: float, a: int) -> int:
    """Tm(beta, a) = round-half-down(2^32 / (1 + exp(2 beta a)))."""
    return int(lib().oracle_minority_threshold(float(beta), int(a)))


def threshold_table(beta, amax: int) -> np.ndarray:
    """uint32 [S][amax+1] table of minority thresholds."""
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    out = np.empty((beta.size, amax + 1), dtype=np.uint32)
    for s, b in enumerate(beta):
        for a in range(amax + 1):
            out[s, a] = minority_threshold(b, a)
    return out


# ---------------------------------------------------------------- graphs

class Graph:
    """Bond list + fields + colouring: the oracle's input form of a problem."""

    def __init__(self, n, bi, bj, bJ, h, colour, n_colours):
        self.n = int(n)
        self.bi = np.ascontiguousarray(bi, dtype=np.int32)
        self.bj = np.ascontiguousarray(bj, dtype=np.int32)
        self.bJ = np.ascontiguousarray(bJ, dtype=np.int8)
        self.h = None if h is None else np.ascontiguousarray(h, dtype=np.int8).reshape(-1)
        self.colour = np.ascontiguousarray(colour, dtype=np.uint8)
        self.n_colours = int(n_colours)

    @property
    def n_bonds(self) -> int:
        return int(self.bi.size)


def ea_site(x, y, z, dims):
    Lx, Ly, _ = dims
    return x + Lx * (y + Ly * z)


def ea_graph(dims, J, h=None) -> Graph:
    """Periodic 3D cube; J is int8 [3][N] with J[d][i] the bond (i, i + e_d)."""
    Lx, Ly, Lz = (int(v) for v in dims)
    N = Lx * Ly * Lz
    J = np.asarray(J, dtype=np.int8).reshape(3, N)
    bi, bj, bJ = [], [], []
    colour = np.zeros(N, dtype=np.uint8)
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = ea_site(x, y, z, (Lx, Ly, Lz))
                colour[i] = (x + y + z) % 2
                nbrs = (ea_site((x + 1) % Lx, y, z, (Lx, Ly, Lz)),
                        ea_site(x, (y + 1) % Ly, z, (Lx, Ly, Lz)),
                        ea_site(x, y, (z + 1) % Lz, (Lx, Ly, Lz)))
                for d in range(3):
                    bi.append(i)
                    bj.append(nbrs[d])
                    bJ.append(J[d, i])
    return Graph(N, bi, bj, bJ, h, colour, 2)


def biclique_graph(na, nb, J, h=None) -> Graph:
    """K_{na,nb}; J is int8 [na][nb] with J[a][b] the bond (a, na + b)."""
    na, nb = int(na), int(nb)
    J = np.asarray(J, dtype=np.int8).reshape(na, nb)
    a_idx, b_idx = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
    colour = np.concatenate([np.zeros(na, np.uint8), np.ones(nb, np.uint8)])
    return Graph(na + nb, a_idx.reshape(-1), na + b_idx.reshape(-1), J.reshape(-1), h, colour, 2)


def graph_from_bonds(n, bond_i, bond_j, bond_J, h=None, colour=None, n_colours=None) -> Graph:
    """General graph; without a colouring, the greedy colouring of the paper
    (Sec. 1.2.2): vertices in ascending order, smallest free colour."""
    if colour is None:
        colour, n_colours = greedy_colouring(n, bond_i, bond_j)
    return Graph(n, bond_i, bond_j, bond_J, h, colour, n_colours)


def greedy_colouring(n, bond_i, bond_j):
    """Colour vertices 0..n-1 in order, each with the smallest colour not used
    by an already coloured neighbour.  Returns (colour[n], number of colours)."""
    nbrs = [[] for _ in range(n)]
    for a, b in zip(np.asarray(bond_i).tolist(), np.asarray(bond_j).tolist()):
        nbrs[a].append(b)
        nbrs[b].append(a)
    colour = np.zeros(n, np.uint8)
    used = 0
    for v in range(n):
        taken = {int(colour[u]) for u in nbrs[v] if u < v}
        c = 0
        while c in taken:
            c += 1
        colour[v] = c
        used = max(used, c + 1)
    return colour, used


# ---------------------------------------------------------------- energy / anneal

def energy(g: Graph, spins) -> np.ndarray:
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1, g.n)
    out = np.zeros(s.shape[0], dtype=np.int64)
    rc = lib().oracle_energy(g.n, g.n_bonds, _ptr(g.bi), _ptr(g.bj), _ptr(g.bJ), _ptr(g.h),
                             _ptr(s), s.shape[0], _ptr(out))
    if rc != ORACLE_OK:
        raise RuntimeError("oracle_energy failed: %d" % rc)
    return out


class AnnealResult:
    def __init__(self, spins, energies, energy_trace, spin_trace):
        self.spins = spins
        self.energies = energies
        self.energy_trace = energy_trace
        self.spin_trace = spin_trace


def anneal(g: Graph, beta, n_replicas: int, seed: int, sweep_offset: int = 0, replica_offset: int = 0,
           init_spins=None, order=None, trace_every: int = 0, trace_spins: bool = False) -> AnnealResult:
    """Run the oracle's sweep.  ``beta[s]`` is used for absolute sweep ``sweep_offset + s``."""
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
    S = beta.size
    R = int(n_replicas)
    init = None if init_spins is None else np.ascontiguousarray(init_spins, dtype=np.int8).reshape(R, g.n)
    ordr = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    spins = np.zeros((R, g.n), dtype=np.int8)
    energies = np.zeros(R, dtype=np.int64)
    n_snap = S // trace_every if trace_every > 0 else 0
    e_trace = np.zeros((n_snap, R), dtype=np.int64) if n_snap else None
    s_trace = np.zeros((n_snap, R, g.n), dtype=np.int8) if (n_snap and trace_spins) else None
    rc = lib().oracle_anneal(g.n, g.n_bonds, _ptr(g.bi), _ptr(g.bj), _ptr(g.bJ), _ptr(g.h),
                             _ptr(g.colour), g.n_colours,
                             _ptr(beta), S, int(sweep_offset), R, int(replica_offset),
                             ctypes.c_uint64(int(seed) & (2**64 - 1)),
                             _ptr(init), _ptr(ordr), _ptr(spins), _ptr(energies),
                             int(trace_every), _ptr(e_trace), _ptr(s_trace))
    if rc != ORACLE_OK:
        raise RuntimeError("oracle_anneal failed: %d" % rc)
    return AnnealResult(spins, energies, e_trace, s_trace)


# ---------------------------------------------------------------- Algorithm 1

def alg1_minimal_budget(pc, G: float, i_start: int, i_step: int, t: int, p: float, p_succ: float,
                        beta_i: float, beta_f: float, i_max: int):
    """Algorithm 1 (Sec. 1.3.3) in the paper's order: for budget i, run the t
    trials one at a time, count those whose energy v exceeds theta = p G,
    leave the trial loop as soon as the count exceeds m_max, and return the
    first i whose count stays within m_max; otherwise try i + i_step.

    ``pc(i, beta, j)`` is the solver: the final energy of trial j annealed
    over the schedule ``beta`` of i sweeps.  Readings: the budget counts
    sweeps; the schedule starts at beta_i and grows by the algorithm's step
    delta_beta = (beta_f - beta_i) / i after every sweep (so its last value is
    beta_f - delta_beta); the search gives up (returns None) past ``i_max``.
    Returns (i_min, [(i, fails counted, trials run) ...])."""
    theta = p * G
    m_max = int(np.floor(t * (1.0 - p_succ) + 0.5))
    history = []
    i = i_start
    while i <= i_max:
        delta_beta = (beta_f - beta_i) / i
        beta = np.array([beta_i + k * delta_beta for k in range(i)], np.float64)
        m = 0
        ran = 0
        for j in range(t):
            v = pc(i, beta, j)
            ran += 1
            if v > theta:
                m += 1
                if m > m_max:
                    break
        history.append((i, m, ran))
        if m <= m_max:
            return i, history
        i += i_step
    return None, history


def alg1_trial(g: Graph, seed_of):
    """The solver of Algorithm 1 on the oracle: trial j is replica j of the
    anneal seeded by ``seed_of(i)``."""
    def pc(i, beta, j):
        return int(anneal(g, beta, 1, seed_of(i), replica_offset=j).energies[0])
    return pc
