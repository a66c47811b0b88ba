"""Test-side formulas written independently of the oracle's code.

Dense couplings, energies and Boltzmann weights are built here straight from
the problem statement (paper Sec. 1.1.1 Eq. 1 with the sign and field reading
used throughout, Sec. 1.2.1 Boltzmann law), with numpy and explicit lattice
coordinates, so that they can pin the oracle rather than repeat it.
"""
import itertools

import numpy as np


def ea_dense(dims, J, h=None):
    """Dense symmetric coupling matrix of a periodic cube and its field vector."""
    Lx, Ly, Lz = dims
    N = Lx * Ly * Lz
    Jf = np.zeros((N, N), dtype=np.int64)
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = x + Lx * (y + Ly * z)
                for d, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    j = (x + dx) % Lx + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))
                    Jf[i, j] += int(J[d][i])
                    Jf[j, i] += int(J[d][i])
    hv = np.zeros(N, np.int64) if h is None else np.asarray(h, np.int64)
    return Jf, hv


def biclique_dense(J, h=None):
    na, nb = J.shape
    N = na + nb
    Jf = np.zeros((N, N), dtype=np.int64)
    Jf[:na, na:] = J
    Jf[na:, :na] = J.T
    hv = np.zeros(N, np.int64) if h is None else np.asarray(h, np.int64)
    return Jf, hv


def dense_energy(Jf, hv, spins):
    """E = -1/2 m^T J m - h.m for every row of spins (bonds counted once)."""
    m = np.asarray(spins, dtype=np.int64).reshape(-1, Jf.shape[0])
    return -(np.einsum("ri,ij,rj->r", m, Jf, m) // 2) - m @ hv


def ea_energy_roll(dims, J, h, spins):
    """Energy of a periodic cube from shifted copies of the lattice (no bond list)."""
    Lx, Ly, Lz = dims
    m = np.asarray(spins, dtype=np.int64).reshape(-1, Lz, Ly, Lx)
    Jr = np.asarray(J, dtype=np.int64).reshape(3, Lz, Ly, Lx)
    e = np.zeros(m.shape[0], dtype=np.int64)
    for d, axis in ((0, 3), (1, 2), (2, 1)):
        e -= (Jr[d][None] * m * np.roll(m, -1, axis=axis)).sum(axis=(1, 2, 3))
    if h is not None:
        e -= (np.asarray(h, np.int64).reshape(1, Lz, Ly, Lx) * m).sum(axis=(1, 2, 3))
    return e


def all_states(N):
    """All 2^N configurations, row k has spin i = +1 iff bit i of k is 0."""
    k = np.arange(2 ** N, dtype=np.int64)[:, None]
    bits = (k >> np.arange(N, dtype=np.int64)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)


def state_index(spins):
    """Inverse of all_states: index of each configuration row."""
    bits = (np.asarray(spins, dtype=np.int64) < 0).astype(np.int64)
    return (bits << np.arange(bits.shape[1], dtype=np.int64)[None, :]).sum(axis=1)


def boltzmann(energies, beta):
    w = np.exp(-beta * (energies - energies.min()))
    return w / w.sum()
