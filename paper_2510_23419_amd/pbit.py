"""ctypes binding of libpbit (the MI355X p-bit sweep library).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
libpbit.so.  The functions keep the C names; see ``include/pbit.h`` for the
meaning of every argument, the layouts and the error codes.  If the library is
not built, loading fails with an error; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libpbit.so"

PBIT_OK = 0
PBIT_PENDING = 1
PBIT_E_ARG = -1
PBIT_E_COLOURING = -2
PBIT_E_RANGE = -3
PBIT_E_NOMEM = -4
PBIT_E_BUSY = -5
PBIT_E_HANDLE = -6
PBIT_E_DEVICE = -7
PBIT_E_UNSUPPORTED = -8

PBIT_EA3D = 1
PBIT_BICLIQUE = 2
PBIT_GRAPH = 3
PBIT_CHECK_SWEEPS = 100
PBIT_NOALLOC_SCRATCH_BYTES = 64 << 20
PBIT_PROBE_PHILOX = 1
PBIT_PROBE_COPY = 2
PBIT_PROBE_MFMA = 3

EXPORTS = ("pbit_create", "pbit_destroy", "pbit_last_error", "pbit_bytes_in_use", "pbit_load_problem",
           "pbit_unload_problem", "pbit_problem_spins", "pbit_anneal", "pbit_anneal_dev", "pbit_energy",
           "pbit_submit", "pbit_poll", "pbit_progress", "pbit_threshold_table", "pbit_version",
           "pbit_profile_enable", "pbit_profile_read", "pbit_anneal_batch", "pbit_serve_config",
           "pbit_load_graph", "pbit_problem_colouring", "pbit_greedy_colouring", "pbit_profile_variant",
           "pbit_profile_ea_path", "pbit_anneal_dev_noalloc", "pbit_probe", "pbit_profile_graph", "pbit_profile_tiles",
           "pbit_profile_graph_path")


class PbitError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (code %d)" % (message, code))
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dims", ctypes.c_int32 * 3),
                ("J", ctypes.c_void_p), ("h", ctypes.c_void_p)]


class AnnealDesc(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("n_sweeps", ctypes.c_int32), ("sweep_offset", ctypes.c_int32),
                ("n_replicas", ctypes.c_int32), ("replica_offset", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("init_spins", ctypes.c_void_p), ("trace_every", ctypes.c_int32), ("has_target", ctypes.c_int32),
                ("target_energy", ctypes.c_int64)]


class Result(ctypes.Structure):  # noqa: E302
    _fields_ = [("spins", ctypes.c_void_p), ("energies", ctypes.c_void_p), ("best_energy", ctypes.c_int64),
                ("best_replica", ctypes.c_int32), ("sweeps_done", ctypes.c_int32),
                ("energy_trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int32), ("trace_len", ctypes.c_int32),
                ("spin_trace", ctypes.c_void_p)]


class GraphDesc(ctypes.Structure):
    _fields_ = [("n_spins", ctypes.c_int32), ("n_bonds", ctypes.c_int32), ("bond_i", ctypes.c_void_p),
                ("bond_j", ctypes.c_void_p), ("bond_J", ctypes.c_void_p), ("h", ctypes.c_void_p),
                ("colour", ctypes.c_void_p), ("n_colours", ctypes.c_int32)]


class BatchJob(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_uint64), ("desc", ctypes.POINTER(AnnealDesc)),
                ("result", ctypes.POINTER(Result))]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpbit.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError("libpbit.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libpbit bind to that one copy, so that one process holds
        # a single HIP runtime and torch's memory and streams are valid here.
        import torch  # noqa: F401
        L = ctypes.CDLL(str(LIB_PATH))
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "pbit_create": ([ctypes.POINTER(P), ctypes.c_int, u64], ctypes.c_int),
            "pbit_destroy": ([P], None),
            "pbit_last_error": ([], ctypes.c_char_p),
            "pbit_bytes_in_use": ([P], u64),
            "pbit_load_problem": ([P, ctypes.POINTER(ProblemDesc), ctypes.POINTER(u64)], ctypes.c_int),
            "pbit_unload_problem": ([P, u64], ctypes.c_int),
            "pbit_problem_spins": ([P, u64], i64),
            "pbit_anneal": ([P, u64, ctypes.POINTER(AnnealDesc), ctypes.POINTER(Result)], ctypes.c_int),
            "pbit_anneal_dev": ([P, u64, ctypes.POINTER(AnnealDesc), P, i32, P, P], ctypes.c_int),
            "pbit_anneal_dev_noalloc": ([P, u64, ctypes.POINTER(AnnealDesc), P, i32, P, P], ctypes.c_int),
            "pbit_probe": ([P, i32, i64, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                           ctypes.c_int),
            "pbit_energy": ([P, u64, P, i32, P], ctypes.c_int),
            "pbit_submit": ([P, u64, ctypes.POINTER(AnnealDesc), ctypes.POINTER(u64)], ctypes.c_int),
            "pbit_poll": ([P, u64, ctypes.POINTER(Result)], ctypes.c_int),
            "pbit_progress": ([P], ctypes.c_int),
            "pbit_threshold_table": ([P, i32, i32, P], ctypes.c_int),
            "pbit_version": ([], ctypes.c_char_p),
            "pbit_profile_enable": ([P, i32], ctypes.c_int),
            "pbit_profile_read": ([P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32], ctypes.c_int),
            "pbit_profile_variant": ([P, ctypes.POINTER(i32)], ctypes.c_int),
            "pbit_profile_graph_path": ([P, ctypes.POINTER(i32)], ctypes.c_int),
            "pbit_profile_ea_path": ([P, ctypes.POINTER(i32)], ctypes.c_int),
            "pbit_profile_graph": ([P, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
            "pbit_profile_tiles": ([P, ctypes.POINTER(i64), ctypes.POINTER(i32)], ctypes.c_int),
            "pbit_anneal_batch": ([P, ctypes.POINTER(BatchJob), i32], ctypes.c_int),
            "pbit_serve_config": ([P, i32, i32, i32], ctypes.c_int),
            "pbit_load_graph": ([P, ctypes.POINTER(GraphDesc), ctypes.POINTER(u64)], ctypes.c_int),
            "pbit_problem_colouring": ([P, u64, P, ctypes.POINTER(i32)], ctypes.c_int),
            "pbit_greedy_colouring": ([i32, i32, P, P, P, ctypes.POINTER(i32)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise PbitError(rc, lib().pbit_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- C-named calls

def pbit_version() -> str:
    return lib().pbit_version().decode()


def pbit_create(device: int = 0, hbm_budget_bytes: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib().pbit_create(ctypes.byref(ctx), int(device), int(hbm_budget_bytes)))
    return ctx


def pbit_destroy(ctx) -> None:
    lib().pbit_destroy(ctx)


def pbit_bytes_in_use(ctx) -> int:
    return int(lib().pbit_bytes_in_use(ctx))


def _problem_desc(kind, dims, J, h):
    J = np.ascontiguousarray(J, dtype=np.int8)
    h = None if h is None else np.ascontiguousarray(h, dtype=np.int8)
    d = ProblemDesc()
    d.kind = int(kind)
    dd = list(dims) + [0] * (3 - len(dims))
    for k in range(3):
        d.dims[k] = int(dd[k])
    d.J = J.ctypes.data
    d.h = None if h is None else h.ctypes.data
    return d, (J, h)


def pbit_load_problem(ctx, kind: int, dims, J, h=None) -> int:
    d, keep = _problem_desc(kind, dims, J, h)
    out = ctypes.c_uint64()
    _check(lib().pbit_load_problem(ctx, ctypes.byref(d), ctypes.byref(out)))
    del keep
    return int(out.value)


def pbit_load_graph(ctx, n_spins: int, bond_i, bond_j, bond_J, h=None, colour=None, n_colours: int = 0) -> int:
    bi = np.ascontiguousarray(bond_i, dtype=np.int32)
    bj = np.ascontiguousarray(bond_j, dtype=np.int32)
    bJ = np.ascontiguousarray(bond_J, dtype=np.int8)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.int8)
    col = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
    d = GraphDesc(int(n_spins), int(bi.size), bi.ctypes.data if bi.size else None, bj.ctypes.data if bj.size else None,
                  bJ.ctypes.data if bJ.size else None, None if hh is None else hh.ctypes.data,
                  None if col is None else col.ctypes.data, int(n_colours))
    out = ctypes.c_uint64()
    _check(lib().pbit_load_graph(ctx, ctypes.byref(d), ctypes.byref(out)))
    del bi, bj, bJ, hh, col
    return int(out.value)


def pbit_problem_colouring(ctx, problem: int):
    """(colour[N] uint8, number of colours) of a loaded problem."""
    N = pbit_problem_spins(ctx, problem)
    col = np.zeros(N, np.uint8)
    nc = ctypes.c_int32()
    _check(lib().pbit_problem_colouring(ctx, int(problem), _ptr(col), ctypes.byref(nc)))
    return col, int(nc.value)


def pbit_greedy_colouring(n: int, bond_i, bond_j):
    bi = np.ascontiguousarray(bond_i, dtype=np.int32)
    bj = np.ascontiguousarray(bond_j, dtype=np.int32)
    col = np.zeros(int(n), np.uint8)
    nc = ctypes.c_int32()
    _check(lib().pbit_greedy_colouring(int(n), int(bi.size), _ptr(bi) if bi.size else None,
                                       _ptr(bj) if bj.size else None, _ptr(col), ctypes.byref(nc)))
    return col, int(nc.value)


def load_instance(ctx, inst) -> int:
    """Load a problem dict as produced by the synthetic generators."""
    if inst["kind"] == "graph":
        return pbit_load_graph(ctx, inst["n"], inst["bond_i"], inst["bond_j"], inst["bond_J"], inst.get("h"),
                               inst.get("colour"), inst.get("n_colours", 0))
    kind = PBIT_EA3D if inst["kind"] == "ea3d" else PBIT_BICLIQUE
    return pbit_load_problem(ctx, kind, inst["dims"], inst["J"], inst.get("h"))


def pbit_unload_problem(ctx, problem: int) -> None:
    _check(lib().pbit_unload_problem(ctx, int(problem)))


def pbit_problem_spins(ctx, problem: int) -> int:
    return int(_check(lib().pbit_problem_spins(ctx, int(problem))))


def _anneal_desc(beta, n_replicas, seed, sweep_offset=0, replica_offset=0, init_spins=None, trace_every=0,
                 target=None):
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
    init = None if init_spins is None else np.ascontiguousarray(init_spins, dtype=np.int8)
    d = AnnealDesc()
    d.beta = beta.ctypes.data if beta.size else None
    d.n_sweeps = beta.size
    d.sweep_offset = int(sweep_offset)
    d.n_replicas = int(n_replicas)
    d.replica_offset = int(replica_offset)
    d.seed = int(seed) & (2**64 - 1)
    d.init_spins = None if init is None else init.ctypes.data
    d.trace_every = int(trace_every)
    d.has_target = 0 if target is None else 1
    d.target_energy = 0 if target is None else int(target)
    return d, (beta, init)


class AnnealOutput:
    def __init__(self, spins, energies, best_energy, best_replica, sweeps_done, energy_trace, spin_trace):
        self.spins = spins
        self.energies = energies
        self.best_energy = best_energy
        self.best_replica = best_replica
        self.sweeps_done = sweeps_done
        self.energy_trace = energy_trace
        self.spin_trace = spin_trace


def _result_buffers(R, N, S, trace_every, want_spins, trace_spins):
    spins = np.zeros((R, N), np.int8) if want_spins else None
    energies = np.zeros(R, np.int64)
    cap = S // trace_every if trace_every > 0 else 0
    etrace = np.zeros((cap, R), np.int64) if cap else None
    strace = np.zeros((cap, R, N), np.int8) if (cap and trace_spins) else None
    res = Result()
    res.spins = None if spins is None else spins.ctypes.data
    res.energies = energies.ctypes.data
    res.energy_trace = None if etrace is None else etrace.ctypes.data
    res.trace_cap = cap
    res.spin_trace = None if strace is None else strace.ctypes.data
    return res, spins, energies, etrace, strace


def _output(res, spins, energies, etrace, strace):
    n = res.trace_len
    return AnnealOutput(spins, energies, int(res.best_energy), int(res.best_replica), int(res.sweeps_done),
                        None if etrace is None else etrace[:n], None if strace is None else strace[:n])


def pbit_anneal(ctx, problem: int, beta, n_replicas: int, seed: int, sweep_offset: int = 0, replica_offset: int = 0,
                init_spins=None, trace_every: int = 0, target=None, want_spins: bool = True,
                trace_spins: bool = False) -> AnnealOutput:
    N = pbit_problem_spins(ctx, problem)
    d, keep = _anneal_desc(beta, n_replicas, seed, sweep_offset, replica_offset, init_spins, trace_every, target)
    res, spins, energies, etrace, strace = _result_buffers(int(n_replicas), N, d.n_sweeps, int(trace_every),
                                                           want_spins, trace_spins)
    _check(lib().pbit_anneal(ctx, int(problem), ctypes.byref(d), ctypes.byref(res)))
    del keep
    return _output(res, spins, energies, etrace, strace)


def pbit_anneal_dev(ctx, problem: int, beta, n_replicas: int, seed: int, d_spins, spins_in: bool = False,
                    d_energies=None, stream=None, sweep_offset: int = 0, replica_offset: int = 0,
                    noalloc: bool = False) -> None:
    """Device-buffer anneal.  ``d_spins`` (int8 [R][N]) and ``d_energies``
    (int64 [R]) are torch CUDA tensors; the work runs on ``stream`` (a torch
    stream, default: torch's current stream) and is finished on return.  With
    ``noalloc`` the call goes to pbit_anneal_dev_noalloc (working buffers in the
    library's static device array)."""
    import torch

    N = pbit_problem_spins(ctx, problem)
    R = int(n_replicas)
    if d_spins.dtype != torch.int8 or not d_spins.is_cuda or not d_spins.is_contiguous() or d_spins.numel() != R * N:
        raise ValueError("d_spins must be a contiguous int8 CUDA tensor of R*N elements")
    if d_energies is not None and (d_energies.dtype != torch.int64 or not d_energies.is_cuda
                                   or d_energies.numel() != R):
        raise ValueError("d_energies must be an int64 CUDA tensor of R elements")
    st = stream if stream is not None else torch.cuda.current_stream(d_spins.device)
    d, keep = _anneal_desc(beta, R, seed, sweep_offset, replica_offset)
    fn = lib().pbit_anneal_dev_noalloc if noalloc else lib().pbit_anneal_dev
    _check(fn(ctx, int(problem), ctypes.byref(d), ctypes.c_void_p(d_spins.data_ptr()), 1 if spins_in else 0,
              None if d_energies is None else ctypes.c_void_p(d_energies.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    del keep


def pbit_energy(ctx, problem: int, spins) -> np.ndarray:
    s = np.ascontiguousarray(spins, dtype=np.int8)
    N = pbit_problem_spins(ctx, problem)
    s = s.reshape(-1, N)
    out = np.zeros(s.shape[0], np.int64)
    _check(lib().pbit_energy(ctx, int(problem), _ptr(s), s.shape[0], _ptr(out)))
    return out


def pbit_profile_enable(ctx, every: int) -> None:
    _check(lib().pbit_profile_enable(ctx, int(every)))


def pbit_profile_read(ctx, kind: int, reset: bool = False):
    """(device milliseconds, launches) of the bracketed half-sweep launches of a problem kind."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().pbit_profile_read(ctx, int(kind), ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return float(ms.value), int(n.value)


def pbit_profile_variant(ctx) -> int:
    """Biclique half-sweep kernel variant of the latest biclique anneal (0: none yet)."""
    v = ctypes.c_int32(0)
    _check(lib().pbit_profile_variant(ctx, ctypes.byref(v)))
    return int(v.value)


def pbit_profile_graph_path(ctx) -> int:
    """General-graph path of the latest graph anneal: 1 one launch per colour class, 2
    LDS-resident tiles for runs of sweeps (0: none yet)."""
    v = ctypes.c_int32(0)
    _check(lib().pbit_profile_graph_path(ctx, ctypes.byref(v)))
    return int(v.value)


def pbit_probe(ctx, probe: int, size: int, reps: int = 20):
    """Mean launch time (ms) and work per launch of a ceiling kernel (PBIT_PROBE_*)."""
    ms, work = ctypes.c_double(), ctypes.c_double()
    _check(lib().pbit_probe(ctx, int(probe), int(size), int(reps), ctypes.byref(ms), ctypes.byref(work)))
    return ms.value, work.value


def pbit_threshold_table(beta, A: int) -> np.ndarray:
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
    out = np.zeros((beta.size, int(A) + 1), np.uint32)
    _check(lib().pbit_threshold_table(_ptr(beta), beta.size, int(A), _ptr(out)))
    return out


def pbit_profile_graph(ctx):
    """(captures, graph launches) of pbit_anneal_dev's sweep graph on this context."""
    c, n = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().pbit_profile_graph(ctx, ctypes.byref(c), ctypes.byref(n)))
    return c.value, n.value


def pbit_profile_tiles(ctx):
    """(tile timings run, cached tile shapes) of the batched engine on this context."""
    t, n = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().pbit_profile_tiles(ctx, ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def pbit_profile_ea_path(ctx) -> int:
    """Cube path of the latest cube anneal: 1 streaming stencil, 2 LDS-resident (0: none yet)."""
    v = ctypes.c_int32(0)
    _check(lib().pbit_profile_ea_path(ctx, ctypes.byref(v)))
    return int(v.value)


def pbit_submit(ctx, problem: int, beta, n_replicas: int, seed: int, sweep_offset: int = 0, replica_offset: int = 0,
                init_spins=None, trace_every: int = 0, target=None) -> int:
    d, keep = _anneal_desc(beta, n_replicas, seed, sweep_offset, replica_offset, init_spins, trace_every, target)
    out = ctypes.c_uint64()
    _check(lib().pbit_submit(ctx, int(problem), ctypes.byref(d), ctypes.byref(out)))
    del keep
    return int(out.value)


def pbit_poll(ctx, job: int, n_replicas: int, n_spins: int, n_sweeps: int = 0, trace_every: int = 0,
              want_spins: bool = True):
    """Returns None while the job is pending, else an AnnealOutput."""
    res, spins, energies, etrace, strace = _result_buffers(int(n_replicas), int(n_spins), int(n_sweeps),
                                                           int(trace_every), want_spins, False)
    rc = _check(lib().pbit_poll(ctx, int(job), ctypes.byref(res)))
    if rc == PBIT_PENDING:
        return None
    return _output(res, spins, energies, etrace, strace)


def pbit_progress(ctx) -> None:
    _check(lib().pbit_progress(ctx))


def pbit_serve_config(ctx, max_queue: int = 0, max_running: int = 0, round_sweeps: int = 0) -> None:
    _check(lib().pbit_serve_config(ctx, int(max_queue), int(max_running), int(round_sweeps)))


def pbit_anneal_batch(ctx, jobs, want_spins: bool = True):
    """Run many jobs in the persistent batched kernels.  ``jobs`` is a list of
    dicts with keys problem, beta, n_replicas, seed and optionally
    sweep_offset, replica_offset, init_spins, trace_every, target.  Returns one
    AnnealOutput per job."""
    n = len(jobs)
    arr = (BatchJob * max(n, 1))()
    keep, outs = [], []
    for k, jb in enumerate(jobs):
        N = pbit_problem_spins(ctx, jb["problem"])
        d, kd = _anneal_desc(jb["beta"], jb["n_replicas"], jb["seed"], jb.get("sweep_offset", 0),
                             jb.get("replica_offset", 0), jb.get("init_spins"), jb.get("trace_every", 0),
                             jb.get("target"))
        S = len(np.asarray(jb["beta"]).reshape(-1))
        res, spins, energies, etrace, strace = _result_buffers(int(jb["n_replicas"]), N, S,
                                                               int(jb.get("trace_every", 0)), want_spins, False)
        keep.append((d, kd, res))
        outs.append((res, spins, energies, etrace, strace))
        arr[k].problem = int(jb["problem"])
        arr[k].desc = ctypes.pointer(d)
        arr[k].result = ctypes.pointer(res)
    _check(lib().pbit_anneal_batch(ctx, arr, n))
    del keep
    return [_output(*o) for o in outs]


class Context:
    """Owns one libpbit context; closes it on exit."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ctx = pbit_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx:
            pbit_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
