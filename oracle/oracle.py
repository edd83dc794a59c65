"""ctypes binding for the MARS CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  The arithmetic lives in ``mars_oracle.c``; this file builds it
with gcc and marshals arguments.  Instances and schedules are duck-typed: any
object with the attributes of the containers in the input-generator module
works.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mars_oracle.c")
_OUT = os.path.join(_HERE, "_build", "libmars_oracle.so")
_lock = threading.Lock()
_lib = None

DENSE, CSR, LATTICE = 0, 1, 2
GEOMETRIC, LINEAR = 0, 1
PHASED, JACOBI = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off so every rounding is explicit)."""
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_OUT), exist_ok=True)
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


class _Inst(C.Structure):
    _fields_ = [("kind", C.c_int), ("N", C.c_int), ("J", C.c_void_p), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("dim", C.c_int), ("L", C.c_int * 3),
                ("bond", C.c_void_p), ("h", C.c_void_p)]


class _Sched(C.Structure):
    _fields_ = [("kind", C.c_int), ("T_lo", C.c_double), ("T_hi", C.c_double), ("T_end", C.c_double),
                ("c_step", C.c_double), ("steps", C.c_int), ("max_sweeps", C.c_int), ("d_min", C.c_double),
                ("update", C.c_int), ("phases", C.c_int), ("damping", C.c_double),
                ("first_level", C.c_int), ("level_count", C.c_int)]


def _bind(path):
    L = C.CDLL(path)
    L.orc_splitmix64.restype = C.c_uint64
    L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_initial_m.restype = C.c_double
    L.orc_initial_m.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
    L.orc_initial_T.restype = C.c_double
    L.orc_initial_T.argtypes = [C.c_uint64, C.c_int64, C.c_double, C.c_double]
    L.orc_exact_sum.restype = C.c_double
    L.orc_exact_sum.argtypes = [C.c_void_p, C.c_int64]
    L.orc_energy.restype = C.c_double
    L.orc_energy.argtypes = [C.POINTER(_Inst), C.c_void_p]
    L.orc_phases.restype = C.c_int
    L.orc_phases.argtypes = [C.POINTER(_Inst), C.POINTER(_Sched), C.c_void_p]
    L.orc_levels.restype = C.c_int
    L.orc_levels.argtypes = [C.POINTER(_Sched), C.c_double, C.c_void_p, C.c_int]
    L.orc_solve.restype = C.c_int
    L.orc_solve.argtypes = [C.POINTER(_Inst), C.POINTER(_Sched), C.c_uint64, C.c_int, C.c_int] + \
        [C.c_void_p] * 10 + [C.c_int]
    L.orc_solve_levels.restype = C.c_int
    L.orc_solve_levels.argtypes = [C.POINTER(_Inst), C.POINTER(_Sched), C.c_uint64, C.c_int, C.c_int] + \
        [C.c_void_p] * 10 + [C.c_int] + [C.c_void_p] * 4 + [C.c_int]
    L.orc_best.restype = C.c_int
    L.orc_best.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]
    return L


_override = None


def lib():
    global _lib
    if _override is not None:
        return _override
    with _lock:
        if _lib is None:
            _lib = _bind(build())
    return _lib


class use_library:
    """Context manager: route every call to another build of the oracle source
    (used by the tests that plant mistakes in a copy of the oracle)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _override
        _override = _bind(self.path)
        return _override

    def __exit__(self, *exc):
        global _override
        _override = None
        return False


def build_variant(source_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (same flags as build())."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-pthread", "-o", out_path, src, "-lm"])
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


# ----------------------------------------------------------------------------
# marshalling
# ----------------------------------------------------------------------------


class Instance:
    """Keeps the numpy buffers alive next to the C view of an instance."""

    def __init__(self, inst):
        self.keep = []
        s = _Inst()
        h = getattr(inst, "h", None)
        if hasattr(inst, "J"):
            J = np.ascontiguousarray(inst.J, dtype=np.float32)
            s.kind, s.N, s.J = DENSE, J.shape[0], J.ctypes.data
            self.keep.append(J)
        elif hasattr(inst, "rowptr"):
            rp = np.ascontiguousarray(inst.rowptr, dtype=np.int32)
            co = np.ascontiguousarray(inst.col, dtype=np.int32)
            va = np.ascontiguousarray(inst.val, dtype=np.int8)
            s.kind, s.N = CSR, int(inst.N)
            s.rowptr, s.col, s.val = rp.ctypes.data, co.ctypes.data, va.ctypes.data
            self.keep += [rp, co, va]
        elif hasattr(inst, "bond"):
            b = np.ascontiguousarray(inst.bond, dtype=np.int8)
            s.kind, s.N, s.dim = LATTICE, int(np.prod(inst.L)), len(inst.L)
            for a, x in enumerate(inst.L):
                s.L[a] = int(x)
            s.bond = b.ctypes.data
            self.keep.append(b)
        else:
            raise TypeError(type(inst))
        if h is not None:
            hh = np.ascontiguousarray(h, dtype=np.float32)
            s.h = hh.ctypes.data
            self.keep.append(hh)
        self.c = s
        self.N = s.N


def _sched(sc) -> _Sched:
    s = _Sched()
    s.kind = GEOMETRIC if sc.kind == "geometric" else LINEAR
    s.T_lo, s.T_hi, s.T_end, s.c_step = float(sc.T_lo), float(sc.T_hi), float(sc.T_end), float(sc.c_step)
    s.steps, s.max_sweeps, s.d_min = int(sc.steps), int(sc.max_sweeps), float(sc.d_min)
    if sc.update not in ("phased", "jacobi", "sequential"):
        raise ValueError("unknown update %r" % (sc.update,))
    s.update = JACOBI if sc.update == "jacobi" else PHASED
    s.phases, s.damping = int(sc.phases), float(sc.damping)
    if sc.update == "sequential":
        # every spin its own phase in index order (Algorithm 1 with the
        # per-spin assignment of the GPU description): phases = N, which the
        # dense phase rule reaches by clamping
        s.phases = 2**31 - 1
    s.first_level, s.level_count = int(sc.first_level), int(sc.level_count)
    return s


def _ptr(a):
    return None if a is None else a.ctypes.data


# ----------------------------------------------------------------------------
# API
# ----------------------------------------------------------------------------


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), counter & (2**64 - 1)))


def initial_m(seed: int, runs: int, N: int) -> np.ndarray:
    """Initial magnetisations, spin-major [N, runs] float64."""
    L = lib()
    out = np.empty((N, runs), dtype=np.float64)
    for r in range(runs):
        for i in range(N):
            out[i, r] = L.orc_initial_m(seed, r, i)
    return out


def initial_T(seed: int, runs: int, T_lo: float, T_hi: float) -> np.ndarray:
    L = lib()
    return np.array([L.orc_initial_T(seed, r, T_lo, T_hi) for r in range(runs)], dtype=np.float64)


def exact_sum(x) -> float:
    a = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_exact_sum(a.ctypes.data, a.shape[0]))


def energy(inst, spins) -> np.ndarray:
    """Exact energies of spin vectors; ``spins`` is [N] or run-major [R, N] of +-1."""
    ci = inst if isinstance(inst, Instance) else Instance(inst)
    s = np.ascontiguousarray(np.atleast_2d(spins), dtype=np.int8)
    L = lib()
    return np.array([L.orc_energy(C.byref(ci.c), s[r].ctypes.data) for r in range(s.shape[0])])


def phases(inst, sched):
    ci = inst if isinstance(inst, Instance) else Instance(inst)
    ph = np.empty(ci.N, dtype=np.int32)
    n = lib().orc_phases(C.byref(ci.c), C.byref(_sched(sched)), ph.ctypes.data)
    return ph, int(n)


def levels(sched, T0: float) -> np.ndarray:
    s = _sched(sched)
    n = lib().orc_levels(C.byref(s), float(T0), None, 0)
    out = np.empty(max(n, 1), dtype=np.float64)
    lib().orc_levels(C.byref(s), float(T0), out.ctypes.data, n)
    return out[:n]


def solve(inst, runs: int, sched, seed: int, *, run_begin: int = 0, run_count: int | None = None,
          m0=None, T0=None, nthreads: int | None = None, levels_cap: int = 0, replay=None) -> dict:
    """Run MARS on runs [run_begin, run_begin + run_count) of a ``runs``-run solve.

    Runs are independent, so any subset gives the same per-run results as the
    full solve.  ``m0`` ([N, run_count]) and ``T0`` ([run_count]) replace the
    generator's draws when given.

    ``levels_cap`` > 0 adds per-level records of the first ``levels_cap``
    visited levels of every run ([run_count, levels_cap] each; 0 past a run's
    levels): ``sweeps_per_level``, ``own_per_level`` (where the oracle's own
    stopping rule ends the level; count + 1 under replay when it would have
    gone on) and ``d_per_level`` (the largest change of that sweep).
    ``replay`` ([run_count, levels_cap] int32) runs exactly that many sweeps at
    each level (entries <= 0: the stopping rule) -- the sweep counts another
    implementation reports."""
    del runs  # per-run results do not depend on the total
    ci = inst if isinstance(inst, Instance) else Instance(inst)
    N = ci.N
    rc = int(run_count if run_count is not None else 0)
    if run_count is None:
        raise ValueError("run_count is required")
    m0a = None if m0 is None else np.ascontiguousarray(m0, dtype=np.float64).reshape(N, rc)
    T0a = None if T0 is None else np.ascontiguousarray(T0, dtype=np.float64).reshape(rc)
    out = {
        "m": np.empty((N, rc), dtype=np.float64),
        "spins": np.empty((rc, N), dtype=np.int8),
        "energy": np.empty(rc, dtype=np.float64),
        "T0": np.empty(rc, dtype=np.float64),
        "sweeps": np.empty(rc, dtype=np.int64),
        "levels": np.empty(rc, dtype=np.int64),
        "cap_hits": np.empty(rc, dtype=np.int64),
        "last_T": np.empty(rc, dtype=np.float64),
    }
    cap = int(levels_cap)
    rep = None
    if replay is not None:
        if cap < 1:
            raise ValueError("replay needs levels_cap")
        rep = np.ascontiguousarray(replay, dtype=np.int32).reshape(rc, cap)
    if cap > 0:
        out["sweeps_per_level"] = np.zeros((rc, cap), dtype=np.int32)
        out["own_per_level"] = np.zeros((rc, cap), dtype=np.int32)
        out["d_per_level"] = np.zeros((rc, cap), dtype=np.float64)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rcode = lib().orc_solve_levels(C.byref(ci.c), C.byref(_sched(sched)), seed & (2**64 - 1), int(run_begin), rc,
                                   _ptr(m0a), _ptr(T0a), out["m"].ctypes.data, out["spins"].ctypes.data,
                                   out["energy"].ctypes.data, out["T0"].ctypes.data, out["sweeps"].ctypes.data,
                                   out["levels"].ctypes.data, out["cap_hits"].ctypes.data,
                                   out["last_T"].ctypes.data, int(nthreads), _ptr(rep),
                                   _ptr(out.get("sweeps_per_level")), _ptr(out.get("own_per_level")),
                                   _ptr(out.get("d_per_level")), cap)
    if rcode != 0:
        raise RuntimeError("oracle solve failed")
    return out


def best(energies):
    e = np.ascontiguousarray(energies, dtype=np.float64)
    hits = C.c_int64(0)
    idx = lib().orc_best(e.ctypes.data, e.shape[0], C.byref(hits))
    return int(idx), int(hits.value)


def coupling_matrix(inst) -> np.ndarray:
    """J as a dense float64 matrix, written out from each container's
    definition: dense J as given; CSR entry (i, col[k]) = val[k]; lattice bond
    bond[a, i] couples site i (x0 fastest) with its neighbour one step along
    axis a in the positive direction, wrapping around (test infrastructure)."""
    if hasattr(inst, "J"):
        return np.asarray(inst.J, dtype=np.float64).copy()
    N = int(inst.N)
    M = np.zeros((N, N), dtype=np.float64)
    if hasattr(inst, "rowptr"):
        for i in range(N):
            for k in range(int(inst.rowptr[i]), int(inst.rowptr[i + 1])):
                M[i, int(inst.col[k])] += float(inst.val[k])
        return M
    L = tuple(int(x) for x in inst.L)
    strides = [1]
    for a in range(len(L) - 1):
        strides.append(strides[-1] * L[a])
    for i in range(N):
        for a in range(len(L)):
            xa = (i // strides[a]) % L[a]
            j = i + (((xa + 1) % L[a]) - xa) * strides[a]
            M[i, j] += float(inst.bond[a, i])
            M[j, i] += float(inst.bond[a, i])
    return M


def spectrum(inst):
    """(lambda_min, lambda_max) of J, from the symmetric eigensolver."""
    w = np.linalg.eigvalsh(coupling_matrix(inst))
    return float(w[0]), float(w[-1])
