"""Thin Python binding of the MARS HIP library (include/mars.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
binding fails loudly when the compiled library is missing; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from . import inputs as _inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libmars.so")

MARS_GEOMETRIC, MARS_LINEAR = 0, 1
MARS_PHASED, MARS_JACOBI, MARS_SEQUENTIAL = 0, 1, 2
_UPDATE = {"phased": MARS_PHASED, "jacobi": MARS_JACOBI, "sequential": MARS_SEQUENTIAL}
MARS_FP32, MARS_FP64, MARS_BF16, MARS_FP16 = 0, 1, 2, 3
_PRECISION = {"fp32": MARS_FP32, "fp64": MARS_FP64, "bf16": MARS_BF16, "fp16": MARS_FP16}

STATUS = {0: "MARS_OK", 1: "MARS_E_ARG", 2: "MARS_E_ASYMMETRIC", 3: "MARS_E_DIAGONAL", 4: "MARS_E_NONFINITE",
          5: "MARS_E_RANGE", 6: "MARS_E_OOM", 7: "MARS_E_DEVICE", 8: "MARS_E_UNSUPPORTED"}


class MarsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Schedule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("T_lo", C.c_double), ("T_hi", C.c_double), ("T_end", C.c_double),
                ("c_step", C.c_double), ("steps", C.c_int32), ("max_sweeps", C.c_int32), ("d_min", C.c_double),
                ("update", C.c_int32), ("phases", C.c_int32), ("damping", C.c_double),
                ("precision", C.c_int32), ("first_level", C.c_int32), ("level_count", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("best_energy", C.c_double), ("best_cut", C.c_double), ("mean_energy", C.c_double),
                ("best_T0", C.c_double), ("best_run", C.c_int32), ("runs", C.c_int32), ("hit_count", C.c_int64),
                ("sweeps_executed", C.c_int64), ("spin_updates", C.c_int64), ("cap_hits", C.c_int64),
                ("levels_executed", C.c_int64), ("seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["mars_create", "mars_create_csr", "mars_create_lattice", "mars_destroy", "mars_describe", "mars_solve",
           "mars_solve_ex", "mars_solve_async", "mars_solve_group_async", "mars_energy", "mars_energy_noalloc", "mars_spectrum",
           "mars_auto_temperatures", "mars_batch_create", "mars_batch_add", "mars_batch_step", "mars_batch_destroy", "mars_status_str",
           "mars_last_error"]

_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH):
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("MARS HIP library not built (%s); run __graft_entry__.build()" % path)
        L = C.CDLL(path)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        L.mars_create.argtypes = [vp, vp, i32, C.POINTER(vp)]
        L.mars_create_csr.argtypes = [i32, vp, vp, vp, vp, C.POINTER(vp)]
        L.mars_create_lattice.argtypes = [i32, vp, vp, vp, C.POINTER(vp)]
        L.mars_destroy.argtypes = [vp]
        L.mars_destroy.restype = None
        L.mars_describe.argtypes = [vp, C.POINTER(Schedule), C.POINTER(i32), C.POINTER(i32)]
        L.mars_solve.argtypes = [vp, i32, C.POINTER(Schedule), u64, vp, vp, C.POINTER(Result)]
        L.mars_solve_ex.argtypes = [vp, i32, C.POINTER(Schedule), u64, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                                    C.POINTER(Result), vp]
        L.mars_solve_async.argtypes = [vp, i32, C.POINTER(Schedule), u64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.mars_solve_group_async.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.mars_energy.argtypes = [vp, vp, i32, vp, vp]
        L.mars_energy_noalloc.argtypes = [vp, vp, i32, vp, vp]
        L.mars_spectrum.argtypes = [vp, i32, u64, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
        L.mars_auto_temperatures.argtypes = [vp, i32, u64, C.POINTER(Schedule), vp]
        L.mars_batch_create.argtypes = [vp, C.POINTER(vp)]
        L.mars_batch_add.argtypes = [vp, vp, i32, C.POINTER(Schedule), u64, C.c_int64, vp, vp]
        L.mars_batch_step.argtypes = [vp, i32, vp, i32, C.POINTER(i32), C.POINTER(i32)]
        L.mars_batch_destroy.argtypes = [vp]
        L.mars_batch_destroy.restype = None
        L.mars_status_str.argtypes = [C.c_int]
        L.mars_status_str.restype = C.c_char_p
        L.mars_last_error.argtypes = []
        L.mars_last_error.restype = C.c_char_p
        for f in ("mars_create", "mars_create_csr", "mars_create_lattice", "mars_describe", "mars_solve",
                  "mars_solve_ex", "mars_solve_async", "mars_solve_group_async", "mars_energy", "mars_energy_noalloc", "mars_spectrum",
                  "mars_auto_temperatures", "mars_batch_create", "mars_batch_add", "mars_batch_step"):
            getattr(L, f).restype = C.c_int
        _lib = L
        return L


def _check(status: int):
    if status != 0:
        msg = load().mars_last_error().decode(errors="replace")
        raise MarsError(status, msg)


def make_schedule(sc) -> Schedule:
    """ctypes schedule from an ``inputs.Schedule`` (or any object with its fields)."""
    s = Schedule()
    s.kind = MARS_GEOMETRIC if sc.kind == "geometric" else MARS_LINEAR
    s.T_lo, s.T_hi, s.T_end, s.c_step = float(sc.T_lo), float(sc.T_hi), float(sc.T_end), float(sc.c_step)
    s.steps, s.max_sweeps, s.d_min = int(sc.steps), int(sc.max_sweeps), float(sc.d_min)
    s.update = _UPDATE[sc.update]
    s.phases, s.damping = int(sc.phases), float(sc.damping)
    s.precision = _PRECISION[sc.precision]
    s.first_level, s.level_count = int(sc.first_level), int(sc.level_count)
    return s


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Instance:
    """An Ising instance resident on the current GPU."""

    def __init__(self, handle: C.c_void_p, N: int):
        self._h = handle
        self.N = N

    # -- construction -------------------------------------------------------
    @classmethod
    def dense(cls, J, h=None) -> "Instance":
        J = np.ascontiguousarray(J, dtype=np.float32)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float32)
        out = C.c_void_p()
        _check(load().mars_create(_ptr(J), _ptr(hh), int(J.shape[0]), C.byref(out)))
        return cls(out, int(J.shape[0]))

    @classmethod
    def csr(cls, N, rowptr, col, val, h=None) -> "Instance":
        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        co = np.ascontiguousarray(col, dtype=np.int32)
        va = np.ascontiguousarray(val, dtype=np.int8)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float32)
        out = C.c_void_p()
        _check(load().mars_create_csr(int(N), _ptr(rp), _ptr(co), _ptr(va), _ptr(hh), C.byref(out)))
        return cls(out, int(N))

    @classmethod
    def lattice(cls, L, bond, h=None) -> "Instance":
        Ls = np.ascontiguousarray(L, dtype=np.int32)
        b = np.ascontiguousarray(bond, dtype=np.int8)
        hh = None if h is None else np.ascontiguousarray(h, dtype=np.float32)
        out = C.c_void_p()
        _check(load().mars_create_lattice(int(Ls.shape[0]), _ptr(Ls), _ptr(b), _ptr(hh), C.byref(out)))
        return cls(out, int(np.prod(Ls)))

    @classmethod
    def from_inputs(cls, inst) -> "Instance":
        if isinstance(inst, _inputs.DenseInstance):
            return cls.dense(inst.J, inst.h)
        if isinstance(inst, _inputs.CsrInstance):
            return cls.csr(inst.N, inst.rowptr, inst.col, inst.val, inst.h)
        if isinstance(inst, _inputs.LatticeInstance):
            return cls.lattice(inst.L, inst.bond, inst.h)
        raise TypeError(type(inst))

    def close(self):
        if self._h:
            load().mars_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    # -- queries ------------------------------------------------------------
    def describe(self, schedule):
        n, p = C.c_int32(), C.c_int32()
        s = make_schedule(schedule)
        _check(load().mars_describe(self._h, C.byref(s), C.byref(n), C.byref(p)))
        return int(n.value), int(p.value)

    # -- solves -------------------------------------------------------------
    def solve(self, runs: int, schedule, seed: int):
        """Host outputs: (best_spins int8[N], energies float64[runs], result dict)."""
        best = np.empty(self.N, dtype=np.int8)
        E = np.empty(runs, dtype=np.float64)
        res = Result()
        s = make_schedule(schedule)
        _check(load().mars_solve(self._h, int(runs), C.byref(s), seed & (2**64 - 1), _ptr(best), _ptr(E),
                                 C.byref(res)))
        return best, E, res.as_dict()

    def solve_ex(self, runs: int, schedule, seed: int, *, m0=None, T0=None, want_T0=False, want_m=False,
                 want_spins=False, want_energies=True, want_best=True, levels_cap: int = 0, sync=True,
                 stream=None) -> dict:
        """Device outputs as torch tensors on the current device and stream.

        ``m0`` ([N, runs], float32, or float64 for fp64 schedules) and ``T0``
        ([runs] float64) are device tensors or None.  ``levels_cap`` > 0 adds
        ``sweeps_per_level`` ([runs, levels_cap] int32): the sweeps each run
        ran at each level it visited."""
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        mdt = torch.float64 if schedule.precision == "fp64" else torch.float32
        out = {}
        if want_T0:
            out["T0"] = torch.empty(runs, dtype=torch.float64, device=dev)
        if want_m:
            out["m"] = torch.empty((self.N, runs), dtype=mdt, device=dev)
        if want_spins:
            out["spins"] = torch.empty((runs, self.N), dtype=torch.int8, device=dev)
        if want_energies:
            out["energies"] = torch.empty(runs, dtype=torch.float64, device=dev)
        if want_best:
            out["best_spins"] = torch.empty(self.N, dtype=torch.int8, device=dev)
        if levels_cap > 0:
            out["sweeps_per_level"] = torch.empty((runs, levels_cap), dtype=torch.int32, device=dev)
        for name, t, dt in (("m0", m0, mdt), ("T0", T0, torch.float64)):
            if t is not None:
                if t.device.type != "cuda" or t.dtype != dt or not t.is_contiguous():
                    raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dt))
        if stream is None:
            stream = torch.cuda.current_stream()
        s = make_schedule(schedule)
        res = Result()
        _check(load().mars_solve_ex(self._h, int(runs), C.byref(s), seed & (2**64 - 1), _ptr(m0), _ptr(T0),
                                    _ptr(out.get("T0")), _ptr(out.get("m")), _ptr(out.get("spins")),
                                    _ptr(out.get("energies")), _ptr(out.get("best_spins")),
                                    _ptr(out.get("sweeps_per_level")), int(max(levels_cap, 0)),
                                    C.byref(res) if sync else None, C.c_void_p(stream.cuda_stream)))
        if sync:
            out["result"] = res.as_dict()
        return out

    def solve_async(self, runs: int, schedule, seed: int, result_buf, *, stream, want_energies=False,
                    want_best=True, want_spins=False) -> dict:
        """Enqueue a solve on `stream`; `result_buf` is a pinned uint8 tensor of
        at least sizeof(Result) bytes that receives the summary asynchronously.
        Returns the device output tensors (valid once the stream has passed)."""
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        out = {}
        if want_energies:
            out["energies"] = torch.empty(runs, dtype=torch.float64, device=dev)
        if want_best:
            out["best_spins"] = torch.empty(self.N, dtype=torch.int8, device=dev)
        if want_spins:
            out["spins"] = torch.empty((runs, self.N), dtype=torch.int8, device=dev)
        s = make_schedule(schedule)
        _check(load().mars_solve_async(self._h, int(runs), C.byref(s), seed & (2**64 - 1), None, None, None,
                                       _ptr(out.get("spins")), _ptr(out.get("energies")),
                                       _ptr(out.get("best_spins")), result_buf.data_ptr(),
                                       C.c_void_p(stream.cuda_stream)))
        return out

    @staticmethod
    def solve_group_async(members, result_buf, *, stream, want_energies=False, want_best=True) -> list:
        """mars_solve_group_async: `members` is a list of (Instance, runs,
        schedule, seed) lattice/sparse solves enqueued together on `stream`;
        `result_buf` a pinned uint8 tensor of at least len(members) *
        sizeof(Result) bytes (read_result(result_buf, i) decodes member i).
        Returns each member's device outputs (valid once the stream has
        passed the enqueued work)."""
        import torch

        n = len(members)
        if result_buf.numel() < n * C.sizeof(Result):
            raise ValueError("result_buf holds fewer than %d results" % n)
        dev = torch.device("cuda", torch.cuda.current_device())
        outs = []
        for inst, runs, _, _ in members:
            o = {}
            if want_energies:
                o["energies"] = torch.empty(int(runs), dtype=torch.float64, device=dev)
            if want_best:
                o["best_spins"] = torch.empty(inst.N, dtype=torch.int8, device=dev)
            outs.append(o)
        handles = (C.c_void_p * n)(*[m[0]._h for m in members])
        runs = (C.c_int32 * n)(*[int(m[1]) for m in members])
        scheds = (Schedule * n)(*[make_schedule(m[2]) for m in members])
        seeds = (C.c_uint64 * n)(*[int(m[3]) & (2**64 - 1) for m in members])
        best = (C.c_void_p * n)(*[_ptr(o.get("best_spins")) for o in outs])
        ens = (C.c_void_p * n)(*[_ptr(o.get("energies")) for o in outs])
        _check(load().mars_solve_group_async(n, handles, runs, scheds, seeds, best, ens, result_buf.data_ptr(),
                                             C.c_void_p(stream.cuda_stream)))
        return outs

    @staticmethod
    def read_result(result_buf, index: int = 0) -> dict:
        """Decode a pinned result buffer filled by solve_async (or member
        `index` of solve_group_async), after the stream passed it."""
        k = C.sizeof(Result)
        raw = bytes(result_buf.cpu().numpy()[index * k: (index + 1) * k])
        return Result.from_buffer_copy(raw).as_dict()

    def energy_noalloc(self, spins, energies):
        """mars_energy_noalloc: exact energies of device spins [R, N] int8 into
        the caller's float64 [R] tensor, with no device allocation by the
        library (current stream)."""
        import torch

        if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != self.N or not spins.is_contiguous():
            raise ValueError("spins must be a contiguous int8 [R, N] CUDA tensor")
        if energies.dtype != torch.float64 or energies.shape != (spins.shape[0],) or not energies.is_contiguous():
            raise ValueError("energies must be a contiguous float64 [R] CUDA tensor")
        _check(load().mars_energy_noalloc(self._h, _ptr(spins), int(spins.shape[0]), _ptr(energies),
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return energies

    def spectrum(self, steps: int = 100, seed: int = 1):
        """(lambda_min, lambda_max) of J by `steps` Lanczos steps on the device."""
        import torch

        lo, hi = C.c_double(), C.c_double()
        _check(load().mars_spectrum(self._h, int(steps), seed & (2**64 - 1), C.byref(lo), C.byref(hi),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return lo.value, hi.value

    def auto_temperatures(self, schedule, steps: int = 100, seed: int = 1):
        """`schedule` (an inputs.Schedule) with T_lo, T_hi, T_end set from the
        spectrum of J by the library (mars_auto_temperatures)."""
        import torch

        s = make_schedule(schedule)
        _check(load().mars_auto_temperatures(self._h, int(steps), seed & (2**64 - 1), C.byref(s),
                                             C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return schedule.replace(T_lo=s.T_lo, T_hi=s.T_hi, T_end=s.T_end)

    def energy(self, spins):
        """Exact energies of device spins [R, N] int8 -> float64 [R] (current stream)."""
        import torch

        if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != self.N or not spins.is_contiguous():
            raise ValueError("spins must be a contiguous int8 [R, N] CUDA tensor")
        E = torch.empty(spins.shape[0], dtype=torch.float64, device=spins.device)
        _check(load().mars_energy(self._h, _ptr(spins), int(spins.shape[0]), _ptr(E),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return E


class Batch:
    """Batched BF16 solver (mars_batch_*): dense instances solved in MARS_BF16
    with one sweep per level advance together on one stream, one launch per
    phase for all members; members join and leave at sweep boundaries."""

    MAX_MEMBERS = 16

    def __init__(self, stream):
        h = C.c_void_p()
        _check(load().mars_batch_create(C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        self._stream = stream
        self._keep = {}  # tag -> (instance, outputs) held until the member finishes

    def add(self, inst: Instance, runs: int, schedule, seed: int, tag: int, result_buf, *, want_best=True) -> dict:
        """Join a solve of `inst`; `result_buf` (pinned uint8, >= sizeof(Result))
        receives its summary when it finishes.  Returns the device outputs."""
        import torch

        if tag in self._keep:
            raise ValueError("tag %d is already in the batch" % tag)
        out = {}
        if want_best:
            out["best_spins"] = torch.empty(inst.N, dtype=torch.int8, device=torch.device("cuda", torch.cuda.current_device()))
        s = make_schedule(schedule)
        _check(load().mars_batch_add(self._h, inst._h, int(runs), C.byref(s), seed & (2**64 - 1), int(tag),
                                     _ptr(out.get("best_spins")), result_buf.data_ptr()))
        self._keep[tag] = (inst, out, result_buf)
        return out

    def step(self, sweeps: int, cap: int = 64):
        """Advance every member by up to `sweeps` sweeps; returns (tags of the
        members that finished, number still active)."""
        tags = (C.c_int64 * max(cap, 1))()
        nf, na = C.c_int32(), C.c_int32()
        _check(load().mars_batch_step(self._h, int(sweeps), tags, int(cap), C.byref(nf), C.byref(na)))
        done = [int(tags[i]) for i in range(nf.value)]
        for t in done:
            self._keep.pop(t, None)
        return done, na.value

    def __len__(self):
        return len(self._keep)

    def close(self):
        if self._h:
            load().mars_batch_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status_str(status: int) -> str:
    return load().mars_status_str(status).decode()
