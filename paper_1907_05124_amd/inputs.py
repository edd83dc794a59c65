"""Seeded synthetic Ising instances and inputs.

This module only *makes inputs*: coupling matrices, sparse graphs, lattice
bonds, spin vectors and schedule parameters, all drawn from NumPy's
``default_rng`` with an explicit seed.  It contains none of the method's
arithmetic (no fields, no annealing, no energies), so both the CPU oracle
tests and the GPU library's tests may use it.

Instance families follow the paper's workloads:

* Sherrington-Kirkpatrick (SK) couplings: symmetric, zero diagonal, iid
  Gaussian off-diagonal entries (paper, section "Ising Spin Glass Model",
  eq. (2) and the sentence after it).  The variance is a parameter; the
  workloads here use 1/N so that local fields are O(1).
* Erdos-Renyi max-cut graphs with unit or +-1 edge weights, stored as CSR
  with couplings J = -w (section "MAX-CUT" and eq. (3); the G-set random
  graphs have densities of a few percent and weights in {+1, -1}).
* Edwards-Anderson +-J lattices with periodic boundaries in 2D and 3D
  (section "Ising Spin Glass Model", first paragraph).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# instance containers
# ----------------------------------------------------------------------------


@dataclass
class DenseInstance:
    """Dense symmetric couplings ``J`` (N x N, float32, zero diagonal) and field ``h``."""

    J: np.ndarray
    h: np.ndarray | None = None

    @property
    def N(self) -> int:
        return int(self.J.shape[0])


@dataclass
class CsrInstance:
    """Sparse symmetric integer couplings in CSR form (sorted columns, no self loops)."""

    N: int
    rowptr: np.ndarray  # int32 [N+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # int8 [nnz]
    h: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


@dataclass
class LatticeInstance:
    """Hypercubic +-J lattice with periodic boundaries.

    Site index ``i = x0 + L0*(x1 + L1*x2)`` (x0 fastest).  ``bond[a, i]`` is
    the coupling between site ``i`` and its neighbour one step along axis
    ``a`` in the positive direction (wrapping around).
    """

    L: tuple
    bond: np.ndarray  # int8 [dim, N]
    h: np.ndarray | None = None

    @property
    def dim(self) -> int:
        return len(self.L)

    @property
    def N(self) -> int:
        return int(np.prod(self.L))


@dataclass
class Schedule:
    """Annealing schedule parameters (mirrors ``mars_schedule`` in include/mars.h)."""

    kind: str = "geometric"  # "geometric" | "linear"
    T_lo: float = 0.5
    T_hi: float = 3.0
    T_end: float = 0.02
    c_step: float = 1.0
    steps: int = 300
    max_sweeps: int = 1
    d_min: float = 1e-4
    update: str = "phased"  # "phased" | "jacobi" | "sequential" (dense fp32: every spin its own phase)
    phases: int = 2
    damping: float = 1.0
    precision: str = "fp32"  # "fp64" | "fp32" | "bf16" | "fp16"
    first_level: int = 0
    level_count: int = -1  # -1: all levels from first_level on

    def replace(self, **kw) -> "Schedule":
        d = dict(self.__dict__)
        d.update(kw)
        return Schedule(**d)


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------


def sk_instance(N: int, seed: int, variance: float | None = None, field_scale: float = 0.0) -> DenseInstance:
    """SK couplings: J_ij = J_ji ~ N(0, variance) for i < j, J_ii = 0 (float32).

    ``variance`` defaults to 1/N.  With ``field_scale > 0`` a Gaussian external
    field h_i ~ N(0, field_scale^2) is added (float32)."""
    if variance is None:
        variance = 1.0 / N
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((N, N)) * math.sqrt(variance)
    up = np.triu(g, 1)
    J = (up + up.T).astype(np.float32)
    np.fill_diagonal(J, 0.0)
    h = None
    if field_scale > 0.0:
        h = (rng.standard_normal(N) * field_scale).astype(np.float32)
    return DenseInstance(J=J, h=h)


def er_instance(N: int, seed: int, *, p: float | None = None, avg_degree: float | None = None,
                weights: str = "unit") -> CsrInstance:
    """Erdos-Renyi graph as a max-cut instance, CSR with J = -w.

    Exactly one of ``p`` (edge density) or ``avg_degree`` is given.  Edges are
    drawn independently for each unordered pair with probability p.  Weights
    are +1 (``"unit"``) or uniform +-1 (``"pm1"``)."""
    if (p is None) == (avg_degree is None):
        raise ValueError("give exactly one of p, avg_degree")
    if p is None:
        p = avg_degree / (N - 1)
    rng = np.random.default_rng(seed)
    m_expect = p * N * (N - 1) / 2
    if N <= 4096:
        iu, ju = np.triu_indices(N, 1)
        keep = rng.random(iu.shape[0]) < p
        ei, ej = iu[keep], ju[keep]
    else:
        # sample the number of edges, then distinct unordered pairs
        m = rng.binomial(N * (N - 1) // 2, p)
        pairs = set()
        while len(pairs) < m:
            a = rng.integers(0, N, size=2 * (m - len(pairs)) + 16)
            b = rng.integers(0, N, size=a.shape[0])
            for x, y in zip(a.tolist(), b.tolist()):
                if x == y:
                    continue
                if x > y:
                    x, y = y, x
                pairs.add((x, y))
                if len(pairs) >= m:
                    break
        arr = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
        ei, ej = arr[:, 0], arr[:, 1]
    del m_expect
    if weights == "unit":
        w = np.ones(ei.shape[0], dtype=np.int8)
    elif weights == "pm1":
        w = np.where(rng.random(ei.shape[0]) < 0.5, 1, -1).astype(np.int8)
    else:
        raise ValueError(weights)
    return csr_from_edges(N, ei, ej, (-w).astype(np.int8))


def csr_from_edges(N: int, ei: np.ndarray, ej: np.ndarray, val: np.ndarray) -> CsrInstance:
    """Symmetric CSR (both directions stored, columns sorted) from an undirected edge list."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    val = np.asarray(val, dtype=np.int8)
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([val, val])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(N + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return CsrInstance(N=N, rowptr=rowptr, col=cols.astype(np.int32), val=vals.astype(np.int8))


def lattice_instance(L, seed: int, *, ferro: bool = False) -> LatticeInstance:
    """Edwards-Anderson +-J lattice: each bond uniform in {+1, -1} (or all +1 if ``ferro``)."""
    L = tuple(int(x) for x in L)
    N = int(np.prod(L))
    rng = np.random.default_rng(seed)
    if ferro:
        bond = np.ones((len(L), N), dtype=np.int8)
    else:
        bond = np.where(rng.random((len(L), N)) < 0.5, 1, -1).astype(np.int8)
    return LatticeInstance(L=L, bond=bond)


def lattice_neighbour(L, i: int, axis: int, step: int) -> int:
    """Index of the site one step (+1 or -1) along ``axis`` from site ``i`` (periodic)."""
    coords = []
    rem = i
    for a in range(len(L)):
        coords.append(rem % L[a])
        rem //= L[a]
    coords[axis] = (coords[axis] + step) % L[axis]
    idx = 0
    for a in reversed(range(len(L))):
        idx = idx * L[a] + coords[a]
    return idx


def lattice_dense(inst: LatticeInstance) -> DenseInstance:
    """The same lattice written out as a dense float32 coupling matrix."""
    N = inst.N
    J = np.zeros((N, N), dtype=np.float32)
    for a in range(inst.dim):
        for i in range(N):
            j = lattice_neighbour(inst.L, i, a, +1)
            J[i, j] += inst.bond[a, i]
            J[j, i] += inst.bond[a, i]
    return DenseInstance(J=J, h=inst.h)


def csr_dense(inst: CsrInstance) -> DenseInstance:
    """The same sparse instance written out as a dense float32 coupling matrix."""
    N = inst.N
    J = np.zeros((N, N), dtype=np.float32)
    for i in range(N):
        a, b = inst.rowptr[i], inst.rowptr[i + 1]
        J[i, inst.col[a:b]] = inst.val[a:b]
    return DenseInstance(J=J, h=inst.h)


def random_spins(N: int, R: int, seed: int) -> np.ndarray:
    """Uniform random +-1 spins, run-major [R, N] int8."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((R, N)) < 0.5, 1, -1).astype(np.int8)


def random_magnetisation(N: int, R: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Uniform magnetisations in (-1, 1), spin-major [N, R] (runs contiguous)."""
    rng = np.random.default_rng(seed)
    return (rng.random((N, R)) * 2.0 - 1.0).astype(dtype)


def random_temperatures(R: int, seed: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=R).astype(np.float64)


def field_scale(inst) -> float:
    """sigma_Phi = sqrt(mean_i sum_j J_ij^2): the scale of local fields for +-1 spins.

    Used only to place temperature ranges of synthetic workloads on the same
    relative scale across instance families."""
    if isinstance(inst, DenseInstance):
        J = inst.J.astype(np.float64)
        return float(math.sqrt(np.mean(np.sum(J * J, axis=1))))
    if isinstance(inst, CsrInstance):
        v = inst.val.astype(np.float64)
        return float(math.sqrt(np.sum(v * v) / inst.N))
    if isinstance(inst, LatticeInstance):
        b = inst.bond.astype(np.float64)
        return float(math.sqrt(2.0 * np.sum(b * b) / inst.N))
    raise TypeError(type(inst))


# ----------------------------------------------------------------------------
# named workloads (shapes of the paper's experiments, synthetic data)
# ----------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    instance: object
    runs: int
    schedule: Schedule
    notes: dict = field(default_factory=dict)


def workload(name: str, *, seed: int = 1) -> Workload:
    """Synthetic stand-ins for the paper's workload shapes.

    ``ea2d_L16``   2D +-J lattice 16x16 (N=256), 1024 runs, T0~U[0.5,3], 300 geometric levels to 0.02, fp64.
    ``ea2d_L4``    2D +-J lattice 4x4 (N=16): brute-force checkable.
    ``sk2000``     SK N=2000, J~N(0,1/N), 4096 runs, T0~U[0.25,1.5] sigma, 300 levels to 0.01 sigma, 2 phases.
    ``er800``      ER N=800 p=0.06 (+-1 weights), 8192 runs.
    ``er800u``     ER N=800 p=0.06 unit weights, 8192 runs.
    ``er20000``    ER N=20000 average degree 4 (+-1 weights), 8192 runs.
    ``ea3d_L32``   3D +-J lattice 32^3, 2048 runs, 1000 levels, fp16 magnetisation storage.
    """
    if name == "ea2d_L16":
        inst = lattice_instance((16, 16), seed)
        sch = Schedule(T_lo=0.5, T_hi=3.0, T_end=0.02, steps=300, precision="fp64")
        return Workload(name, inst, 1024, sch)
    if name == "ea2d_L4":
        inst = lattice_instance((4, 4), seed)
        sch = Schedule(T_lo=0.5, T_hi=3.0, T_end=0.02, steps=300, precision="fp64")
        return Workload(name, inst, 1024, sch)
    if name == "sk2000":
        inst = sk_instance(2000, seed)
        s = field_scale(inst)
        sch = Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, phases=2, precision="fp32")
        return Workload(name, inst, 4096, sch, {"sigma_phi": s})
    if name in ("er800", "er800u"):
        inst = er_instance(800, seed, p=0.06, weights="pm1" if name == "er800" else "unit")
        s = field_scale(inst)
        sch = Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, precision="fp32")
        return Workload(name, inst, 8192, sch, {"sigma_phi": s})
    if name == "er20000":
        inst = er_instance(20000, seed, avg_degree=4.0, weights="pm1")
        s = field_scale(inst)
        sch = Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, precision="fp32")
        return Workload(name, inst, 8192, sch, {"sigma_phi": s})
    if name == "ea3d_L32":
        inst = lattice_instance((32, 32, 32), seed)
        s = field_scale(inst)
        sch = Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=1000, precision="fp16")
        return Workload(name, inst, 2048, sch, {"sigma_phi": s})
    raise KeyError(name)
