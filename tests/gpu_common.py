"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import math
import sys

import numpy as np

from oracle import oracle as O


def require_gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU (run them with -m gpu on the GPU box)"
    return torch


def announce(*parts):
    """Name the case on stdout before a GPU step (flushed)."""
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()


UNIT = {"fp32": 2.0**-24, "fp64": 2.0**-53}
BASE = {"fp32": 1e-5, "fp64": 1e-9}


def amplification(inst, runs, sched, seed, ref, run_begin=0, trials=2, eps=1e-9):
    """Per-run growth of a tiny change of the initial state through the anneal,
    measured with the oracle alone: max_i |dm_i(final)| / eps over `trials`
    random +-eps perturbations of m0."""
    N = ref["m"].shape[0]
    rc = ref["m"].shape[1]
    m0 = np.empty((N, rc))
    for q in range(rc):
        for i in range(N):
            m0[i, q] = O.lib().orc_initial_m(seed, run_begin + q, i)
    A = np.zeros(rc)
    for t in range(trials):
        rng = np.random.default_rng(1000 + t)
        pert = np.clip(m0 + eps * np.where(rng.random(m0.shape) < 0.5, -1.0, 1.0), -1 + 1e-12, 1 - 1e-12)
        alt = O.solve(inst, runs, sched, seed, run_begin=run_begin, run_count=rc, m0=pert, T0=ref["T0"])
        A = np.maximum(A, np.max(np.abs(alt["m"] - ref["m"]), axis=0) / eps)
    return A


def dense_couplings(inst):
    from paper_1907_05124_amd import inputs as I

    if isinstance(inst, I.DenseInstance):
        return inst.J.astype(np.float64)
    if isinstance(inst, I.CsrInstance):
        return I.csr_dense(inst).J.astype(np.float64)
    return I.lattice_dense(inst).J.astype(np.float64)


def trajectory_tolerance(inst, ref, A, precision):
    """Elementwise bar for a GPU trajectory against the oracle, from the
    arithmetic of the GPU form (unit roundoff u):
        base                               the stated bar (1e-5 fp32, 1e-9 fp64)
      + 34 u * A_r                         per-level rounding (measured < 34 u at
                                           level 1) carried by the run's growth A_r
      + 4 u sqrt(N) S_ir (1 - m_ir^2) / T  rounding of the last level's field
                                           (S = sum_j |J_ij m_j|) through tanh at T
    Every quantity comes from the oracle, none from the GPU."""
    u = UNIT[precision]
    J = dense_couplings(inst)
    S = np.abs(J) @ np.abs(ref["m"])
    N = J.shape[0]
    T = ref["last_T"][None, :]
    T = np.where(np.isfinite(T), T, np.inf)
    return BASE[precision] + 34 * u * A[None, :] + 4 * u * np.sqrt(N) * S * (1 - ref["m"] ** 2) / T


def check_trajectory(m_gpu, inst, runs, sched, seed, ref, precision, run_begin=0, spins=None):
    """Assert |m_gpu - m_oracle| <= trajectory_tolerance elementwise; return the
    fraction of runs that also meet the plain base bar.

    With `spins` (the GPU's run-major rounded spins) also assert that they equal
    the oracle's wherever the oracle's magnetisation is farther from zero than
    the tolerance: only there is the sign decided at the GPU form's precision
    (with integer couplings many spins sit at exactly zero field)."""
    A = amplification(inst, runs, sched, seed, ref, run_begin=run_begin)
    tol = trajectory_tolerance(inst, ref, A, precision)
    err = np.abs(np.asarray(m_gpu, dtype=np.float64) - ref["m"])
    worst = float(np.max(err / tol))
    assert worst <= 1.0, "trajectory error exceeds the derived bound by %.2fx" % worst
    if spins is not None:
        decided = np.abs(ref["m"]) > tol
        mismatch = (np.asarray(spins).T != ref["spins"].T) & decided
        assert not mismatch.any(), "%d decided spins differ" % int(mismatch.sum())
    return float(np.mean(np.max(err, axis=0) <= BASE[precision]))


def energy_fsum_dense(J, h, s):
    """Exact energy of one spin vector by math.fsum over the eq. (2) terms
    (independent of both the oracle and the library)."""
    s = s.astype(np.float64)
    J = J.astype(np.float64)
    terms = (-(J * s[:, None]) * s[None, :])
    np.fill_diagonal(terms, 0.0)
    lst = terms.ravel().tolist()
    if h is not None:
        lst += (-(h.astype(np.float64) * s)).tolist()
    return math.fsum(lst)
