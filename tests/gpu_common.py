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


def conditioned_runs(inst, runs, sched, seed, ref, eps=1e-9, move=1e-6, nthreads=None):
    """Runs whose oracle trajectory is well conditioned: rerunning the oracle
    from m0 perturbed by +-eps (random signs) moves the final m by at most
    `move`.  Ill-conditioned runs sit near a bifurcation of the anneal where
    any rounding difference is amplified; their final state is not a stable
    function of the input at fp32 precision."""
    N = ref["m"].shape[0]
    m0 = O.initial_m(seed, runs, N)
    rng = np.random.default_rng(12345)
    pert = np.clip(m0 + eps * np.where(rng.random(m0.shape) < 0.5, -1.0, 1.0), -1 + 1e-12, 1 - 1e-12)
    alt = O.solve(inst, runs, sched, seed, run_count=runs, m0=pert, T0=ref["T0"], nthreads=nthreads)
    dev = np.max(np.abs(alt["m"] - ref["m"]), axis=0)
    return dev <= move


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
