"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import math
import sys

import numpy as np

from oracle import oracle as O


def require_gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU (run them with -m gpu on a machine with an MI355X)"
    return torch


def announce(*parts):
    """Name the case on stdout before a GPU step (flushed)."""
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()


BASE = {"fp32": 1e-5, "fp64": 1e-9}


def _initial_m(seed, run_begin, N, rc):
    m0 = np.empty((N, rc))
    for q in range(rc):
        for i in range(N):
            m0[i, q] = O.lib().orc_initial_m(seed, run_begin + q, i)
    return m0


def _ulp_shifted(inst, sign):
    """The dense instance with every coupling J_ij = J_ji (and field value)
    moved by one fp32 ulp, in direction sign * xi (xi drawn once, so that
    sign = +1 and -1 are mirror images)."""
    from paper_1907_05124_amd import inputs as I

    rng = np.random.default_rng(500)
    J = np.asarray(inst.J, dtype=np.float32)
    N = J.shape[0]
    up = (rng.random((N, N)) < 0.5) == (sign > 0)
    P = np.where(up, np.nextafter(J, np.float32(np.inf)), np.nextafter(J, np.float32(-np.inf)))
    P = np.triu(P, 1)
    h = None
    if inst.h is not None:
        hh = np.asarray(inst.h, dtype=np.float32)
        hu = (rng.random(N) < 0.5) == (sign > 0)
        h = np.where(hu, np.nextafter(hh, np.float32(np.inf)), np.nextafter(hh, np.float32(-np.inf)))
        h = np.where(hh == 0, hh, h).astype(np.float32)
    return I.DenseInstance(J=(P + P.T).astype(np.float32), h=h)


def conditioning(inst, runs, sched, seed, ref, *, run_begin=0, replay=None, levels_cap=0, precision="fp32"):
    """How far each run's final magnetisation moves in the oracle itself (no
    GPU input), two arrays over the runs of `ref` (max over a random pattern
    and its mirror image):

      move_m0  under a +-1e-9 change of every initial magnetisation: the
               sensitivity to the start, by which the reading of the paper's
               "agree within 1e-5" excludes runs;
      move_fp  (fp32 forms; zeros for fp64) under the changes an fp32
               evaluation makes at every level rather than at the start: every
               starting temperature moved by one fp32 ulp (so every level's
               1/T moves by about one), and for dense couplings every J_ij
               moved by one fp32 ulp (the rounding of the field product).
               A change of m0 decays at temperatures above the run's
               instability and so misses runs whose outcome is decided later
               in the anneal, when 1/T amplifies any change of the field;
               these changes act there.

    With `replay`, the perturbed oracle runs replay the same per-level sweep
    counts."""
    from paper_1907_05124_amd import inputs as I

    N, rc = ref["m"].shape
    kw = dict(levels_cap=levels_cap, replay=replay) if replay is not None else {}
    m0 = _initial_m(seed, run_begin, N, rc)
    xi = np.where(np.random.default_rng(1000).random(m0.shape) < 0.5, -1.0, 1.0)

    def move(alt):
        return np.max(np.abs(alt["m"] - ref["m"]), axis=0)

    move_m0 = np.zeros(rc)
    move_fp = np.zeros(rc)
    for sign in (1.0, -1.0):
        pert = np.clip(m0 + sign * 1e-9 * xi, -1 + 1e-12, 1 - 1e-12)
        move_m0 = np.maximum(move_m0, move(O.solve(inst, runs, sched, seed, run_begin=run_begin, run_count=rc,
                                                   m0=pert, T0=ref["T0"], **kw)))
        if precision != "fp32":
            continue
        T0 = ref["T0"] * (1.0 + sign * 2.0**-23)
        move_fp = np.maximum(move_fp, move(O.solve(inst, runs, sched, seed, run_begin=run_begin, run_count=rc,
                                                   m0=m0, T0=T0, **kw)))
        if isinstance(inst, I.DenseInstance):
            move_fp = np.maximum(move_fp, move(O.solve(_ulp_shifted(inst, sign), runs, sched, seed,
                                                       run_begin=run_begin, run_count=rc, m0=m0, T0=ref["T0"],
                                                       **kw)))
    return move_m0, move_fp


def c16_parity(m_gpu, inst, runs, sched, seed, ref, precision, *, run_begin=0, replay=None, levels_cap=0,
               max_excluded=0.0, label=""):
    """The elementwise bar on the runs the oracle finds well conditioned: a run
    is excluded when its final m moves in the oracle by more than 1e-6 under
    a 1e-9 change of m0 (the stated reading), or, for fp32 forms, by more
    than a quarter of the bar under the fp32-sized changes of `conditioning`;
    every element of every other run must agree with the oracle within the
    bar (1e-5 fp32, 1e-9 fp64).  Prints the excluded fraction by criterion,
    asserts its ceiling and returns it."""
    bar = BASE[precision]
    move_m0, move_fp = conditioning(inst, runs, sched, seed, ref, run_begin=run_begin, replay=replay,
                                    levels_cap=levels_cap, precision=precision)
    out_m0 = move_m0 > 1e-6
    out_fp = move_fp > 0.25 * bar
    out = out_m0 | out_fp
    err = np.max(np.abs(np.asarray(m_gpu, dtype=np.float64) - ref["m"]), axis=0)
    frac = float(np.mean(out))
    print("[parity] %s: %d runs, excluded %.3f (m0 %.3f, fp32-sized %.3f), worst kept %.3g, worst excluded %.3g"
          % (label, len(err), frac, float(np.mean(out_m0)), float(np.mean(out_fp)),
             float(np.max(err[~out], initial=0.0)), float(np.max(err[out], initial=0.0))), flush=True)
    bad = np.flatnonzero(~out & (err > bar))
    assert bad.size == 0, "runs %s differ from the oracle by %s (> %g)" % (
        (bad + run_begin).tolist()[:8], err[bad][:8].tolist(), bar)
    assert frac <= max_excluded, "excluded fraction %.3f above %.3f" % (frac, max_excluded)
    return frac


def _blocks(sample):
    """Contiguous blocks (first, count) of a sorted list of run indices."""
    out = []
    for r in sorted(sample):
        if out and out[-1][0] + out[-1][1] == r:
            out[-1][1] += 1
        else:
            out.append([r, 1])
    return out


def check_replay(m_gpu, spl, inst, runs, sched, seed, precision, sample, *, max_excluded=0.1, label=""):
    """Parity of the paper's scheduler by replay (the reading of Algorithm 1's
    repeat ... until decided in two precisions): the oracle runs exactly the
    per-level sweep counts `spl` [runs x cap] the GPU reports, for the runs in
    `sample`.  Asserts that it followed them, that wherever its own rule
    (d < d_min, or the cap) would have ended a level at another sweep its d
    at the deciding sweep is within 1e-5 of d_min, and the elementwise bar of
    `c16_parity` on m_gpu [N x runs].  Returns (levels checked, levels whose
    decision differs, largest |d - d_min| among those)."""
    cap = spl.shape[1]
    levels = disagree = 0
    worst_dd = excl = 0.0
    for r0, n in _blocks(sample):
        rep = np.ascontiguousarray(spl[r0:r0 + n])
        ref = O.solve(inst, runs, sched, seed, run_begin=r0, run_count=n, levels_cap=cap, replay=rep)
        assert np.array_equal(ref["sweeps_per_level"], rep), "replay not followed at runs %d.." % r0
        nlev = np.count_nonzero(rep, axis=1)
        assert np.array_equal(nlev, ref["levels"]), "level counts differ at runs %d.." % r0
        assert np.all(nlev < cap), "a run visits more levels than the record holds"
        diff = (rep > 0) & (ref["own_per_level"] != rep)
        dd = np.abs(ref["d_per_level"][diff] - sched.d_min)
        assert np.all(dd <= 1e-5), "a differing stop decision %g away from d_min" % float(np.max(dd))
        levels += int(nlev.sum())
        disagree += int(diff.sum())
        worst_dd = max(worst_dd, float(np.max(dd, initial=0.0)))
        excl += n * c16_parity(np.asarray(m_gpu)[:, r0:r0 + n], inst, runs, sched, seed, ref, precision,
                               run_begin=r0, replay=rep, levels_cap=cap, max_excluded=1.0,
                               label="%s replay runs %d..%d" % (label, r0, r0 + n - 1))
    frac = excl / len(sample)
    print("[replay] %s: %d runs, %d levels, %d stop decisions differ (max |d - d_min| %.3g), excluded %.3f"
          % (label, len(sample), levels, disagree, worst_dd, frac), flush=True)
    assert frac <= max_excluded, "excluded fraction %.3f above %.3f" % (frac, max_excluded)
    return levels, disagree, worst_dd


def solve_summary(res: dict) -> dict:
    """A solve's summary without its timing (`seconds`, the device time of the
    solve, which differs between otherwise identical solves); asserts that the
    timing is positive."""
    assert res["seconds"] > 0.0, res
    return {k: v for k, v in res.items() if k != "seconds"}


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
