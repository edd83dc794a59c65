"""Pins for the CPU oracle: checks against facts that the paper and the
mathematics fix, independent of the oracle's own code.

Each test names what it pins.  None of them re-types the oracle's update
formula; they use published generator outputs, brute-force enumeration,
library routines (math.fsum, fractions, scipy root finding), exact integer
arithmetic, symmetries of the dynamics, and the mean-field free energy as a
Lyapunov function.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import optimize, stats

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# generator
# ---------------------------------------------------------------------------


def test_splitmix64_published_vector():
    """The generator is SplitMix64: its first outputs from state 0 are published."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.strip() and l[0] != "#"]
    for c, v in rows:
        assert O.splitmix64(0, int(c)) == int(v, 16)


def test_initial_m_grid_and_distribution():
    """rand(-1,1) of Algorithm 1: odd multiples of 2^-24 in (-1, 1), uniform, symmetric."""
    m = O.initial_m(12345, 64, 200)
    assert np.all(np.abs(m) < 1.0)
    k = m * 2**24
    assert np.all(k == np.round(k)) and np.all(np.abs(k) % 2 == 1)
    assert stats.kstest((m.ravel() + 1) / 2, "uniform").pvalue > 1e-4
    assert abs(m.mean()) < 0.02
    # distinct counters give distinct values (the output function is a bijection)
    assert len(np.unique(m)) > 0.99 * m.size
    # different seeds decorrelate
    m2 = O.initial_m(12346, 64, 200)
    assert abs(np.corrcoef(m.ravel(), m2.ravel())[0, 1]) < 0.02


def test_initial_T_range_and_distribution():
    """Random starting temperature drawn in [T_lo, T_hi) (section MARS, first paragraph)."""
    T = O.initial_T(99, 4000, 0.5, 3.0)
    assert np.all(T >= 0.5) and np.all(T < 3.0)
    assert stats.kstest((T - 0.5) / 2.5, "uniform").pvalue > 1e-4


# ---------------------------------------------------------------------------
# exact summation and energies
# ---------------------------------------------------------------------------


def test_exact_sum_matches_fsum_and_fractions():
    """The long accumulator is the correctly rounded sum (math.fsum and exact rationals)."""
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(1, 3000))
        scale = 10.0 ** rng.integers(-30, 30, size=n)
        x = rng.standard_normal(n) * scale
        if trial % 3 == 0:  # heavy cancellation
            x = np.concatenate([x, -x[: n // 2] * (1 + 2**-52)])
        x = x.astype(np.float32).astype(np.float64) if trial % 2 else x
        got = O.exact_sum(x)
        assert got == math.fsum(x.tolist())
        if trial < 10:
            assert got == float(sum(Fraction(v) for v in x.tolist()))
    assert O.exact_sum([1e300, 1.0, -1e300]) == 1.0
    assert O.exact_sum([]) == 0.0
    assert O.exact_sum([2.0**-1074, 2.0**-1074]) == 2.0**-1073
    # a tie that must round to even
    assert O.exact_sum([1.0, 2.0**-53]) == 1.0
    assert O.exact_sum([1.0, 2.0**-53, 2.0**-106]) == 1.0 + 2.0**-52


def _energy_fsum_dense(J, h, s):
    """eq. (2) written out term by term, summed with math.fsum (correct rounding)."""
    N = J.shape[0]
    terms = []
    for i in range(N):
        for j in range(N):
            if i != j:
                terms.append(-float(J[i, j]) * s[i] * s[j])
        if h is not None:
            terms.append(-float(h[i]) * s[i])
    return math.fsum(terms)


def test_energy_dense_real_couplings_exact():
    """Exact energy of real couplings equals the correctly rounded ordered-pair sum."""
    inst = I.sk_instance(60, 3, field_scale=0.7)
    S = I.random_spins(60, 12, 4)
    E = O.energy(inst, S)
    for r in range(S.shape[0]):
        assert E[r] == _energy_fsum_dense(inst.J, inst.h, S[r].astype(np.int64))


def test_energy_integer_couplings_match_integer_arithmetic():
    """For +-1 couplings the energy is an integer: -s^T J s computed in int64."""
    for inst in (I.er_instance(300, 1, p=0.05, weights="pm1"), I.lattice_instance((8, 6), 2),
                 I.lattice_instance((4, 4, 6), 3)):
        Jd = (I.csr_dense(inst) if hasattr(inst, "rowptr") else I.lattice_dense(inst)).J.astype(np.int64)
        S = I.random_spins(inst.N, 20, 7).astype(np.int64)
        want = -np.einsum("ri,ij,rj->r", S, Jd, S)
        assert np.array_equal(O.energy(inst, S.astype(np.int8)), want.astype(np.float64))


def test_cut_identity_eq3():
    """eq. (3): cut weight = (sum_ij w_ij - sum_ij w_ij s_i s_j)/4 equals the directly counted cut."""
    inst = I.er_instance(200, 11, p=0.08, weights="pm1")  # J = -w
    S = I.random_spins(200, 10, 3)
    E = O.energy(inst, S)
    W = -float(inst.val.astype(np.int64).sum())  # sum over ordered pairs of w
    for r in range(S.shape[0]):
        cut = 0
        for i in range(inst.N):
            for k in range(inst.rowptr[i], inst.rowptr[i + 1]):
                j = inst.col[k]
                if i < j and S[r, i] != S[r, j]:
                    cut += -int(inst.val[k])
        assert (W - E[r]) / 4 == cut


# ---------------------------------------------------------------------------
# brute force ground states (N <= 20)
# ---------------------------------------------------------------------------


def _brute_force_gs(Jd, h=None):
    """Minimum of E over all 2^N spin vectors, enumerated in numpy."""
    N = Jd.shape[0]
    idx = np.arange(2**N, dtype=np.int64)
    S = 1 - 2 * ((idx[:, None] >> np.arange(N)[None, :]) & 1)
    S = S.astype(np.float64)
    E = -np.einsum("ki,ij,kj->k", S, Jd.astype(np.float64), S)
    if h is not None:
        E -= S @ h.astype(np.float64)
    return E.min()


@pytest.mark.parametrize("kind", ["ea2d_L4", "sk16", "er20", "ea2d_4x5"])
def test_brute_force_ground_state_is_reached(kind):
    """MARS never reports an energy below the true ground state, and with 1024
    runs it reaches it (the paper's success probability P > 0)."""
    if kind == "ea2d_L4":
        w = I.workload("ea2d_L4", seed=3)
        inst, sch = w.instance, w.schedule
        Jd = I.lattice_dense(inst).J
    elif kind == "ea2d_4x5":
        inst = I.lattice_instance((4, 6), 5)
        sch = I.Schedule(T_lo=0.5, T_hi=3.0, T_end=0.02, steps=300)
        Jd = I.lattice_dense(inst).J
    elif kind == "sk16":
        inst = I.sk_instance(16, 8)
        s = I.field_scale(inst)
        sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, phases=4)
        Jd = inst.J
    else:
        inst = I.er_instance(20, 9, p=0.3, weights="pm1")
        s = I.field_scale(inst)
        sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300)
        Jd = I.csr_dense(inst).J
    gs = _brute_force_gs(Jd)
    r = O.solve(inst, 1024, sch, 17, run_count=1024)
    assert np.all(r["energy"] >= gs - 1e-9 * abs(gs))
    b, hits = O.best(r["energy"])
    assert abs(r["energy"][b] - gs) <= 1e-9 * abs(gs)
    assert hits >= 1


# ---------------------------------------------------------------------------
# symmetries of the dynamics
# ---------------------------------------------------------------------------


def _gauge(inst, xi):
    J = (inst.J * xi[:, None] * xi[None, :]).astype(np.float32)
    h = None if inst.h is None else (inst.h * xi).astype(np.float32)
    return I.DenseInstance(J=J, h=h)


@pytest.mark.parametrize("update,phases", [("phased", 2), ("phased", 3), ("jacobi", 1)])
def test_gauge_covariance_bitwise(update, phases):
    """J' = DJD, h' = Dh, m0' = D m0 (D = diag of +-1) gives m' = D m exactly and
    the same energies: the dynamics is odd and every sign flip is exact."""
    N, R = 40, 6
    inst = I.sk_instance(N, 21, field_scale=0.3)
    xi = np.where(np.random.default_rng(2).random(N) < 0.5, -1.0, 1.0)
    s = I.field_scale(inst)
    sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=40, update=update, phases=phases)
    m0 = O.initial_m(4, R, N)
    T0 = O.initial_T(4, R, sch.T_lo, sch.T_hi)
    a = O.solve(inst, R, sch, 0, run_count=R, m0=m0, T0=T0)
    b = O.solve(_gauge(inst, xi), R, sch, 0, run_count=R, m0=m0 * xi[:, None], T0=T0)
    assert np.array_equal(b["m"], a["m"] * xi[:, None])
    assert np.array_equal(b["energy"], a["energy"])


def test_global_flip_covariance_h0():
    """With h = 0, E(s) = E(-s) and the trajectory from -m0 is -m (special case D = -I)."""
    inst = I.lattice_instance((6, 6), 4)
    sch = I.Schedule(T_lo=0.5, T_hi=3.0, T_end=0.02, steps=50)
    m0 = O.initial_m(1, 5, 36)
    T0 = O.initial_T(1, 5, 0.5, 3.0)
    a = O.solve(inst, 5, sch, 0, run_count=5, m0=m0, T0=T0)
    b = O.solve(inst, 5, sch, 0, run_count=5, m0=-m0, T0=T0)
    assert np.array_equal(b["m"], -a["m"])


def test_jacobi_sublattice_two_cycle_symmetry():
    """Bipartite lattice, synchronous (Jacobi) update: with the staggered gauge D
    (DJD = -J), the trajectory from D m0 is (-1)^k D m(k), bitwise."""
    L = (6, 4)
    inst = I.lattice_instance(L, 13)
    N = 24
    D = np.array([(-1.0) ** ((i % L[0]) + (i // L[0])) for i in range(N)])
    m0 = O.initial_m(3, 4, N)
    T0 = np.full(4, 1.3)
    for k in (1, 2, 7, 8):
        sch = I.Schedule(T_lo=1.3, T_hi=1.3, T_end=0.2, steps=20, update="jacobi", level_count=k)
        a = O.solve(inst, 4, sch, 0, run_count=4, m0=m0, T0=T0)
        b = O.solve(inst, 4, sch, 0, run_count=4, m0=D[:, None] * m0, T0=T0)
        assert np.array_equal(b["m"], ((-1.0) ** k) * D[:, None] * a["m"])


def test_permutation_covariance_jacobi():
    """Relabelling the spins relabels the trajectory (synchronous update; FP64 up to summation order)."""
    N, R = 30, 4
    inst = I.sk_instance(N, 31, field_scale=0.2)
    perm = np.random.default_rng(1).permutation(N)
    P = I.DenseInstance(J=inst.J[np.ix_(perm, perm)].copy(), h=inst.h[perm].copy())
    s = I.field_scale(inst)
    sch = I.Schedule(T_lo=0.5 * s, T_hi=1.5 * s, T_end=0.3 * s, steps=25, update="jacobi")
    m0 = O.initial_m(9, R, N)
    T0 = O.initial_T(9, R, sch.T_lo, sch.T_hi)
    a = O.solve(inst, R, sch, 0, run_count=R, m0=m0, T0=T0)
    b = O.solve(P, R, sch, 0, run_count=R, m0=m0[perm], T0=T0)
    assert np.max(np.abs(b["m"] - a["m"][perm])) < 1e-12


# ---------------------------------------------------------------------------
# closed forms and the free energy
# ---------------------------------------------------------------------------


def test_zero_couplings_closed_form():
    """J = 0: the field is h/2, so one sweep gives m = tanh(h / (2T)) from any start."""
    N, R = 7, 3
    h = np.array([0.3, -1.2, 0.0, 2.5, -0.01, 0.7, -3.0], dtype=np.float32)
    inst = I.DenseInstance(J=np.zeros((N, N), np.float32), h=h)
    T0 = np.array([0.4, 1.0, 2.2])
    sch = I.Schedule(T_lo=0.4, T_hi=2.2, T_end=0.1, steps=5, level_count=1)
    r = O.solve(inst, R, sch, 5, run_count=R, T0=T0)
    for q in range(R):
        for i in range(N):
            assert abs(r["m"][i, q] - math.tanh(float(h[i]) / (2 * T0[q]))) < 1e-15


@pytest.mark.parametrize("gamma", [0.3, 0.7])
def test_zero_couplings_damped_closed_form(gamma):
    """J = 0 with damping g: every sweep moves m a fraction g of the way to the
    fixed point t = tanh(h / (2T)), so after n sweeps at one temperature
    m_n = t + (1 - g)^n (m_0 - t) (the closed form of the iterated convex
    combination; the fixed point itself does not depend on g)."""
    N, R = 6, 2
    h = np.array([0.9, -1.3, 0.05, 2.0, -0.4, 0.0], dtype=np.float32)
    inst = I.DenseInstance(J=np.zeros((N, N), np.float32), h=h)
    T0 = np.array([0.5, 1.7])
    m0 = np.array([[0.8, -0.6], [0.1, 0.9], [-0.95, 0.3], [0.0, -0.2], [0.5, 0.5], [-0.7, 0.25]])
    for n in (1, 2, 5, 17):
        sch = I.Schedule(T_lo=0.5, T_hi=1.7, steps=1, max_sweeps=n, d_min=0.0, damping=gamma)
        r = O.solve(inst, R, sch, 0, run_count=R, m0=m0, T0=T0)
        for q in range(R):
            for i in range(N):
                t = math.tanh(float(h[i]) / (2 * T0[q]))
                want = t + (1 - gamma) ** n * (m0[i, q] - t)
                assert abs(r["m"][i, q] - want) < 1e-14, (n, q, i)
        # d_min = 0 is never undercut: the cap ends the level
        assert np.all(r["sweeps"] == n) and np.all(r["cap_hits"] == (1 if n > 1 else 0))


@pytest.mark.parametrize("gamma", [0.3, 0.7])
def test_damped_sweep_count_closed_form(gamma):
    """J = 0 with damping: the change of sweep n is g (1 - g)^(n-1) |m_0 - t|
    (largest over the spins), so the level ends at the first n where that is
    below d_min -- a count fixed in closed form, which pins the stopping rule
    of the repeat ... until loop and the per-level sweep record."""
    N = 4
    h = np.array([1.0, -0.5, 0.25, 0.0], dtype=np.float32)
    inst = I.DenseInstance(J=np.zeros((N, N), np.float32), h=h)
    T = 0.8
    m0 = np.array([[0.3], [0.9], [-0.6], [0.45]])
    t = np.tanh(h.astype(np.float64) / (2 * T))
    dev = float(np.max(np.abs(m0[:, 0] - t)))
    for d_min in (1e-2, 1e-4, 1e-7):
        n = 1
        while not (gamma * (1 - gamma) ** (n - 1) * dev < d_min):
            n += 1
        sch = I.Schedule(T_lo=T, T_hi=T, steps=1, max_sweeps=10000, d_min=d_min, damping=gamma)
        r = O.solve(inst, 1, sch, 0, run_count=1, m0=m0, T0=np.array([T]), levels_cap=2)
        assert int(r["sweeps"][0]) == n and int(r["cap_hits"][0]) == 0, (d_min, n, r["sweeps"])
        assert r["sweeps_per_level"][0, 0] == n and r["own_per_level"][0, 0] == n
        assert r["sweeps_per_level"][0, 1] == 0  # one level only
        # a cap below n ends the level early and is counted; max_sweeps = 1 is
        # one sweep per level by definition and counts no cap
        for cap in (1, 2, n - 1):
            if cap < 1 or cap >= n:
                continue
            sc2 = I.Schedule(T_lo=T, T_hi=T, steps=1, max_sweeps=cap, d_min=d_min, damping=gamma)
            r2 = O.solve(inst, 1, sc2, 0, run_count=1, m0=m0, T0=np.array([T]))
            assert int(r2["sweeps"][0]) == cap
            assert int(r2["cap_hits"][0]) == (1 if cap > 1 else 0), (cap, n)


def test_cap_hits_count_levels_cut_by_the_cap():
    """Over a whole schedule, cap_hits is the number of levels the sweep cap
    ended: every level when d_min = 0 (never undercut) and max_sweeps > 1,
    none when each level converges within the cap, none when max_sweeps = 1."""
    inst = I.DenseInstance(J=np.array([[0, 0.9], [0.9, 0]], dtype=np.float32))
    T0 = np.array([1.3, 2.9, 0.7])
    m0 = np.array([[0.6, -0.2, 0.9], [0.1, 0.4, -0.3]])
    sch = I.Schedule(kind="linear", T_lo=0.5, T_hi=3.0, c_step=0.1, max_sweeps=3, d_min=0.0, phases=2)
    r = O.solve(inst, 3, sch, 0, run_count=3, m0=m0, T0=T0)
    assert np.all(r["levels"] > 0) and np.array_equal(r["cap_hits"], r["levels"])
    assert np.array_equal(r["sweeps"], 3 * r["levels"])
    sch1 = I.Schedule(kind="linear", T_lo=0.5, T_hi=3.0, c_step=0.1, max_sweeps=1, d_min=0.0, phases=2)
    r1 = O.solve(inst, 3, sch1, 0, run_count=3, m0=m0, T0=T0)
    assert np.all(r1["cap_hits"] == 0) and np.array_equal(r1["sweeps"], r1["levels"])
    sch2 = I.Schedule(kind="linear", T_lo=0.5, T_hi=3.0, c_step=0.1, max_sweeps=100000, d_min=1e-6, phases=2)
    r2 = O.solve(inst, 3, sch2, 0, run_count=3, m0=m0, T0=T0)
    assert np.all(r2["cap_hits"] == 0) and np.all(r2["sweeps"] > r2["levels"])


def test_replay_of_own_counts_and_of_other_counts():
    """Replaying the oracle's own per-level sweep counts reproduces its run bit
    for bit; replaying one sweep per level equals the max_sweeps = 1 schedule;
    under a replay the own-rule record marks exactly the levels whose replayed
    count differs from the rule's, with the d of the deciding sweep."""
    inst = I.sk_instance(40, 8)
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=3 * s, c_step=0.3 * s, max_sweeps=500, d_min=1e-4, phases=2)
    R, cap = 6, 16
    r = O.solve(inst, R, sch, 11, run_count=R, levels_cap=cap)
    assert np.array_equal(r["sweeps_per_level"].sum(axis=1), r["sweeps"])
    assert np.array_equal(r["own_per_level"], r["sweeps_per_level"])
    assert np.all(r["d_per_level"][r["sweeps_per_level"] > 0] < 1e-4)
    rr = O.solve(inst, R, sch, 11, run_count=R, levels_cap=cap, replay=r["sweeps_per_level"])
    assert np.array_equal(rr["m"], r["m"]) and np.array_equal(rr["sweeps"], r["sweeps"])
    ones = np.where(r["sweeps_per_level"] > 0, 1, 0).astype(np.int32)
    r1 = O.solve(inst, R, sch, 11, run_count=R, levels_cap=cap, replay=ones)
    sc1 = I.Schedule(kind="linear", T_lo=0.0, T_hi=3 * s, c_step=0.3 * s, max_sweeps=1, d_min=1e-4, phases=2)
    ref1 = O.solve(inst, R, sc1, 11, run_count=R)
    assert np.array_equal(r1["m"], ref1["m"])
    live = r["sweeps_per_level"] > 1
    # with one sweep replayed where the rule needs more, the rule would go on
    assert np.all(r1["own_per_level"][live] == 2) and np.all(r1["d_per_level"][live] >= 1e-4)


def test_single_spin():
    """N = 1: no couplings, the field is zero, m becomes 0 and rounds to +1 with E = 0."""
    inst = I.DenseInstance(J=np.zeros((1, 1), np.float32))
    r = O.solve(inst, 3, I.Schedule(steps=4), 1, run_count=3)
    assert np.all(r["m"] == 0.0) and np.all(r["spins"] == 1) and np.all(r["energy"] == 0.0)


@pytest.mark.parametrize("Jv,T", [(0.8, 0.5), (-1.1, 0.6), (0.3, 1.0)])
def test_two_spin_fixed_point(Jv, T):
    """N = 2 at fixed T relaxes to the fixed point m1 = tanh(J m2/T), m2 = tanh(J m1/T)
    (the root found by scipy's brentq; the paramagnet 0 when |J|/T < 1)."""
    inst = I.DenseInstance(J=np.array([[0, Jv], [Jv, 0]], dtype=np.float32))
    Jd = float(np.float32(Jv))
    sch = I.Schedule(T_lo=T, T_hi=T, steps=1, max_sweeps=100000, d_min=1e-15, phases=2)
    m0 = np.array([[0.9], [0.4]])
    r = O.solve(inst, 1, sch, 0, run_count=1, m0=m0, T0=np.array([T]))
    m1, m2 = r["m"][:, 0]
    if abs(Jd) / T > 1:
        x = optimize.brentq(lambda x: x - math.tanh(abs(Jd) * x / T), 1e-6, 1.0, xtol=1e-15)
        assert abs(abs(m1) - x) < 1e-10 and abs(abs(m2) - x) < 1e-10
        assert np.sign(m1) * np.sign(m2) == np.sign(Jd)
    else:
        assert abs(m1) < 1e-6 and abs(m2) < 1e-6


def _free_energy(Jd, h, m, T):
    """Mean-field free energy whose coordinate-wise minimiser is m_i = tanh(Phi_i/T):
    F = -sum_{i!=j} J_ij m_i m_j - sum_i h_i m_i - 2T sum_i S(m_i), S the binary entropy."""
    p = np.clip((1 + m) / 2, 1e-300, 1)
    q = np.clip((1 - m) / 2, 1e-300, 1)
    S = -(p * np.log(p) + q * np.log(q))
    e = -m @ Jd @ m - (0.0 if h is None else h @ m)
    return e - 2 * T * S.sum()


@pytest.mark.parametrize("inst_kind,gamma", [("lattice2d", 1.0), ("lattice3d", 1.0), ("er", 1.0),
                                             ("lattice2d", 0.3), ("er", 0.7)])
def test_free_energy_is_nonincreasing_over_sweeps(inst_kind, gamma):
    """Updating an independent set of spins (a lattice sublattice or a colour
    class) minimises the mean-field free energy over them, so F never rises
    from sweep to sweep at fixed T.  F is convex in each such spin, so a damped
    step (a convex combination of the old value and the minimiser) cannot
    raise it either.  A sign error in the field or the update, or a wrong
    neighbour, breaks this."""
    if inst_kind == "lattice2d":
        inst = I.lattice_instance((8, 8), 2)
        Jd = I.lattice_dense(inst).J.astype(np.float64)
    elif inst_kind == "lattice3d":
        inst = I.lattice_instance((4, 4, 4), 2)
        Jd = I.lattice_dense(inst).J.astype(np.float64)
    else:
        inst = I.er_instance(60, 4, p=0.1, weights="pm1")
        Jd = I.csr_dense(inst).J.astype(np.float64)
    N = Jd.shape[0]
    m0 = O.initial_m(8, 3, N)
    for T in (0.3, 1.0, 2.5):
        prev = None
        for sweeps in range(1, 12):
            sch = I.Schedule(T_lo=T, T_hi=T, steps=1, max_sweeps=sweeps, d_min=0.0, damping=gamma)
            r = O.solve(inst, 3, sch, 0, run_count=3, m0=m0, T0=np.full(3, T))
            F = np.array([_free_energy(Jd, None, r["m"][:, q], T) for q in range(3)])
            if prev is not None:
                assert np.all(F <= prev + 1e-9 * np.abs(prev)), (T, sweeps)
            prev = F


def test_fixed_point_residual_after_convergence():
    """When a level ends on d < d_min the state is a fixed point of the mean-field
    equations up to a small multiple of d_min (checked with an independent
    numpy field computation of the converged state)."""
    inst = I.sk_instance(80, 6, field_scale=0.2)
    Jd = inst.J.astype(np.float64)
    h = inst.h.astype(np.float64)
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=3.0 * s, c_step=0.5 * s, max_sweeps=5000, d_min=1e-9,
                     phases=8)
    r = O.solve(inst, 8, sch, 3, run_count=8)
    for q in range(8):
        if r["levels"][q] == 0:
            continue
        T = r["last_T"][q]
        m = r["m"][:, q]
        resid = np.max(np.abs(m - np.tanh((Jd @ m + h / 2) / T)))
        assert resid < 1e-6, (q, resid, T)
    assert np.all(r["cap_hits"] == 0)


# ---------------------------------------------------------------------------
# schedule, phases, resume
# ---------------------------------------------------------------------------


def test_geometric_levels():
    sch = I.Schedule(T_end=0.02, steps=300)
    T = O.levels(sch, 2.7)
    assert len(T) == 300 and T[0] == 2.7 and abs(T[-1] - 0.02) < 1e-15
    ratio = T[1:] / T[:-1]
    assert np.max(np.abs(ratio - ratio.mean())) < 1e-12
    assert len(O.levels(sch.replace(steps=1), 1.5)) == 1 and O.levels(sch.replace(steps=0), 1.5).size == 0


def test_linear_levels_paper_schedule():
    """Algorithm 1: T decreases by C_step before each relaxation and stops at T <= 0."""
    sch = I.Schedule(kind="linear", c_step=1.0)
    T = O.levels(sch, 30.0)
    assert list(T) == [float(x) for x in range(29, 0, -1)]
    assert len(O.levels(sch, 3.7)) == 3 and len(O.levels(sch, 0.5)) == 0


def test_phase_partitions():
    inst = I.sk_instance(11, 1)
    ph, n = O.phases(inst, I.Schedule(phases=3))
    assert n == 3 and list(ph) == [0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2]
    lat = I.lattice_instance((4, 6), 1)
    ph, n = O.phases(lat, I.Schedule())
    Jd = I.lattice_dense(lat).J
    assert n == 2
    for i, j in zip(*np.nonzero(Jd)):
        assert ph[i] != ph[j]
    g = I.er_instance(400, 2, p=0.05)
    ph, n = O.phases(g, I.Schedule())
    deg = np.diff(g.rowptr)
    assert n <= deg.max() + 1
    for i in range(g.N):
        assert np.all(ph[g.col[g.rowptr[i]:g.rowptr[i + 1]]] != ph[i])
    ph, n = O.phases(g, I.Schedule(update="jacobi"))
    assert n == 1 and np.all(ph == 0)


def test_resume_equals_full_solve():
    """Levels are a checkpoint unit: levels [0,k) then [k,K) from the saved state equal one solve."""
    inst = I.sk_instance(50, 2)
    s = I.field_scale(inst)
    sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=60)
    full = O.solve(inst, 5, sch, 77, run_count=5)
    a = O.solve(inst, 5, sch.replace(level_count=17), 77, run_count=5)
    b = O.solve(inst, 5, sch.replace(first_level=17), 77, run_count=5, m0=a["m"], T0=a["T0"])
    assert np.array_equal(b["m"], full["m"]) and np.array_equal(b["energy"], full["energy"])


def test_run_subsets_are_independent():
    """Runs are independent: a subset of runs equals the same runs of the full solve."""
    inst = I.lattice_instance((8, 8), 1)
    sch = I.Schedule(steps=30)
    full = O.solve(inst, 40, sch, 5, run_count=40, nthreads=3)
    part = O.solve(inst, 40, sch, 5, run_begin=13, run_count=9, nthreads=1)
    assert np.array_equal(part["m"], full["m"][:, 13:22])
    assert np.array_equal(part["energy"], full["energy"][13:22])


def test_best_run_ties_lowest_index():
    e = np.array([3.0, -2.0, 5.0, -2.0, -1.0])
    assert O.best(e) == (1, 2)


def test_phased_beats_jacobi_on_lattice():
    """Qualitative: the synchronous reading 2-cycles on bipartite lattices (mean
    energy near 0); the phased update relaxes (mean well below 0)."""
    w = I.workload("ea2d_L16", seed=1)
    a = O.solve(w.instance, 128, w.schedule, 1, run_count=128)
    b = O.solve(w.instance, 128, w.schedule.replace(update="jacobi"), 1, run_count=128)
    N = w.instance.N
    assert a["energy"].mean() / N < -2.4
    assert abs(b["energy"].mean() / N) < 0.5


def test_sequential_is_one_phase_per_spin():
    """The sequential update (dense) is the phased update with every spin its
    own phase in index order: the oracle's phase map and a one-level result
    equal those of phases = N."""
    from oracle import oracle as O
    from paper_1907_05124_amd import inputs as I

    inst = I.sk_instance(24, 3, field_scale=0.3)
    seq = I.Schedule(steps=3, phases=2, update="sequential")
    ph, n = O.phases(inst, seq)
    assert n == 24 and list(ph) == list(range(24))
    a = O.solve(inst, 5, seq, 7, run_count=5)
    b = O.solve(inst, 5, seq.replace(update="phased", phases=24), 7, run_count=5)
    assert np.array_equal(a["m"], b["m"])
    # one level written out as a plain Gauss-Seidel loop in index order
    one = seq.replace(level_count=1, precision="fp64")
    got = O.solve(inst, 5, one, 7, run_count=5)
    J = inst.J.astype(np.float64)
    h = inst.h.astype(np.float64)
    m = O.initial_m(7, 5, 24).astype(np.float64)
    T0 = got["T0"]
    for r in range(5):
        for i in range(24):
            m[i, r] = math.tanh((sum(J[i, j] * m[j, r] for j in range(24)) + h[i] / 2) / T0[r])
    assert np.allclose(got["m"], m, rtol=0, atol=1e-12)
