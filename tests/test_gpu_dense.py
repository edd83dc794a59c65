"""GPU parity of the dense path (matrix-core field product + fused update)
against the CPU oracle, through the C interface.

Tolerance: the fp32 form must match the oracle's magnetisations within 1e-5
(absolute) on the same seeds; energies of equal spin vectors are bit-exact.
Sizes span several 128 x 128 tiles with ragged tails in both the spin and
the run dimension."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, c16_parity, energy_fsum_dense, require_gpu

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


def _sched(inst, **kw):
    s = I.field_scale(inst)
    base = dict(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, phases=2)
    base.update(kw)
    return I.Schedule(**base)


def test_generator_bitwise():
    """m0 and T0 come from the same counter generator on both sides: bitwise equal."""
    M = _mars()
    N, R, seed = 37, 300, 12345
    inst = I.sk_instance(N, 1)
    sch = I.Schedule(T_lo=0.3, T_hi=2.0, steps=0)
    announce("generator", N, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, seed, want_T0=True, want_m=True)
    assert np.array_equal(out["m"].cpu().numpy().astype(np.float64), O.initial_m(seed, R, N))
    assert np.array_equal(out["T0"].cpu().numpy(), O.initial_T(seed, R, 0.3, 2.0))


@pytest.mark.parametrize("N,R,phases,update,damping,field", [
    (1000, 300, 2, "phased", 1.0, 0.0),
    (1000, 300, 2, "phased", 1.0, 0.5),
    (517, 129, 3, "phased", 0.6, 0.0),
    (300, 77, 1, "jacobi", 1.0, 0.0),
    (129, 1, 5, "phased", 1.0, 0.3),
])
def test_one_level_parity(N, R, phases, update, damping, field):
    """One level of Algorithm 1 (every phase once) from the generator's state."""
    M = _mars()
    inst = I.sk_instance(N, 2, field_scale=field)
    sch = _sched(inst, phases=phases, update=update, damping=damping, level_count=1)
    announce("dense one level", N, R, phases, update, damping, field)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 99, want_m=True)
    ref = O.solve(inst, R, sch, 99, run_count=R)
    err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
    assert err <= TOL_FP32, err


# ceilings of the excluded fraction (the oracle's own sensitivity, measured
# 0, 0.25, 0.06 and 0.11 on this instance: at level 10 many runs are near the
# temperature where their descent picks a direction; at the last levels
# 1/T = 100/sigma amplifies any change of the field of a weakly pinned spin)
CHECKPOINT_EXCLUDED = {1: 0.0, 10: 0.35, 100: 0.15, 300: 0.2}


@pytest.mark.parametrize("levels", [1, 10, 100, 300])
def test_anneal_parity_checkpoints(levels):
    """Full anneal (300 geometric levels) checked at levels 1, 10, 100 and 300:
    every run the oracle finds well conditioned agrees within 1e-5 in every
    element (runs excluded when a 1e-9 change of m0 moves their final m by
    more than 1e-6, or fp32-sized changes of T0 and J by more than 2.5e-6;
    the excluded fraction bounded); spins agree wherever such a run's |m|
    exceeds the bar, and energies of equal spin vectors are equal."""
    M = _mars()
    N, R, seed = 256, 64, 5
    inst = I.sk_instance(N, 4)
    sch = _sched(inst, level_count=levels)
    announce("dense anneal", N, R, levels)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, seed, want_m=True, want_spins=True)
    ref = O.solve(inst, R, sch, seed, run_count=R)
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    m = out["m"].cpu().numpy()
    c16_parity(m, inst, R, sch, seed, ref, "fp32", max_excluded=CHECKPOINT_EXCLUDED[levels],
               label="dense sk256 level %d" % levels)
    close = np.max(np.abs(m.astype(np.float64) - ref["m"]), axis=0) <= TOL_FP32
    decided = np.abs(ref["m"]) > TOL_FP32
    assert not np.any((S.T != ref["spins"].T) & decided & close[None, :])
    same = np.all(S == ref["spins"], axis=1)
    assert np.array_equal(E[same], ref["energy"][same])


def test_energy_exact():
    """Exact energies of given spins: bitwise equal to the oracle's long accumulator."""
    M = _mars()
    torch = require_gpu()
    inst = I.sk_instance(500, 6, field_scale=0.7)
    S = I.random_spins(500, 64, 3)
    announce("dense energy", 500, 64)
    with M.Instance.from_inputs(inst) as g:
        E = g.energy(torch.from_numpy(S).cuda()).cpu().numpy()
    assert np.array_equal(E, O.energy(inst, S))


def test_energy_exact_wide_range():
    """Couplings spanning ~60 bits of binary range use 128-bit row sums: still exact."""
    M = _mars()
    torch = require_gpu()
    inst = I.sk_instance(300, 7)
    inst.J[0, 1] = inst.J[1, 0] = np.float32(2.0**-40)
    inst.J[5, 9] = inst.J[9, 5] = np.float32(-3.0 * 2.0**-41)
    S = I.random_spins(300, 40, 8)
    announce("dense energy wide", 300, 40)
    with M.Instance.from_inputs(inst) as g:
        E = g.energy(torch.from_numpy(S).cuda()).cpu().numpy()
    assert np.array_equal(E, O.energy(inst, S))


def test_result_summary_is_consistent():
    """best = min energy (ties to the lowest run), hits, mean, best spins; the
    reported best energy is the exact energy of the returned spins (checked
    with math.fsum, independently of the library and the oracle)."""
    M = _mars()
    N, R = 96, 777
    inst = I.sk_instance(N, 11, field_scale=0.1)
    sch = _sched(inst, steps=60)
    announce("dense summary", N, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 3, want_spins=True)
    E = out["energies"].cpu().numpy()
    S = out["spins"].cpu().numpy()
    res = out["result"]
    b = int(np.argmin(E))
    assert res["best_run"] == b and res["best_energy"] == E[b]
    assert res["hit_count"] == int(np.sum(E == E[b]))
    assert abs(res["mean_energy"] - E.mean()) <= 1e-12 * max(1.0, abs(E.mean()))
    assert res["sweeps_executed"] == R * 60 and res["levels_executed"] == R * 60
    assert res["spin_updates"] == R * 60 * N
    assert np.array_equal(out["best_spins"].cpu().numpy(), S[b])
    assert energy_fsum_dense(inst.J, inst.h, S[b]) == E[b]
    for r in (0, R // 2, R - 1):
        assert energy_fsum_dense(inst.J, inst.h, S[r]) == E[r]


def test_deterministic_bitwise():
    M = _mars()
    inst = I.sk_instance(300, 12)
    sch = _sched(inst, steps=40)
    announce("dense determinism", 300, 200)
    with M.Instance.from_inputs(inst) as g:
        a = g.solve_ex(200, sch, 9, want_m=True)
        b = g.solve_ex(200, sch, 9, want_m=True)
    assert np.array_equal(a["m"].cpu().numpy(), b["m"].cpu().numpy())
    assert np.array_equal(a["energies"].cpu().numpy(), b["energies"].cpu().numpy())


def test_gauge_covariance_bitwise():
    """J' = DJD, h' = Dh, m0' = D m0 gives m' = D m bit for bit on the GPU."""
    M = _mars()
    torch = require_gpu()
    N, R = 200, 50
    inst = I.sk_instance(N, 13, field_scale=0.3)
    xi = np.where(np.random.default_rng(1).random(N) < 0.5, -1.0, 1.0).astype(np.float32)
    ginst = I.DenseInstance(J=(inst.J * xi[:, None] * xi[None, :]).astype(np.float32),
                            h=(inst.h * xi).astype(np.float32))
    sch = _sched(inst, steps=30)
    m0 = O.initial_m(4, R, N).astype(np.float32)
    announce("dense gauge", N, R)
    with M.Instance.from_inputs(inst) as g, M.Instance.from_inputs(ginst) as gg:
        a = g.solve_ex(R, sch, 4, m0=torch.from_numpy(m0).cuda(), want_m=True)
        b = gg.solve_ex(R, sch, 4, m0=torch.from_numpy(m0 * xi[:, None]).cuda(), want_m=True)
    ma = a["m"].cpu().numpy()
    mb = b["m"].cpu().numpy()
    assert np.array_equal(mb, ma * xi[:, None])
    assert np.array_equal(a["energies"].cpu().numpy(), b["energies"].cpu().numpy())


def test_resume_equals_full_solve():
    """Levels [0, 11) then [11, K) from the saved state and temperatures equal one solve."""
    M = _mars()
    N, R = 150, 40
    inst = I.sk_instance(N, 14)
    sch = _sched(inst, steps=50)
    announce("dense resume", N, R)
    with M.Instance.from_inputs(inst) as g:
        full = g.solve_ex(R, sch, 21, want_m=True)
        a = g.solve_ex(R, sch.replace(level_count=11), 21, want_m=True, want_T0=True)
        b = g.solve_ex(R, sch.replace(first_level=11), 21, m0=a["m"], T0=a["T0"], want_m=True)
    assert np.array_equal(b["m"].cpu().numpy(), full["m"].cpu().numpy())
    assert np.array_equal(b["energies"].cpu().numpy(), full["energies"].cpu().numpy())


@pytest.mark.parametrize("phases,damping", [(4, 1.0), (2, 1.0), (2, 0.7)])
def test_paper_schedule_replay(phases, damping):
    """The paper's scheduler (linear decrement, sweeps repeated until
    d < d_min = 1e-4, Algorithm 1's repeat ... until) by replay: the oracle
    runs the per-level sweep counts the GPU reports and must agree within
    1e-5 on every well-conditioned run; wherever its own d-versus-d_min
    decision differs from the GPU's count, its d at the deciding sweep is
    within 1e-5 of d_min (an fp32 d near d_min may round either way)."""
    from tests.gpu_common import check_replay

    M = _mars()
    N, R, cap = 128, 64, 64
    inst = I.sk_instance(N, 15)
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=3.0 * s, c_step=0.25 * s, max_sweeps=1000, d_min=1e-4,
                     phases=phases, damping=damping)
    announce("dense paper schedule replay", N, R, phases, damping)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 31, want_m=True, levels_cap=cap)
    spl = out["sweeps_per_level"].cpu().numpy()
    res = out["result"]
    own = O.solve(inst, R, sch, 31, run_count=R)
    assert res["levels_executed"] == int(own["levels"].sum())  # levels follow from T0 alone
    assert res["sweeps_executed"] == int(spl.sum())
    check_replay(out["m"].cpu().numpy(), spl, inst, R, sch, 31, "fp32", list(range(R)), max_excluded=0.15,
                 label="dense sk128")


def test_bench_configuration_sampled_runs():
    """SK N=2000, 4096 runs, 300 levels (the benchmark's launch configuration):
    32 sampled runs recomputed by the oracle match within 1e-5 in every
    element where well conditioned (excluded fraction measured 0.34, at most
    0.5), and their energies are equal where the spins are."""
    M = _mars()
    w = I.workload("sk2000", seed=1)
    inst, sch, R = w.instance, w.schedule, w.runs
    announce("dense sk2000 full", inst.N, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 1, want_m=True, want_spins=True)
    m = out["m"].cpu().numpy()
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    # 32 runs spread over the run range, contiguous blocks of 8 (oracle subsets)
    excl = 0.0
    for r0 in (0, 1300, 2704, 4088):
        one = O.solve(inst, R, sch, 1, run_begin=r0, run_count=8)
        excl += c16_parity(m[:, r0:r0 + 8], inst, R, sch, 1, one, "fp32", run_begin=r0, max_excluded=1.0,
                           label="sk2000 runs %d..%d" % (r0, r0 + 7))
        for q in range(8):
            if np.array_equal(S[r0 + q], one["spins"][q]):
                assert E[r0 + q] == one["energy"][q]
    assert excl / 4 <= 0.5, excl / 4
    # the summary refers to the full set of runs
    res = out["result"]
    assert res["best_energy"] == E.min() and res["spin_updates"] == R * 300 * inst.N


@pytest.mark.parametrize("N", [5, 300, 1100])
def test_dense_create_validation(N):
    """Instance validation (parallel, tiled scan): each malformed input gets its
    status; with several faults the first one in row-by-row order decides: a
    non-finite value anywhere first, then the lowest row with a diagonal
    entry or an asymmetric pair (j > i), the diagonal first within a row."""
    M = _mars()
    base = I.sk_instance(N, 8).J

    def status(J):
        try:
            M.Instance.dense(J).close()
        except M.MarsError as e:
            return e.status
        return 0

    assert status(base) == 0
    A = base.copy()
    A[N - 1, 0] = np.nextafter(A[N - 1, 0], np.float32(2.0))  # pair (0, N-1) differs: found in row 0
    assert status(A) == 2
    AD = A.copy()
    AD[N // 2, N // 2] = 0.5  # a later row's diagonal does not win over row 0
    assert status(AD) == 2
    D = base.copy()
    D[N // 2, N // 2] = 0.5
    assert status(D) == 3
    DA = D.copy()
    DA[N // 2, N - 1] += np.float32(1.0)  # same row: the diagonal wins
    assert status(DA) == 3
    F = DA.copy()
    F[N - 1, N - 2] = np.nan  # a non-finite value anywhere wins
    assert status(F) == 4


@pytest.mark.parametrize("kind", ["subnormal", "wide"])
def test_dense_exponent_range_pins(kind):
    """The fixed point covers every coupling exactly (subnormal couplings, or
    normal ones spanning ~50 bits): energies equal the exactly rounded sums."""
    M = _mars()
    torch = require_gpu()
    N = 40
    rng = np.random.default_rng(9)
    J = rng.standard_normal((N, N)).astype(np.float32)
    if kind == "subnormal":
        J = (J * np.float32(1e-40)).astype(np.float32)
        assert np.all(np.abs(J[J != 0]) < np.finfo(np.float32).tiny)
    else:
        J[0, 1] = np.float32(2.0**20 + 1.0)
    J = np.triu(J, 1)
    J = (J + J.T).astype(np.float32)
    inst = I.DenseInstance(J=J, h=None)
    S = I.random_spins(N, 12, 4)
    with M.Instance.from_inputs(inst) as g:
        E = g.energy(torch.from_numpy(S).cuda()).cpu().numpy()
    assert np.array_equal(E, O.energy(inst, S))


@pytest.mark.parametrize("N,R,levels,damping,field", [
    (130, 200, 1, 1.0, 0.0),   # blocks of 64, 64, 2
    (300, 1031, 1, 1.0, 0.3),  # ragged runs, field
    (64, 77, 1, 0.5, 0.0),     # one full block, damped
    (65, 129, 3, 1.0, 0.2),    # a one-spin last block, three levels
    (517, 300, 2, 1.0, 0.0),
])
def test_sequential_parity(N, R, levels, damping, field):
    """Sequential update (every spin its own phase, in index order; blocks of
    64 spins with the in-block correction) against the oracle with one phase
    per spin: fp32 within 1e-5 after one level; over several levels within
    1e-5 on every run the oracle finds well conditioned (at most 10 %
    excluded)."""
    M = _mars()
    inst = I.sk_instance(N, 3, field_scale=field)
    sch = _sched(inst, update="sequential", damping=damping, level_count=levels)
    announce("dense sequential", N, R, levels, damping, field)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 31, want_m=True)
        _, phases = g.describe(sch)
    assert phases == N
    ref = O.solve(inst, R, sch, 31, run_count=R)
    if levels == 1:
        err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
        assert err <= TOL_FP32, err
    else:
        c16_parity(out["m"].cpu().numpy(), inst, R, sch, 31, ref, "fp32", max_excluded=0.15,
                   label="sequential N=%d levels %d" % (N, levels))


def test_sequential_unsupported_forms():
    M = _mars()
    inst = I.sk_instance(100, 3)
    with M.Instance.from_inputs(inst) as g:
        with pytest.raises(M.MarsError) as e:
            g.solve_ex(16, _sched(inst, update="sequential", precision="bf16"), 1)
        assert e.value.status == 8
    with M.Instance.from_inputs(I.lattice_instance((8, 8), 1)) as g:
        with pytest.raises(M.MarsError) as e:
            g.solve_ex(16, _sched(I.lattice_instance((8, 8), 1), update="sequential", precision="fp32"), 1)
        assert e.value.status == 8
