"""GPU checks of the BF16 form of the dense path (bf16 couplings and
magnetisations, fp32 accumulation; rounding and energies exact).

This form changes the method's arithmetic, so there is no 1e-5 bar:
* one level from the same draws: the oracle runs on the bf16-rounded
  couplings and initial state (rounded here in the test), so the remaining
  difference is the bf16 rounding of the new magnetisation (at most 2^-9 for
  |m| <= 1) plus fp32 accumulation;
* whole anneals: the fraction of rounded spins that differ from the FP64
  oracle's, and the best-energy gap against the oracle on the same seeds,
  compared with the fp32 form's."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, energy_fsum_dense, require_gpu

pytestmark = pytest.mark.gpu


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _sched(inst, **kw):
    s = I.field_scale(inst)
    base = dict(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, phases=2, precision="bf16")
    base.update(kw)
    return I.Schedule(**base)


@pytest.mark.parametrize("N,R,phases,field", [(1000, 300, 1, 0.0), (517, 129, 1, 0.4), (130, 1, 1, 0.0),
                                              (1000, 300, 2, 0.0), (517, 129, 3, 0.4)])
def test_bf16_one_level(N, R, phases, field):
    """With one phase every field comes from the same (rounded) state, so the
    only differences are the bf16 rounding of the result (<= 2^-9) and fp32
    accumulation.  With several phases, later phases also see earlier phases'
    rounded results: each of those differs by <= 2^-9 |m_j|, which moves
    Phi_i by at most 2^-9 sum_j |J_ij m_j| over the earlier phases."""
    M = _mars()
    inst = I.sk_instance(N, 2, field_scale=field)
    update = "jacobi" if phases == 1 else "phased"
    sch = _sched(inst, phases=phases, update=update, level_count=1)
    announce("bf16 one level", N, R, phases, field)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 99, want_m=True, want_T0=True)
    rinst = I.DenseInstance(J=bf16_round(inst.J), h=inst.h)
    m0 = bf16_round(O.initial_m(99, R, N).astype(np.float32)).astype(np.float64)
    ref = O.solve(rinst, R, sch.replace(precision="fp32"), 99, run_count=R, m0=m0)
    tol = np.full(ref["m"].shape, 2.0**-9 + 1e-5)
    if phases > 1:
        ph, _ = O.phases(rinst, sch)
        Jr = np.abs(rinst.J.astype(np.float64))
        earlier = ph[None, :] < ph[:, None]
        prop = (Jr * earlier) @ np.abs(ref["m"]) * 2.0**-9
        tol += (1 - ref["m"] ** 2) * prop / ref["T0"][None, :] * 1.01
    err = np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"])
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("tile", ["0", "1", "2", "3", "4"])
def test_bf16_tile_variants_bitwise(tile, monkeypatch):
    """The autotuner may pick any tile variant: every variant reduces each
    element over K in the same order, so a 20-level anneal with a forced
    variant equals the tuner's choice bit for bit (ragged runs and phase
    widths, nonzero field)."""
    M = _mars()
    inst = I.sk_instance(517, 4, field_scale=0.3)
    sch = _sched(inst, steps=20, phases=3)
    announce("bf16 tile variant", tile)
    monkeypatch.delenv("MARS_BF16_TILE", raising=False)
    with M.Instance.from_inputs(inst) as g:
        a = g.solve_ex(300, sch, 3, want_m=True, want_spins=True)
        monkeypatch.setenv("MARS_BF16_TILE", tile)
        b = g.solve_ex(300, sch, 3, want_m=True, want_spins=True)
    assert np.array_equal(a["m"].cpu().numpy(), b["m"].cpu().numpy())
    assert np.array_equal(a["spins"].cpu().numpy(), b["spins"].cpu().numpy())
    assert np.array_equal(a["energies"].cpu().numpy(), b["energies"].cpu().numpy())


@pytest.mark.parametrize("tile", ["1", "2", "3", "4"])
def test_bf16_one_level_small_tiles(tile, monkeypatch):
    """One level on each forced non-default variant, same bar as the default tile."""
    monkeypatch.setenv("MARS_BF16_TILE", tile)
    test_bf16_one_level(517, 129, 3, 0.4)


def test_bf16_anneal_quality_vs_fp32_and_oracle():
    """Whole anneal: the bf16 form's best-energy gap to the FP64 oracle (same
    seeds) is no worse than the fp32 form's by more than 0.2 % of |E|, and its
    spin-mismatch fraction is reported."""
    M = _mars()
    N, R = 384, 256
    inst = I.sk_instance(N, 21)
    sch = _sched(inst)
    announce("bf16 anneal quality", N, R)
    with M.Instance.from_inputs(inst) as g:
        b = g.solve_ex(R, sch, 7, want_spins=True)
        f = g.solve_ex(R, sch.replace(precision="fp32"), 7, want_spins=True)
    ref = O.solve(inst, R, sch.replace(precision="fp64"), 7, run_count=R)
    Eo = ref["energy"].min()
    gap_b = (b["result"]["best_energy"] - Eo) / abs(Eo)
    gap_f = (f["result"]["best_energy"] - Eo) / abs(Eo)
    Sb = b["spins"].cpu().numpy()
    mismatch = float(np.mean(np.minimum(np.mean(Sb != ref["spins"], axis=1), np.mean(Sb != -ref["spins"], axis=1))))
    print("best-energy gap bf16 %.4f%% fp32 %.4f%%; spin mismatch %.3f" % (100 * gap_b, 100 * gap_f, mismatch))
    assert gap_b <= gap_f + 2e-3
    # the bf16 form's energies are exact for its own spins
    Eb = b["energies"].cpu().numpy()
    r = int(np.argmin(Eb))
    assert energy_fsum_dense(inst.J, inst.h, Sb[r]) == Eb[r]


def test_bf16_paper_schedule_runs():
    """The paper's scheduler (several sweeps per level) on the bf16 form: level
    counts equal the oracle's (same draws), every run finishes."""
    M = _mars()
    inst = I.sk_instance(200, 3)
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=3.0 * s, c_step=0.25 * s, max_sweeps=200, d_min=1e-3,
                     phases=4, precision="bf16")
    announce("bf16 paper schedule")
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(64, sch, 5)
    ref = O.solve(inst, 64, sch.replace(precision="fp64"), 5, run_count=64)
    assert out["result"]["levels_executed"] == int(ref["levels"].sum())
    assert out["result"]["sweeps_executed"] >= out["result"]["levels_executed"]


def test_bf16_bench_configuration():
    """SK N=2000 x 4096 runs x 300 levels in bf16: sampled runs against the
    FP64 oracle (spin agreement up to a global flip), exact best energy."""
    M = _mars()
    w = I.workload("sk2000", seed=1)
    sch = w.schedule.replace(precision="bf16")
    announce("bf16 sk2000", w.runs)
    with M.Instance.from_inputs(w.instance) as g:
        out = g.solve_ex(w.runs, sch, 1, want_spins=True)
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    agree = []
    for r in (0, 2048, 4095):
        one = O.solve(w.instance, w.runs, w.schedule.replace(precision="fp64"), 1, run_begin=r, run_count=1)
        agree.append(max(np.mean(S[r] == one["spins"][0]), np.mean(S[r] == -one["spins"][0])))
        assert abs(E[r] - one["energy"][0]) <= 0.03 * abs(one["energy"][0])
    print("sampled spin agreement with the oracle:", agree)
    b = int(np.argmin(E))
    assert energy_fsum_dense(w.instance.J, None, S[b]) == E[b] == out["result"]["best_energy"]
