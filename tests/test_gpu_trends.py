"""The paper's quality trends (best and mean energy and the success
probability against the number of runs and against the temperature range,
section "Parameter sensitivity analysis") measured on the GPU and checked
against the CPU oracle run on the same seeds: SK N = 256, fp32 form."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, require_gpu

pytestmark = pytest.mark.gpu

COUNTS = (64, 256, 1024)


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


def _summary(E, best_ref=None):
    best = float(np.min(E))
    ref = best if best_ref is None else best_ref
    return {"best": best, "mean": float(np.mean(E)), "hits": int(np.sum(E == ref)), "runs": len(E)}


@pytest.fixture(scope="module")
def trend_data():
    """GPU and oracle energies and spins for SK N = 256 at 64, 256 and 1024
    runs under two temperature ranges: sigma_Phi x [0.25, 1.5] to 0.01 sigma
    (the benchmark's rule) and lambda_max x [0.5, 1.5] to 0.005 lambda_max
    (the spectrum's rule, with lambda_max from the oracle's eigensolver)."""
    M = _mars()
    inst = I.sk_instance(256, 21)
    s = I.field_scale(inst)
    lam = float(O.spectrum(inst)[1])
    ranges = {"sigma": I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300, phases=2),
              "lambda": I.Schedule(T_lo=0.5 * lam, T_hi=1.5 * lam, T_end=0.005 * lam, steps=300, phases=2)}
    out = {}
    with M.Instance.from_inputs(inst) as g:
        for name, sch in ranges.items():
            ref = O.solve(inst, max(COUNTS), sch, 7, run_count=max(COUNTS))
            for R in COUNTS:
                announce("trends", name, R)
                o = g.solve_ex(R, sch, 7, want_spins=True)
                out[(name, R)] = {"E": o["energies"].cpu().numpy(), "S": o["spins"].cpu().numpy(),
                                  "res": o["result"], "E_o": ref["energy"][:R], "S_o": ref["spins"][:R]}
    return out


@pytest.mark.parametrize("rng", ["sigma", "lambda"])
@pytest.mark.parametrize("R", COUNTS)
def test_trend_point_matches_oracle(trend_data, rng, R):
    """One point of the trend: the GPU summary (best energy, its hit count,
    mean) is that of its own exact energies; on the runs whose rounded spins
    equal the oracle's (up to the global flip of h = 0; at least 95 % of the
    runs) the energies are the oracle's bit for bit, so best, mean and hits
    over those runs are the oracle's too."""
    d = trend_data[(rng, R)]
    E, S, res, E_o, S_o = d["E"], d["S"], d["res"], d["E_o"], d["S_o"]
    mine = _summary(E)
    assert res["best_energy"] == mine["best"] and res["hit_count"] == mine["hits"]
    assert abs(res["mean_energy"] - mine["mean"]) <= 1e-12 * abs(mine["mean"])
    match = np.all(S == S_o, axis=1) | np.all(S == -S_o, axis=1)
    print("[trend] %s R=%d: best %.6f mean %.6f hits %d, spins match on %.4f of runs"
          % (rng, R, mine["best"] / 256, mine["mean"] / 256, mine["hits"], match.mean()), flush=True)
    assert match.mean() >= 0.95
    assert np.array_equal(E[match], E_o[match])
    gm, om = _summary(E[match]), _summary(E_o[match])
    assert gm == om


@pytest.mark.parametrize("rng", ["sigma", "lambda"])
def test_trend_with_runs(trend_data, rng):
    """Against the number of runs (Table 3_2's axis): run r is the same
    descent whatever the run count (counter-based draws), so the GPU's
    energies of the first 64 and 256 runs are those of the 1024-run solve bit
    for bit, and the best energy can only fall as runs are added, on the GPU
    and in the oracle."""
    E = {R: trend_data[(rng, R)]["E"] for R in COUNTS}
    Eo = trend_data[(rng, max(COUNTS))]["E_o"]
    for a, b in zip(COUNTS, COUNTS[1:]):
        assert np.array_equal(E[b][:a], E[a])
        assert E[b].min() <= E[a].min() and Eo[:b].min() <= Eo[:a].min()


def test_trend_with_temperature_range(trend_data):
    """Against the temperature range (Table 3_3's axis): the range from the
    spectrum, [0.5, 1.5] x lambda_max, reaches a lower mean energy than
    sigma x [0.25, 1.5] on the GPU and in the oracle alike (a start above
    lambda_max decays towards m = 0 before the cooling picks a direction, so
    many runs forget their random start)."""
    R = max(COUNTS)
    g_sig, g_lam = trend_data[("sigma", R)]["E"].mean(), trend_data[("lambda", R)]["E"].mean()
    o_sig, o_lam = trend_data[("sigma", R)]["E_o"].mean(), trend_data[("lambda", R)]["E_o"].mean()
    print("[trend] mean per spin at R=%d: sigma range %.5f / %.5f (GPU / oracle), lambda range %.5f / %.5f"
          % (R, g_sig / 256, o_sig / 256, g_lam / 256, o_lam / 256), flush=True)
    assert g_lam < g_sig and o_lam < o_sig
