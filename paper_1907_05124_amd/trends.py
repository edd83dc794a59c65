"""Solution-quality trends on synthetic instances (the shape of the paper's
tables of best energy, mean energy and success probability against the
number of runs and against the temperature range), measured with the HIP
library on the current GPU.

    python -m paper_1907_05124_amd.trends runs     # SK: best / mean / P / TTS99 vs runs
    python -m paper_1907_05124_amd.trends trange   # temperature ranges, sigma- vs spectrum-scaled

Each line printed is one JSON record; a markdown table follows.  Instances are
the seeded generators' (stand-ins for the paper's unpublished SK matrices and
graph sets)."""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs as I


def _solve(g, R, sch, seed):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = g.solve_ex(R, sch, seed)
    torch.cuda.synchronize()
    return out["energies"].cpu().numpy(), time.perf_counter() - t0


def _tts99(P, t_run):
    if P <= 0.0:
        return None
    if P >= 0.99:
        return t_run
    return t_run * max(1.0, math.log(0.01) / math.log(1.0 - P))


def runs_trend(N=1000, seed=11, counts=(64, 256, 1024, 4096, 8192), forms=("fp32", "bf16")):
    """Best / mean energy per spin and the success probability P (fraction of
    runs within 0.1 % of the best energy found over all runs and forms) as the
    number of runs grows, for SK N(0, 1/N) couplings; TTS99 from P and the
    per-run time at the solve's throughput."""
    from . import mars as M

    inst = I.sk_instance(N, seed)
    s = I.field_scale(inst)
    rows = []
    with M.Instance.from_inputs(inst) as g:
        sched = g.auto_temperatures(I.Schedule(steps=300, phases=2), steps=150, seed=3)
        res = {}
        for form in forms:
            sch = sched.replace(precision=form)
            _solve(g, 64, sch, 1)  # warm-up (tuner, buffers)
            for R in counts:
                E, dt = _solve(g, R, sch, 1)
                res[(form, R)] = (E, dt)
        best = min(float(E.min()) for E, _ in res.values())
        target = best + 1e-3 * abs(best)
        for (form, R), (E, dt) in sorted(res.items()):
            P = float(np.mean(E <= target))
            rows.append({"instance": "sk%d" % N, "form": form, "runs": R, "best_per_spin": float(E.min()) / N,
                         "mean_per_spin": float(E.mean()) / N, "P": P, "solve_ms": dt * 1e3,
                         "tts99_ms": _tts99(P, dt * 1e3 / R), "sigma": s})
    return rows


def trange_trend():
    """Best energy, mean energy and the fraction of runs within 0.5 % of the
    best for temperature ranges scaled by sigma_Phi or by lambda_max."""
    from . import mars as M

    fams = [("sk1000", I.sk_instance(1000, 11), 1024),
            ("er800", I.er_instance(800, 12, p=0.06, weights="pm1"), 1024),
            ("er20000", I.er_instance(20000, 13, avg_degree=4.0, weights="pm1"), 512),
            ("ea2d_32", I.lattice_instance((32, 32), 14), 1024),
            ("ea3d_16", I.lattice_instance((16, 16, 16), 15), 512)]
    rows = []
    for name, inst, R in fams:
        sig = I.field_scale(inst)
        with M.Instance.from_inputs(inst) as g:
            lo, hi = g.spectrum(200, seed=3)
            rules = [("sigma x [0.25, 1.5], end 0.01", 0.25 * sig, 1.5 * sig, 0.01 * sig)]
            for a, b in ((0.1, 0.5), (0.2, 1.0), (0.3, 1.25), (0.5, 1.5), (0.3, 2.0)):
                rules.append(("lambda_max x [%g, %g], end 0.005" % (a, b), a * hi, b * hi, 0.005 * hi))
            res = []
            for rn, tl, th, te in rules:
                sch = I.Schedule(T_lo=tl, T_hi=th, T_end=te, steps=300, phases=2, precision="fp32")
                E, _ = _solve(g, R, sch, 5)
                res.append((rn, E))
            best = min(float(E.min()) for _, E in res)
            for rn, E in res:
                rows.append({"instance": name, "N": inst.N, "runs": R, "lambda_min": lo, "lambda_max": hi,
                             "sigma": sig, "range": rn, "best_per_spin": float(E.min()) / inst.N,
                             "mean_per_spin": float(E.mean()) / inst.N,
                             "gap_to_best": (float(E.min()) - best) / abs(best),
                             "within_0.5pct": float(np.mean(E <= best + 5e-3 * abs(best)))})
    return rows


def _table(rows, cols):
    out = ["| " + " | ".join(cols) + " |", "|" + "---|" * len(cols)]
    for r in rows:
        cells = []
        for c in cols:
            v = r[c]
            cells.append("%.5g" % v if isinstance(v, float) else ("—" if v is None else str(v)))
        out.append("| " + " | ".join(cells) + " |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["runs", "trange"])
    a = ap.parse_args()
    import torch

    # the device is set up through torch before the library makes its first HIP call
    if not torch.cuda.is_available():
        raise SystemExit("trends needs a GPU")
    torch.cuda.set_device(0)
    if a.what == "runs":
        rows = runs_trend()
        cols = ["instance", "form", "runs", "best_per_spin", "mean_per_spin", "P", "solve_ms", "tts99_ms"]
    else:
        rows = trange_trend()
        cols = ["instance", "range", "best_per_spin", "mean_per_spin", "gap_to_best", "within_0.5pct"]
    for r in rows:
        print(json.dumps(r), flush=True)
    print(_table(rows, cols), flush=True)


if __name__ == "__main__":
    main()
