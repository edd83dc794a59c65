"""MARS benchmark: spin-updates/s of whole solves on one MI355X.

One step = one complete solve of the workload (initial draws, every
temperature level and phase, rounding, exact energies, best-of-runs), with
the instance already resident in HBM.  Prints one JSON line.

Default workload: dense SK N=2000, J ~ N(0, 1/N) fp32, 4096 runs, 300
geometric levels, 2 update phases per sweep (the shape of the paper's
largest SK experiment).  Dense workloads are measured in both forms (fp32
and bf16 matrix cores) on the same seeds; the reported value is the fastest
form whose best energy is no worse than the fp32 form's (equal best-energy
gap), and "forms" lists both.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin-updates/s (runs×N×steps) at equal best-energy gap; p50/p99 solve latency"
# TFLOP/s except hbm (GB/s).  *_valu: vector FMA without packed-fp32 issue
# (the library is built without it): 256 CUs x 64 lanes x 2 flops x 2.4 GHz.
PEAK = {"fp32_mfma": 157.3, "bf16_mfma": 2500.0, "hbm": 8000.0, "fp32_valu": 78.6, "fp64_valu": 78.6}

# HBM bytes of one launch of the dominant kernel from rocprofv3 FETCH_SIZE /
# WRITE_SIZE (KiB per dispatch), scaled by the counters' reading of a plain
# 256 MiB copy, by (workload, form).  Valid only for the kernel sources they
# were taken on (sha256 over the listed files in order).  The LDS-resident
# solvers read almost nothing from HBM: what they write is the rounded spins
# (one byte per spin and run) and run counters.
_CSRC = "paper_1907_05124_amd/csrc/"
KERNEL_SOURCES = {
    "k_dense_phase_f32": [_CSRC + "dense_phase.h", _CSRC + "k_dense.hip", _CSRC + "common_device.h"],
    "k_dense_phase_bf16": [_CSRC + "dense_phase_bf16.h", _CSRC + "k_dense_bf16.hip", _CSRC + "common_device.h"],
    "k_lattice_solve": [_CSRC + "k_lattice.hip", _CSRC + "lds_state.h", _CSRC + "common_device.h"],
    "k_sparse_solve": [_CSRC + "sparse_solve.h", _CSRC + "k_sparse.hip", _CSRC + "k_sparse_split.hip",
                       _CSRC + "lds_state.h", _CSRC + "common_device.h"],
}
TRAFFIC_RECORD = {
    ("sk2000", "fp32"): {"kernel": "k_dense_phase_f32", "sha256_prefix": "5e141b5bb4edf753",
        "fetch_kib": 60399.2, "write_kib": 27264.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_dense_phase_f32_sk2000.md"},
    ("sk2000", "bf16"): {"kernel": "k_dense_phase_bf16", "sha256_prefix": "abd9cf6588efd30d",
        "fetch_kib": 26429.7, "write_kib": 8256.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_dense_phase_bf16_sk2000.md"},
    ("er800", "fp32"): {"kernel": "k_sparse_solve", "sha256_prefix": "5c4273a474ee9f48",
        "fetch_kib": 1210.9, "write_kib": 6656.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_sparse_solve_er800.md"},
    ("er800", "fp16"): {"kernel": "k_sparse_solve", "sha256_prefix": "5c4273a474ee9f48",
        "fetch_kib": 1210.9, "write_kib": 6656.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_sparse_solve_er800.md"},
    ("er20000", "fp16"): {"kernel": "k_sparse_solve", "sha256_prefix": "5c4273a474ee9f48",
        "fetch_kib": 3424.0, "write_kib": 165309.7, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_sparse_solve_er20000.md"},
    ("ea2d_L16", "fp64"): {"kernel": "k_lattice_solve", "sha256_prefix": "cbc9d812e2337556",
        "fetch_kib": 115.2, "write_kib": 288.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_lattice_solve_ea2d_L16.md"},
    ("ea2d_L16", "fp32"): {"kernel": "k_lattice_solve", "sha256_prefix": "cbc9d812e2337556",
        "fetch_kib": 111.9, "write_kib": 288.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_lattice_solve_ea2d_L16.md"},
    ("ea3d_L32", "fp16"): {"kernel": "k_lattice_solve", "sha256_prefix": "cbc9d812e2337556",
        "fetch_kib": 1030.6, "write_kib": 65600.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "summary": "profiles/k_lattice_solve_ea3d_L32.md"},
}


DESCRIPTION = {
    "sk2000": "SK N=2000 J~N(0,1/N) (fp32 input), 4096 runs, T0~U[0.25,1.5]*sigma, 300 geometric levels to "
              "0.01*sigma, 2 phases; fp32 and bf16 matrix-core forms",
    "ea2d_L16": "2D +-J lattice 16x16 periodic, 1024 runs, T0~U[0.5,3], 300 geometric levels to 0.02, fp64",
    "er800": "Erdos-Renyi N=800 p=0.06 +-1 weights (J=-w), 8192 runs, 300 levels, greedy-colour phases, fp32",
    "er20000": "Erdos-Renyi N=20000 avg degree 4 +-1 weights (J=-w), 8192 runs, 300 levels, fp32",
    "ea3d_L32": "3D +-J lattice 32^3 periodic, 2048 runs, 1000 levels, fp16 magnetisation storage",
    "served": "served mixed stream: Poisson arrivals, N log-uniform in [100,10000], half dense SK (bf16 form), "
              "half ER degree-4 +-1 (fp32), 256-4096 runs each, 300 levels; admission by HBM footprint, "
              "concurrent solves on 4 streams",
}


def sources_sha(kernel):
    """sha256 prefix over the sources a kernel is built from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, precision):
    """Bytes per launch from the recorded counters, or None if the kernel changed since."""
    rec = TRAFFIC_RECORD.get((workload, precision))
    if rec is None or sources_sha(rec["kernel"]) != rec["sha256_prefix"]:
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def tts99(m, E_target, R):
    """Time to reach E_target with probability 0.99 (the time-to-solution of
    the paper's evaluation, with the runs of one solve as the samples): the
    per-run time at the solve's throughput, ms / R, times the number of runs
    ln(0.01) / ln(1 - P) needed, P = fraction of runs with E <= E_target
    (at least one run; None if no run reaches it)."""
    import numpy as np

    P = float(np.mean(m["energies"] <= E_target))
    if P <= 0.0:
        return None
    t_run = m["ms_per_step"] / R
    if P >= 0.99:
        return t_run
    return t_run * max(1.0, math.log(0.01) / math.log(1.0 - P))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, seed, budget_s=12.0):
    """Time the CPU oracle (FP64, threads over runs) on a bounded sample of runs."""
    from oracle import oracle as O

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    N = w.instance.N
    sch = w.schedule.replace(precision="fp64") if w.schedule.precision != "fp64" else w.schedule
    n = cores
    total_runs, total_t, total_upd = 0, 0.0, 0
    spins, energies = [], []
    while True:
        t0 = time.perf_counter()
        r = O.solve(w.instance, w.runs, sch, seed, run_begin=total_runs, run_count=n, nthreads=cores)
        dt = time.perf_counter() - t0
        total_runs += n
        total_t += dt
        total_upd += int(r["sweeps"].sum()) * N
        spins.append(r["spins"])
        energies.append(r["energy"])
        if total_t >= budget_s or total_runs >= w.runs:
            break
        # grow the sample towards the budget
        n = max(cores, min(w.runs - total_runs, int(n * max(1.0, (budget_s - total_t) / max(dt, 1e-3)))))
    import numpy as np

    out = {"value": total_upd / total_t, "unit": "spin-updates/s", "cores": cores, "kind": "oracle",
           "sample": "%d of %d runs at full N=%d and full schedule, %.1f s" % (total_runs, w.runs, N, total_t)}
    return out, np.concatenate(spins), np.concatenate(energies)


def vs_oracle(m, spins, energies, symmetric):
    """The form's rounded spins and best energy against the FP64 oracle on
    the oracle's sample of runs (the first runs, same seeds): mean fraction of
    spins that differ (up to a global flip when h = 0, where s and -s have the
    same energy) and the relative gap of the sample's best energies."""
    import numpy as np

    n = len(energies)
    S = m["spins"][:n]
    diff = np.mean(S != spins, axis=1)
    if symmetric:
        diff = np.minimum(diff, np.mean(S != -spins, axis=1))
    Eo = float(np.min(energies))
    Eg = float(np.min(m["energies"][:n]))
    return {"runs": int(n), "spin_mismatch": float(np.mean(diff)), "best_gap": (Eg - Eo) / abs(Eo) if Eo else 0.0}


def copy_calibration():
    """One plain device-to-device copy of 256 MiB (after a warm-up copy): the
    reference for scaling FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch

    n = (256 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "ms": ms,
                      "GB/s": 2 * n * 4 / ms / 1e6}), flush=True)


def work_roofline(done, requests, makespan_s):
    """The capacity pass against the roofline of its own work mix: every
    completed request's algorithmic flops (2 per coupling term and update:
    2N per spin-update for dense J, 2 nnz / N for sparse J) at the peak of
    the unit that bounds its kernel (bf16 MFMA for dense requests, the fp32
    vector ALU for sparse ones), summed into the time a perfectly fed GPU
    would take; frac = that time / the measured makespan."""
    by = {r.rid: r for r in requests}
    flops = {"dense": 0.0, "sparse": 0.0}
    ideal = 0.0
    for c in done:
        r = by[c.rid]
        upd = float(c.result["spin_updates"])
        if r.dense:
            f = 2.0 * r.N * upd
            ideal += f / (PEAK["bf16_mfma"] * 1e12)
            flops["dense"] += f
        else:
            f = 2.0 * r.instance.nnz / r.N * upd
            ideal += f / (PEAK["fp32_valu"] * 1e12)
            flops["sparse"] += f
    return {"dense_flop": flops["dense"], "sparse_flop": flops["sparse"], "dense_peak_tflops": PEAK["bf16_mfma"],
            "sparse_peak_tflops": PEAK["fp32_valu"], "ideal_s": ideal, "makespan_s": makespan_s,
            "frac": ideal / makespan_s if makespan_s > 0 else None}


def served_cpu_baseline(base, seed_budget_s=12.0):
    """The CPU oracle on a bounded sample of the served stream: requests in
    stream order, each with as many runs as there are cores (full N and
    schedule, fp64), skipping requests whose estimated cost would overrun the
    budget; spin-updates/s over the sample."""
    from oracle import oracle as O

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    t_tot, upd, n_req, n_runs = 0.0, 0, 0, 0
    for r in base:
        terms = r.N * r.N if r.dense else r.instance.nnz
        est = terms * r.schedule.steps * cores / (cores * 4e8)  # ~4e8 coupling terms/s per core
        if t_tot + est > seed_budget_s:
            continue
        n = min(cores, r.runs)
        t0 = time.perf_counter()
        res = O.solve(r.instance, r.runs, r.schedule.replace(precision="fp64"), r.seed, run_count=n, nthreads=cores)
        t_tot += time.perf_counter() - t0
        upd += int(res["sweeps"].sum()) * r.N
        n_req += 1
        n_runs += n
        if t_tot >= seed_budget_s:
            break
    return {"value": upd / t_tot if t_tot > 0 else None, "unit": "spin-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d runs of %d of the stream's requests (in stream order, full N and schedule, fp64), %.1f s"
                      % (n_runs, n_req, t_tot)}


def served(args):
    """Served mixed stream: a capacity pass (all requests at t = 0), then
    Poisson passes at the given fractions of that capacity (default 0.7);
    latency is arrival to result.  The same instances serve every pass (the
    arrival times differ)."""
    import torch

    from paper_1907_05124_amd import serve as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    server = S.MarsServer(max_active=8, n_streams=4, batching=not args.no_batching, grouping=not args.no_batching)
    fracs = [float(x) for x in args.rates.split(",")]

    base = S.mixed_stream(args.requests, 1e9, seed=args.seed)
    # synthetic inputs are generated before the clock starts (threads: the
    # generators spend their time in numpy, outside the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as pool:
        for k, inst in enumerate(pool.map(lambda r: r.materialize(), base)):
            base[k].instance = inst
            if (k + 1) % 200 == 0:
                log("materialised %d / %d instances" % (k + 1, len(base)))

    def make(rate):
        reqs = S.mixed_stream(args.requests, rate, seed=args.seed)
        for r, b in zip(reqs, base):
            assert r.runs == b.runs and r.N == b.N
            r.instance = b.instance
        return reqs

    warm = S.mixed_stream(4, 1e9, seed=args.seed + 7, n_hi=500)
    server.run(warm)
    log("capacity pass: %d requests" % len(base))
    done, cap = server.run(base, progress=log)
    cap["work_roofline"] = work_roofline(done, base, cap["makespan_s"])
    capacity = cap["requests"] / cap["makespan_s"]
    log("capacity", cap, "-> %.2f req/s" % capacity)
    sweep = []
    for f in fracs:
        rate = f * capacity
        _, st = server.run(make(rate), progress=log)
        log("load pass at %.2f of capacity (%.2f req/s)" % (f, rate), st)
        sweep.append({"fraction_of_capacity": f, "offered_rate_per_s": rate, **st})
    head = next((x for x in sweep if abs(x["fraction_of_capacity"] - 0.7) < 1e-9), sweep[-1])
    line = {
        "metric": METRIC, "value": head["spin_updates_per_s"], "unit": "spin-updates/s", "n_gpus": 1,
        "steps": head["requests"], "warmup": len(warm),
        "ms_per_step": head["makespan_s"] * 1e3 / max(1, head["requests"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (dense) / f32 (sparse)",
        "data": "synthetic",
        "config": {"workload": "served", "description": DESCRIPTION["served"], "requests": head["requests"],
                   "offered_rate_per_s": head["offered_rate_per_s"],
                   "fraction_of_capacity": head["fraction_of_capacity"], "batching": not args.no_batching,
                   "parallelism": "single GPU, concurrent streams"},
        "latency_ms": {"p50": head["latency_p50_ms"], "p99": head["latency_p99_ms"]},
        "capacity": cap, "load_sweep": sweep,
    }
    # the capacity pass against the roofline of its own work mix: the flops of
    # every request at the peak of the unit bounding its kernel, over the makespan
    wr = cap["work_roofline"]
    total = wr["dense_flop"] + wr["sparse_flop"]
    line["roofline"] = {"bound": "mfma", "work_weighted": True,
                        "achieved": round(total / wr["makespan_s"] / 1e12, 3),
                        "peak": round(total / wr["ideal_s"] / 1e12, 3), "unit": "TFLOP/s",
                        "frac": round(wr["frac"], 4), "traffic": None,
                        "mix": {"dense_flop": wr["dense_flop"], "sparse_flop": wr["sparse_flop"],
                                "dense_peak_tflops": wr["dense_peak_tflops"],
                                "sparse_peak_tflops": wr["sparse_peak_tflops"]}}
    line["cpu_baseline"] = None if args.no_cpu_baseline else served_cpu_baseline(base)
    if line["cpu_baseline"]:
        log("cpu baseline", line["cpu_baseline"])
    print(json.dumps(line), flush=True)


SUB_CONFIGS = ["ea2d_L16", "er800", "er20000", "ea3d_L32"]


def bench_workload(name, args, *, cpu_budget_s, steps, warmup):
    """Time every form of one workload (K whole solves on the library's stream,
    after W untimed ones), its dominant kernel against its roofline, and the
    CPU oracle on a bounded sample of the same runs.  Returns the fields of a
    bench line."""
    import numpy as np
    import torch

    from paper_1907_05124_amd import inputs as I
    from paper_1907_05124_amd import mars as M

    w = I.workload(name, seed=args.seed)
    N, R = w.instance.N, w.runs
    log("workload", name, "N=%d R=%d" % (N, R))
    inst = M.Instance.from_inputs(w.instance)
    stream = torch.cuda.current_stream()
    dense = isinstance(w.instance, I.DenseInstance)
    if args.precision:
        forms = [args.precision]
    elif dense:
        forms = ["fp32", "bf16"]  # the exact-arithmetic form and the bf16 matrix-core form
    elif isinstance(w.instance, I.CsrInstance) and w.schedule.precision == "fp32":
        forms = ["fp32", "fp16"]  # fp32 state, and fp16 state storage with fp32 fields (twice the runs per CU)
    elif isinstance(w.instance, I.LatticeInstance) and w.schedule.precision == "fp64":
        forms = ["fp64", "fp32"]  # the fp64 form the oracle is compared with, and fp32 state
    else:
        forms = [w.schedule.precision]

    def measure(prec, update=None):
        sch = w.schedule.replace(precision=prec)
        if update is not None:
            sch = sch.replace(update=update)

        def solve(sc):
            return inst.solve_ex(R, sc, args.seed, want_best=True, sync=False, stream=stream)

        for i in range(warmup):
            solve(sch)
            torch.cuda.synchronize()
            log(name, prec, "warmup", i + 1, "done")
        # timed region: K whole solves, events on the library's stream
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(steps):
            solve(sch)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        ms = float(np.mean(step_ms))
        log("%s %s%s: timed %d steps: %.3f ms/step (wall %.3f s)"
            % (name, prec, "" if update is None else " " + update, steps, ms, wall))
        # the same solve once more with host results: update count and summary
        once = inst.solve_ex(R, sch, args.seed, want_best=True, want_spins=True, sync=True, stream=stream)
        res = once["result"]
        out = {"precision": prec, "ms_per_step": ms, "value": int(res["spin_updates"]) / (ms * 1e-3),
               "step_ms": step_ms, "result": res, "roofline": None, "energies": once["energies"].cpu().numpy(),
               "spins": once["spins"].cpu().numpy()}
        del once
        # solve with no levels (draws, rounding, energies, best-of-runs), timed
        # with events on the same stream: the solve minus it is the time of
        # the anneal kernels
        zero = sch.replace(steps=0)
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        solve(zero)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            solve(zero)
        e1.record(stream)
        torch.cuda.synchronize()
        base_ms = e0.elapsed_time(e1) / reps
        if dense:
            # dominant kernel: the field product of one phase (one launch per
            # phase and level)
            _, phases = inst.describe(sch)
            launches = sch.steps * phases
            per_launch_s = max(ms - base_ms, 1e-6) * 1e-3 / launches
            # algorithmic flops of one phase launch: 2 * (rows of the phase) * N * R
            flops = 2.0 * (N / phases) * N * R
            achieved = flops / per_launch_s / 1e12
            peak = PEAK["bf16_mfma"] if prec == "bf16" else PEAK["fp32_mfma"]
            kname = "k_dense_phase_bf16" if prec == "bf16" else "k_dense_phase_f32"
            out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                               "frac": round(achieved / peak, 4),
                               "traffic": recorded_traffic(name, prec),
                               "kernel": kname, "launches": launches, "launch_us": round(per_launch_s * 1e6, 3),
                               "flops_per_launch": flops}
        else:
            # one launch of the LDS-resident solver holds the whole anneal; its
            # algorithmic work is 2 flops per coupling term: sweeps x nnz terms
            lat = isinstance(w.instance, I.LatticeInstance)
            nnz = 2 * w.instance.dim * N if lat else w.instance.nnz
            per_launch_s = max(ms - base_ms, 1e-6) * 1e-3
            flops = 2.0 * float(res["sweeps_executed"]) * nnz
            achieved = flops / per_launch_s / 1e12
            peak = PEAK["fp64_valu"] if prec == "fp64" else PEAK["fp32_valu"]
            out["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                               "frac": round(achieved / peak, 4),
                               "traffic": recorded_traffic(name, prec),
                               "kernel": "k_lattice_solve" if lat else "k_sparse_solve", "launches": 1,
                               "launch_us": round(per_launch_s * 1e6, 3), "flops_per_launch": flops}
        return out

    measured = {p: measure(p) for p in forms}
    # headline: the fastest form whose best energy (same seeds, exact energies)
    # is no worse than the reference form's, i.e. at an equal best-energy gap
    ref_form = forms[0]
    E_ref = measured[ref_form]["result"]["best_energy"]
    tol = 1e-9 * max(1.0, abs(E_ref))
    eligible = [p for p in forms if measured[p]["result"]["best_energy"] <= E_ref + tol]
    head = max(eligible, key=lambda p: measured[p]["value"])
    hm = measured[head]
    forms_out = {p: {"value": measured[p]["value"], "ms_per_step": measured[p]["ms_per_step"],
                     "best_energy": measured[p]["result"]["best_energy"],
                     "equal_gap": p in eligible, "tts99_ms": tts99(measured[p], E_ref + tol, R),
                     "roofline": measured[p]["roofline"]} for p in forms}
    w.schedule = w.schedule.replace(precision=head)
    # literal reading of the pseudocode (one synchronous phase) on the 2D
    # lattice, timed like the forms: a fidelity row, never the headline (its
    # runs fall into the 2-cycles of the synchronous update)
    fidelity = None
    if name == "ea2d_L16" and not args.precision:
        jm = measure("fp64", update="jacobi")
        jr = jm["result"]
        fidelity = {"jacobi_fp64": {"value": jm["value"], "ms_per_step": jm["ms_per_step"],
                                    "best_energy": jr["best_energy"],
                                    "best_energy_per_spin": jr["best_energy"] / N,
                                    "mean_energy_per_spin": jr["mean_energy"] / N,
                                    "positive_energy_runs": float(np.mean(jm["energies"] > 0))}}
        del jm

    cpu = None
    if not args.no_cpu_baseline:
        log(name, "cpu baseline ...")
        cpu, o_spins, o_energies = cpu_baseline(w, args.seed, budget_s=cpu_budget_s)
        log(name, "cpu baseline", cpu)
        h = getattr(w.instance, "h", None)
        symmetric = h is None or not np.any(h)
        for p in forms:
            forms_out[p]["vs_oracle"] = vs_oracle(measured[p], o_spins, o_energies, symmetric)
        log(name, "vs oracle", {p: forms_out[p]["vs_oracle"] for p in forms})
    inst.close()

    res = hm["result"]
    dtype = {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "fp16": "f16-store/f32"}[head]
    return {
        "value": hm["value"], "ms_per_step": hm["ms_per_step"], "dtype": dtype,
        "config": {"workload": name, "description": DESCRIPTION[name], "N": N, "runs": R,
                   "levels": w.schedule.steps, "parallelism": "single GPU, runs batched"},
        "latency_ms": {"p50": float(np.percentile(hm["step_ms"], 50)),
                       "p99": float(np.percentile(hm["step_ms"], 99))},
        "forms": forms_out,
        **({"fidelity": fidelity} if fidelity else {}),
        "result": {"best_energy": res["best_energy"], "best_energy_per_spin": res["best_energy"] / N,
                   "mean_energy_per_spin": res["mean_energy"] / N, "hit_count": res["hit_count"]},
        "roofline": hm["roofline"], "cpu_baseline": cpu,
        **({"vs_oracle": forms_out[head]["vs_oracle"]} if cpu else {}),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sk2000", choices=sorted(DESCRIPTION))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16", "fp16"],
                    help="override the workload's arithmetic form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="default workload only: leave out the per-configuration records of the other workloads")
    ap.add_argument("--rates", default="0.7",
                    help="served workload: offered loads as fractions of the measured capacity, comma separated")
    ap.add_argument("--no-batching", action="store_true",
                    help="served workload: run every request alone on the stream pool (no dense batch, no sparse groups)")
    ap.add_argument("--requests", type=int, default=200, help="served workload: number of requests")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (to scale rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print("bench.py measures one GPU and has no multi-GPU path (runs would shard by index across GPUs, "
              "with one all-reduce-min of the best energies per instance).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "served":
        return served(args)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    head = bench_workload(args.workload, args, cpu_budget_s=12.0, steps=args.steps, warmup=args.warmup)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "spin-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic", **{k: v for k, v in head.items()
                                                                            if k not in ("value", "ms_per_step",
                                                                                         "dtype")},
    }
    if args.workload == "sk2000" and not args.no_configs and not args.precision:
        # the other configurations of the measurement table, same protocol,
        # smaller CPU samples (a few seconds each)
        line["configs"] = {}
        for name in SUB_CONFIGS:
            line["configs"][name] = bench_workload(name, args, cpu_budget_s=4.0, steps=args.steps,
                                                   warmup=args.warmup)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
