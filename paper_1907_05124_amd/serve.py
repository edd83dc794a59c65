"""Serving loop: continuous batching of Ising solve requests on one GPU.

Requests (an instance, a number of runs, a schedule, a seed and an arrival
time) are admitted as soon as they have arrived and both an active slot and
enough HBM are free; each admitted request keeps its couplings and run state
resident on the GPU while its solve runs on one of a pool of streams, so the
work of different requests overlaps on the device.  An admitted request's
dense instance is created on a worker thread (host validation of the
couplings, encodings and upload: about 0.1 s for N = 10^4), and its solve is
enqueued once it is ready, so that creation overlaps the GPU's work.  Completed requests free
their slot at once and their memory when the GPU is idle or as soon as an
arrived request waits for memory (releasing device memory synchronises the
device, so it is not done while it would only stall running solves).

Dense requests in the BF16 form that are too small to fill the GPU on their
own (fewer 128 x 128 output tiles per update phase than the chip has compute
units) join a batch instead (``mars_batch_*``): every update phase of all
batch members is one launch, and members join and leave between sweeps.
Larger requests run alone on the stream pool, where they fill the GPU
anyway, and do not hold small members back to their pace.  Sparse requests
admitted in the same pass are enqueued together (``mars_solve_group_async``):
those on the same instantiation of the LDS-resident solver share its launch,
which fills the GPU with the workgroups of several small requests at once.

Every solve is independent and deterministic (counter-based draws, fixed
reduction orders), so a request's result is the same whether it runs alone
or in the mix; ``tests/test_gpu_serve.py`` checks that bit for bit.

The scheduling policy (``Scheduler``) is separate from the GPU executor so
that it can be exercised without a GPU.
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I

GROUP_MAX = 64  # solves per mars_solve_group_async call
RESULT_BYTES = 256  # room for one mars_result in a pinned result buffer

# ---------------------------------------------------------------------------
# requests and footprints
# ---------------------------------------------------------------------------


@dataclass
class InstanceSpec:
    """A synthetic instance described by kind, size and seed; materialised on
    admission (dense N = 10^4 couplings are 400 MB of host memory)."""

    kind: str  # "sk" | "er"
    N: int
    seed: int
    avg_degree: float = 4.0

    @property
    def nnz(self) -> int:
        return int(self.avg_degree * self.N) if self.kind == "er" else self.N * self.N

    def materialize(self):
        if self.kind == "sk":
            return I.sk_instance(self.N, self.seed)
        return I.er_instance(self.N, self.seed, avg_degree=min(self.avg_degree, self.N - 1.0), weights="pm1")


@dataclass
class Request:
    rid: int
    instance: object  # an inputs.*Instance or an InstanceSpec
    runs: int
    schedule: I.Schedule
    seed: int
    arrival: float = 0.0  # seconds after the start of the stream

    @property
    def N(self) -> int:
        return self.instance.N

    @property
    def dense(self) -> bool:
        if isinstance(self.instance, InstanceSpec):
            return self.instance.kind == "sk"
        return isinstance(self.instance, I.DenseInstance)

    def materialize(self):
        if isinstance(self.instance, InstanceSpec):
            return self.instance.materialize()
        return self.instance


@dataclass
class Completion:
    rid: int
    result: dict
    best_spins: np.ndarray
    arrival: float
    admitted: float
    finished: float
    footprint: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def footprint_bytes(req: Request) -> int:
    """Upper estimate of the device memory a request holds while it runs
    (instance encodings plus solve workspace), from the library's layouts."""
    inst, R, sc = req.instance, req.runs, req.schedule
    N = inst.N
    levels = sc.steps if sc.kind == "geometric" else int(math.ceil(sc.T_hi / sc.c_step)) + 1
    if req.dense:
        Np = _round_up(N, 128) + 128
        Ke = _round_up(N, 128)
        ldr = _round_up(R, 256)
        inst_b = Np * Np * 4 + 8 * Ke * Ke + N * N * 8  # J fp32, digits, transient fixed point
        if sc.precision == "bf16":
            inst_b += Np * Np * 2
            state = 2 * ldr * Np * 2
        else:
            state = 2 * Np * _round_up(R, 128) * 4
        work = state + ldr * Ke + levels * ldr * 4 + (Ke // 128) * R * 16 + R * 64
    else:
        nnz = getattr(inst, "nnz", 2 * getattr(inst, "dim", 3) * N)
        inst_b = nnz * 4 + N * 16
        work = R * N + R * 64 + levels * 4
    return int((inst_b + work) * 1.05) + (1 << 20)


BATCH_TILES = 256  # one tile per compute unit


def phase_tiles(req: Request) -> int:
    """Output tiles (128 runs x 128 spins) of one update phase of a dense solve."""
    sc = req.schedule
    phases = 1 if sc.update == "jacobi" else max(1, min(sc.phases, req.N))
    width = -(-req.N // phases)
    return -(-req.runs // 128) * -(-width // 128)


def batchable(req: Request, tiles: int = BATCH_TILES) -> bool:
    """A request that the batched BF16 solver takes: dense, BF16 form, one
    sweep per level, and too small to fill the GPU alone."""
    sc = req.schedule
    return req.dense and sc.precision == "bf16" and sc.max_sweeps == 1 and phase_tiles(req) < tiles


class Scheduler:
    """Admission policy: FIFO by arrival, admit while a slot and memory are free.

    A request larger than the whole budget is rejected (never admitted) rather
    than blocking the queue forever."""

    def __init__(self, hbm_budget: int, max_active: int):
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.in_use = 0
        self.active = 0
        self.queue: list = []  # heap of (arrival, rid, request)
        self.rejected: list = []

    def submit(self, req: Request):
        if footprint_bytes(req) > self.budget:
            self.rejected.append(req)
            return
        heapq.heappush(self.queue, (req.arrival, req.rid, req))

    def admissible(self, now: float, accept=None):
        """Pop the requests that can start now (arrived, slot and memory free,
        and `accept(req)` true if given: the executor's own slot classes)."""
        out = []
        while self.queue and self.queue[0][0] <= now and self.active < self.max_active:
            req = self.queue[0][2]
            fp = footprint_bytes(req)
            if self.in_use + fp > self.budget:
                break  # FIFO: wait for memory rather than overtake
            if accept is not None and not accept(req):
                break  # FIFO: wait for a slot of the request's class
            heapq.heappop(self.queue)
            self.in_use += fp
            self.active += 1
            out.append((req, fp))
        return out

    def finish(self):
        """A solve completed: its slot is free (its memory is freed later)."""
        self.active -= 1

    def free(self, fp: int):
        """A finished request's device memory was released."""
        self.in_use -= fp

    def next_arrival(self):
        return self.queue[0][0] if self.queue else None

    def blocked_on_memory(self, now: float) -> bool:
        """The request at the head of the queue has arrived and has a slot,
        but its footprint does not fit the memory still held."""
        if not self.queue or self.queue[0][0] > now or self.active >= self.max_active:
            return False
        return self.in_use + footprint_bytes(self.queue[0][2]) > self.budget

    def should_release(self, now: float, running: int) -> bool:
        """Release the memory of finished requests now: when nothing runs (the
        synchronising free then stalls nothing) or when an arrived request
        waits for memory (continuous batching: it is admitted while others
        still run, instead of after the GPU drains)."""
        return running == 0 or self.blocked_on_memory(now)


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------


class MarsServer:
    """Runs a stream of requests with continuous batching on the current GPU."""

    def __init__(self, hbm_budget: int | None = None, max_active: int = 8, n_streams: int = 4, batching: bool = True,
                 batch_sweeps: int = 8, grouping: bool = True, create_workers: int = 4):
        import torch

        from . import mars as M

        self.torch = torch
        self.M = M
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        # default-priority streams (torch creates them non-blocking)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.batching = batching
        self.batch_sweeps = int(batch_sweeps)
        self.batch_stream = torch.cuda.Stream() if batching else None
        self.grouping = grouping
        from concurrent.futures import ThreadPoolExecutor

        # instance creation off the serving loop (the library releases the
        # interpreter lock in its calls)
        self.creator = ThreadPoolExecutor(max_workers=max(1, int(create_workers)))

    def run(self, requests, time_scale: float = 1.0, verbose: bool = False, progress=None,
            progress_every_s: float = 30.0):
        """Serve `requests` (arrival times in seconds, scaled by time_scale);
        returns (completions, stats).  `progress(msg)`, if given, is called
        every progress_every_s seconds with the number of requests served."""
        torch, M = self.torch, self.M
        cap = self.M.Batch.MAX_MEMBERS if self.batching else 0
        # the batch's members have slots of their own beside the stream pool's
        sched = Scheduler(self.hbm_budget, self.max_active + cap)
        for r in requests:
            sched.submit(r)
        batch = M.Batch(self.batch_stream) if self.batching else None
        inflight = []  # events after the batch's recent steps (at most two queued)
        running = []  # dicts: req, inst, event, outs, buf, fp, admitted, stream (-1: batch)
        by_tag = {}
        graveyard = []  # finished instances awaiting release (frees synchronise the device)
        done = []
        stream_load = [0] * len(self.streams)
        peak_running = peak_batch = 0
        n_grouped = 0  # requests enqueued in groups of two or more
        reserved = {"batch": 0, "solo": 0}  # admitted, instance still being created
        t0 = time.perf_counter()
        last_report = t0
        try:
            while sched.queue or running:
                if progress is not None and time.perf_counter() - last_report >= progress_every_s:
                    last_report = time.perf_counter()
                    progress("served %d / %d requests, %d running" % (len(done), len(requests), len(running)))
                now = (time.perf_counter() - t0) / time_scale
                progressed = False
                # retire finished requests
                still = []
                for job in running:
                    if job["event"] is not None and job["event"].query():
                        if "group_buf" in job:
                            res = M.Instance.read_result(job["group_buf"], job["group_index"])
                        else:
                            res = M.Instance.read_result(job["buf"])
                        best = job["outs"]["best_spins"].cpu().numpy()
                        fin = (time.perf_counter() - t0) / time_scale
                        done.append(Completion(job["req"].rid, res, best, job["req"].arrival, job["admitted"], fin,
                                               job["fp"]))
                        graveyard.append((job["inst"], job["fp"]))
                        sched.finish()
                        if job["stream"] >= 0:
                            stream_load[job["stream"]] -= 1
                        progressed = True
                    else:
                        still.append(job)
                running = still
                # release device memory when nothing runs or a request waits
                # for memory: a free synchronises the device, which stalls the
                # running solves, so it is not done while it would only cost
                if graveyard and sched.should_release(now, len(running)):
                    for inst, fp in graveyard:
                        inst.close()
                        sched.free(fp)
                    graveyard = []
                    progressed = True
                # admit: batch members up to the batch's capacity, other
                # requests up to max_active on the stream pool (counting the
                # admitted requests whose instance is still being created)
                room = {"batch": cap - len(batch) - reserved["batch"] if batch is not None else 0,
                        "solo": self.max_active - sum(stream_load) - reserved["solo"]}

                decided = {}

                def accept(req):
                    cls = "batch" if room["batch"] > 0 and batchable(req) else "solo"
                    if room[cls] <= 0:
                        return False
                    room[cls] -= 1
                    decided[req.rid] = cls
                    return True

                for req, fp in sched.admissible(now, accept):
                    cls = decided[req.rid]
                    reserved[cls] += 1
                    # a dense instance (host validation of N^2 couplings,
                    # encodings, upload) is created on a worker thread while
                    # the GPU runs the others; a sparse one (about a
                    # millisecond) here, so that the sparse requests admitted
                    # together are ready together and share launches
                    if req.dense:
                        creating = self.creator.submit(M.Instance.from_inputs, req.materialize())
                    else:
                        from concurrent.futures import Future

                        creating = Future()
                        creating.set_result(M.Instance.from_inputs(req.materialize()))
                    job = {"req": req, "inst": None, "event": None, "fp": fp, "cls": cls, "creating": creating,
                           "buf": torch.empty(256, dtype=torch.uint8, pin_memory=True),
                           "admitted": (time.perf_counter() - t0) / time_scale}
                    running.append(job)
                    if verbose:
                        print("admit", req.rid, "N", req.N, "runs", req.runs, cls, flush=True)
                    progressed = True
                # enqueue the admitted requests whose instance is ready
                grouped = []  # sparse requests ready in this pass: enqueued together
                for job in running:
                    if job["inst"] is not None or not job["creating"].done():
                        continue
                    job["inst"] = job.pop("creating").result()
                    req, inst, buf = job["req"], job["inst"], job["buf"]
                    reserved[job["cls"]] -= 1
                    progressed = True
                    if job["cls"] == "batch":
                        with torch.cuda.stream(self.batch_stream):
                            job["outs"] = batch.add(inst, req.runs, req.schedule, req.seed, req.rid, buf)
                        job["stream"] = -1
                        by_tag[req.rid] = job
                    elif self.grouping and not req.dense:
                        grouped.append(job)
                    else:
                        k = int(np.argmin(stream_load))
                        stream = self.streams[k]
                        job["outs"] = inst.solve_async(req.runs, req.schedule, req.seed, buf, stream=stream)
                        ev = torch.cuda.Event()
                        ev.record(stream)
                        job["event"] = ev
                        job["stream"] = k
                        stream_load[k] += 1
                # sparse requests ready together share the solver's launches
                # (mars_solve_group_async): one stream, one completion event
                for g0 in range(0, len(grouped), GROUP_MAX):
                    part = grouped[g0:g0 + GROUP_MAX]
                    k = int(np.argmin(stream_load))
                    stream = self.streams[k]
                    if len(part) == 1:
                        j = part[0]
                        j["outs"] = j["inst"].solve_async(j["req"].runs, j["req"].schedule, j["req"].seed, j["buf"],
                                                          stream=stream)
                    else:
                        n_grouped += len(part)
                        gbuf = torch.empty(len(part) * RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
                        outs = M.Instance.solve_group_async(
                            [(j["inst"], j["req"].runs, j["req"].schedule, j["req"].seed) for j in part], gbuf,
                            stream=stream)
                        for i, j in enumerate(part):
                            j["outs"] = outs[i]
                            j["group_buf"], j["group_index"] = gbuf, i
                    ev = torch.cuda.Event()
                    ev.record(stream)
                    for j in part:
                        j["event"] = ev
                        j["stream"] = k
                    stream_load[k] += len(part)
                # advance the batch, keeping at most two steps queued ahead of the GPU
                while inflight and inflight[0].query():
                    inflight.pop(0)
                if batch is not None and len(batch) and len(inflight) < 2:
                    peak_batch = max(peak_batch, len(batch))
                    fin_tags, _ = batch.step(self.batch_sweeps, cap=cap)
                    ev = torch.cuda.Event()
                    ev.record(self.batch_stream)
                    inflight.append(ev)
                    for t in fin_tags:
                        by_tag.pop(t)["event"] = ev
                    progressed = True
                peak_running = max(peak_running, len(running))
                if not progressed:
                    nxt = sched.next_arrival()
                    wait = 2e-4
                    if nxt is not None and not running:
                        wait = max(0.0, min(0.05, (nxt - now) * time_scale))
                    time.sleep(wait)
        finally:
            if batch is not None:
                batch.close()
        for inst, fp in graveyard:
            inst.close()
            sched.free(fp)
        makespan = (time.perf_counter() - t0) / time_scale
        lat = np.array([c.latency for c in done]) if done else np.zeros(1)
        updates = sum(int(c.result["spin_updates"]) for c in done)
        stats = {"requests": len(done), "rejected": len(sched.rejected), "makespan_s": makespan,
                 "peak_concurrent": peak_running, "peak_batch": peak_batch, "grouped_requests": n_grouped,
                 "spin_updates": updates, "spin_updates_per_s": updates / makespan if makespan > 0 else 0.0,
                 "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
                 "latency_p99_ms": float(np.percentile(lat, 99) * 1e3)}
        return sorted(done, key=lambda c: c.rid), stats


# ---------------------------------------------------------------------------
# the served mixed stream (shape of the paper's two workload families)
# ---------------------------------------------------------------------------


def mixed_stream(n_requests: int, rate: float, seed: int = 0, n_lo: int = 100, n_hi: int = 10000,
                 runs_lo: int = 256, runs_hi: int = 4096, levels: int = 300):
    """Poisson arrivals at `rate` requests/s; N log-uniform in [n_lo, n_hi];
    half dense SK couplings N(0, 1/N) solved in the bf16 form, half
    Erdos-Renyi average degree 4 with +-1 weights (J = -w) solved in fp32;
    runs uniform in [runs_lo, runs_hi]; geometric schedules scaled to each
    instance's field scale (sqrt(N * 1/N) = 1 for SK, sqrt(degree) for the
    +-1 graphs)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        runs = int(rng.integers(runs_lo, runs_hi + 1))
        if k % 2 == 0:
            spec = InstanceSpec("sk", N, seed * 100003 + k)
            prec, s = "bf16", math.sqrt((N - 1) / N)
        else:
            spec = InstanceSpec("er", N, seed * 100003 + k)
            prec, s = "fp32", math.sqrt(min(4.0, N - 1.0))
        sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=levels, phases=2, precision=prec)
        reqs.append(Request(k, spec, runs, sch, seed=1000 + k, arrival=t))
    return reqs
