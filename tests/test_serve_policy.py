"""CPU checks of the serving admission policy (no GPU): memory and slot
limits are never exceeded, arrivals are served first-come first-served,
oversized requests are rejected instead of blocking the queue, and every
admissible request is eventually admitted."""
import numpy as np

from paper_1907_05124_amd import inputs as I
from paper_1907_05124_amd import serve as S


def _reqs(n, seed=0, rate=50.0):
    return S.mixed_stream(n, rate, seed=seed, n_lo=50, n_hi=800, runs_lo=64, runs_hi=512, levels=20)


def _simulate(reqs, budget, max_active, service=0.05):
    """Discrete-event run of the scheduler with a fake executor (fixed service time)."""
    sched = S.Scheduler(budget, max_active)
    for r in reqs:
        sched.submit(r)
    t, running, order, peak_mem, peak_active = 0.0, [], [], 0, 0
    while sched.queue or running:
        for req, fp in sched.admissible(t):
            running.append((t + service * (1 + req.N / 800), req, fp))
            order.append(req.rid)
        peak_mem = max(peak_mem, sched.in_use)
        peak_active = max(peak_active, sched.active)
        assert sched.in_use <= budget and sched.active <= max_active
        nxt = [e for e, _, _ in running]
        if sched.queue and sched.queue[0][0] > t:
            nxt.append(sched.queue[0][0])  # the next arrival
        assert nxt, "queue head arrived but was not admitted with nothing running"
        t = min(nxt)
        keep = []
        for e, req, fp in running:
            if e <= t:
                sched.finish()
                sched.free(fp)
            else:
                keep.append((e, req, fp))
        running = keep
    return order, peak_mem, peak_active, sched


def test_limits_and_fifo():
    reqs = _reqs(60)
    budget = 4 * max(S.footprint_bytes(r) for r in reqs)
    order, peak_mem, peak_active, sched = _simulate(reqs, budget, max_active=3)
    assert sorted(order) == [r.rid for r in reqs]  # every request served
    arrivals = {r.rid: r.arrival for r in reqs}
    assert all(arrivals[a] <= arrivals[b] for a, b in zip(order, order[1:]))  # FIFO
    assert peak_active <= 3 and peak_mem <= budget
    assert not sched.rejected


def test_oversized_request_is_rejected_not_blocking():
    reqs = _reqs(10)
    budget = max(S.footprint_bytes(r) for r in reqs) + 1
    big = S.Request(999, S.InstanceSpec("sk", 4000, 1), 64, reqs[0].schedule, 1, arrival=0.0)
    order, _, _, sched = _simulate(reqs + [big], budget, max_active=2)
    assert [r.rid for r in sched.rejected] == [999]
    assert sorted(order) == [r.rid for r in reqs]


def test_footprint_grows_with_size():
    base = S.Request(0, I.sk_instance(300, 1), 512, I.Schedule(steps=50, precision="bf16"), 1)
    bigger_n = S.Request(1, I.sk_instance(600, 1), 512, base.schedule, 1)
    more_runs = S.Request(2, base.instance, 2048, base.schedule, 1)
    assert S.footprint_bytes(bigger_n) > S.footprint_bytes(base)
    assert S.footprint_bytes(more_runs) > S.footprint_bytes(base)


def test_mixed_stream_shape():
    reqs = S.mixed_stream(200, 10.0, seed=3)
    Ns = np.array([r.N for r in reqs])
    assert Ns.min() >= 100 and Ns.max() <= 10000
    assert abs(np.mean(np.log(Ns)) - (np.log(100) + np.log(10000)) / 2) < 0.5
    kinds = [r.dense for r in reqs]
    assert sum(kinds) == 100
    gaps = np.diff([r.arrival for r in reqs])
    assert np.all(gaps >= 0) and abs(gaps.mean() - 0.1) < 0.03


def test_batchable_requests():
    """Only dense BF16 one-sweep-per-level requests smaller than one tile per
    compute unit per phase join the batch."""
    sch = I.Schedule(phases=2, precision="bf16")
    small = S.Request(0, S.InstanceSpec("sk", 1000, 1), 1024, sch, seed=1)
    assert S.phase_tiles(small) == 8 * 4 and S.batchable(small)
    big = S.Request(1, S.InstanceSpec("sk", 10000, 1), 4096, sch, seed=1)
    assert S.phase_tiles(big) == 32 * 40 and not S.batchable(big)
    assert not S.batchable(S.Request(2, S.InstanceSpec("sk", 1000, 1), 1024, sch.replace(precision="fp32"), seed=1))
    assert not S.batchable(S.Request(3, S.InstanceSpec("er", 1000, 1), 1024, sch, seed=1))
    jac = S.Request(4, S.InstanceSpec("sk", 1000, 1), 1024, sch.replace(update="jacobi"), seed=1)
    assert S.phase_tiles(jac) == 8 * 8
    slow = S.Request(5, S.InstanceSpec("sk", 1000, 1), 1024,
                     sch.replace(kind="linear", max_sweeps=10, c_step=0.1), seed=1)
    assert not S.batchable(slow)


def test_accept_predicate_keeps_fifo():
    """A request refused by the executor's slot classes blocks the queue
    behind it (first come, first served) without being lost."""
    reqs = _reqs(6, seed=3, rate=0.0)
    sched = S.Scheduler(1 << 40, 10)
    for r in reqs:
        sched.submit(r)
    first = sched.admissible(1.0, accept=lambda r: r.rid < 2)
    assert [r.rid for r, _ in first] == [0, 1] and sched.active == 2
    rest = sched.admissible(1.0)
    assert [r.rid for r, _ in rest] == [2, 3, 4, 5]


def test_memory_of_finished_requests_is_released_while_others_run():
    """The executor's release rule (Scheduler.should_release): a finished
    request's memory is held back (a device free synchronises the device)
    only until an arrived request waits for it.  With a budget for two
    requests, one long and three short requests arriving at once, the third
    request must start while the long one still runs, as soon as the first
    short one has finished."""
    reqs = _reqs(4, seed=5, rate=0.0)
    fps = [S.footprint_bytes(r) for r in reqs]
    budget = fps[0] + max(fps[1:]) + 1
    assert sum(fps) > budget
    sched = S.Scheduler(budget, max_active=8)
    for r in reqs:
        sched.submit(r)
    duration = {reqs[0].rid: 10.0, reqs[1].rid: 1.0, reqs[2].rid: 1.0, reqs[3].rid: 1.0}
    t, running, graveyard, started = 0.0, [], [], {}
    while sched.queue or running:
        if graveyard and sched.should_release(t, len(running)):
            for fp in graveyard:
                sched.free(fp)
            graveyard = []
        for req, fp in sched.admissible(t):
            running.append((t + duration[req.rid], req, fp))
            started[req.rid] = t
        assert sched.in_use <= budget
        t = min(e for e, _, _ in running)
        keep = []
        for e, req, fp in running:
            if e <= t:
                sched.finish()
                graveyard.append(fp)  # memory held until the release rule frees it
            else:
                keep.append((e, req, fp))
        running = keep
    # requests 0 and 1 start at once; 2 starts when 1 finishes (t = 1), while 0 runs until t = 10
    assert started[reqs[0].rid] == 0.0 and started[reqs[1].rid] == 0.0
    assert started[reqs[2].rid] == 1.0 < started[reqs[0].rid] + duration[reqs[0].rid]
    assert started[reqs[3].rid] == 2.0


def test_release_rule_holds_memory_while_nothing_waits():
    """Without a waiting request the finished memory stays held while solves
    run (no synchronising free), and is released once nothing runs."""
    reqs = _reqs(2, seed=6, rate=0.0)
    sched = S.Scheduler(10 * sum(S.footprint_bytes(r) for r in reqs), max_active=8)
    for r in reqs:
        sched.submit(r)
    admitted = sched.admissible(0.0)
    assert len(admitted) == 2
    sched.finish()
    assert not sched.should_release(0.0, running=1)
    sched.finish()
    assert sched.should_release(0.0, running=0)
