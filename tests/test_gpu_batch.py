"""GPU checks of the batched BF16 solver (mars_batch_*): members of uneven
size that join and leave at different sweeps give bit for bit the results of
the same solves run alone, and the batch refuses what it does not hold."""
import ctypes

import numpy as np
import pytest

from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, require_gpu, solve_summary

pytestmark = pytest.mark.gpu


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


def _case(N, R, phases, levels, field, seed):
    inst = I.sk_instance(N, seed, field_scale=field)
    s = I.field_scale(inst)
    sch = I.Schedule(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=levels, phases=phases, precision="bf16")
    return inst, R, sch, 1000 + seed


# uneven N, unaligned phase starts (517/3, 130/4), a single run, a single
# level, a zero-level solve, Jacobi updates
CASES = [
    (517, 129, 3, 25, 0.4, 1),
    (1000, 300, 2, 40, 0.0, 2),
    (130, 1, 4, 12, 0.0, 3),
    (2000, 520, 1, 30, 0.0, 4),
    (64, 64, 2, 1, 0.2, 5),
    (300, 33, 5, 18, 0.0, 6),
]


def _pinned(M):
    import torch

    return torch.zeros(256, dtype=torch.uint8, pin_memory=True)


MODES = {"persistent": ("1", "1"), "graph": ("0", "1"), "eager": ("0", "0")}


def _mode(mode, monkeypatch):
    persist, graph = MODES[mode]
    monkeypatch.setenv("MARS_BATCH_PERSIST", persist)
    monkeypatch.setenv("MARS_BATCH_GRAPH", graph)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("tile", ["", "0", "3"])
def test_batch_equals_alone(mode, tile, monkeypatch):
    """Steps run as one persistent cooperative launch (while no member has
    more than four phases: the five-phase member below sends the steps it
    takes part in down the graph path), as one captured graph per membership
    (replayed while the membership holds) or sweep by sweep; every way equals
    the solves alone."""
    _mode(mode, monkeypatch)
    if tile:
        monkeypatch.setenv("MARS_BATCH_TILE", tile)  # phase tiles 128 x 128 (0) or 64 x 64 (3) forced
    else:
        monkeypatch.delenv("MARS_BATCH_TILE", raising=False)
    M = _mars()
    import torch

    cases = [_case(*c) for c in CASES]
    cases.append(_case(257, 96, 1, 10, 0.0, 7))
    cases[-1] = (cases[-1][0], cases[-1][1], cases[-1][2].replace(update="jacobi"), cases[-1][3])
    cases.append(_case(90, 40, 2, 8, 0.0, 8))
    cases[-1] = (cases[-1][0], cases[-1][1], cases[-1][2].replace(level_count=0), cases[-1][3])
    announce("batch vs alone", len(cases), mode, tile)
    handles = [M.Instance.from_inputs(c[0]) for c in cases]
    alone = [h.solve_ex(R, sch, seed, want_best=True) for h, (_, R, sch, seed) in zip(handles, cases)]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    bufs = [_pinned(M) for _ in cases]
    outs = {}
    finished = []
    with torch.cuda.stream(stream):
        batch = M.Batch(stream)
        # the first half joins at once, the rest one at a time between steps;
        # a small tag capacity makes steps stop early
        for i in range(4):
            outs[i] = batch.add(handles[i], cases[i][1], cases[i][2], cases[i][3], i, bufs[i])
        nxt = 4
        while len(finished) < len(cases):
            done, active = batch.step(3, cap=2)
            finished += done
            assert len(done) <= 2 and active == len(batch)
            if nxt < len(cases):
                outs[nxt] = batch.add(handles[nxt], cases[nxt][1], cases[nxt][2], cases[nxt][3], nxt, bufs[nxt])
                nxt += 1
        batch.close()
    stream.synchronize()
    assert sorted(finished) == list(range(len(cases)))
    for i, (a, h) in enumerate(zip(alone, handles)):
        res = M.Instance.read_result(bufs[i])
        assert solve_summary(res) == solve_summary(a["result"]), (i, res, a["result"])
        assert np.array_equal(outs[i]["best_spins"].cpu().numpy(), a["best_spins"].cpu().numpy()), i
        h.close()


@pytest.mark.parametrize("mode", list(MODES))
def test_batch_full_and_refusals(mode, monkeypatch):
    _mode(mode, monkeypatch)
    M = _mars()
    import torch

    announce("batch refusals")
    stream = torch.cuda.Stream()
    dense = I.sk_instance(200, 11)
    sch = I.Schedule(steps=5, phases=2, precision="bf16")
    with torch.cuda.stream(stream):
        batch = M.Batch(stream)
        handles = [M.Instance.from_inputs(dense) for _ in range(M.Batch.MAX_MEMBERS + 1)]
        bufs = [_pinned(M) for _ in handles]
        batch.add(handles[0], 64, sch, 0, 0, bufs[0])
        # a member's instance is owned by the batch
        with pytest.raises(M.MarsError) as e:
            handles[0].solve_ex(8, sch, 1)
        assert e.value.status == 1
        with pytest.raises(M.MarsError) as e:
            batch.add(handles[0], 64, sch, 5, 100, bufs[0])
        assert e.value.status == 1
        # what the batch does not hold
        other = handles[-1]
        for bad in (sch.replace(precision="fp32"), sch.replace(max_sweeps=4, kind="linear", c_step=0.5)):
            with pytest.raises(M.MarsError) as e:
                batch.add(other, 64, bad, 1, 200, _pinned(M))
            assert e.value.status == 8
        with M.Instance.from_inputs(I.lattice_instance((8, 8), 3)) as g:
            with pytest.raises(M.MarsError) as e:
                batch.add(g, 64, sch.replace(precision="fp32"), 1, 201, _pinned(M))
            assert e.value.status == 8
        for t in range(1, M.Batch.MAX_MEMBERS):
            batch.add(handles[t], 64, sch, t, t, bufs[t])
        with pytest.raises(M.MarsError) as e:
            batch.add(other, 64, sch, 99, 99, _pinned(M))
        assert e.value.status == 8 and "full" in str(e.value)
        total = []
        while len(batch):
            done, _ = batch.step(2, cap=16)
            total += done
        # a second round on the same batch: members join again, the step
        # graph is captured anew and replayed
        for t in range(4):
            batch.add(handles[t], 64, sch, 100 + t, 100 + t, bufs[t])
        while len(batch):
            done, _ = batch.step(3, cap=16)
            total += done
        batch.close()
    stream.synchronize()
    assert sorted(total) == list(range(M.Batch.MAX_MEMBERS)) + [100, 101, 102, 103]
    # released: the instances solve alone again, with the batch's results
    for t in range(4):
        r_alone = handles[t].solve_ex(64, sch, 100 + t)["result"]
        assert solve_summary(r_alone) == solve_summary(M.Instance.read_result(bufs[t]))
    for h in handles:
        h.close()


def test_batch_destroy_with_members():
    """Destroying a batch that still holds members releases them."""
    M = _mars()
    import torch

    announce("batch destroy")
    stream = torch.cuda.Stream()
    inst = I.sk_instance(300, 12)
    sch = I.Schedule(steps=50, phases=2, precision="bf16")
    with M.Instance.from_inputs(inst) as g:
        with torch.cuda.stream(stream):
            batch = M.Batch(stream)
            batch.add(g, 128, sch, 3, 0, _pinned(M))
            done, active = batch.step(5)
            assert done == [] and active == 1
            batch.close()
        out = g.solve_ex(128, sch, 3)
        assert out["result"]["levels_executed"] > 0
