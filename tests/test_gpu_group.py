"""mars_solve_group_async: lattice and sparse solves enqueued together, sparse
members on one instantiation of the LDS-resident solver sharing one launch.
Every member's outputs must equal those of the same solve alone, bit for bit
(each run's trajectory is independent of the others: Algorithm 1 per run)."""
import ctypes as C

import numpy as np
import pytest

from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, require_gpu, solve_summary
from tests.test_gpu_graph import _mars, _rel_sched, _with_field

pytestmark = pytest.mark.gpu


def _members():
    """(label, instance, runs, schedule, seed): three short-row ±1 ER solves
    with at least 1024 runs (four runs per lane group) share one launch; two
    long-row ones share another (two lanes per slot); a field, fp16 and fp64
    storage, a synchronous update, few runs (one run per workgroup) and a
    lattice take launches of their own."""
    out = []

    def add(label, inst, R, seed, **kw):
        out.append((label, inst, R, _rel_sched(inst, **kw), seed))

    add("er300", I.er_instance(300, 1, p=0.02, weights="pm1"), 1031, 11, precision="fp32")
    add("er500", I.er_instance(500, 2, avg_degree=5.0, weights="pm1"), 2048, 12, precision="fp32")
    add("er800", I.er_instance(800, 3, p=0.01, weights="pm1"), 1500, 13, precision="fp32")
    add("er300 long", I.er_instance(300, 4, p=0.12, weights="pm1"), 1100, 14, precision="fp32")
    add("er400 long", I.er_instance(400, 5, p=0.08, weights="pm1"), 4100, 15, precision="fp32")
    add("er field", _with_field(I.er_instance(200, 6, p=0.05, weights="pm1"), 0.4), 1031, 16, precision="fp32")
    add("er fp16", I.er_instance(600, 7, avg_degree=4.0, weights="pm1"), 2000, 17, precision="fp16")
    add("er fp64", I.er_instance(250, 8, p=0.03, weights="pm1"), 1024, 18, precision="fp64")
    add("er jacobi", I.er_instance(300, 9, p=0.02, weights="pm1"), 1031, 19, precision="fp32", update="jacobi")
    add("er few runs", I.er_instance(300, 10, p=0.02, weights="pm1"), 96, 20, precision="fp32")
    add("lattice", I.lattice_instance((8, 8, 8), 3), 1024, 21, precision="fp32")
    return out


def test_group_equals_alone():
    M = _mars()
    torch = require_gpu()
    members = _members()
    insts = [M.Instance.from_inputs(m[1]) for m in members]
    try:
        alone = []
        for (label, _, R, sch, seed), g in zip(members, insts):
            announce("group: alone", label, R)
            alone.append(g.solve_ex(R, sch, seed, want_best=True, want_energies=True))
        stream = torch.cuda.Stream()
        buf = torch.zeros(len(members) * C.sizeof(M.Result), dtype=torch.uint8, pin_memory=True)
        announce("group: together", len(members))
        outs = M.Instance.solve_group_async([(g, m[2], m[3], m[4]) for g, m in zip(insts, members)], buf,
                                            stream=stream, want_energies=True)
        stream.synchronize()
        for i, ((label, _, R, _, _), a) in enumerate(zip(members, alone)):
            res = M.Instance.read_result(buf, i)
            assert solve_summary(res) == solve_summary(a["result"]), label
            assert np.array_equal(outs[i]["energies"].cpu().numpy(), a["energies"].cpu().numpy()), label
            assert np.array_equal(outs[i]["best_spins"].cpu().numpy(), a["best_spins"].cpu().numpy()), label
    finally:
        for g in insts:
            g.close()


def test_group_of_one_and_repeat():
    """A group of one equals the solve alone; the same instances grouped
    twice in a row (the leader's descriptor rewritten) give the same
    results."""
    M = _mars()
    torch = require_gpu()
    members = _members()[:3]
    insts = [M.Instance.from_inputs(m[1]) for m in members]
    try:
        stream = torch.cuda.Stream()
        bufs = [torch.zeros(len(members) * C.sizeof(M.Result), dtype=torch.uint8, pin_memory=True)
                for _ in range(2)]
        outs = []
        for b in bufs:
            outs.append(M.Instance.solve_group_async([(g, m[2], m[3], m[4]) for g, m in zip(insts, members)], b,
                                                     stream=stream, want_energies=True))
        one = torch.zeros(C.sizeof(M.Result), dtype=torch.uint8, pin_memory=True)
        single = M.Instance.solve_group_async([(insts[0], members[0][2], members[0][3], members[0][4])], one,
                                              stream=stream, want_energies=True)
        stream.synchronize()
        for i in range(len(members)):
            assert solve_summary(M.Instance.read_result(bufs[0], i)) == \
                solve_summary(M.Instance.read_result(bufs[1], i))
            assert np.array_equal(outs[0][i]["energies"].cpu().numpy(), outs[1][i]["energies"].cpu().numpy())
        assert solve_summary(M.Instance.read_result(one, 0)) == solve_summary(M.Instance.read_result(bufs[0], 0))
        assert np.array_equal(single[0]["best_spins"].cpu().numpy(), outs[0][0]["best_spins"].cpu().numpy())
    finally:
        for g in insts:
            g.close()


def test_group_rejects():
    """Validation precedes any enqueued work: an instance twice, a dense
    instance, an empty group."""
    M = _mars()
    torch = require_gpu()
    a = M.Instance.from_inputs(I.er_instance(100, 1, p=0.05, weights="pm1"))
    d = M.Instance.from_inputs(I.sk_instance(64, 1))
    try:
        sch = _rel_sched(I.er_instance(100, 1, p=0.05, weights="pm1"), precision="fp32")
        stream = torch.cuda.Stream()
        buf = torch.zeros(4 * C.sizeof(M.Result), dtype=torch.uint8, pin_memory=True)
        with pytest.raises(M.MarsError) as e:
            M.Instance.solve_group_async([(a, 64, sch, 1), (a, 64, sch, 2)], buf, stream=stream)
        assert "twice" in str(e.value)
        with pytest.raises(M.MarsError) as e:
            M.Instance.solve_group_async([(a, 64, sch, 1), (d, 64, sch, 2)], buf, stream=stream)
        assert "lattice and sparse" in str(e.value)
        with pytest.raises(M.MarsError):
            M.Instance.solve_group_async([], buf, stream=stream)
        stream.synchronize()
    finally:
        a.close()
        d.close()


def test_group_with_unshared_paths():
    """Members that cannot share a launch sit beside ones that do: a solve
    with no temperature level (start-only path), a sparse instance beyond LDS
    (device-memory solver) and a lattice beyond LDS; every member equals its
    solve alone."""
    M = _mars()
    torch = require_gpu()
    big = I.er_instance(48000, 3, p=4.0 / 47999, weights="pm1")
    lat = I.lattice_instance((28, 28, 28), 5)
    small = [I.er_instance(300, 1, p=0.02, weights="pm1"), I.er_instance(500, 2, avg_degree=5.0, weights="pm1"),
             I.er_instance(400, 6, p=0.015, weights="pm1")]
    members = [("small a", small[0], 1031, _rel_sched(small[0], precision="fp32"), 1),
               ("no level", small[1], 1100, _rel_sched(small[1], precision="fp32", steps=0), 2),
               ("beyond LDS", big, 64, _rel_sched(big, precision="fp32", steps=30), 3),
               ("lattice beyond LDS", lat, 32, _rel_sched(lat, precision="fp64", steps=20), 4),
               ("small b", small[2], 2048, _rel_sched(small[2], precision="fp32"), 5)]
    insts = [M.Instance.from_inputs(m[1]) for m in members]
    try:
        alone = []
        for (label, _, R, sch, seed), g in zip(members, insts):
            announce("group unshared: alone", label, R)
            alone.append(g.solve_ex(R, sch, seed, want_best=True, want_energies=True))
        stream = torch.cuda.Stream()
        buf = torch.zeros(len(members) * C.sizeof(M.Result), dtype=torch.uint8, pin_memory=True)
        announce("group unshared: together", len(members))
        outs = M.Instance.solve_group_async([(g, m[2], m[3], m[4]) for g, m in zip(insts, members)], buf,
                                            stream=stream, want_energies=True)
        stream.synchronize()
        for i, ((label, _, R, _, _), a) in enumerate(zip(members, alone)):
            assert solve_summary(M.Instance.read_result(buf, i)) == solve_summary(a["result"]), label
            assert np.array_equal(outs[i]["energies"].cpu().numpy(), a["energies"].cpu().numpy()), label
            assert np.array_equal(outs[i]["best_spins"].cpu().numpy(), a["best_spins"].cpu().numpy()), label
    finally:
        for g in insts:
            g.close()
