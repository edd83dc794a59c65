"""Error paths of creation and solves, driven by the library's allocation
test hook (MARS_TEST_FAIL_ALLOC=1: every instance and workspace allocation
fails as out of memory).  A refused creation leaves nothing behind; a refused
solve leaves the instance usable, and its later solves equal the ones before
bit for bit."""
import numpy as np
import pytest

from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, require_gpu, solve_summary

pytestmark = pytest.mark.gpu

MARS_E_OOM = 6


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


@pytest.mark.parametrize("kind", ["dense", "csr", "lattice"])
def test_injected_allocation_failure(kind, monkeypatch):
    M = _mars()
    monkeypatch.delenv("MARS_TEST_FAIL_ALLOC", raising=False)
    if kind == "dense":
        inst = I.sk_instance(96, 3)
        sch = I.Schedule(steps=6, phases=2, precision="fp32")
    elif kind == "csr":
        inst = I.er_instance(200, 4, p=0.03, weights="pm1")
        sch = I.Schedule(steps=6, precision="fp32")
    else:
        inst = I.lattice_instance((8, 8), 5)
        sch = I.Schedule(steps=6, precision="fp32")
    announce("injected allocation failure", kind)
    monkeypatch.setenv("MARS_TEST_FAIL_ALLOC", "1")
    with pytest.raises(M.MarsError) as e:
        M.Instance.from_inputs(inst)
    assert e.value.status == MARS_E_OOM
    monkeypatch.delenv("MARS_TEST_FAIL_ALLOC")
    with M.Instance.from_inputs(inst) as g:
        first = g.solve_ex(32, sch, 11, want_best=True)
        # a solve that needs larger workspaces is refused while the hook is set
        monkeypatch.setenv("MARS_TEST_FAIL_ALLOC", "1")
        with pytest.raises(M.MarsError) as e:
            g.solve_ex(4096, sch, 12, want_best=True)
        assert e.value.status == MARS_E_OOM
        monkeypatch.delenv("MARS_TEST_FAIL_ALLOC")
        again = g.solve_ex(32, sch, 11, want_best=True)
        big = g.solve_ex(4096, sch, 12, want_best=True)
    assert solve_summary(again["result"]) == solve_summary(first["result"])
    assert np.array_equal(again["best_spins"].cpu().numpy(), first["best_spins"].cpu().numpy())
    with M.Instance.from_inputs(inst) as h:
        fresh = h.solve_ex(4096, sch, 12, want_best=True)
    assert solve_summary(big["result"]) == solve_summary(fresh["result"])
