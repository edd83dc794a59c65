"""mars_energy_noalloc (the entry point for callers that cannot allocate)
against mars_energy, through the C interface: bit-identical energies on two
calls in a row, the second with fewer spin vectors (the scratch array keeps
the first call's contents), for dense, lattice and sparse instances; a
request beyond the fixed scratch is refused and writes nothing."""
import numpy as np
import pytest

from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, require_gpu

pytestmark = pytest.mark.gpu


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


@pytest.mark.parametrize("make", [
    lambda: I.sk_instance(1000, 3, field_scale=0.4),  # several spin tiles, ragged, with a field
    lambda: I.sk_instance(300, 7),
    lambda: I.lattice_instance((16, 16, 8), 2),
    lambda: I.er_instance(800, 5, p=0.06, weights="pm1"),
])
def test_noalloc_equals_energy(make):
    M = _mars()
    torch = require_gpu()
    inst = make()
    with M.Instance.from_inputs(inst) as g:
        for R, seed in ((517, 1), (129, 2)):
            S = torch.from_numpy(I.random_spins(inst.N, R, seed)).cuda()
            announce("energy noalloc", type(inst).__name__, inst.N, R)
            want = g.energy(S)
            got = torch.full((R,), float("nan"), dtype=torch.float64, device="cuda")
            g.energy_noalloc(S, got)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (R, int((got != want).sum()))


def test_noalloc_refuses_beyond_scratch():
    M = _mars()
    torch = require_gpu()
    inst = I.sk_instance(4000, 1)
    R = 9000  # 9088 x 4096 spin bytes alone exceed 32 MiB
    with M.Instance.from_inputs(inst) as g:
        S = torch.ones((R, inst.N), dtype=torch.int8, device="cuda")
        E = torch.full((R,), 7.0, dtype=torch.float64, device="cuda")
        announce("energy noalloc refusal", inst.N, R)
        with pytest.raises(M.MarsError) as e:
            g.energy_noalloc(S, E)
        assert e.value.status == 8
        torch.cuda.synchronize()
        assert torch.all(E == 7.0)
        # a request that fits still works after the refusal
        E2 = torch.empty(64, dtype=torch.float64, device="cuda")
        g.energy_noalloc(S[:64].contiguous(), E2)
        assert torch.equal(E2, g.energy(S[:64].contiguous()))
