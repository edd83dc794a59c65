"""GPU check of the serving loop: requests that run concurrently on several
streams give bit-for-bit the same results as the same requests solved alone,
and the solves really overlapped."""
import numpy as np
import pytest

from tests.gpu_common import announce, require_gpu, solve_summary

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("batching,grouping", [(True, True), (False, False), (False, True)])
def test_served_results_equal_alone(batching, grouping):
    require_gpu()
    from paper_1907_05124_amd import mars as M
    from paper_1907_05124_amd import serve as S

    # a burst (every request arrives at t = 0): the first admission pass takes
    # several sparse requests at once, which grouping then enqueues together
    reqs = S.mixed_stream(16, rate=1e9, seed=5, n_lo=100, n_hi=1500, runs_lo=256, runs_hi=1024, levels=60)
    for r in reqs:
        r.instance = r.materialize()
    announce("serve mixed", len(reqs), "batching", batching, "grouping", grouping)
    server = S.MarsServer(max_active=6, n_streams=4, batching=batching, grouping=grouping)
    done, stats = server.run(reqs)
    print(stats)
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    assert stats["peak_concurrent"] >= 2
    if batching:
        assert stats["peak_batch"] >= 2
    if grouping:
        assert stats["grouped_requests"] >= 2
    else:
        assert stats["grouped_requests"] == 0
    for c, r in zip(done, reqs):
        assert c.rid == r.rid
        with M.Instance.from_inputs(r.instance) as g:
            alone = g.solve_ex(r.runs, r.schedule, r.seed, want_best=True)
        assert solve_summary(alone["result"]) == solve_summary(c.result), r.rid
        assert np.array_equal(alone["best_spins"].cpu().numpy(), c.best_spins), r.rid
