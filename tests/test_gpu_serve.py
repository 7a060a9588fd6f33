"""The continuous-batching serving loop: every request, admitted while others run and propagated
in a changing batch, returns the dipole it gives alone (bit for bit); with a tight HBM budget the
loop admits fewer requests at a time and still completes them all."""
import numpy as np
import pytest

from paper_2601_17164_amd import inputs as I
from tests.common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    yield sfhk, torch


def _requests(n, rate, scale):
    from paper_2601_17164_amd import serve
    t = serve.poisson_arrivals(rate, n, seed=11)
    return [serve.Request(k, float(t[k]), I.serving_request(k, traj_scale=scale)) for k in range(n)]


def _alone(sfhk, ctx, inst, precision):
    job = sfhk.make_job(ctx, inst, precision=precision)
    assert job.propagate(0)
    d = job.dipole().cpu().numpy()
    job.close()
    return d


@pytest.mark.parametrize("precision", [0, 1])
def test_serving_results_equal_alone(S, precision):
    sfhk, torch = S
    from paper_2601_17164_amd import serve
    ctx = sfhk.Context(0)
    reqs = _requests(8, 200.0, 1.0 / 128)
    srv = serve.Server(ctx, precision=precision, chunk=700, workers_per_cu=0, max_jobs=8,
                       max_tiles=sum(sfhk.tiles_of(r.inst) for r in reqs), keep_results=True)
    res = srv.run(reqs)
    srv.close()
    assert [r.req_id for r in res] == list(range(len(reqs)))
    for r in res:
        np.testing.assert_array_equal(r.dipole, _alone(sfhk, ctx, reqs[r.req_id].inst, precision))
        assert r.finished >= r.admitted >= r.arrival - 1e-9
    summ = serve.summarize(res)
    print("serving summary", summ, flush=True)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    ctx.close()


def test_serving_with_tight_hbm_budget(S):
    sfhk, torch = S
    from paper_2601_17164_amd import serve
    reqs = _requests(6, 500.0, 1.0 / 128)
    need = max(sfhk.job_footprint(r.inst.n_traj, r.inst.grid.n_steps) for r in reqs)
    ctx = sfhk.Context(0, hbm_budget_bytes=int(need * 1.5))
    srv = serve.Server(ctx, chunk=900, max_jobs=6, max_tiles=sum(sfhk.tiles_of(r.inst) for r in reqs),
                       keep_results=True)
    res = srv.run(reqs)
    srv.close()
    assert len(res) == len(reqs)
    ref_ctx = sfhk.Context(0)
    for r in res:
        np.testing.assert_array_equal(r.dipole, _alone(sfhk, ref_ctx, reqs[r.req_id].inst, 0))
    assert ctx.bytes_in_use() == 0
    ref_ctx.close()
    ctx.close()


def test_serving_sfa_born_requests(S):
    """Requests with SFA birth samples: the loop runs the birth step on the device at admission;
    each result equals the same request born and propagated alone, bit for bit."""
    sfhk, torch = S
    from paper_2601_17164_amd import serve
    ctx = sfhk.Context(0)
    t = serve.poisson_arrivals(200.0, 6, seed=12)
    reqs = [serve.Request(k, float(t[k]), I.serving_request(k, traj_scale=1.0 / 128, sfa=True))
            for k in range(6)]
    srv = serve.Server(ctx, chunk=800, max_jobs=6,
                       max_tiles=sum(sfhk.tiles_of(r.inst) for r in reqs), keep_results=True)
    res = srv.run(reqs)
    srv.close()
    assert len(res) == len(reqs)
    for r in res:
        job = serve._create_job(ctx, reqs[r.req_id].inst, 0, None)
        assert job.propagate(0)
        alone = job.dipole().cpu().numpy()
        job.close()
        np.testing.assert_array_equal(r.dipole, alone)
    ctx.close()
