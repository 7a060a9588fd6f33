"""Batched, graph-captured propagation (persistent queue and hardware dispatch) through the C ABI:
every job's result must equal its result propagated alone, bit for bit, whatever the batch
composition, worker count, chunk size and replay count."""
import numpy as np
import pytest

from paper_2601_17164_amd import inputs as I
from tests.common import pulse_table, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    ctx = sfhk.Context(0)
    yield sfhk, ctx, torch
    ctx.close()


def _instances():
    rng = np.random.default_rng(21)
    out = [I.random_instance(rng, 500 + k, f"b{k}", traj_scale=1.0 / 256) for k in range(5)]
    out.append(I.config0(n_birth=8, n_per_birth=20, seed=7))
    return out


def _alone(S, inst, precision):
    sfhk, ctx, torch = S
    job = sfhk.make_job(ctx, inst, precision=precision)
    assert job.propagate(0)
    d = job.dipole().cpu().numpy()
    job.close()
    return d


@pytest.mark.parametrize("workers,chunk", [(8, 0), (4, 700), (0, 0), (0, 1500)])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_jobs_alone(S, workers, chunk, precision):
    sfhk, ctx, torch = S
    insts = _instances()
    alone = [_alone(S, x, precision) for x in insts]
    jobs = [sfhk.make_job(ctx, x, precision=precision) for x in insts]
    b = sfhk.Batch(ctx, len(jobs), sum(sfhk.tiles_of(x) for x in insts), chunk, workers)
    b.set_jobs(jobs)
    replays = 0
    while not b.run():
        replays += 1
        # eager work and a synchronisation between replays
        torch.ones(1000, device="cuda").sum().item()
        assert replays < 10000
    for job, ref in zip(jobs, alone):
        np.testing.assert_array_equal(job.dipole().cpu().numpy(), ref)
        job.close()
    b.close()


def test_batch_jobs_join_and_leave_between_replays(S):
    """Continuous batching: a job admitted after others have started, and finished jobs dropped
    from the table, still give the results they give alone."""
    sfhk, ctx, torch = S
    insts = _instances()
    alone = [_alone(S, x, 0) for x in insts]
    jobs = [sfhk.make_job(ctx, x) for x in insts]
    b = sfhk.Batch(ctx, len(jobs), sum(sfhk.tiles_of(x) for x in insts), 400, 8)
    active = jobs[:2]
    waiting = list(jobs[2:])
    b.set_jobs(active)
    finished = []
    for _ in range(10000):
        b.run()
        still = []
        for j in active:
            if j.stats().tiles_done == j.stats().tiles_total:
                finished.append(j)
            else:
                still.append(j)
        if waiting:
            still.append(waiting.pop(0))
        active = still
        if not active:
            break
        b.set_jobs(active)
    assert not waiting and not active
    for job, ref in zip(jobs, alone):
        np.testing.assert_array_equal(job.dipole().cpu().numpy(), ref)
        job.close()
    b.close()


def test_batch_capacity_errors(S):
    sfhk, ctx, torch = S
    inst = I.config0(n_birth=4, n_per_birth=16)
    jobs = [sfhk.make_job(ctx, inst), sfhk.make_job(ctx, inst)]
    b = sfhk.Batch(ctx, 1, 100, 0, 8)
    with pytest.raises(sfhk.SfhkError) as ei:
        b.set_jobs(jobs)
    assert ei.value.status == sfhk.SFHK_E_INVALID
    b.close()
    b = sfhk.Batch(ctx, 2, 1, 0, 8)
    with pytest.raises(sfhk.SfhkError):
        b.set_jobs(jobs)
    b.close()
    for j in jobs:
        j.close()


def _kind_instances():
    """One instance of each potential kind (none, soft-core, screened, harmonic): each runs in its
    own kernel instance."""
    pulse = I.Pulse(800.0, 1e14, 2.0)
    grid = I.time_grid(pulse, 0.1)
    e = pulse_table(pulse, grid)
    rng = np.random.default_rng(5)
    n = 96
    t0 = np.sort(grid.t_a + rng.integers(0, grid.n_steps, n) * grid.h)
    q0 = rng.normal(0.0, 1.0, (3, n))
    p0 = rng.normal(0.0, 0.5, (3, n))
    none = I.Instance("none", I.Potential(I.POT_NONE, 0, 0, 1, 0, 0), I.gto_h1s(), pulse, grid, e,
                      t0, q0, p0)
    ho = I.Instance("ho", I.Potential(I.POT_HARMONIC, 0, 0, 1, 0, 0.3), I.gto_h1s(), pulse, grid,
                    e, t0, q0, p0)
    soft = I.config0(n_birth=4, n_per_birth=24, seed=3)
    scr = I.config1_birth_subset(I.config1(), [700, 900], 40)
    return [none, soft, scr, ho]


@pytest.mark.parametrize("precision", [0, 1])
def test_all_potential_kinds_in_one_batch_and_one_call(S, precision):
    """Jobs of all four potential kinds together (one kernel instance per kind and precision) in
    a batch replay, hardware dispatch and persistent form, and in one sfhk_propagate_many call:
    each equals the job alone."""
    sfhk, ctx, torch = S
    insts = _kind_instances()
    alone = [_alone(S, x, precision) for x in insts]
    n_tiles = sum(sfhk.tiles_of(x) for x in insts)
    for workers in (0, 8):
        jobs = [sfhk.make_job(ctx, x, precision=precision) for x in insts]
        b = sfhk.Batch(ctx, len(jobs), n_tiles, 0, workers)
        b.set_jobs(jobs)
        assert b.run()
        for job, ref in zip(jobs, alone):
            np.testing.assert_array_equal(job.dipole().cpu().numpy(), ref)
            job.close()
        b.close()
    jobs = [sfhk.make_job(ctx, x, precision=precision) for x in insts]
    while not sfhk.propagate_many(jobs, 300):
        pass
    for job, ref in zip(jobs, alone):
        np.testing.assert_array_equal(job.dipole().cpu().numpy(), ref)
        job.close()


def test_a_replay_needs_a_staged_table(S):
    """Before any sfhk_batch_set_jobs (or after a failed one) a replay is refused rather than
    reported finished; an empty table is finished at once."""
    sfhk, ctx, torch = S
    b = sfhk.Batch(ctx, 2, 16, 0, 0)
    with pytest.raises(sfhk.SfhkError) as ei:
        b.run()
    assert ei.value.status == sfhk.SFHK_E_INVALID
    b.set_jobs([])
    assert b.run()
    b.close()
