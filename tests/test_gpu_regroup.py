"""Regrouping of live trajectories (sfhk_params.compact_every, k_propagate_rg): four tiles of one
first birth step run in one workgroup and, at every multiple of compact_every steps, move the
trajectories not removed by the Kay test (Sec. III.A) into their first tiles. Trajectories must be
unchanged bit for bit (against the oracle and against the job without regrouping), the dipole equal
to the oracle's within the FP64 bar and to the unregrouped job's at rounding level, and the result
bitwise reproducible whether propagated in one call, in chunks, or across a checkpoint."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2601_17164_amd import inputs as I
from tests.common import rel_l2, require_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    ctx = sfhk.Context(0)
    yield sfhk, ctx, torch
    ctx.close()


def _run(S, inst, every=0, chunk=0, precision=0):
    sfhk, ctx, torch = S
    job = sfhk.make_job(ctx, inst, precision=precision, compact_every=every)
    if chunk:
        while not job.propagate(chunk):
            pass
    else:
        assert job.propagate(0)
    d, f = job.dipole(want_f=True)
    y, c, death = job.trajectories()
    st = job.stats()
    torch.cuda.synchronize()
    out = dict(d=d.cpu().numpy(), F=(f[0] + 1j * f[1]).cpu().numpy(), y=y.cpu().numpy(),
               c=(c[0] + 1j * c[1]).cpu().numpy(), death=death.cpu().numpy(), stats=st)
    job.close()
    return out


def _softcore_groups(births=(0, 100, 200, 300, 511)):
    """Whole birth groups of the full soft-core workload (1024 samples each: 16 tiles, four groups
    of four tiles per birth step), 28% of them removed by the Kay test at various steps."""
    return I.config1_birth_subset(I.softcore_full(), list(births))


def _check_vs_oracle(name, g, r):
    print(f"[{name}] rel-L2(F) = {rel_l2(g['F'], r.F):.2e}, removed {np.sum(r.death >= 0)}"
          f"/{r.death.size}", flush=True)
    np.testing.assert_array_equal(g["death"], r.death)
    np.testing.assert_array_equal(g["y"], r.y_final)
    assert g["stats"].steps_evaluated == r.steps_evaluated
    assert g["stats"].kay_removed == r.kay_removed
    assert g["stats"].nonfinite_removed == r.nonfinite_removed
    assert rel_l2(g["F"], r.F) <= TOL
    alive = r.death < 0
    if alive.any():
        assert np.max(np.abs(g["c"][alive] - r.c_final[alive]) / np.abs(r.c_final[alive])) < 1e-12


@pytest.mark.parametrize("every", [16, 256, 1000])
def test_regrouped_softcore_matches_oracle_and_the_plain_job(S, every):
    inst = _softcore_groups()
    print(f"[regroup every {every}] {inst.n_traj} trajectories x {inst.grid.n_steps} steps",
          flush=True)
    r = run_oracle(inst)
    g = _run(S, inst, every=every)
    _check_vs_oracle(f"every {every}", g, r)
    plain = _run(S, inst)
    np.testing.assert_array_equal(g["y"], plain["y"])
    np.testing.assert_array_equal(g["death"], plain["death"])
    assert g["stats"].integrands_evaluated == plain["stats"].integrands_evaluated
    assert g["stats"].prims_evaluated == plain["stats"].prims_evaluated
    assert rel_l2(g["F"], plain["F"]) < 1e-13  # only the grouping of the per-tile sums differs


def test_regrouped_chunked_repeat_and_checkpoint_are_bitwise(S):
    sfhk, ctx, torch = S
    inst = _softcore_groups((3, 250, 400))
    one = _run(S, inst, every=512)
    again = _run(S, inst, every=512)
    np.testing.assert_array_equal(one["F"], again["F"])
    for chunk in (700, 512, 97):
        ch = _run(S, inst, every=512, chunk=chunk)
        np.testing.assert_array_equal(ch["F"], one["F"])
        np.testing.assert_array_equal(ch["y"], one["y"])
        np.testing.assert_array_equal(ch["death"], one["death"])
        assert ch["stats"].steps_evaluated == one["stats"].steps_evaluated
    a = sfhk.make_job(ctx, inst, compact_every=512)
    assert not a.propagate(3000)
    ck = a.checkpoint()
    a.close()
    b = sfhk.make_job(ctx, inst, compact_every=512)
    b.restore(ck)
    while not b.propagate(1100):
        pass
    d, f = b.dipole(want_f=True)
    y, c, death = b.trajectories()
    torch.cuda.synchronize()
    np.testing.assert_array_equal((f[0] + 1j * f[1]).cpu().numpy(), one["F"])
    np.testing.assert_array_equal(y.cpu().numpy(), one["y"])
    assert b.stats().steps_evaluated == one["stats"].steps_evaluated
    b.close()
    # a checkpoint of the unregrouped job does not restore into a regrouping one
    p = sfhk.make_job(ctx, inst)
    assert not p.propagate(3000)
    ckp = p.checkpoint()
    p.close()
    q = sfhk.make_job(ctx, inst, compact_every=512)
    with pytest.raises(sfhk.SfhkError) as e:
        q.restore(ckp)
    assert e.value.status == sfhk.SFHK_E_INVALID
    q.close()


@pytest.mark.parametrize("case", ["config0", "ragged", "all_removed", "screened"])
def test_regrouping_with_partial_groups_and_edge_cases(S, case):
    """config 0 has 32 samples per birth, so no four tiles share a first birth step (every
    workgroup runs four independent tiles); 'ragged' has 288 samples per birth (4.5 tiles: some
    groups, some not) and a padded last tile; 'all_removed' removes every trajectory early (every
    wave of every group retires at a boundary); 'screened' is the p-wave potential."""
    if case == "config0":
        inst = I.config0()
    elif case == "ragged":
        inst = I.softcore_full(n_birth=512, n_per_birth=288)
        inst = inst.subset(np.concatenate([np.arange(288 * b, 288 * b + 288) for b in (7, 300)]
                                          + [np.arange(288 * 450, 288 * 450 + 100)]))
    elif case == "all_removed":
        inst = replace(_softcore_groups((10, 300)), kay_max=1e2)
    else:
        inst = I.config1_birth_subset(I.config1(), [0, 512], 256)
    r = run_oracle(inst)
    g = _run(S, inst, every=64)
    _check_vs_oracle(case, g, r)
    if case == "all_removed":
        assert np.all(r.death >= 0)


def test_regrouping_refusals(S):
    sfhk, ctx, torch = S
    inst = I.config0(n_birth=4, n_per_birth=64)
    for kw in (dict(compact_every=8), dict(compact_every=1 << 25),
               dict(compact_every=256, precision=sfhk.SFHK_FP32_MIXED)):
        with pytest.raises(sfhk.SfhkError) as e:
            sfhk.make_job(ctx, inst, **kw)
        assert e.value.status == sfhk.SFHK_E_INVALID
    job = sfhk.make_job(ctx, inst, compact_every=256)
    with pytest.raises(sfhk.SfhkError) as e:
        sfhk.propagate_many([job])
    assert e.value.status == sfhk.SFHK_E_INVALID
    b = sfhk.Batch(ctx, max_jobs=2, max_tiles=64)
    with pytest.raises(sfhk.SfhkError) as e:
        b.set_jobs([job])
    assert e.value.status == sfhk.SFHK_E_INVALID
    b.close()
    assert job.propagate(0)
    job.close()


def test_regrouped_full_size_sampled_trajectories(S):
    """The full soft-core workload (2^19 trajectories) regrouped every 1024 steps, as the
    benchmark's soft-core leg runs it: sampled trajectories bit for bit against the oracle and the
    counters against the per-trajectory removal steps."""
    sfhk, ctx, torch = S
    inst = I.softcore_full()
    g = _run(S, inst, every=1024)
    died = g["death"] >= 0
    rng = np.random.default_rng(23)
    idx = np.sort(np.concatenate([rng.choice(np.flatnonzero(died), 8, replace=False),
                                  rng.choice(np.flatnonzero(~died), 8, replace=False)]))
    r = run_oracle(inst.subset(idx))
    np.testing.assert_array_equal(g["death"][idx], r.death)
    np.testing.assert_array_equal(g["y"][:, idx], r.y_final)
    st = g["stats"]
    n0 = np.clip(np.ceil((inst.t0 - inst.grid.t_a) / inst.grid.h - 0.5), 0, inst.grid.n_steps)
    expect = np.where(died, g["death"] - n0 + 1, inst.grid.n_steps - n0 + 1).sum()
    assert st.steps_evaluated == expect
    assert st.kay_removed + st.nonfinite_removed == died.sum()


def test_regrouping_with_velocity_and_partial_waves(S):
    """The dipole velocity's accumulators and the partial-wave filter under regrouping: V and F
    agree with the unregrouped job at rounding level, trajectories bit for bit."""
    sfhk, ctx, torch = S
    inst = _softcore_groups((20, 260))
    out = {}
    for every in (0, 128):
        job = sfhk.make_job(ctx, inst, compact_every=every, velocity=True, pw_mask=0x1FD,
                            pw_radius=3.0)
        assert job.propagate(0)
        _, f = job.dipole(want_f=True)
        _, vf = job.velocity(want_v=True)
        y, _, death = job.trajectories()
        torch.cuda.synchronize()
        out[every] = ((f[0] + 1j * f[1]).cpu().numpy(), (vf[0] + 1j * vf[1]).cpu().numpy(),
                      y.cpu().numpy(), death.cpu().numpy())
        job.close()
    (f0, v0, y0, d0), (f1, v1, y1, d1) = out[0], out[128]
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(d1, d0)
    assert np.linalg.norm(f0) > 0 and np.linalg.norm(v0) > 0
    assert rel_l2(f1, f0) < 1e-13 and rel_l2(v1, v0) < 1e-13
