"""The partial-wave filter (Sec. III.A) on the GPU: jobs created with pw_mask != 0 keep only the
steps near the core whose angular momentum |q x p| lies in the selected bands (s, p, d, ...) or,
with the far bit, the steps beyond the radius. Against the oracle's filter on the same inputs (the
decision is reproducible bit for bit: it is taken from the bitwise-equal trajectory state with one
fixed sequence), for the dipole and the dipole velocity; masks partition the unfiltered dipole."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I
from tests.common import e_half, oracle_ground, oracle_potential, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-9
S_, P_, D_, FAR = 1, 2, 4, 256


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    ctx = sfhk.Context(0)
    yield sfhk, ctx, torch
    ctx.close()


def _oracle(inst, mask, velocity=False):
    return O.propagate(oracle_potential(inst.potential), oracle_ground(inst.ground), e_half(inst),
                       inst.grid.t_a, inst.grid.h, inst.grid.n_steps, inst.t0, inst.q0, inst.p0,
                       inst.w, inst.gamma, inst.kay_max, inst.overlap_cut, 0, velocity=velocity,
                       pw_mask=mask, pw_radius=3.0)


def _gpu(S, inst, mask, velocity=False, precision=0):
    sfhk, ctx, torch = S
    job = sfhk.make_job(ctx, inst, precision=precision, velocity=velocity, pw_mask=mask,
                        pw_radius=3.0)
    assert job.propagate(0)
    _, f = job.dipole(want_f=True)
    F = (f[0] + 1j * f[1]).cpu().numpy()
    V = None
    if velocity:
        _, vf = job.velocity(want_v=True)
        V = (vf[0] + 1j * vf[1]).cpu().numpy()
    torch.cuda.synchronize()
    job.close()
    return F, V


def _close(g, r):
    if np.max(np.abs(r)) == 0.0:
        return np.max(np.abs(g)) == 0.0
    return rel_l2(g, r) <= TOL


@pytest.mark.parametrize("mask", [P_, S_ | D_, FAR, P_ | FAR])
def test_softcore_filter_matches_oracle(S, mask):
    inst = I.config0()
    ref = _oracle(inst, mask)
    F, _ = _gpu(S, inst, mask)
    print(f"mask {mask:#x}: rel-L2 {rel_l2(F, ref.F) if np.any(ref.F) else 0.0:.3e}", flush=True)
    assert _close(F, ref.F)


def test_screened_p_ground_state_s_and_d_waves(S):
    """A p-wave ground state (the argon analogue): s and d waves, dipole and velocity."""
    full = I.config1(n_out=0)
    inst = I.config1_birth_subset(full, [200, 480, 512, 800], n_per_birth=64)
    ref = _oracle(inst, S_ | D_, velocity=True)
    F, V = _gpu(S, inst, S_ | D_, velocity=True)
    assert _close(F, ref.F) and _close(V, ref.V)


def test_masks_partition_the_dipole(S):
    inst = I.config0(n_birth=32, n_per_birth=16)
    full, _ = _gpu(S, inst, 0)
    allbits, _ = _gpu(S, inst, 0x1FF)
    np.testing.assert_array_equal(allbits, full)
    parts = [_gpu(S, inst, 1 << k)[0] for k in range(9)]
    assert np.max(np.abs(np.sum(parts, axis=0) - full)) <= 1e-12 * np.max(np.abs(full))


def test_mixed_precision_full_mask_equals_unfiltered(S):
    inst = I.config0(n_birth=16, n_per_birth=16)
    a, _ = _gpu(S, inst, 0, precision=1)
    b, _ = _gpu(S, inst, 0x1FF, precision=1)
    np.testing.assert_array_equal(a, b)


def test_filter_argument_errors(S):
    sfhk, ctx, torch = S
    inst = I.config0(n_birth=4, n_per_birth=8)
    for mask, radius in ((0x200, 3.0), (-1, 3.0), (P_, 0.0), (P_, float("inf"))):
        with pytest.raises(sfhk.SfhkError) as ei:
            sfhk.make_job(ctx, inst, pw_mask=mask, pw_radius=radius)
        assert ei.value.status == sfhk.SFHK_E_INVALID


def test_checkpoint_refused_by_a_job_with_other_parameters(S):
    """A checkpoint carries a fingerprint of the job's parameters: restoring it into a job of the
    same shape but another filter, Kay limit or coherent-state width is refused."""
    sfhk, ctx, torch = S
    inst = I.config0(n_birth=8, n_per_birth=32)
    a = sfhk.make_job(ctx, inst, pw_mask=P_, pw_radius=3.0)
    assert not a.propagate(500)
    ck = a.checkpoint()
    a.close()
    from dataclasses import replace
    for other in (dict(pw_mask=P_ | FAR, pw_radius=3.0), dict(pw_mask=P_, pw_radius=2.5),
                  dict(pw_mask=P_, pw_radius=3.0, inst=replace(inst, kay_max=1e20)),
                  dict(pw_mask=P_, pw_radius=3.0, inst=replace(inst, gamma=0.6))):
        x = other.pop("inst", inst)
        b = sfhk.make_job(ctx, x, **other)
        with pytest.raises(sfhk.SfhkError) as ei:
            b.restore(ck)
        assert ei.value.status == sfhk.SFHK_E_INVALID
        b.close()
    same = sfhk.make_job(ctx, inst, pw_mask=P_, pw_radius=3.0)
    same.restore(ck)
    while not same.propagate(700):
        pass
    ref, _ = _gpu(S, inst, P_)
    _, f = same.dipole(want_f=True)
    np.testing.assert_array_equal((f[0] + 1j * f[1]).cpu().numpy(), ref)
    same.close()
