"""The laser field behind the C ABI: the library tabulates a pulse's field itself (Sec. II.B field,
E = -dA/dt of the sin^2 pulse of App. A) in the fixed sequence its header states, the same one the
oracle's field table follows, so a job given only the pulse runs in the oracle's field bit for bit;
a job given both a table and a pulse is refused when the two disagree."""
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


def _run(S, inst, e_half, pulse):
    sfhk, ctx, torch = S
    a = sfhk.to_device(inst, f"cuda:{ctx.device}")
    e = None if e_half is None else torch.from_numpy(np.ascontiguousarray(e_half)).to(a["t0"].device)
    g = inst.grid
    job = sfhk.Job(ctx, inst.potential, inst.ground, g.t_a, g.h, g.n_steps, e, a["t0"], a["q0"],
                   a["p0"], a["w"], inst.gamma, inst.kay_max, inst.overlap_cut, pulse=pulse)
    assert job.propagate(0)
    d, f = job.dipole(want_f=True)
    y, _, death = job.trajectories()
    torch.cuda.synchronize()
    out = (f.cpu().numpy(), y.cpu().numpy(), death.cpu().numpy())
    job.close()
    return out


def _cases():
    c0 = I.config0(16, 8)
    pl = c0.pulse
    cep = I.Pulse(pl.wavelength_nm, pl.intensity_wcm2, pl.n_cycles, cep=0.7)
    from dataclasses import replace
    c0_cep = replace(c0, pulse=cep)
    c1 = I.config1_birth_subset(I.config1(1024, 16), [100, 512, 900])
    return {"config0": c0, "config0_cep": c0_cep, "config1_3x16": c1}


@pytest.mark.parametrize("name", ["config0", "config0_cep", "config1_3x16"])
def test_a_pulse_job_runs_in_the_oracles_field_bit_for_bit(S, name):
    inst = _cases()[name]
    print(f"[field] {name}: {inst.t0.size} trajectories, {inst.grid.n_steps} steps", flush=True)
    table = pulse_table(inst.pulse, inst.grid)
    f_pulse, y_pulse, d_pulse = _run(S, inst, None, inst.pulse)
    f_tab, y_tab, d_tab = _run(S, inst, table, None)
    np.testing.assert_array_equal(y_pulse, y_tab)
    np.testing.assert_array_equal(d_pulse, d_tab)
    np.testing.assert_array_equal(f_pulse, f_tab)
    # and with both given (they agree exactly): the same again
    f_both, y_both, _ = _run(S, inst, table, inst.pulse)
    np.testing.assert_array_equal(y_both, y_tab)
    np.testing.assert_array_equal(f_both, f_tab)


def test_a_table_that_is_not_the_pulses_field_is_refused(S):
    sfhk, ctx, torch = S
    inst = I.config0(4, 4)
    table = pulse_table(inst.pulse, inst.grid)
    e0 = inst.pulse.e0
    # within 1e-9 e0 at every half step: accepted
    near = table + 1e-11 * e0 * np.sin(np.arange(table.size))
    _run(S, inst, near, inst.pulse)
    # one entry off by 1e-6 e0: refused, and the context stays usable
    bad = table.copy()
    bad[table.size // 3] += 1e-6 * e0
    with pytest.raises(RuntimeError, match="pulse"):
        _run(S, inst, bad, inst.pulse)
    # a different CEP: refused
    pl = inst.pulse
    other = pulse_table(I.Pulse(pl.wavelength_nm, pl.intensity_wcm2, pl.n_cycles, cep=0.3),
                        inst.grid)
    with pytest.raises(RuntimeError, match="pulse"):
        _run(S, inst, other, inst.pulse)
    _run(S, inst, table, inst.pulse)


def test_a_grid_without_field_is_refused(S):
    inst = I.config0(4, 4)
    with pytest.raises(RuntimeError, match="e_half or a pulse"):
        _run(S, inst, None, None)
    pl = inst.pulse
    bad = I.Pulse(pl.wavelength_nm, pl.intensity_wcm2, 0.0)
    with pytest.raises(RuntimeError, match="n_cycles"):
        _run(S, inst, None, bad)
