"""The C ABI used from plain C: tests/native/c_api_driver.c (gcc, the HIP runtime API and
libsfhk.so, no Python) runs an instance through job creation with the pulse, chunked propagation,
the dipole and the spectrum; its F must equal the oracle's within the FP64 bar and the Python
binding's result bit for bit (the same library behind both)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I
from tests.common import rel_l2, require_gpu, run_oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2601_17164_amd")


def _write_instance(path, inst, chunk):
    g, p, gs, pot = inst.grid, inst.pulse, inst.ground, inst.potential
    alpha = np.asarray(gs.alpha, dtype=np.float64)
    hdr = np.array([inst.n_traj, g.n_steps, alpha.size, gs.l, pot.kind, chunk], dtype=np.int64)
    par = np.array([g.t_a, g.h, p.e0, p.omega, p.n_cycles, p.cep, inst.gamma, inst.kay_max,
                    inst.overlap_cut, gs.ip, pot.z_inf, pot.z_in, pot.r_scr, pot.soft2,
                    pot.omega_ho], dtype=np.float64)
    with open(path, "wb") as f:
        for a in (hdr, par, alpha, np.asarray(gs.coef, dtype=np.float64),
                  np.asarray(inst.t0, dtype=np.float64), np.asarray(inst.q0, dtype=np.float64),
                  np.asarray(inst.p0, dtype=np.float64)):
            f.write(np.ascontiguousarray(a).tobytes())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("case", ["config0", "screened_4x64"])
def test_the_path_from_plain_c(tmp_path, case):
    require_gpu()
    if case == "config0":
        inst = I.config0(n_birth=16, n_per_birth=32)
    else:
        inst = I.config1_birth_subset(I.config1(), [0, 300, 600, 900], 64)
    exe = str(tmp_path / "c_api_driver")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    f"-I{rocm}/include", f"-I{os.path.join(ROOT, 'include')}", "-o", exe,
                    os.path.join(HERE, "native", "c_api_driver.c"), f"-L{PKG}", "-lsfhk",
                    f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{rocm}/lib"],
                   check=True, capture_output=True, text=True)
    inp, out = str(tmp_path / "inst.bin"), str(tmp_path / "out.bin")
    _write_instance(inp, inst, chunk=700)
    print(f"[c api] {case}: {inst.n_traj} trajectories, {inst.grid.n_steps} steps", flush=True)
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout.strip(), flush=True)
    m = inst.grid.n_steps + 1
    v = np.fromfile(out, dtype=np.float64)
    F = v[:m] + 1j * v[m:2 * m]
    d = v[2 * m:3 * m]
    power = v[3 * m:]
    ref = run_oracle(inst)
    assert rel_l2(F, ref.F) <= 1e-9
    np.testing.assert_array_equal(d, -2.0 * F.real)
    T = inst.grid.h * inst.grid.n_steps
    _, p_ref, _ = O.spectrum(O.dipole(ref.F), inst.grid.t_a, inst.grid.h, T / 2)
    big = p_ref > 1e-12 * p_ref.max()
    assert np.max(np.abs(power[big] - p_ref[big]) / p_ref[big]) < 1e-6
    # the Python binding over the same library, same chunking: bit for bit
    import torch
    from paper_2601_17164_amd import sfhk
    ctx = sfhk.Context(0)
    job = sfhk.make_job(ctx, inst)
    while not job.propagate(700):
        pass
    _, f = job.dipole(want_f=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal((f[0] + 1j * f[1]).cpu().numpy(), F)
    job.close()
    ctx.close()
