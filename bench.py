"""Benchmark of the SFHK hot path on one MI355X.

One step = one pass of the whole path over one synthetic instance whose inputs are already in
HBM: job creation (birth snapping, initial state), propagation of every trajectory (RK4 of the 43
ODEs, HK prefactor, Kay removal, dipole integrand, per-step reduction), the fixed-order reduction
into d(t) with resampling, and the Hann-windowed spectrum.

Workload: screened SAE potential, 1600 nm, 1.5e14 W/cm^2, 8-cycle sin^2 pulse, 1024 birth times x
1024 Gaussian phase-space samples (2^20 trajectories), gamma = 0.5, RK4 dt = 0.05, FP64, dipole
resampled onto 2^15 points.

Prints one JSON line. The CPU baseline is the plain oracle on a bounded sample of the same
workload (it is test infrastructure; the product path never calls it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CUs x 2.4 GHz x 128 FP64 operations per CU-clock
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "propagate_traffic.json")


def kernel_source_hash() -> str:
    """sha256 of the sources the FP64 propagate kernel is compiled from (the host runtime in
    sfhk.hip does not enter)."""
    h = hashlib.sha256()
    for f in ("sfhk_kernels.hpp", "sfhk_device.hpp", "sfhk_exact_sum.hpp"):
        with open(os.path.join(ROOT, "paper_2601_17164_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(n_traj: int):
    """HBM bytes of one propagate launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE runs recorded
    with the profile, if they were taken on this kernel source and this workload; else None."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("n_traj") != n_traj:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64"], default="fp64")
    ap.add_argument("--n-birth", type=int, default=1024)
    ap.add_argument("--n-per-birth", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-mixed pass over the same inputs")
    ap.add_argument("--cpu-births", type=int, default=64,
                    help="birth groups (spread over the pulse) in the oracle's sample")
    ap.add_argument("--cpu-per-birth", type=int, default=384)
    ap.add_argument("--batch", action="store_true",
                    help="instead: the 64-instance uneven batch in one graph-captured launch per "
                         "precision (FP64 and FP32-mixed), autotuned launch form")
    ap.add_argument("--batch-size", type=int, default=64)
    ap.add_argument("--batch-sweep", action="store_true",
                    help="instead: every launch form of the autotuner on the full batch, the "
                         "tuner's trial beside it, and the batch split by potential kind")
    ap.add_argument("--batch-forms", default="",
                    help="with --batch-sweep: only these forms (';'-separated, as the tuner names "
                         "them, e.g. 'workers=0,chunk=0;workers=8,chunk=0')")
    ap.add_argument("--serve", action="store_true",
                    help="instead: the serving sweep (Poisson arrivals at --rates, FP64 and mixed)")
    ap.add_argument("--rates", default="5,10,20,50")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--serve-warmup", type=int, default=20)
    ap.add_argument("--serve-chunk", type=int, default=1024)
    ap.add_argument("--default-requests", type=int, default=100,
                    help="measured requests per rate in the default line's serving sweep")
    ap.add_argument("--default-serve-warmup", type=int, default=10)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving sweep (--rates, both forms) of the default benchmark")
    ap.add_argument("--no-sfa", action="store_true",
                    help="skip the SFA birth step leg (birth kernel timing, SFA-born propagation)")
    ap.add_argument("--sfa-reps", type=int, default=5)
    ap.add_argument("--gabor-only", action="store_true",
                    help="time only the Gabor map (512 x 2048) of a seeded 2^15-sample signal")
    ap.add_argument("--no-velocity", action="store_true",
                    help="skip the dipole-velocity leg (one propagation with both accumulators)")
    ap.add_argument("--sfa-only", action="store_true",
                    help="time only the SFA birth step (2^20 samples) and print its JSON line")
    ap.add_argument("--no-softcore", action="store_true",
                    help="skip the soft-core leg (config 0's atom at config 1's pulse, 2^19 "
                         "trajectories)")
    ap.add_argument("--softcore-regroup", default="1024",
                    help="regrouping intervals (steps, comma-separated; empty: none) timed on the "
                         "soft-core leg besides the plain form")
    ap.add_argument("--softcore-kay", type=float, default=None,
                    help="Kay limit D_t of the soft-core leg (default: the workload's 1e30)")
    ap.add_argument("--softcore-only", action="store_true",
                    help="time only the soft-core leg and print its JSON line")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven-batch pass of the default benchmark")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (calibrates the "
                         "HBM traffic counters) and exit")
    return ap.parse_args()


def _device_info():
    """The GPU the line was measured on (boxes of one model differ by a few % in sustained FP64
    clock, so the figures are read together with this)."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    return {"name": pr.name, "arch": getattr(pr, "gcnArchName", None),
            "compute_units": pr.multi_processor_count,
            "memory_gib": round(pr.total_memory / 2 ** 30, 1)}


def _ints(text):
    """comma-separated integers (empty: none)"""
    return [int(x) for x in text.split(",") if x.strip()]


def copy_probe(nbytes):
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8}), flush=True)


def cpu_baseline(inst, n_births, n_per, ctx=None):
    """Oracle trajectory-steps/s on a bounded sample: n_births birth groups spread evenly over
    the pulse, the first n_per samples of each. With a context, the device also propagates the
    same sample and its F is compared with the oracle's (relative L2)."""
    from oracle import oracle as O  # test infrastructure: the CPU-baseline leg only
    from tests.common import run_oracle
    O.build(force=False)
    stride = max(1, inst.n_birth // n_births)
    births = list(range(0, inst.n_birth, stride))[:n_births]
    from paper_2601_17164_amd import inputs as I
    sub = I.config1_birth_subset(inst, births, n_per)
    threads = min(os.cpu_count() or 1, 16)
    t = time.perf_counter()
    r = run_oracle(sub, n_threads=threads)
    dt = time.perf_counter() - t
    c0 = I.config0()  # the small configuration in full, beside the sample
    t = time.perf_counter()
    r0 = run_oracle(c0, n_threads=threads)
    dt0 = time.perf_counter() - t
    parity = None
    if ctx is not None:
        import torch
        from paper_2601_17164_amd import sfhk
        job = sfhk.make_job(ctx, sub)
        assert job.propagate(0)
        _, f = job.dipole(want_f=True)
        F = (f[0] + 1j * f[1]).cpu().numpy()
        torch.cuda.synchronize()
        job.close()
        parity = float(np.linalg.norm(F - r.F) / np.linalg.norm(r.F))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": r.steps_evaluated / dt, "unit": "trajectory-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(births)} birth groups x {n_per} samples = {sub.n_traj} trajectories "
                      f"({r.steps_evaluated} trajectory-steps, {dt:.1f} s)",
            "per_core": r.steps_evaluated / dt / threads, "cpu_model": model,
            "host_cpus": os.cpu_count(),
            "gpu_vs_oracle_rel_l2_F": parity,
            "config0_full": {"value": r0.steps_evaluated / dt0, "trajectories": c0.n_traj,
                             "trajectory_steps": r0.steps_evaluated, "seconds": dt0}}


def mixed_form(step, stream, inst, arrays, ref_spectrum, flops):
    """One pass of the FP32-mixed form over the same inputs: its rate, its spectral error against
    the FP64 kernel's spectrum (which matches the FP64 oracle to 1e-9), and beside it the
    conditioning floor of the workload: the FP64 spectrum of the samples with q0 moved by one ulp
    against the unmoved one."""
    import torch
    from paper_2601_17164_amd import metrics
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    job, (om, pw, x) = step(ev, precision=1)
    st = job.stats(stream)
    wall = time.perf_counter() - t
    drift = _det_drift(job)
    job.close()
    kms = ev[0].elapsed_time(ev[1])
    fl = flops.flops(inst.potential.kind, inst.ground.l, st.steps_evaluated, st.prims_evaluated,
                     st.integrands_evaluated)
    om_r, _, x_r = ref_spectrum
    band = lambda xx: metrics.spectral_report(om_r.cpu().numpy(), xx.cpu().numpy(),
                                              x_r.cpu().numpy(), inst.ground.ip, inst.pulse.up,
                                              inst.pulse.omega)
    q0 = arrays["q0"]
    arrays["q0"] = torch.nextafter(q0, torch.full_like(q0, float("inf")))
    job, (_, _, x_p) = step([torch.cuda.Event(enable_timing=True) for _ in range(2)])
    torch.cuda.synchronize()
    drift64 = _det_drift(job)
    job.close()
    arrays["q0"] = q0
    return {"value": st.steps_evaluated / wall, "unit": "trajectory-steps/s",
            "kernel_ms": kms,
            "frac_of_fp64_vector_peak": fl / (kms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "fp64_step_fraction": st.steps_fp64 / max(1, st.steps_evaluated),
            "spectral_error_vs_fp64": band(x), "fp64_one_ulp_floor": band(x_p),
            "det_M_drift": drift, "fp64_det_M_drift": drift64, "kay_max": inst.kay_max}


def _det_drift(job):
    """At each trajectory's last evaluated step (the removal step for removed ones): |det M - 1|
    and the scale-free symplectic defect max|M^T J M - J| / ||M||_F^2, median and max over the
    job. With the Kay limit at 1e30 |det M - 1| is dominated by the cancellation in det M of
    large monodromy matrices; the defect is the meaningful figure."""
    from paper_2601_17164_amd import metrics
    y, _, _ = job.trajectories()
    y = y.cpu().numpy()
    out = {}
    for name, v in (("det", metrics.det_monodromy_drift(y)),
                    ("symplectic_defect", metrics.symplectic_defect(y))):
        v = v[np.isfinite(v)]
        out[name] = {"median": float(np.median(v)), "max": float(np.max(v))} if v.size else None
    return out


def serving_run(ctx, rate, n_req, warmup, precision, chunk, reqs=None, verbose=False):
    """Poisson arrivals at `rate` of requests drawn from the uneven-batch distribution (request r
    has seed 4000 + r); returns latency percentiles and throughput over the non-warm-up requests."""
    from paper_2601_17164_amd import inputs as I, serve, sfhk
    n = warmup + n_req
    if reqs is None:
        reqs = [I.serving_request(k) for k in range(n)]
    t = serve.poisson_arrivals(rate, n, seed=4000 + int(round(rate * 1000)))
    requests = [serve.Request(k, float(t[k]), reqs[k]) for k in range(n)]
    max_tiles = sum(sfhk.tiles_of(x) for x in reqs)
    srv = serve.Server(ctx, precision=precision, chunk=chunk, workers_per_cu=0,
                       max_jobs=min(64, n), max_tiles=max_tiles)
    res = srv.run(requests)
    srv.close()
    kept = [r for r in res if r.req_id >= warmup]
    summ = serve.summarize(kept)
    summ.update({"offered_rate": rate, "served_rate": len(kept) / summ["span_s"],
                 "precision": "fp32_mixed" if precision else "fp64", "chunk": chunk})
    summ.update(srv.stats)
    if verbose:
        print(json.dumps(summ), flush=True)
    return summ


def serving_sweep(ctx, a):
    """The serving loop at each offered rate of --rates, in both forms, with --default-requests
    measured requests after --default-serve-warmup warm-up ones (the default line's leg)."""
    from paper_2601_17164_amd import inputs as I
    n = a.default_serve_warmup + a.default_requests
    reqs = [I.serving_request(k) for k in range(n)]
    runs = []
    for prec in (0, 1):
        for rate in [float(x) for x in a.rates.split(",")]:
            r = serving_run(ctx, rate, a.default_requests, a.default_serve_warmup, prec,
                            a.serve_chunk, reqs)
            runs.append({k: r[k] for k in ("precision", "offered_rate", "served_rate", "requests",
                                           "p50_ms", "p99_ms", "trajectory_steps_per_s",
                                           "max_active", "max_queued")})
            print(json.dumps({"serving_progress": runs[-1]}), file=sys.stderr, flush=True)
    return {"requests_per_rate": a.default_requests, "warmup": a.default_serve_warmup,
            "chunk": a.serve_chunk, "runs": runs}


def run_serve(a):
    import torch
    from paper_2601_17164_amd import inputs as I, sfhk
    ctx = sfhk.Context(0)
    n = a.serve_warmup + a.requests
    reqs = [I.serving_request(k) for k in range(n)]
    out = {"metric": "serving: p50/p99 spectrum latency and trajectory-steps/s",
           "data": "synthetic", "n_gpus": 1, "requests_per_rate": a.requests,
           "warmup": a.serve_warmup, "runs": []}
    for prec in (0, 1):
        for rate in [float(x) for x in a.rates.split(",")]:
            out["runs"].append(serving_run(ctx, rate, a.requests, a.serve_warmup, prec,
                                           a.serve_chunk, reqs, verbose=True))
    print(json.dumps(out), flush=True)


def batch_results(ctx, batch_size):
    """The uneven batch: `batch_size` instances (wavelength 800-2000 nm, 0.8-3e14 W/cm^2, 2-10
    cycles, potential of either workload, 2^14-2^20 trajectories each), all tiles of all instances
    in one graph replay with the autotuned launch form, in FP64 and then in the FP32-mixed form."""
    import torch
    from paper_2601_17164_amd import autotune, inputs as I, sfhk
    insts = I.batch_instances(batch_size, seed=3)
    arrays = [sfhk.to_device(x, "cuda:0") for x in insts]
    n_tiles = sum(sfhk.tiles_of(x) for x in insts)
    out = {"metric": "HK trajectory-steps/s, uneven batch in one graph-captured launch",
           "unit": "trajectory-steps/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"{len(insts)} uneven instances", "instances": len(insts),
                      "trajectories": int(sum(x.n_traj for x in insts)), "tiles": n_tiles}}
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        tuned = autotune.tune(ctx, prec, verbose=True)
        jobs = [sfhk.make_job(ctx, x, arr, precision=prec) for x, arr in zip(insts, arrays)]
        b = sfhk.Batch(ctx, len(jobs), n_tiles, tuned["chunk"], tuned["workers_per_cu"])
        b.set_jobs(jobs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        replays = 1
        while not b.run():
            replays += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        st = [j.stats() for j in jobs]
        steps = sum(x.steps_evaluated for x in st)
        out[name] = {"value": steps / wall, "seconds": wall, "trajectory_steps": steps,
                     "replays": replays, "workers_per_cu": tuned["workers_per_cu"],
                     "chunk": tuned["chunk"], "autotune_rates": tuned["rates"],
                     "autotune_confirm_rates": tuned.get("confirm_rates"),
                     "fp64_step_fraction": sum(x.steps_fp64 for x in st) / max(1, steps)}
        for j in jobs:
            j.close()
        b.close()
    return out


def _batch_rate(ctx, insts, arrays, prec, workers, chunk):
    """trajectory-steps/s of one batch of `insts` in one launch form (all replays to the end)"""
    import torch
    from paper_2601_17164_amd import sfhk
    jobs = [sfhk.make_job(ctx, x, arr, precision=prec) for x, arr in zip(insts, arrays)]
    b = sfhk.Batch(ctx, len(jobs), sum(sfhk.tiles_of(x) for x in insts), chunk, workers)
    b.set_jobs(jobs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    while not b.run():
        pass
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    steps = sum(j.stats().steps_evaluated for j in jobs)
    for j in jobs:
        j.close()
    b.close()
    return steps, steps / wall


def batch_sweep(ctx, batch_size, forms=None):
    """The autotuner's candidates on the full uneven batch, beside the tuner's own trial rates
    (does the scaled-down trial rank the forms as the full batch does?), and the batch split by
    potential kind: each kind's instances alone in hardware dispatch, with the work-weighted
    combination of the two rates that the whole batch can be expected to reach."""
    from paper_2601_17164_amd import autotune, inputs as I, sfhk
    insts = I.batch_instances(batch_size, seed=3)
    arrays = [sfhk.to_device(x, "cuda:0") for x in insts]
    out = {"instances": len(insts)}
    for prec, name in ((0, "fp64"), (1, "fp32_mixed")):
        trial = autotune.tune(ctx, prec, use_cache=False, verbose=True)
        full = {}
        for form in (forms or autotune.forms()):
            w, k = autotune.parse(form)
            full[form] = _batch_rate(ctx, insts, arrays, prec, w, k)[1]
            print(json.dumps({"batch_sweep": name, "form": form, "full": full[form],
                              "trial": trial["rates"][form]}), flush=True)
        kinds = {}
        for kind in sorted({x.potential.kind for x in insts}):
            sel = [i for i, x in enumerate(insts) if x.potential.kind == kind]
            steps, rate = _batch_rate(ctx, [insts[i] for i in sel], [arrays[i] for i in sel], prec,
                                      0, 0)
            kinds[str(kind)] = {"instances": len(sel), "trajectory_steps": steps, "rate": rate}
        tot = sum(v["trajectory_steps"] for v in kinds.values())
        mix = tot / sum(v["trajectory_steps"] / v["rate"] for v in kinds.values())
        out[name] = {"chosen": autotune.choose(trial["rates"]), "trial": trial["rates"],
                     "full": full, "by_kind": kinds, "work_weighted_rate": mix}
        print(json.dumps({"batch_sweep": name, "by_kind": kinds, "work_weighted_rate": mix}),
              flush=True)
    return out


def run_batch(a):
    from paper_2601_17164_amd import sfhk
    ctx = sfhk.Context(0)
    print(json.dumps(batch_results(ctx, a.batch_size)), flush=True)
    ctx.close()


def gabor_only(a):
    """The Gabor map of the screened workload's shape (2^15 samples over the 8-cycle 1600 nm
    pulse) on a seeded signal of harmonic bursts; the kernel's work does not depend on the values."""
    import torch
    from paper_2601_17164_amd import inputs as I
    inst = I.config1(n_birth=1, n_per_birth=1)
    T = inst.grid.h * inst.grid.n_steps
    n = inst.n_out
    t = inst.grid.t_a + (T / n) * np.arange(n)
    rng = np.random.default_rng(5)
    d = np.zeros(n)
    for _ in range(16):
        tb, wb = rng.uniform(-0.4 * T, 0.4 * T), inst.pulse.omega * rng.uniform(5, 160)
        d += np.exp(-(t - tb) ** 2 / 50.0) * np.cos(wb * t)
    v = torch.from_numpy(d).to("cuda:0")
    out = gabor_results(torch.cuda.current_stream(), inst, v, reps=a.sfa_reps)
    print(json.dumps({"workload": "Gabor map, 2^15 samples over the screened workload's pulse, "
                                  "512 centres x 2048 frequencies", **out}), flush=True)


def sfa_saddle_work(inst, tt):
    """March steps and algorithmic FP64 operations of the saddle-point kernel for the t_t it
    returned (the march stops at k = ceil(t_t / dtau), dtau = 1 / (4 (omega + omega/n_cycles)))."""
    from paper_2601_17164_amd import flops
    om = inst.pulse.omega
    dtau = 0.25 / (om + om / inst.pulse.n_cycles)
    ok = np.isfinite(tt)
    k = np.ceil(tt[ok] / dtau)
    fl = flops.sfa_saddle_flops(int(k.sum()), int(ok.sum()))
    return {"march_steps_mean": float(k.mean()) if ok.any() else 0.0, "saddle_flop": fl}


def sfa_only(a):
    """Only the SFA birth step on the 2^20 samples of the screened 1600 nm workload."""
    import torch
    from paper_2601_17164_amd import inputs as I, sfhk
    inst = I.sfa_config1()
    stream = torch.cuda.current_stream()
    t0 = torch.from_numpy(inst.t0).to("cuda:0")
    kp = torch.from_numpy(inst.meta["kperp"]).to("cuda:0")
    u = torch.from_numpy(inst.meta["u"]).to("cuda:0")
    for _ in range(a.warmup):
        sfhk.sfa_birth(inst.pulse, inst.ground, t0, kp, u, sfhk.SFHK_BIRTH_GTO, stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(a.sfa_reps):
        b = sfhk.sfa_birth(inst.pulse, inst.ground, t0, kp, u, sfhk.SFHK_BIRTH_GTO, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / a.sfa_reps
    w = sfa_saddle_work(inst, b["tt"].cpu().numpy())
    print(json.dumps({"workload": "SFA births, screened-SAE 1600nm 1.5e14 W/cm2 8-cycle, "
                                  "1024x1024 samples", "n": inst.n_traj, "reps": a.sfa_reps,
                      "birth_ms": ms, "births_per_s": inst.n_traj / ms * 1e3, **w}), flush=True)


def velocity_results(ctx, stream, inst, arrays, plain_ms):
    """One propagation of the benchmark workload with the dipole velocity (App. C.2) accumulated
    beside the dipole: kernel time against the dipole-only launch of the timed steps."""
    import torch
    from paper_2601_17164_amd import sfhk
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    job = sfhk.make_job(ctx, inst, arrays, velocity=True)
    ev[0].record(stream)
    assert job.propagate(0)
    ev[1].record(stream)
    v = job.velocity()
    st = job.stats(stream)
    ok = bool(torch.isfinite(v).all())
    job.close()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    return {"propagate_kernel_ms": ms, "dipole_only_kernel_ms": plain_ms,
            "overhead": ms / plain_ms - 1.0,
            "trajectory_steps_per_s": st.steps_evaluated / ms * 1e3, "finite": ok,
            "gabor": gabor_results(stream, inst, v)}


GABOR_CUT = 9.2  # the kernel sums the samples within this many sigma of each centre


def gabor_results(stream, inst, v, reps=5):
    """Gabor map (sfhk_gabor) of the dipole velocity on the 2^15-point output grid: 512 centres
    over the pulse, 2048 frequencies in steps of omega/10 (beyond the cutoff), sigma = 1/(3 omega).
    Mean kernel time over `reps` launches (HIP events on the launch stream) and the algorithmic
    rate at 7 FP64 operations per (centre, frequency, sample) update (one Horner step: a complex
    multiplication by e^{i w dt} and the sample's addition)."""
    import torch
    from paper_2601_17164_amd import sfhk
    T = inst.grid.h * inst.grid.n_steps
    n = int(v.shape[0])
    dt = T / n
    w0 = inst.pulse.omega
    sigma, n_c, n_w, ws = 1.0 / (3.0 * w0), 512, 2048, w0 / 10
    tc0, tcs = inst.grid.t_a + T / 1024, T / 512
    args = (inst.grid.t_a, dt, sigma, tc0, tcs, n_c, ws, n_w)
    sfhk.gabor(v, *args, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(reps):
        pw, G = sfhk.gabor(v, *args, stream=stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    tc = tc0 + tcs * np.arange(n_c)
    lo = np.ceil(np.clip((tc - GABOR_CUT * sigma - inst.grid.t_a) / dt, 0, n))
    hi = np.floor(np.clip((tc + GABOR_CUT * sigma - inst.grid.t_a) / dt, -1, n - 1))
    updates = float(np.sum(np.maximum(hi - lo + 1, 0))) * n_w
    fl = 7.0 * updates
    return {"n": n, "n_centres": n_c, "n_freq": n_w, "sigma": sigma, "kernel_ms": ms,
            "updates": updates, "achieved_tflops": fl / (ms * 1e-3) / 1e12,
            "frac_of_fp64_vector_peak": fl / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "finite": bool(torch.isfinite(pw).all())}


def sfa_results(ctx, stream, reps):
    """The SFA birth step (sfhk_sfa_birth) on the 2^20 samples of the screened 1600 nm workload:
    mean duration of the birth kernel over `reps` launches (HIP events on the launch stream), then
    one propagation of the trajectories it bore."""
    import torch
    from paper_2601_17164_amd import flops, inputs as I, sfhk
    inst = I.sfa_config1()
    dev = sfhk.to_device(inst, "cuda:0")
    kp = torch.from_numpy(inst.meta["kperp"]).to("cuda:0")
    u = torch.from_numpy(inst.meta["u"]).to("cuda:0")
    b = sfhk.sfa_birth(inst.pulse, inst.ground, dev["t0"], kp, u, sfhk.SFHK_BIRTH_GTO, stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        b = sfhk.sfa_birth(inst.pulse, inst.ground, dev["t0"], kp, u, sfhk.SFHK_BIRTH_GTO, stream)
    ev[1].record(stream)
    dev.update(q0=b["q0"], p0=b["p0"], w=b["w"])
    job = sfhk.make_job(ctx, inst, dev)
    ev[2].record(stream)
    assert job.propagate(0)
    ev[3].record(stream)
    st = job.stats(stream)
    no_saddle = int(torch.isnan(b["tt"]).sum())
    job.close()
    torch.cuda.synchronize()
    birth_ms = ev[0].elapsed_time(ev[1]) / reps
    prop_ms = ev[2].elapsed_time(ev[3])
    tt = b["tt"].cpu().numpy()
    fl = flops.flops(inst.potential.kind, inst.ground.l, st.steps_evaluated, st.prims_evaluated,
                     st.integrands_evaluated)
    envelope = mixed_envelope(ctx, inst, dev, stream)
    return {"workload": "screened-SAE 1600nm 1.5e14 W/cm2 8-cycle, 1024x1024 SFA births "
                        "(GTO tunnelling element), dt 0.05",
            "mixed_vs_fp64_by_kay_limit": envelope,
            "n": inst.n_traj, "birth_kernel_ms": birth_ms, "births_per_s": inst.n_traj / birth_ms * 1e3,
            "no_saddle": no_saddle, **sfa_saddle_work(inst, tt),
            "propagate_kernel_ms": prop_ms,
            "trajectory_steps": st.steps_evaluated,
            "trajectory_steps_per_s": st.steps_evaluated / prop_ms * 1e3,
            "propagate_fp64_frac": fl / (prop_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "kay_removed": st.kay_removed, "prims_per_step": st.prims_evaluated / max(1, st.steps_evaluated)}


def mixed_envelope(ctx, inst, dev, stream, limits=(1e6, 1e8, 1e30)):
    """The FP32-mixed form against the FP64 kernel (which matches the FP64 oracle to 1e-9) on the
    SFA-born trajectories at several Kay limits: E_dB over the plateau and cutoff bands of the
    2^15-point spectrum, and the trajectories the Kay test removed. The FP32 state resolves
    trajectories stretched by up to a few hundred, which limits of 1e6 to 1e8 keep."""
    from dataclasses import replace
    import torch
    from paper_2601_17164_amd import metrics, sfhk
    T = inst.grid.h * inst.grid.n_steps
    dt_out = T / inst.n_out
    out = {}
    for kay in limits:
        ik = replace(inst, kay_max=kay)
        spec, removed = {}, 0
        for prec in (0, 1):
            job = sfhk.make_job(ctx, ik, dev, precision=prec)
            assert job.propagate(0)
            om, _, x = sfhk.spectrum(job.dipole(), inst.grid.t_a, dt_out, T / 2)
            if prec == 0:
                removed = job.stats(stream).kay_removed
            job.close()
            spec[prec] = (om.cpu().numpy(), x.cpu().numpy())
        torch.cuda.synchronize()
        rep = metrics.spectral_report(spec[0][0], spec[1][1], spec[0][1], inst.ground.ip,
                                      inst.pulse.up, inst.pulse.omega)
        out[f"{kay:.0e}"] = {"kay_removed": removed,
                             **{band: round(e["E_dB"], 2) for band, e in rep.items()}}
    return out


def softcore_results(ctx, stream, regroup=(1024,), kay_max=None):
    """The propagate kernel on the soft-core atom at full size (inputs.softcore_full): per form
    (plain, and regrouped every E steps for E in `regroup`) one untimed launch, then one timed with
    HIP events on the launch stream. The soft-core instances are half of the batch and serving
    mix; on these Gaussian samples, placed inside the potential, their kernel is held back by the
    s-wave dipole element, needed at most steps near the nucleus, and by lanes idle after the Kay
    test (28% of the trajectories are removed), which regrouping (sfhk_params.compact_every) gives
    back. `sfa_born`: the same atom, pulse and sizes with SFA births at the tunnel exit."""
    import torch
    from paper_2601_17164_amd import flops, inputs as I, sfhk
    inst = I.softcore_full()
    if kay_max is not None:
        from dataclasses import replace
        inst = replace(inst, kay_max=kay_max)
    arrays = sfhk.to_device(inst, "cuda:0")

    def timed(every, inst=inst, arrays=arrays):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for it in range(2):
            job = sfhk.make_job(ctx, inst, arrays, compact_every=every)
            ev[0].record(stream)
            assert job.propagate(0)
            ev[1].record(stream)
            st = job.stats(stream)
            job.close()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        fl = flops.flops(inst.potential.kind, inst.ground.l, st.steps_evaluated,
                         st.prims_evaluated, st.integrands_evaluated)
        return {"kernel": "k_propagate_rg" if every else "k_propagate_fp64", "kernel_ms": ms,
                "trajectory_steps": st.steps_evaluated,
                "trajectory_steps_per_s": st.steps_evaluated / ms * 1e3,
                "frac_of_fp64_vector_peak": fl / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                "kay_removed_frac": st.kay_removed / inst.n_traj,
                "prims_per_step": st.prims_evaluated / max(1, st.steps_evaluated)}

    plain = timed(0)
    forms = {f"regroup_every_{e}": timed(e) for e in regroup}
    best = min(forms.items(), key=lambda kv: kv[1]["kernel_ms"]) if forms else None
    out = {"workload": "soft-core H (config 0 atom) 1600nm 1.5e14 W/cm2 8-cycle, "
                       f"{inst.n_birth}x{inst.n_per_birth} trajectories, dt 0.1, FP64",
           "n_traj": inst.n_traj, "n_steps": inst.grid.n_steps, "kay_max": inst.kay_max}
    if best and best[1]["kernel_ms"] < plain["kernel_ms"]:
        out.update(best[1])
        out["form"] = best[0]
    else:
        out.update(plain)
        out["form"] = "plain"
    out["plain"] = plain
    out.update(forms)
    # the same atom, pulse and sizes with the paper's initial conditions: SFA births at the tunnel
    # exit (sfhk_sfa_birth on the device) instead of Gaussian samples placed inside the potential
    sfa = I.softcore_sfa_full()
    if kay_max is not None:
        from dataclasses import replace
        sfa = replace(sfa, kay_max=kay_max)
    dev = sfhk.to_device(sfa, "cuda:0")
    b = sfhk.sfa_birth(sfa.pulse, sfa.ground, dev["t0"], torch.from_numpy(sfa.meta["kperp"]).cuda(),
                       torch.from_numpy(sfa.meta["u"]).cuda(), sfhk.SFHK_BIRTH_GTO, stream)
    dev.update(q0=b["q0"], p0=b["p0"], w=b["w"])
    out["sfa_born"] = {"workload": "soft-core H 1600nm 1.5e14 W/cm2 8-cycle, "
                                   f"{sfa.n_birth}x{sfa.n_per_birth} SFA births, dt 0.1, FP64",
                       **timed(0, sfa, dev)}
    return out


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs one job on one GPU; a multi-GPU path (sharding "
                                   "by birth groups with one reduction of d(t)) is not built",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.batch:
        run_batch(a)
        return
    if a.batch_sweep:
        from paper_2601_17164_amd import sfhk
        ctx = sfhk.Context(0)
        forms = [f for f in a.batch_forms.split(";") if f] or None
        print(json.dumps({"batch_sweep": batch_sweep(ctx, a.batch_size, forms)}), flush=True)
        ctx.close()
        return
    if a.serve:
        run_serve(a)
        return
    if a.sfa_only:
        sfa_only(a)
        return
    if a.gabor_only:
        gabor_only(a)
        return
    if a.softcore_only:
        import torch
        from paper_2601_17164_amd import sfhk
        ctx = sfhk.Context(0)
        print(json.dumps({"softcore": softcore_results(ctx, torch.cuda.current_stream(),
                                                       _ints(a.softcore_regroup),
                                                       a.softcore_kay)}), flush=True)
        ctx.close()
        return
    import torch
    from paper_2601_17164_amd import flops, inputs as I, sfhk

    inst = I.config1(n_birth=a.n_birth, n_per_birth=a.n_per_birth)
    dev = torch.device("cuda:0")
    arrays = sfhk.to_device(inst, "cuda:0")
    ctx = sfhk.Context(0)
    stream = torch.cuda.current_stream()
    T = inst.grid.h * inst.grid.n_steps
    n_out = inst.n_out
    dt_out = T / n_out

    def step(ev, precision=0):
        job = sfhk.make_job(ctx, inst, arrays, precision=precision)  # arrays: read at each call
        ev[0].record(stream)
        done = job.propagate(0)
        ev[1].record(stream)
        assert done
        d = job.dipole()
        om, pw, x = sfhk.spectrum(d, inst.grid.t_a, dt_out, T / 2)
        return job, (om, pw, x)

    for _ in range(a.warmup):
        job, spec = step([torch.cuda.Event(enable_timing=True) for _ in range(2)])
        torch.cuda.synchronize()
        job.close()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(a.steps)]
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(a.steps):
        job, spec = step(evs[k])
        marks[k + 1].record(stream)
        stats.append(job.stats(stream))  # synchronises the stream
        job.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    steps_eval = sum(s.steps_evaluated for s in stats)
    kern_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    lat_ms = np.array([marks[k].elapsed_time(marks[k + 1]) for k in range(a.steps)])
    s0 = stats[0]
    fl = flops.flops(inst.potential.kind, inst.ground.l, s0.steps_evaluated, s0.prims_evaluated,
                     s0.integrands_evaluated)
    achieved = fl / (kern_ms.mean() * 1e-3) / 1e12
    out = {
        "metric": "HK trajectory-steps/s (3D, w/ monodromy) at 1 GPU; p50/p99 spectrum latency",
        "value": steps_eval / wall,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "screened-SAE 1600nm 1.5e14 W/cm2 8-cycle, "
                               f"{inst.n_birth}x{inst.n_per_birth} trajectories, dt 0.05, "
                               "2^15-point dipole, FP64",
                   "n_traj": inst.n_traj, "n_steps": inst.grid.n_steps,
                   "trajectory_steps_per_step": s0.steps_evaluated},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99))},
        "roofline": {"bound": "alu", "kernel": "k_propagate_fp64 (screened)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": recorded_traffic(inst.n_traj),
                     "kernel_ms": float(kern_ms.mean()),
                     "flop_per_launch": fl},
        "stats": {"kay_removed": s0.kay_removed, "nonfinite_removed": s0.nonfinite_removed,
                  "prims_per_step": s0.prims_evaluated / max(1, s0.steps_evaluated)},
        "device": _device_info(),
    }
    if not a.no_mixed:
        out["fp32_mixed"] = mixed_form(step, stream, inst, arrays, spec, flops)
    if not a.no_serving:
        out["serving"] = serving_sweep(ctx, a)
    if not a.no_batch:
        out["batch"] = batch_results(ctx, a.batch_size)
    if not a.no_velocity:
        out["velocity"] = velocity_results(ctx, stream, inst, arrays, float(kern_ms.mean()))
    if not a.no_sfa:
        out["sfa_birth"] = sfa_results(ctx, stream, a.sfa_reps)
    if not a.no_softcore:
        out["softcore"] = softcore_results(ctx, stream, _ints(a.softcore_regroup))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, a.cpu_births, a.cpu_per_birth, ctx)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
