"""Autotuner of the batched propagation: chooses the launch form (persistent queue with a given
number of resident workgroups per compute unit, or hardware dispatch of one workgroup per tile)
and the step chunk for a precision, by timing trials of the candidates through the C ABI on
batches drawn from the uneven-batch distribution, in two stages:
  1. every candidate (WORKERS x CHUNKS) on a small batch: 16 instances with a quarter of their
     trajectories (1/16 of the 64-instance batch's work);
  2. for each resident-workgroup count, its best chunk from stage 1, again on a batch of the full
     batch's shape: 64 instances with half their trajectories. The small batch ranks the chunks
     as the full batch does but not the forms (it has too few long tiles for the tails of the
     persistent forms to even out), so the form is chosen on the second.
Results are cached per device name and precision in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

# resident workgroups per compute unit (0 = hardware dispatch); 8 and 12 fill the wave slots of
# the FP64 (two waves per SIMD) and the FP32-mixed (three) kernels
WORKERS = (0, 4, 8, 12, 16)
CHUNKS = (0, 256, 1024, 4096)    # steps per replay; 0 = to the end in one replay
# on a small trial a persistent form must beat the best hardware-dispatch form by this factor:
# near-ties there have not carried over to full-size batches (stage 2 compares with no margin)
PERSISTENT_MARGIN = 1.05


def forms():
    """Every candidate launch form, as the keys of the rates the tuner reports."""
    return [f"workers={w},chunk={k}" for w in WORKERS for k in CHUNKS]


def parse(form: str):
    """(workers_per_cu, chunk) of a form key"""
    w, k = (int(v.split("=")[1]) for v in form.split(","))
    return w, k


def _trial(sfhk, ctx, arrays_list, insts, precision, workers, chunk, torch):
    jobs = [sfhk.make_job(ctx, x, a, precision=precision) for x, a in zip(insts, arrays_list)]
    b = sfhk.Batch(ctx, len(jobs), sum(sfhk.tiles_of(x) for x in insts), chunk, workers)
    b.set_jobs(jobs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    while not b.run():
        pass
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    steps = sum(j.stats().steps_evaluated for j in jobs)
    for j in jobs:
        j.close()
    b.close()
    return steps / dt


def choose(rates: dict, margin: float = PERSISTENT_MARGIN) -> str:
    """The fastest candidate, with hardware dispatch kept unless a persistent form is faster by
    `margin`."""
    best = max(rates, key=rates.get)
    hw = [k for k in rates if k.startswith("workers=0,")]
    if hw and not best.startswith("workers=0,"):
        best_hw = max(hw, key=rates.get)
        if rates[best] < margin * rates[best_hw]:
            return best_hw
    return best


def finalists(rates: dict) -> list:
    """For each resident-workgroup count, its form with the best rate."""
    out = {}
    for form, r in rates.items():
        w, _ = parse(form)
        if w not in out or r > rates[out[w]]:
            out[w] = form
    return [out[w] for w in sorted(out)]


def tune(ctx, precision: int = 0, n_instances: int = 16, traj_scale: float = 1.0 / 4,
         seed: int = 77, use_cache: bool = True, verbose: bool = False,
         confirm_instances: int = 64, confirm_scale: float = 0.5) -> dict:
    """Returns {"workers_per_cu": w, "chunk": k, "rates": {stage 1}, "confirm_rates": {stage 2}}
    for this device and precision (confirm_instances = 0: stage 1 only)."""
    import torch
    from . import inputs as I, sfhk
    dev = torch.cuda.get_device_name(ctx.device)
    key = f"{dev}|precision={precision}"
    cache = {}
    if os.path.exists(CACHE):
        try:
            with open(CACHE) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]
    insts = I.batch_instances(n_instances, seed=seed, traj_scale=traj_scale)
    arrays_list = [sfhk.to_device(x, f"cuda:{ctx.device}") for x in insts]
    _trial(sfhk, ctx, arrays_list, insts, precision, 8, 0, torch)  # warm-up
    rates = {}
    for form in forms():
        w, k = parse(form)
        r = _trial(sfhk, ctx, arrays_list, insts, precision, w, k, torch)
        rates[form] = r
        if verbose:
            print(f"autotune precision={precision} workers_per_cu={w} chunk={k}: "
                  f"{r:.4e} trajectory-steps/s", flush=True)
    best = choose(rates)
    confirm = {}
    if confirm_instances > 0:
        big = I.batch_instances(confirm_instances, seed=seed, traj_scale=confirm_scale)
        big_arrays = [sfhk.to_device(x, f"cuda:{ctx.device}") for x in big]
        for form in finalists(rates):
            fw, fk = parse(form)
            confirm[form] = _trial(sfhk, ctx, big_arrays, big, precision, fw, fk, torch)
            if verbose:
                print(f"autotune precision={precision} stage 2 workers_per_cu={fw} chunk={fk}: "
                      f"{confirm[form]:.4e} trajectory-steps/s", flush=True)
        del big_arrays
        best = choose(confirm, margin=1.0)
    w, k = parse(best)
    res = {"workers_per_cu": w, "chunk": k, "rates": rates, "confirm_rates": confirm}
    cache[key] = res
    try:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return res
