"""Autotuner of the batched propagation: chooses the launch form (persistent queue with a given
number of resident workgroups per compute unit, or hardware dispatch of one workgroup per tile)
and the step chunk for a precision, by timing short trials of each candidate through the C ABI on
a scaled-down batch drawn from the uneven-batch distribution (16 instances with a quarter of their
trajectories: 1/16 of the 64-instance batch's work, large enough for its tail effects to show).
Results are cached per device name and precision in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

WORKERS = (0, 4, 8, 16)          # 0 = hardware dispatch
CHUNKS = (0, 2048)               # 0 = to the end in one replay
# a persistent form must beat the best hardware-dispatch form by this factor on the scaled-down
# trial: it calls the tile loop out of line, and near-ties on the small trial have not carried
# over to full-size batches
PERSISTENT_MARGIN = 1.05


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


def choose(rates: dict) -> str:
    """The fastest candidate, with hardware dispatch kept unless a persistent form is faster by
    PERSISTENT_MARGIN."""
    best = max(rates, key=rates.get)
    hw = [k for k in rates if k.startswith("workers=0,")]
    if hw and not best.startswith("workers=0,"):
        best_hw = max(hw, key=rates.get)
        if rates[best] < PERSISTENT_MARGIN * rates[best_hw]:
            return best_hw
    return best


def tune(ctx, precision: int = 0, n_instances: int = 16, traj_scale: float = 1.0 / 4,
         seed: int = 77, use_cache: bool = True, verbose: bool = False) -> dict:
    """Returns {"workers_per_cu": w, "chunk": k, "rates": {...}} for this device and precision."""
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
    for w in WORKERS:
        for k in CHUNKS:
            r = _trial(sfhk, ctx, arrays_list, insts, precision, w, k, torch)
            rates[f"workers={w},chunk={k}"] = r
            if verbose:
                print(f"autotune precision={precision} workers_per_cu={w} chunk={k}: "
                      f"{r:.4e} trajectory-steps/s", flush=True)
    best = choose(rates)
    w, k = (int(v.split("=")[1]) for v in best.split(","))
    res = {"workers_per_cu": w, "chunk": k, "rates": rates}
    cache[key] = res
    try:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return res
