"""Continuous-batching serving loop for spectrum requests.

Requests (one SFHK instance each) arrive at given times. Between graph replays of one batch,
arrived requests are admitted in arrival order while their device footprint fits the context's
HBM budget and the batch's capacity; admitted requests keep their trajectory state in HBM and
every replay advances all of them by `chunk` steps (one launch per precision and potential kind
over all their tiles, longest first). A request that has finished gets its dipole and spectrum
computed on the device and copied to pinned host memory; its latency runs from arrival to the
moment the loop sees that copy complete.

The loop is pipelined: replays, dipoles and spectra run on one compute stream, uploads and job
creation on an admission stream, and nothing waits for the replay in flight. Staging the next
replay's table waits only for the replay before it (the batch keeps two staging sets), finished
requests are collected by polling events, and destroyed jobs return their memory in stream order.
Results are identical to each request propagated alone (the batch path is bitwise equal to it).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Request:
    req_id: int
    arrival: float          # seconds after the start of the run
    inst: object            # inputs.Instance


@dataclass
class Result:
    req_id: int
    arrival: float
    admitted: float
    finished: float
    n_traj: int
    steps: int
    omega: Optional[np.ndarray] = None
    power: Optional[np.ndarray] = None
    dipole: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _create_job(ctx, inst, precision, stream):
    """The request's job on `stream`; a request that carries SFA birth samples (``meta`` holds
    k_perp and the Monte-Carlo weights) gets its initial conditions from the SFA birth step on
    the device first (sfhk_sfa_birth), in the same stream."""
    import torch
    from paper_2601_17164_amd import sfhk
    if "kperp" not in inst.meta:
        return sfhk.make_job(ctx, inst, precision=precision, stream=stream)
    dev = sfhk.to_device(inst, f"cuda:{ctx.device}")
    f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev["t0"].device)
    b = sfhk.sfa_birth(inst.pulse, inst.ground, dev["t0"], f64(inst.meta["kperp"]),
                       f64(inst.meta["u"]), inst.meta.get("mode", sfhk.SFHK_BIRTH_GTO), stream)
    dev.update(q0=b["q0"], p0=b["p0"], w=b["w"])
    return sfhk.make_job(ctx, inst, dev_arrays=dev, precision=precision, stream=stream)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))


@dataclass
class _Active:
    req: Request
    job: object
    admitted: float


@dataclass
class _Finishing:
    req: Request
    job: object
    admitted: float
    event: object
    omega: object
    power: object
    dipole: object


class Server:
    def __init__(self, ctx, precision: int = 0, chunk: int = 1024, workers_per_cu: int = 0,
                 max_jobs: int = 64, max_tiles: int = 1 << 20, keep_results: bool = False):
        from . import sfhk
        self.sfhk = sfhk
        self.ctx = ctx
        self.precision = precision
        self.keep = keep_results
        self.max_jobs, self.max_tiles = max_jobs, max_tiles
        self.batch = sfhk.Batch(ctx, max_jobs, max_tiles, chunk, workers_per_cu)
        # occupancy of the last run: replays issued, requests in the batch and waiting for
        # admission (sampled at each replay)
        self.stats = {}

    def close(self):
        self.batch.close()

    def run(self, requests: List[Request]) -> List[Result]:
        import torch
        sfhk = self.sfhk
        dev = torch.device(f"cuda:{self.ctx.device}")
        comp = torch.cuda.Stream(dev)   # replays, dipoles, spectra, copies to the host
        adm = torch.cuda.Stream(dev)    # uploads and job creation
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque = deque()
        active: List[_Active] = []
        finishing: List[_Finishing] = []
        results: List[Result] = []
        tiles_active = 0
        replays, active_sum, active_max, queued_max = 0, 0, 0, 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0

        def collect(f: _Finishing):
            st = f.job.stats(adm)  # the counters were final when the event completed
            results.append(Result(f.req.req_id, f.req.arrival, f.admitted, now(),
                                  f.req.inst.n_traj, st.steps_evaluated,
                                  None if f.omega is None else f.omega.numpy(),
                                  f.power.numpy() if self.keep else None,
                                  None if f.dipole is None else f.dipole.numpy()))
            f.job.close()

        while pending or queue or active or finishing:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            # finished requests whose spectrum has reached host memory
            still = []
            for f in finishing:
                if f.event.query():
                    collect(f)
                else:
                    still.append(f)
            finishing = still
            # admission, in arrival order, by HBM footprint and batch capacity
            while queue and len(active) < self.max_jobs:
                req = queue[0]
                nt = sfhk.tiles_of(req.inst)
                if nt > self.max_tiles:
                    raise ValueError(f"request {req.req_id} has more tiles than the batch holds")
                if tiles_active + nt > self.max_tiles:
                    break
                try:
                    with torch.cuda.stream(adm):
                        job = _create_job(self.ctx, req.inst, self.precision, adm)
                except sfhk.SfhkError as e:
                    if e.status == sfhk.SFHK_E_BUDGET and (active or finishing):
                        break  # wait for running requests to free HBM
                    raise      # does not fit even on an idle device
                queue.popleft()
                active.append(_Active(req, job, now()))
                tiles_active += nt
            if active:
                # waits only for the replay before the one in flight
                self.batch.set_jobs([a.job for a in active], stream=comp)
                self.batch.run(stream=comp)
                replays += 1
                active_sum += len(active)
                active_max = max(active_max, len(active))
                queued_max = max(queued_max, len(queue))
                still = []
                with torch.cuda.stream(comp):
                    for a in active:
                        if not a.job.done:
                            still.append(a)
                            continue
                        d = a.job.dipole(stream=comp)
                        inst = a.req.inst
                        T = inst.grid.h * inst.grid.n_steps
                        dt = T / inst.n_out if inst.n_out else inst.grid.h
                        om, pw, _ = sfhk.spectrum(d, inst.grid.t_a, dt, T / 2, stream=comp)
                        host_pw = torch.empty(pw.shape, dtype=pw.dtype, pin_memory=True)
                        host_pw.copy_(pw, non_blocking=True)
                        host_om = host_d = None
                        if self.keep:
                            host_om = torch.empty(om.shape, dtype=om.dtype, pin_memory=True)
                            host_om.copy_(om, non_blocking=True)
                            host_d = torch.empty(d.shape, dtype=d.dtype, pin_memory=True)
                            host_d.copy_(d, non_blocking=True)
                        ev = torch.cuda.Event()
                        ev.record(comp)
                        finishing.append(_Finishing(a.req, a.job, a.admitted, ev, host_om,
                                                    host_pw, host_d))
                        tiles_active -= sfhk.tiles_of(inst)
                active = still
            elif finishing:
                finishing[0].event.synchronize()
            elif queue:
                comp.synchronize()  # admission waits for memory held by finished requests
            elif pending:
                time.sleep(max(0.0, min(0.05, pending[0].arrival - now())))
        comp.synchronize()
        self.stats = {"replays": replays, "mean_active": active_sum / max(1, replays),
                      "max_active": active_max, "max_queued": queued_max}
        return sorted(results, key=lambda r: r.req_id)


def summarize(results: List[Result], wall: float = None) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    steps = sum(r.steps for r in results)
    span = wall if wall is not None else (max(r.finished for r in results) -
                                          min(r.arrival for r in results))
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "trajectory_steps_per_s": steps / span, "span_s": span}
