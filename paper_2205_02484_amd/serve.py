"""Ensemble stepping and a continuously-batched request loop over the C ABI's grmhd_batch_*.

Jobs are torus runs of different grids, spins, adiabatic indices and field strengths -- the kind
of parameter scan the paper runs over beta_0, disk size and gamma (Sec. 5, Table 1).  Each admitted
job's state stays resident in HBM; all active jobs advance together (one launch per stage kernel
for the whole ensemble, each job with its own CFL step) until they have taken their requested
number of steps.  New jobs are admitted whenever their memory footprint fits, while others run.

This module only orchestrates: every step of the method runs in libgrmhd.so.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import grmhd
from .torus_init import TorusConfig, fm_torus_2d, make_torus


@dataclasses.dataclass
class Job:
    jid: int
    cfg: TorusConfig
    nsteps: int
    arrival: float = 0.0          # seconds after the stream starts
    admitted: Optional[float] = None
    done: Optional[float] = None
    handle: Optional[int] = None
    horizon: Optional[Dict[str, float]] = None   # accretion diagnostics at completion (serve(diagnose=True))
    unfixed: Optional[int] = None                # cells the fixups left unfixed over the run (serve())

    @property
    def zone_updates(self) -> int:
        return self.cfg.zones * self.nsteps


def _torus_exists(cfg: TorusConfig) -> bool:
    ii, jj = np.meshgrid(np.arange(cfg.n1), np.arange(cfg.n2), indexing="ij")
    return bool(fm_torus_2d(cfg, ii, jj)[4].any())


def _random_physics(rng, n1, n2, n3, seed) -> TorusConfig:
    """Spin U[0, 0.98], gamma in {4/3, 13/9, 5/3}, beta_0 in {30, 100, 300}, r_max U[10, 30],
    r_in = r_max/2 (moved out by 0.5 M until a torus exists on the grid), r_out = 1000."""
    spin = float(rng.uniform(0.0, 0.98))
    gam = float(rng.choice([4.0 / 3.0, 13.0 / 9.0, 5.0 / 3.0]))
    beta = float(rng.choice([30.0, 100.0, 300.0]))
    r_max = float(rng.uniform(10.0, 30.0))
    r_in = r_max / 2.0
    cfg = None
    while r_in < r_max:
        cfg = TorusConfig(n1=n1, n2=n2, n3=n3, spin=spin, gam=gam, beta=beta, r_max=r_max, r_in=r_in,
                          r_out=1000.0, delta=0.04, seed=seed, cfl=0.45)
        if _torus_exists(cfg):
            return cfg
        r_in += 0.5
    raise RuntimeError("no torus for this draw")


def ensemble_jobs(seed: int = 4, n2d: int = 24, n3d: int = 24, nsteps: int = 500) -> List[Job]:
    """The uneven 48-torus ensemble: half 2D N x N with N in {64..192}, half 3D N1 x 48 x 48 with
    N1 in {48..96}, physics drawn as in _random_physics."""
    rng = np.random.default_rng(seed)
    jobs = []
    for x in range(n2d + n3d):
        if x < n2d:
            n = int(rng.integers(64, 193))
            cfg = _random_physics(rng, n, n, 1, seed * 1000 + x)
        else:
            n1 = int(rng.integers(48, 97))
            cfg = _random_physics(rng, n1, 48, 48, seed * 1000 + x)
        jobs.append(Job(jid=x, cfg=cfg, nsteps=nsteps))
    return jobs


def served_jobs(rate_hz: float, duration_s: float, seed: int = 5) -> List[Job]:
    """Poisson arrivals over `duration_s`: 2D 128^2 or 3D N^3 (N in [64, 160]) tori requesting
    100..2000 steps, physics as in _random_physics."""
    rng = np.random.default_rng(seed)
    jobs, t, x = [], 0.0, 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        if rng.random() < 0.5:
            cfg = _random_physics(rng, 128, 128, 1, seed * 100000 + x)
        else:
            n = int(rng.integers(64, 161))
            cfg = _random_physics(rng, n, n, n, seed * 100000 + x)
        jobs.append(Job(jid=x, cfg=cfg, nsteps=int(rng.integers(100, 2001)), arrival=t))
        x += 1
    return jobs


def mean_job_zone_updates(seed: int = 5, samples: int = 4000) -> float:
    """E[zones x steps] of the served job mix (sizes and step counts only)."""
    rng = np.random.default_rng(seed + 12345)
    tot = 0.0
    for _ in range(samples):
        if rng.random() < 0.5:
            z = 128 * 128
        else:
            z = int(rng.integers(64, 161)) ** 3
        tot += z * float(rng.integers(100, 2001))
    return tot / samples


def _latency(done: List[float]) -> Dict[str, float]:
    d = np.array(done)
    return {"p50_s": float(np.percentile(d, 50)), "p99_s": float(np.percentile(d, 99))} if len(d) else {}


def run_sequential(jobs: List[Job], stream=None, inputs: Optional[List[np.ndarray]] = None) -> Dict[str, float]:
    """Each job alone with the plain stepper (one context at a time).  Every job counts as
    submitted at the start; its latency is the time until its run has finished."""
    import torch
    if inputs is None:
        inputs = [make_torus(j.cfg) for j in jobs]
    t0 = time.perf_counter()
    zu = 0
    done = []
    for j, P in zip(jobs, inputs):
        ctx = grmhd.Context(j.cfg, P, stream=stream)
        ctx.steps(j.nsteps)
        ctx.get_time()                       # waits for the run
        ctx.close()
        zu += j.zone_updates
        done.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"seconds": el, "zone_updates": zu, "zu_per_s": zu / el, **_latency(done)}


def run_batched(jobs: List[Job], steps_per_launch: int = 25, stream=None,
                keep: Optional[Callable[[Job, np.ndarray], None]] = None,
                inputs: Optional[List[np.ndarray]] = None, autotune_steps: int = 0) -> Dict[str, float]:
    """All jobs resident together, advanced in one kernel chain until each is done (latency: from the
    start, when every job is submitted, until it is retired).  With
    autotune_steps > 0 the launch-shape autotuner first runs that many ordinary steps per candidate
    shape on the whole ensemble (they count towards each job's steps and are timed with the rest)."""
    b = grmhd.Batch(stream=stream)
    if inputs is None:
        inputs = [make_torus(j.cfg) for j in jobs]
    t0 = time.perf_counter()
    by_handle = {}
    for j, P in zip(jobs, inputs):
        h = b.admit(j.cfg, P, j.nsteps)
        if h is None:
            raise RuntimeError("ensemble does not fit the device memory budget")
        j.handle = h
        by_handle[h] = j
    left = len(jobs)
    zu = 0
    done = []
    tuned = b.autotune(autotune_steps) if autotune_steps > 0 else ""
    while left:
        b.advance(steps_per_launch)
        for h in b.poll():
            j = by_handle[h]
            if keep is not None:
                keep(j, b.fetch(h)[0])
            b.release(h)
            zu += j.zone_updates
            left -= 1
            done.append(time.perf_counter() - t0)
    el = time.perf_counter() - t0
    b.close()
    return {"seconds": el, "zone_updates": zu, "zu_per_s": zu / el, **_latency(done),
            "autotune": [ln for ln in tuned.splitlines() if ln.startswith("chosen")]}


def serve(jobs: List[Job], steps_per_launch: int = 20, budget_bytes: int = 0, stream=None,
          log: Optional[Callable[[str], None]] = None, batch=None,
          make_input: Callable[[TorusConfig], np.ndarray] = make_torus,
          clock: Callable[[], float] = time.perf_counter,
          sleep: Callable[[float], None] = time.sleep,
          max_active_cells: int = 0, diagnose: bool = False) -> Dict[str, float]:
    """Replay an arrival stream in real time with continuous batching.

    Arrived jobs wait in a FIFO queue; every pass admits, in order, each queued job whose
    footprint fits the remaining budget (smaller jobs may pass a large head), advances all active
    jobs, and retires finished ones (fetch + release).  With max_active_cells > 0 a job is also
    admitted only while the active jobs' cells stay within that many (a job larger than the cap
    runs when none is active): the active set is kept near what fills the chip, so large jobs run
    close to alone in arrival order instead of sharing the GPU with every arrival, and small ones
    still batch.  A pass lasts as many steps as the active
    job closest to completion still needs, at most `steps_per_launch`: a job is retired at the end
    of the pass in which it takes its last step, never a partial pass later.  Latency is arrival ->
    finished on the host.  Each finished job's count of cells left unfixed is kept in
    `Job.unfixed`, the served stream's numerical-failure report.  With `diagnose`, each finished
    job's horizon diagnostics (Sec. 4.2: Mdot,
    phi_B, Ldot, Edot, the MAD parameter) are taken on the device before its slot is released and
    kept in `Job.horizon`.  `batch`, `make_input`, `clock` and `sleep` can be replaced (host-side
    tests of the scheduling logic)."""
    b = batch if batch is not None else grmhd.Batch(budget_bytes=budget_bytes, stream=stream)
    time_now = clock
    pending = sorted(jobs, key=lambda j: j.arrival)
    inputs: Dict[int, np.ndarray] = {}
    queue: List[Job] = []
    active: Dict[int, Job] = {}
    left: Dict[int, int] = {}          # steps each active job still takes
    finished: List[Job] = []
    passes = 0
    t0 = time_now()
    nxt = 0
    zu = 0
    last_log = t0
    while nxt < len(pending) or queue or active:
        now = time_now() - t0
        while nxt < len(pending) and pending[nxt].arrival <= now:
            j = pending[nxt]
            inputs[j.jid] = make_input(j.cfg)
            queue.append(j)
            nxt += 1
        still = []
        cells = sum(a.cfg.zones for a in active.values())
        for j in queue:
            if max_active_cells > 0 and active and cells + j.cfg.zones > max_active_cells:
                still.append(j)
                continue
            h = b.admit(j.cfg, inputs[j.jid], j.nsteps)
            if h is None:
                still.append(j)
                continue
            j.handle = h
            j.admitted = time_now() - t0
            active[h] = j
            left[h] = j.nsteps
            cells += j.cfg.zones
            del inputs[j.jid]
        queue = still
        if active:
            nstep = max(1, min(steps_per_launch, min(left.values())))
            b.advance(nstep)
            passes += 1
            for h in left:
                left[h] = max(0, left[h] - nstep)
            for h in b.poll():
                j = active.pop(h)
                left.pop(h, None)
                b.fetch(h)
                j.unfixed = b.get_time(h)[2]
                if diagnose:
                    j.horizon = b.diag_full(h)[0]
                b.release(h)
                j.done = time_now() - t0
                zu += j.zone_updates
                finished.append(j)
        elif nxt < len(pending):
            sleep(max(0.0, min(0.05, pending[nxt].arrival - (time_now() - t0))))
        elif queue:
            raise RuntimeError(f"job {queue[0].jid} can never fit the memory budget")
        if log is not None and time_now() - last_log > 30.0:
            last_log = time_now()
            log(f"[serve] t={last_log - t0:.0f}s done={len(finished)} active={len(active)} queued={len(queue)}")
    el = time_now() - t0
    if batch is None:
        b.close()
    lat = np.array([j.done - j.arrival for j in finished])
    return {"jobs": len(finished), "seconds": el, "zone_updates": zu, "zu_per_s": zu / el, "passes": passes,
            "unfixed_cells": int(sum(j.unfixed or 0 for j in finished)),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_s": float(lat.mean()) if len(lat) else math.nan}


def _run_one_plain(job: Job, P: np.ndarray, stream=None) -> None:
    ctx = grmhd.Context(job.cfg, P, stream=stream)
    ctx.steps(job.nsteps)
    ctx.get_prims()                          # the result back on the host, as serve() fetches it
    ctx.close()


def serve_plain(jobs: List[Job], stream=None,
                make_input: Callable[[TorusConfig], np.ndarray] = make_torus,
                run_one: Optional[Callable[[Job, np.ndarray], None]] = None,
                clock: Callable[[], float] = time.perf_counter,
                sleep: Callable[[float], None] = time.sleep) -> Dict[str, float]:
    """The plain baseline for serve(): the same arrival stream in real time, one job at a time
    in arrival order, each run to completion alone with the plain stepper (no batching, no
    overlap).  Latency is arrival -> finished on the host, as in serve().  `run_one`, `clock` and
    `sleep` can be replaced (host-side tests)."""
    if run_one is None:
        def run_one(j, P):
            _run_one_plain(j, P, stream)
    pending = sorted(jobs, key=lambda j: j.arrival)
    t0 = clock()
    zu = 0
    lat = []
    for j in pending:
        wait = j.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        P = make_input(j.cfg)
        run_one(j, P)
        j.done = clock() - t0
        lat.append(j.done - j.arrival)
        zu += j.zone_updates
    el = clock() - t0
    lat = np.array(lat)
    return {"jobs": len(lat), "seconds": el, "zone_updates": zu, "zu_per_s": zu / el if el > 0 else math.nan,
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_s": float(lat.mean()) if len(lat) else math.nan}

