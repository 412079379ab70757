"""Benchmark: FP64 zone-updates/s of the GR-MHD RK2 step on the 256^3 FM torus (one MI355X).

A zone-update is one interior cell advanced one full RK2 step (both stages: ghosts, face fluxes,
CFL step, flux-CT, update with source, inversion, floors, fixups).  Inputs are the seeded
synthetic torus, resident in HBM before the timed region.  The launch-shape autotuner first runs
its candidates on ordinary steps, then W untimed warm-up steps, then exactly K timed steps
replayed from the captured HIP graph (no per-kernel events), bracketed by device synchronisation
and timed with HIP events on the run's stream.  A separate pass of min(K, 20) steps with an event
pair around every kernel gives the per-kernel split and the dominant kernel's duration for its
roofline figure.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic HBM bytes of the method (the state alone, FP64, P-only state): stage 1 reads P^n and
# writes P^{n+1/2} (128 B per cell); stage 2 reads P^{n+1/2} and P^n and writes P^{n+1} (192 B).
# 320 B per zone-update; the update kernel is the one launch per stage that must move them.
ALG_BYTES_STAGE = (128.0, 192.0)
ALG_BYTES_ZU = sum(ALG_BYTES_STAGE)
# Intermediate traffic of this implementation's face kernels (context, not algorithmic): per face
# the 8 primitives of one cell read once per direction and the 7 stored flux slots written.
FACE_BYTES = 120.0
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# committed rocprofv3 counters of the 256^3 workload, per face reconstruction
COUNTERS = {"plm": os.path.join(ROOT, "profiles", "hbm_counters_torus3d_256.json"),
            "ppm": os.path.join(ROOT, "profiles", "hbm_counters_torus3d_256_ppm.json")}
# FP64 operations per zone-update of the method, counted on an op-counting build of the oracle
# (every add/sub/mul/div/sqrt/pow of one RK2 step on the benchmark torus's physics)
FLOP_COUNT = os.path.join(ROOT, "profiles", "oracle_flop_count.json")
FLOP_KEY = "torus3d_256x256x256_physics_at_64cubed"


def oracle_flops_per_zu():
    try:
        with open(FLOP_COUNT) as fh:
            return float(json.load(fh)["per_zone_update"][FLOP_KEY]["total"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("grmhd_dev.h", "grmhd_c2p.h", "grmhd_kernels.hip"):
        with open(os.path.join(ROOT, "paper_2205_02484_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_counters(workload, recon):
    """Per-launch HBM bytes and FP64 FLOP of the committed rocprofv3 passes, or None when the
    kernels have changed since they were taken (source hash) or the workload differs."""
    try:
        with open(COUNTERS[recon]) as fh:
            js = json.load(fh)
    except OSError:
        return None
    if js.get("workload") != workload or js.get("recon", "plm") != recon:
        return None
    if js.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return js["per_launch"]


def units_per_launch(kind, n1, n2, n3, recon="plm"):
    if kind == "flux1":
        return (n1 + 1) * (n2 + 2) * n3
    if kind == "flux2":
        return (n1 + 2) * (n2 + 1) * n3
    if kind == "flux3":
        return (n1 + 2) * (n2 + 2) * n3
    if kind == "update":
        return n1 * n2 * n3
    if kind == "emf":
        return (n1 + 1) * (n2 + 1) * n3
    if kind == "bound":
        g = 3 if recon == "ppm" else 2     # ghost layers a run fills
        return (2 * g * (n2 + 2 * g) + 2 * g * n1) * n3
    return 0


def cpu_baseline(cfg, P, nsteps):
    """The oracle as it stands on the host cores, a bounded sample of the same workload."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    os.environ["OMP_NUM_THREADS"] = str(threads)
    from oracle import oracle as orc
    ocfg = orc.make_cfg(cfg)
    t0 = time.perf_counter()
    orc.step(ocfg, P, nsteps)
    el = time.perf_counter() - t0
    zones = cfg.n1 * cfg.n2 * cfg.n3
    return {"value": zones * nsteps / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{nsteps} RK2 steps of the full {cfg.n1}x{cfg.n2}x{cfg.n3} torus, OpenMP over cells, "
                      f"{el:.1f} s wall"}


def ensemble_legs(args, stream):
    """48 uneven tori batched vs one after another, then a served Poisson stream at 80 % of the
    batched capacity with continuous admission; p50/p99 job latency (arrival -> done)."""
    from paper_2205_02484_amd import serve
    jobs = serve.ensemble_jobs(seed=4, nsteps=args.ensemble_steps)
    from paper_2205_02484_amd.torus_init import make_torus
    inputs = [make_torus(j.cfg) for j in jobs]
    print(f"[bench] ensemble: {len(jobs)} tori x {args.ensemble_steps} steps, batched", file=sys.stderr, flush=True)
    bat = serve.run_batched(jobs, steps_per_launch=25, stream=stream, inputs=inputs, autotune_steps=1)
    print(f"[bench] ensemble batched {bat['zu_per_s']:.3e} ZU/s; sequential", file=sys.stderr, flush=True)
    seq = serve.run_sequential(jobs, stream=stream, inputs=inputs)
    print(f"[bench] ensemble sequential {seq['zu_per_s']:.3e} ZU/s; job latency p50/p99 batched "
          f"{bat['p50_s']:.2f}/{bat['p99_s']:.2f} s, one after another {seq['p50_s']:.2f}/{seq['p99_s']:.2f} s",
          file=sys.stderr, flush=True)
    rate = 0.8 * bat["zu_per_s"] / serve.mean_job_zone_updates(seed=5)
    sjobs = serve.served_jobs(rate_hz=rate, duration_s=args.serve_seconds, seed=5)
    print(f"[bench] served stream: {len(sjobs)} jobs over {args.serve_seconds:.0f} s at {rate:.3f}/s",
          file=sys.stderr, flush=True)
    srv = serve.serve(sjobs, steps_per_launch=20, stream=stream, max_active_cells=args.serve_cap_cells,
                      log=lambda m: print(m, file=sys.stderr, flush=True))
    print(f"[bench] served p50 {srv['p50_s']:.2f} s p99 {srv['p99_s']:.2f} s, {srv['zu_per_s']:.3e} ZU/s",
          file=sys.stderr, flush=True)
    vs_plain = None
    if args.plain_seconds > 0:
        # the first plain_seconds of the same arrivals, served by the batched loop and by the plain
        # baseline (one job at a time, first come first served, the plain stepper)
        def head():
            return [j for j in serve.served_jobs(rate_hz=rate, duration_s=args.serve_seconds, seed=5)
                    if j.arrival < args.plain_seconds]
        hb = serve.serve(head(), steps_per_launch=20, stream=stream, max_active_cells=args.serve_cap_cells)
        print(f"[bench] first {args.plain_seconds:.0f} s of the stream ({hb['jobs']} jobs): batched p50 "
              f"{hb['p50_s']:.2f} s p99 {hb['p99_s']:.2f} s; plain", file=sys.stderr, flush=True)
        hp = serve.serve_plain(head(), stream=stream)
        print(f"[bench] plain p50 {hp['p50_s']:.2f} s p99 {hp['p99_s']:.2f} s, {hp['seconds']:.1f} s",
              file=sys.stderr, flush=True)
        vs_plain = {"arrivals_s": args.plain_seconds, "jobs": hb["jobs"],
                    "batched": {"p50_s": hb["p50_s"], "p99_s": hb["p99_s"], "mean_s": hb["mean_s"],
                                "seconds": hb["seconds"], "zu_per_s": hb["zu_per_s"]},
                    "plain": {"p50_s": hp["p50_s"], "p99_s": hp["p99_s"], "mean_s": hp["mean_s"],
                              "seconds": hp["seconds"], "zu_per_s": hp["zu_per_s"]},
                    "plain_is": "same arrivals, one job at a time in arrival order, plain stepper"}
    return {
        "workload": "48 seeded tori (24 2D 64^2-192^2, 24 3D 48-96 x 48 x 48), spin U[0,0.98], "
                    "gamma {4/3,13/9,5/3}, beta {30,100,300}, r_max U[10,30]",
        "steps_each": args.ensemble_steps,
        "batched_zu_per_s": bat["zu_per_s"], "batched_seconds": bat["seconds"],
        "sequential_zu_per_s": seq["zu_per_s"], "sequential_seconds": seq["seconds"],
        "batched_over_sequential": bat["zu_per_s"] / seq["zu_per_s"],
        "job_latency": {"submitted": "all 48 at t = 0", "batched_p50_s": bat["p50_s"], "batched_p99_s": bat["p99_s"],
                        "sequential_p50_s": seq["p50_s"], "sequential_p99_s": seq["p99_s"]},
        "batched_autotune": bat["autotune"],
        "served": {"duration_s": args.serve_seconds, "rate_hz": rate, "load": 0.8, "jobs": srv["jobs"],
                   "p50_s": srv["p50_s"], "p99_s": srv["p99_s"], "mean_s": srv["mean_s"],
                   "zu_per_s": srv["zu_per_s"], "seconds": srv["seconds"], "passes": srv["passes"],
                   "max_steps_per_pass": 20, "max_active_cells": args.serve_cap_cells,
                   "unfixed_cells": srv["unfixed_cells"],
                   "mix": "2D 128^2 or 3D N^3 (N in [64,160]), 100-2000 steps each"},
        "served_vs_plain": vs_plain,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--autotune-steps", type=int, default=2,
                    help="ordinary steps per candidate launch shape of the autotuner, before the warm-up")
    ap.add_argument("--workload", default="torus3d_256x256x256")
    ap.add_argument("--recon", choices=("plm", "ppm"), default="plm",
                    help="face reconstruction: PLM with the MC limiter (the paper's) or PPM")
    ap.add_argument("--cpu-steps", type=int, default=5, help="oracle steps in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the ensemble and served-stream legs")
    ap.add_argument("--ensemble-steps", type=int, default=500, help="steps of each of the 48 ensemble tori")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="length of the served arrival stream")
    ap.add_argument("--serve-cap-cells", type=int, default=1 << 21,
                    help="served loop: admit a job only while the active jobs hold at most this many cells "
                         "(a larger job runs alone); 0: admit whatever fits the memory budget")
    ap.add_argument("--plain-seconds", type=float, default=10.0,
                    help="arrivals of the stream's head served both batched and by the plain one-at-a-time "
                         "baseline (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size kernel that "
                         "scales the HBM counters of a profiler pass)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2205_02484_amd import grmhd
    from paper_2205_02484_amd.torus_init import make_torus
    from paper_2205_02484_amd.workloads import WORKLOADS

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    grmhd.load()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    cfg = WORKLOADS[args.workload]()
    cfg.recon = args.recon
    P = make_torus(cfg)
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    zones = n1 * n2 * n3
    stream = torch.cuda.Stream()
    ctx = grmhd.Context(cfg, P, stream=stream)
    print(f"[bench] {args.workload}: {zones} zones, warmup {args.warmup}", file=sys.stderr, flush=True)
    # the launch-shape autotuner runs its candidates on ordinary steps before the warm-up (its
    # steps advance the run like any other and are not timed)
    tuned = ctx.autotune(args.autotune_steps) if args.autotune_steps > 0 else ""
    ctx.steps(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.steps(args.steps)                  # graph replays: the product path, no per-kernel events
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t, nstep, nfail = ctx.get_time()
    ms_per_step = ms / args.steps
    value = zones * args.steps / (ms * 1e-3)
    print(f"[bench] {ms_per_step:.3f} ms/step, {value:.3e} ZU/s, t={t:.4f}, failures={nfail}",
          file=sys.stderr, flush=True)
    # per-kernel split: a separate pass with an event pair around every kernel (plain launches)
    nsplit = min(args.steps, 20)
    ctx.kernel_timing(True)
    ctx.steps(nsplit)
    kt = ctx.kernel_times()
    ctx.kernel_timing(False)
    torch.cuda.synchronize()
    split_ms = sum(v[0] * v[1] for v in kt.values()) / max(nsplit, 1)

    # dominant kernel: the update (flux-CT, update with source, inversion, floors), which is the
    # launch per stage that must move the method's state bytes
    tot = {k: v[0] * v[1] for k, v in kt.items()}
    dom = "update"
    avg_ms = kt[dom][0]
    alg_launch = 0.5 * (ALG_BYTES_STAGE[0] + ALG_BYTES_STAGE[1]) * zones   # both stages' launches averaged
    achieved = alg_launch / (avg_ms * 1e-3) / 1e9
    prof = profiled_counters(args.workload, args.recon)
    traffic = None
    if prof and dom in prof:
        traffic = prof[dom]["hbm_read_bytes"] + prof[dom]["hbm_write_bytes"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom, "avg_ms": avg_ms,
                "alg_bytes_per_unit": list(ALG_BYTES_STAGE), "unit_name": "cell (stage 1, stage 2)",
                "units_per_launch": zones, "alg_bytes_per_launch": alg_launch}
    # whole step against the method's own bytes and FP64 operations
    flops_zu = oracle_flops_per_zu()
    t_bytes = ALG_BYTES_ZU * zones / (HBM_PEAK_GBS * 1e9) * 1e3
    t_flops = flops_zu * zones / (FP64_PEAK_TFLOPS * 1e12) * 1e3 if flops_zu else None
    t_roof = max(t_bytes, t_flops or 0.0)
    step_roof = {"alg_bytes_per_zu": ALG_BYTES_ZU, "alg_fp64_ops_per_zu": flops_zu,
                 "t_bytes_ms": t_bytes, "t_fp64_ms": t_flops, "t_roofline_ms": t_roof,
                 "bound": "fp64" if (t_flops or 0.0) > t_bytes else "hbm",
                 "frac": t_roof / ms_per_step,
                 "hbm_frac_alg_bytes": ALG_BYTES_ZU * zones / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    if prof:
        # measured HBM and FP64 rates of every stage kernel at the live durations (context)
        roofline["per_kernel_measured"] = {
            k: {"hbm_GBs": (v["hbm_read_bytes"] + v["hbm_write_bytes"]) / (kt[k][0] * 1e-3) / 1e9,
                "fp64_TFLOPs": v["fp64_flop"] / (kt[k][0] * 1e-3) / 1e12,
                "fp64_frac": v["fp64_flop"] / (kt[k][0] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}
            for k, v in prof.items() if k in kt and kt[k][0] > 0}
        per_step = sum((v["hbm_read_bytes"] + v["hbm_write_bytes"]) * kt[k][1] / max(nsplit, 1)
                       for k, v in prof.items() if k in kt)
        step_roof["traffic_per_step"] = per_step
        step_roof["traffic_over_alg"] = per_step / (ALG_BYTES_ZU * zones)
    kernels = {k: {"avg_ms": v[0], "launches": v[1], "share": tot[k] / max(sum(tot.values()), 1e-30)}
               for k, v in kt.items()}

    out = {
        "metric": "FP64 zone-updates/s (256^3 torus) + ensemble p50/p99 latency vs plain",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Fishbone-Moncrief torus, 4% u perturbation, beta_0 = 100)",
        "config": {"workload": args.workload, "grid": [n1, n2, n3], "zones": zones, "spin": cfg.spin,
                   "gamma": cfg.gam, "r_out": cfg.r_out, "r_in_torus": cfg.r_in, "r_max": cfg.r_max,
                   "cfl": cfg.cfl, "riemann": "llf", "recon": args.recon},
        "roofline": roofline,
        "step_roofline": step_roof,
        "kernels": kernels,
        "kernel_split": {"steps": nsplit, "ms_per_step_with_events": split_ms},
        "autotune": {"steps": 5 * args.autotune_steps,
                     "chosen": [ln for ln in (tuned or "").splitlines() if ln.startswith("chosen")]},
        "sim_time": t,
        "unfixed_cells": nfail,
    }
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if not args.no_ensemble:
        out["ensemble"] = ensemble_legs(args, stream)
    if not args.no_cpu_baseline:
        print(f"[bench] CPU baseline: oracle, {args.cpu_steps} step(s)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, P, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
