#!/usr/bin/env python3
"""Benchmark of the FISH split-MHD step on one MI355X.

Default workload: a 256^3 periodic box of the random-Fourier initialiser
(rms Mach 1, plasma beta 1, wave numbers |k| <= 16, gamma 5/3, CFL 0.5),
20 symmetric Strang steps (each: the device CFL reduction plus the twelve
sub-operators, advancing 2 dt) timed in segments of 5 that each start from
the initial state, since the box loses positivity after 6 steps (the FP64
oracle as well: the scheme has no floors), FP32 storage with FP64 pressure recovery as
the headline value and FP64 beside it.  Inputs are resident in HBM before the
timed region starts.

Prints ONE JSON line on stdout (progress goes to stderr):
  metric/value/unit  cell-updates per second (cells x Strang steps / wall s)
  roofline           dominant kernel (the fluid sweep) vs the 8 TB/s HBM peak,
                     its average launch time measured with hipEvents recorded
                     around each of its launches inside the timed region
  cpu_baseline       the FP64 CPU oracle on a bounded sample of the same box
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s per Strang step (FP32 vs FP64) + % HBM roofline; p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for fn in ("physics.h", "sweeps.h"):
        with open(os.path.join(ROOT, "paper_0910_2854_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(name, esize, cells):
    """HBM bytes per launch of the fluid sweep from the committed counter run,
    or None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except Exception:
        return None
    if rec.get("kernel_hash") != kernel_source_hash() or rec.get("cells") != cells or rec.get("esize") != esize:
        return None
    return rec.get("bytes_per_launch")


def run_gpu(fish, torch, st, n, precision, steps, warmup, cfl, segment):
    """Time `steps` Strang steps (dt from the device CFL step) in segments of at
    most `segment` steps, each started from the initial state: the state is
    re-uploaded and synchronised before a segment's clock starts and checked
    after it stops, so every timed step advances a physically valid state."""
    box = fish.Box(*n, precision=precision, cfl=cfl)
    box.set_state(st)
    for _ in range(warmup):
        box.strang_step(0.0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    box.timing_enable(fish.KERNEL_FLUID, max_launches=8 * steps)
    wall = 0.0
    step_ms = []
    ok = True
    done = 0
    while done < steps:
        k = min(segment, steps - done)
        box.set_state(st)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for s in range(k):
            box.strang_step(0.0)
            ev[s + 1].record(stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        step_ms += [ev[s].elapsed_time(ev[s + 1]) for s in range(k)]
        try:
            box.cfl_dt()
        except fish.FishError:
            ok = False
        done += k
    launches, fluid_ms = box.timing_read()
    box.close()
    return {"wall": wall, "step_ms": sorted(step_ms), "fluid_launches": launches, "fluid_ms": fluid_ms,
            "state_ok": ok}


def pct(sorted_vals, q):
    if not sorted_vals:
        return None
    k = min(len(sorted_vals) - 1, max(0, int(math.ceil(q / 100.0 * len(sorted_vals))) - 1))
    return sorted_vals[k]


def cpu_baseline(st, n, cfl, steps):
    from oracle import Oracle

    cores = len(os.sched_getaffinity(0))
    o = Oracle(*n, cfl=cfl, nthreads=cores)
    o.set_state(st)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.strang_step(0.0)
    dt = time.perf_counter() - t0
    ncell = n[0] * n[1] * n[2]
    return {"value": ncell * steps / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} Strang step(s) of the same {n[0]}x{n[1]}x{n[2]} box from the same initial state, "
                      f"FP64, {cores} OpenMP threads ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--segment", type=int, default=5,
                    help="timed steps per segment before the initial state is restored (the 256^3 Mach 1, beta 1 "
                         "box loses positivity after 6 steps, in the oracle as well)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(boxes are independent; a multi-GPU slab decomposition is a design note, not a run)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_probe} MiB x3")
        return

    import fish_inputs as fi
    import paper_0910_2854_amd as fish

    fish.load_library()
    n = (args.n,) * 3
    ncell = n[0] * n[1] * n[2]
    cfl = 0.5
    log(f"generating {n} random-Fourier state (Mach 1, beta 1, k<=16)")
    t0 = time.perf_counter()
    st = fi.random_fourier_state(n, seed=0, mach=1.0, beta=1.0, kmax=16)
    log(f"  {time.perf_counter() - t0:.1f} s")

    res = {}
    for prec in ("fp32",) + (() if args.no_fp64 else ("fp64",)):
        log(f"GPU {prec}: {args.warmup} warmup + {args.steps} timed steps")
        res[prec] = run_gpu(fish, torch, st, n, prec, args.steps, args.warmup, cfl, args.segment)
        r = res[prec]
        log(f"  {r['wall'] * 1e3 / args.steps:.3f} ms/step, fluid launch avg "
            f"{r['fluid_ms'] / max(1, r['fluid_launches']):.3f} ms, state_ok={r['state_ok']}")

    r = res["fp32"]
    value = ncell * args.steps / r["wall"]
    esize = 4
    fluid_avg_s = r["fluid_ms"] / max(1, r["fluid_launches"]) * 1e-3
    bytes_fluid = ncell * 13 * esize  # reads rho, m, E and the three face fields; writes rho, m, E
    achieved = bytes_fluid / fluid_avg_s / 1e9
    traffic = load_traffic("fluid_sweep_traffic_256.json", esize, ncell)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n[0]}^3 periodic box, random-Fourier initialiser (rms Mach 1, beta 1, |k|<=16, seed 0), "
                        "gamma 5/3, CFL 0.5, symmetric Strang steps with the device CFL step",
            "segments": f"{args.steps} timed steps in segments of at most {args.segment}, each from the initial state "
                        "(this box loses positivity after 6 steps, the FP64 oracle included; there are no floors)",
            "precision": "FP32 storage and arithmetic, FP64 pressure recovery / CFL reduction",
            "cells": ncell,
            "limiter": "van Leer",
        },
        "latency_ms": {"p50": pct(r["step_ms"], 50), "p99": pct(r["step_ms"], 99)},
        "step_roofline": {"bytes_per_cell": 384, "achieved_GBs": value * 384 / 1e9, "peak_GBs": HBM_PEAK_GBS,
                          "frac": value * 384 / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fluid_sweep_kernel (L_x, L_y, L_z)",
                     "avg_launch_ms": fluid_avg_s * 1e3, "launches": r["fluid_launches"],
                     "algorithmic_bytes_per_launch": bytes_fluid},
        "state_ok": r["state_ok"],
    }
    if "fp64" in res:
        r64 = res["fp64"]
        v64 = ncell * args.steps / r64["wall"]
        out["fp64"] = {"value": v64, "ms_per_step": r64["wall"] * 1e3 / args.steps,
                       "latency_ms": {"p50": pct(r64["step_ms"], 50), "p99": pct(r64["step_ms"], 99)},
                       "step_roofline_frac": v64 * 768 / 1e9 / HBM_PEAK_GBS,
                       "fluid_avg_launch_ms": r64["fluid_ms"] / max(1, r64["fluid_launches"]),
                       "state_ok": r64["state_ok"]}
    if not args.no_cpu:
        log(f"CPU oracle baseline: {args.cpu_steps} step(s)")
        out["cpu_baseline"] = cpu_baseline(st, n, cfl, args.cpu_steps)
        log(f"  {out['cpu_baseline']['value']:.3e} cell-updates/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
