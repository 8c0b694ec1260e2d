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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles
# at 2.4 GHz, i.e. 3.93e13 lane-instructions/s (no packed FP32 here)
VALU_PEAK_LANE_INSTS = 256 * 4 * 64 / 4 * 2.4e9
LIMITERS = {"minmod": 0, "vanleer": 1, "switch": 2}
METRIC = "cell-updates/s per Strang step (FP32 vs FP64) + % HBM roofline; p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources' code: line comments, trailing blanks and
    empty lines are dropped, so that a comment edit keeps the counters valid
    while any change to the code invalidates them."""
    h = hashlib.sha256()
    for fn in ("physics.h", "sweeps.h"):
        with open(os.path.join(ROOT, "paper_0910_2854_amd", "csrc", fn), "rb") as f:
            lines = []
            for line in f.read().decode().splitlines():
                code = line.split("//", 1)[0].rstrip()
                if code.strip():
                    lines.append(code)
            h.update("\n".join(lines).encode())
    return h.hexdigest()[:16]


def load_counters(name, esize, cells):
    """(HBM bytes, VALU wave instructions) per launch of the fluid sweep from
    the committed counter runs, or (None, None) if the kernel source changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, None
    try:
        with open(path) as f:
            rec = json.load(f)
    except Exception:
        return None, None
    if rec.get("kernel_hash") != kernel_source_hash() or rec.get("cells") != cells or rec.get("esize") != esize:
        return None, None
    return rec.get("bytes_per_launch"), rec.get("valu_wave_insts_per_launch")


def stretched_widths(n, amp, phase):
    """Cell widths of an irregular mesh (Sect. 2.5) on [0, 1]: proportional to
    1 + amp sin(2 pi x + phase), normalised to sum to 1."""
    xi = (np.arange(n) + 0.5) / n
    w = 1.0 + amp * np.sin(2 * np.pi * xi + phase)
    return w / w.sum()


def run_gpu(fish, torch, st, n, precision, steps, warmup, cfl, segment, autotune=True, limiter=1, stretch=0.0,
            x_strided=0):
    """Time `steps` Strang steps (dt from the device CFL step) in segments of at
    most `segment` steps, each started from the initial state: the state is
    re-uploaded and synchronised before a segment's clock starts and checked
    after it stops, so every timed step advances a physically valid state.

    The same steps then run a second time with the launch-timing hook on (a
    hipEvent on the library's stream before and after every fluid launch)
    for the fluid sweep's average launch time.  The hook's event records add
    a gap of several microseconds at each recorded launch boundary, so the
    headline steps run without it."""
    box = fish.Box(*n, precision=precision, cfl=cfl, limiter=limiter)
    if stretch:
        for a in range(3):
            box.set_spacing(a, stretched_widths(n[a], stretch, float(a)))
    box.set_state(st)
    tuned = box.autotune(reps=5) if autotune else None
    if x_strided:
        # the measured alternative to the lanes policy for the x fluid sweep
        box.set_shape("fluid_x", x_strided, 1, 1)
        if tuned:
            tuned["fluid_x"] = {"target": x_strided, "xcd_remap": 1, "alt_layout": 1}
    for _ in range(warmup):
        box.strang_step(0.0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def segments():
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
        return wall, step_ms, ok

    wall, step_ms, ok = segments()
    box.timing_enable(fish.KERNEL_FLUID, max_launches=8 * steps)
    wall_hooked, _, ok2 = segments()
    launches, fluid_ms = box.timing_read()
    box.timing_enable(0)
    box.close()
    return {"wall": wall, "step_ms": sorted(step_ms), "fluid_launches": launches, "fluid_ms": fluid_ms,
            "state_ok": ok and ok2, "tuned": tuned, "wall_hooked": wall_hooked}


def pct(sorted_vals, q):
    if not sorted_vals:
        return None
    k = min(len(sorted_vals) - 1, max(0, int(math.ceil(q / 100.0 * len(sorted_vals))) - 1))
    return sorted_vals[k]


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy rate in GB/s (bytes read + bytes written): the
    measured stream peak, reported beside the nominal 8 TB/s."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / sec / 1e9


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(st, n, cfl, steps, threads, **kw):
    from oracle import Oracle

    o = Oracle(*n, cfl=cfl, nthreads=threads, **kw)
    o.set_state(st)
    t0 = time.perf_counter()
    for _ in range(steps):
        o.strang_step(0.0)
    dt = time.perf_counter() - t0
    o.close()
    return n[0] * n[1] * n[2] * steps / dt, dt


def cpu_baseline(st, n, cfl, steps, per_core_state=None, **kw):
    """The oracle on the host's cores; with per_core_state = (state, shape,
    steps), also one thread on that sample for a per-core figure."""
    cores = len(os.sched_getaffinity(0))
    rate, dt = _oracle_rate(st, n, cfl, steps, cores, **kw)
    out = {"value": rate, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} Strang step(s) of the same {n[0]}x{n[1]}x{n[2]} box from the same initial state, "
                     f"FP64, {cores} OpenMP threads ({dt:.1f} s)",
           "cpu_model": _cpu_model()}
    if per_core_state is not None:
        st1, n1, steps1 = per_core_state
        rate1, dt1 = _oracle_rate(st1, n1, cfl, steps1, 1, **kw)
        out["per_core"] = {"value": rate1, "unit": "cell-updates/s",
                           "sample": f"{steps1} Strang step(s) of a {n1[0]}x{n1[1]}x{n1[2]} box, FP64, "
                                     f"1 thread ({dt1:.1f} s)"}
    return out


def _gen_states(fi, jobs, workers):
    """Generate states in order with a thread pool (numpy releases the GIL in
    its array loops); yields (job, state) lazily, at most 2 x workers ahead."""
    from concurrent.futures import ThreadPoolExecutor

    def make(job):
        return fi.random_fourier_state(job["n"], seed=job["seed"], mach=job["mach"], beta=job["beta"],
                                       kmax=job["kmax"])

    with ThreadPoolExecutor(max_workers=workers) as ex:
        pending = []
        it = iter(jobs)
        for job in it:
            pending.append((job, ex.submit(make, job)))
            if len(pending) >= 2 * workers:
                break
        while pending:
            job, fut = pending.pop(0)
            nxt = next(it, None)
            if nxt is not None:
                pending.append((nxt, ex.submit(make, nxt)))
            yield job, fut.result()


def bench_batch(args, torch, fish, fi):
    """2048 periodic boxes, edges uniform over {16,24,32,48,64}, Mach U[0.3,2],
    beta log-uniform [0.5,50], |k| <= 4, FP32, autotuned work shapes, one
    graph-captured double step replayed per step; against the same boxes
    stepped one at a time through single-box contexts."""
    specs = fi.batch_box_specs(args.boxes)
    jobs = [{"n": (s["edge"],) * 3, "seed": s["seed"], "mach": s["mach"], "beta": s["beta"], "kmax": 4, "spec": s}
            for s in specs]
    pool = sum(fish.box_pool_bytes(j["n"], "fp32") for j in jobs) + (64 << 20)
    cells = sum(j["n"][0] ** 3 for j in jobs)
    log(f"batch: {len(jobs)} boxes, {cells} cells, pool {pool / 2**30:.2f} GiB")
    stream = torch.cuda.Stream()  # the batch's stream (default priority); events are recorded on it
    b = fish.Batch(pool, max_boxes=len(jobs), precision="fp32", stream=stream.cuda_stream)
    t0 = time.perf_counter()
    ids = []
    for job, st in _gen_states(fi, jobs, args.workers):
        ids.append(b.add(st))
    log(f"  generated and uploaded in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    tuned = b.autotune(reps=3)
    log(f"  autotune {time.perf_counter() - t0:.1f} s: {tuned}")

    def timed(graph, steps, warmup):
        b.use_graph(graph)
        b.step(warmup)
        b.sync()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(steps):
            b.step(1)
            ev[k + 1].record(stream)
        b.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))

    b.use_graph(True)
    b.step(args.warmup)
    b.sync()
    taken0 = [b.steps_taken(i) for i in ids]
    wall_g, ms_g = timed(True, args.steps, 0)
    # the work each box did in the timed steps: double steps with dt > 0 (a
    # box whose state went bad stops with dt = 0 but stays in the launches)
    taken = [b.steps_taken(i) - t0_ for i, t0_ in zip(ids, taken0)]
    valid_updates = sum(j["n"][0] ** 3 * k for j, k in zip(jobs, taken))
    log(f"  graph: {wall_g * 1e3 / args.steps:.3f} ms/step, {valid_updates / wall_g:.3e} valid cell-updates/s")
    wall_e, ms_e = timed(False, args.steps, 0)
    log(f"  eager: {wall_e * 1e3 / args.steps:.3f} ms/step")
    # the fluid sweep's launch time: further eager steps with a hipEvent around
    # every fluid launch (kept out of the timed steps: the records add gaps)
    hooked = max(2, args.steps // 10)
    b.timing_enable(fish.KERNEL_FLUID, 8 * hooked)
    b.step(hooked)
    b.sync()
    launches, fluid_ms = b.timing_read()
    b.timing_enable(0)
    fluid_avg_s = fluid_ms / max(1, launches) * 1e-3
    valid = sum(0 if b.info(i)["bad"] else 1 for i in ids)
    valid_cells = sum(j["n"][0] ** 3 for j, i in zip(jobs, ids) if not b.info(i)["bad"])
    b.close()
    # the plain single-box path: a stratified sample of the same boxes, one
    # context each, stepped one box at a time
    per_edge = {}
    sample = []
    for j in jobs:
        e = j["n"][0]
        if per_edge.get(e, 0) < args.single_sample:
            per_edge[e] = per_edge.get(e, 0) + 1
            sample.append(j)
    sc = 0
    st_time = 0.0
    for job, st in _gen_states(fi, sample, args.workers) if sample else ():
        g = fish.Box(*job["n"], precision="fp32")
        g.set_state(st)
        g.strang_step(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.strang_step(0.0)
        torch.cuda.synchronize()
        st_time += time.perf_counter() - t0
        sc += job["n"][0] ** 3 * args.steps
        g.close()
    single_rate = sc / st_time if st_time else None
    value = valid_updates / wall_g
    raw = cells * args.steps / wall_g
    bytes_fluid = cells * 13 * 4
    traffic, _ = load_counters("fluid_sweep_traffic_batch.json", 4, cells)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_g * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(jobs)} periodic boxes, edges uniform over {{16,24,32,48,64}}, "
                               "random-Fourier initialiser per box (Mach U[0.3,2], beta log-uniform [0.5,50], |k|<=4), "
                               "gamma 5/3, CFL 0.5, per-box CFL step, FP32 with FP64 pressure recovery",
                   "cells": cells, "boxes": len(jobs), "autotuned": tuned,
                   "value_counts": "cell-updates of boxes whose state is valid: each box's cells times the double "
                                   "steps it took with dt > 0 in the timed steps"},
        "latency_ms": {"p50": pct(ms_g, 50), "p99": pct(ms_g, 99)},
        "step_roofline": {"bytes_per_cell": 384, "achieved_GBs": value * 384 / 1e9, "peak_GBs": HBM_PEAK_GBS,
                          "frac": value * 384 / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "achieved": bytes_fluid / fluid_avg_s / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": bytes_fluid / fluid_avg_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fluid sweep class over the whole batch (fluid_lanes_kernel, fluid_strided_kernel), "
                               "every box in each launch",
                     "avg_launch_ms": fluid_avg_s * 1e3, "launches": launches,
                     "timed_with": f"{hooked} further eager double steps with a hipEvent around every fluid launch",
                     "algorithmic_bytes_per_launch": bytes_fluid},
        "all_boxes_rate": {"value": raw, "note": "every box's cells times every timed step, including boxes that "
                                                 "stopped on a bad state (their launches still run)"},
        "eager": {"value": cells * args.steps / wall_e, "ms_per_step": wall_e * 1e3 / args.steps},
        "single_box_path": {"value": single_rate, "boxes_sampled": len(sample),
                            "note": "same boxes, one single-box context each, stepped one box at a time"},
        "speedup_vs_single_box": raw / single_rate if single_rate else None,
        "boxes_valid_at_end": valid,
        "valid_cell_fraction": valid_cells / cells,
        "valid_work_fraction": valid_updates / (cells * args.steps),
        "note": "a box whose state fails the check (the scheme has no floors) stops with dt = 0 but stays "
                "in every launch, so the timed work per step is constant; value counts only the valid boxes' "
                "steps, all_boxes_rate every box's",
    }
    if not args.no_cpu:
        # the oracle on 16 boxes of each edge, one double step each
        from oracle import Oracle

        cores = len(os.sched_getaffinity(0))
        per_edge = {}
        csample = []
        for j in jobs:
            e = j["n"][0]
            if per_edge.get(e, 0) < 16:
                per_edge[e] = per_edge.get(e, 0) + 1
                csample.append(j)
        log(f"CPU oracle baseline: one step of {len(csample)} boxes")
        ccells, ctime = 0, 0.0
        for job, st in _gen_states(fi, csample, args.workers):
            o = Oracle(*job["n"], cfl=0.5, nthreads=cores)
            o.set_state(st)
            t0 = time.perf_counter()
            o.strang_step(0.0)
            ctime += time.perf_counter() - t0
            ccells += job["n"][0] ** 3
            o.close()
        out["cpu_baseline"] = {"value": ccells / ctime, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
                               "sample": f"one double step of {len(csample)} of the boxes (16 per edge), FP64, "
                                         f"{cores} OpenMP threads ({ctime:.1f} s)",
                               "cpu_model": _cpu_model()}
        log(f"  {out['cpu_baseline']['value']:.3e} cell-updates/s")
    print(json.dumps(out), flush=True)


def bench_serve(args, torch, fish, fi):
    """Poisson arrivals of periodic boxes (edge log-uniform in [32,192],
    10-200 double steps, Mach 0.5, beta 10 random-Fourier state per request
    seed), FP32, admission capped by the pool size; p50/p99 latency beside
    aggregate cell-updates/s per arrival rate."""
    pool = int(args.serve_pool_gb * 2**30)

    def jobs_for(reqs):
        return [{"n": (r["edge"],) * 3, "seed": r["seed"], "mach": 0.5, "beta": 10.0, "kmax": 4, "req": r}
                for r in reqs]

    def run(reqs, rate_label, saturate=False):
        srv = fish.Server(pool, chunk_steps=args.chunk, max_boxes=4096, precision="fp32")
        srv.use_graph(True)
        # every request's state exists before the clock starts (host
        # generation is not part of serving)
        gen = iter(list(_gen_states(fi, jobs_for(reqs), args.workers)))
        t_start = time.perf_counter()
        arrival = {}
        complete = {}
        work = {}
        bad = set()
        cell_steps = 0
        pending = None
        n_sub = 0
        while len(complete) < len(reqs):
            now = time.perf_counter() - t_start
            # submit every request that has arrived (and whose state is ready)
            while n_sub < len(reqs):
                if pending is None:
                    pending = next(gen)
                job, st = pending
                r = job["req"]
                if not saturate and r["arrival"] > now:
                    break
                srv.submit(n_sub, st, r["steps"])
                arrival[n_sub] = 0.0 if saturate else r["arrival"]
                work[n_sub] = r["edge"] ** 3 * r["steps"]
                cell_steps += work[n_sub]
                n_sub += 1
                pending = None
            done = srv.pump()
            tnow = time.perf_counter() - t_start
            for tag, status, _ in done:
                complete[tag] = tnow
                if status != fish.FISH_OK:
                    bad.add(tag)
            s = srv.stats()
            if not done and s["resident"] == 0 and s["queued"] == 0 and n_sub < len(reqs):
                nxt = reqs[n_sub]["arrival"] - (time.perf_counter() - t_start)
                if nxt > 0:
                    time.sleep(min(nxt, 0.05))
        wall = time.perf_counter() - t_start
        srv.close()
        lat = sorted((complete[k] - arrival[k]) * 1e3 for k in complete if k >= args.serve_skip)
        # a request whose state went bad is not credited (no floors: its box
        # stops with dt = 0); every request counts in the latency figures
        valid = sum(w for t, w in work.items() if t not in bad)
        return {"rate_label": rate_label, "requests": len(reqs), "wall_s": wall,
                "cell_updates_per_s": valid / wall, "requests_bad_state": len(bad),
                "all_requests_cell_updates_per_s": cell_steps / wall, "requests_per_s": len(reqs) / wall,
                "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)}}

    # saturated throughput mu (requests/s) on this mix: everything queued at t = 0
    sat_reqs = fi.serving_requests(args.serve_sat, rate=1.0, seed=7)
    sat = run(sat_reqs, "saturated", saturate=True)
    mu = sat["requests_per_s"]
    log(f"serve: saturated {mu:.2f} req/s, {sat['cell_updates_per_s']:.3e} cell-updates/s")
    # the plain single-box path on the same saturated mix: one request at a time
    t0 = time.perf_counter()
    sc = 0
    for job, st in _gen_states(fi, jobs_for(sat_reqs), args.workers):
        r = job["req"]
        g = fish.Box(*job["n"], precision="fp32")
        g.set_state(st)
        for _ in range(r["steps"]):
            g.strang_step(0.0)
        g.get_state(check=False)
        g.close()
        sc += r["edge"] ** 3 * r["steps"]
    single = {"cell_updates_per_s": sc / (time.perf_counter() - t0),
              "requests_per_s": len(sat_reqs) / (time.perf_counter() - t0)}
    log(f"serve: single-box path {single['requests_per_s']:.2f} req/s")
    rates = []
    for f in args.serve_rates:
        reqs = fi.serving_requests(args.serve_requests, rate=f * mu, seed=7)
        res = run(reqs, f"{f} x mu")
        res["rate_req_per_s"] = f * mu
        log(f"serve: rate {f} mu: p50 {res['latency_ms']['p50']:.0f} ms p99 {res['latency_ms']['p99']:.0f} ms, "
            f"{res['cell_updates_per_s']:.3e} cell-updates/s")
        rates.append(res)
    best = max(rates, key=lambda r: r["cell_updates_per_s"])
    out = {
        "metric": METRIC, "value": sat["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, periodic boxes of edge log-uniform in [32,192], "
                               "10-200 double steps, random-Fourier state per request (Mach 0.5, beta 10, |k|<=4), "
                               f"FP32, pool {args.serve_pool_gb} GB, chunk {args.chunk} steps",
                   "requests_per_rate": args.serve_requests, "excluded_warm": args.serve_skip},
        "saturated": sat, "mu_req_per_s": mu, "single_box_path": single,
        "speedup_vs_single_box": sat["cell_updates_per_s"] / single["cell_updates_per_s"],
        "rates": rates, "latency_ms": best["latency_ms"],
    }
    print(json.dumps(out), flush=True)


def bench_sphere(args, torch, fish, fi):
    """512^3 stratified sphere: outflow on every face, unsplit gravity and HSE
    subtraction, FP32 with FP64 pressure recovery, autotuned work shapes,
    --steps double steps (20 by default)."""
    n = (args.n if args.n != 256 else 512,) * 3
    ncell = n[0] * n[1] * n[2]
    log(f"sphere {n}: generating")
    t0 = time.perf_counter()
    st = fi.sphere_state(n, seed=0)
    log(f"  {time.perf_counter() - t0:.1f} s")
    box = fish.Box(*n, precision="fp32", bc=(fish.OUTFLOW,) * 3, gravity=args.gravity, hse=True, cfl=0.5)
    box.set_state(st)
    if args.no_cpu:
        del st
    tuned = box.autotune(reps=3) if not args.no_autotune else None
    log(f"  autotuned: {tuned}")
    for _ in range(args.warmup):
        box.strang_step(0.0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        box.strang_step(0.0)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the fluid sweep's launch time: further steps with a hipEvent around every
    # fluid launch (kept out of the headline steps: the event records add gaps)
    hooked = max(2, args.steps // 10)
    box.timing_enable(fish.KERNEL_FLUID, max_launches=8 * hooked)
    for k in range(hooked):
        box.strang_step(0.0)
    launches, fluid_ms = box.timing_read()
    box.timing_enable(0)
    ok = True
    try:
        box.cfl_dt()
    except fish.FishError:
        ok = False
    box.close()
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps))
    value = ncell * args.steps / wall
    fluid_avg_s = fluid_ms / max(1, launches) * 1e-3
    bytes_fluid = ncell * 14 * 4  # the fluid sweep also reads phi
    # the counters were taken on the unsplit-gravity kernels at 512^3
    traffic = (load_counters("fluid_sweep_traffic_512_sphere.json", 4, ncell)[0] if args.gravity == "unsplit"
               else None)
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n[0]}^3 stratified sphere rho = 1/(1+(r/0.1)^2) with 1% noise, matching potential "
                               f"and hydrostatic pressure, beta 100, outflow boundaries, {args.gravity} gravity + HSE, "
                               "gamma 5/3, CFL 0.5, FP32 with FP64 pressure recovery", "cells": ncell,
                   "autotuned": tuned},
        "latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99)},
        "step_roofline": {"bytes_per_cell": 408, "achieved_GBs": value * 408 / 1e9, "peak_GBs": HBM_PEAK_GBS,
                          "frac": value * 408 / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "achieved": bytes_fluid / fluid_avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_fluid / fluid_avg_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fluid sweep class with gravity + HSE (fluid_lanes_kernel, fluid_strided_kernel)",
                     "avg_launch_ms": fluid_avg_s * 1e3, "launches": launches,
                     "timed_with": f"{hooked} further double steps with a hipEvent around every fluid launch",
                     "algorithmic_bytes_per_launch": bytes_fluid},
        "state_ok": ok,
    }
    if not args.no_cpu:
        log("CPU oracle baseline: the first double step of the same box")
        out["cpu_baseline"] = cpu_baseline(st, n, 0.5, 1, bc=(fish.OUTFLOW,) * 3, gravity=args.gravity, hse=True)
        out["cpu_baseline"]["sample"] += " (a prefix of the 50-step run)"
        log(f"  {out['cpu_baseline']['value']:.3e} cell-updates/s")
    print(json.dumps(out), flush=True)


PROBLEMS = (
    ("sedov", "Sedov-Taylor blast 256^3 (Sect. 4.2), until the shock reaches r = 0.45"),
    ("spherical_riemann", "spherical Riemann problem 256^3 (Sect. 4.3), t = 0.09"),
    ("magnetic_explosion", "magnetic explosion 256^3 (Sect. 4.4), minmod, t = 0.03"),
    ("rotor", "rotor 256^2 (Sect. 4.5), t = 0.15"),
    ("mhd_riemann_2d", "2-D MHD Riemann problem 512^2 (Sect. 4.6), t = 0.8"),
)


def _problem_state(fi, name):
    if name == "sedov":
        st, s = fi.sedov_state(256)
        h = s["h"][0]
        eb = (float(st["cell"][4].sum()) - 1e-3 * st["cell"][4].size) * h ** 3
        s["t_end"] = (0.45 / 1.152) ** 2.5 / math.sqrt(eb)  # similarity law R = 1.152 (E t^2/rho)^(1/5)
        return st, s
    return {"spherical_riemann": fi.spherical_riemann_state, "magnetic_explosion": fi.magnetic_explosion_state,
            "rotor": fi.rotor_state, "mhd_riemann_2d": fi.mhd_riemann_2d_state}[name]()


def bench_problems(args, torch, fish, fi):
    """The validation problems of Sect. 4.2-4.6 at the paper's sizes, FP32,
    each run to its end time from a state resident on the GPU with
    fish_advance_to: the device takes the CFL step of every double step and
    shortens the last one to land on the end time, and the steps replay as a
    captured graph on the bench's stream (the explosion, whose fluid launches
    are timed for the roofline, runs them eagerly)."""
    total_cells, total_wall, total_steps, per, roof = 0, 0.0, 0, {}, None
    stream = torch.cuda.Stream()
    for name, desc in PROBLEMS:
        st, s = _problem_state(fi, name)
        h = s["h"]
        box = fish.Box(*s["shape"], dx=h[0], dy=h[1], dz=h[2], gamma=s["gamma"], cfl=s["cfl"], limiter=s["limiter"],
                       bc=s["bc"], precision="fp32", stream=stream.cuda_stream)
        box.set_state(st)
        ncell = s["shape"][0] * s["shape"][1] * s["shape"][2]
        log(f"{name}: {s['shape']} to t = {s['t_end']:.4f}")
        timed = name == "magnetic_explosion"
        if timed:
            box.timing_enable(fish.KERNEL_FLUID, max_launches=6 * 400)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, t = box.advance_to(s["t_end"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if timed:
            launches, fluid_ms = box.timing_read()
            avg_s = fluid_ms / max(1, launches) * 1e-3
            b = ncell * 13 * 4
            roof = {"bound": "hbm", "achieved": b / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": b / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "fluid sweep (L_x, L_y, L_z), magnetic explosion 256^3, minmod",
                    "avg_launch_ms": avg_s * 1e3, "launches": launches, "algorithmic_bytes_per_launch": b}
        x = box.get_state()
        box.close()
        c = x["cell"]
        ke = 0.5 * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0]
        bc = fi.cell_centred_b(x["bx"], x["by"], x["bz"])
        me = 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)
        p = (s["gamma"] - 1.0) * (c[4] - ke - me)
        per[name] = {"problem": desc, "cells": ncell, "steps": k, "wall_s": wall,
                     "value": ncell * k / wall, "ms_per_step": wall * 1e3 / k,
                     "ranges": {"rho": [float(c[0].min()), float(c[0].max())], "p": [float(p.min()), float(p.max())],
                                "e_mag": [float(me.min()), float(me.max())], "e_kin": [float(ke.min()), float(ke.max())]}}
        log(f"  {k} steps, {wall:.2f} s, {ncell * k / wall:.3e} cell-updates/s")
        total_cells += ncell * k
        total_wall += wall
        total_steps += k
        del st, x
    out = {
        "metric": METRIC, "value": total_cells / total_wall, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": total_steps, "warmup": 0, "ms_per_step": total_wall * 1e3 / total_steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "the validation problems of Sect. 4.2-4.6 at the paper's sizes, each from its "
                               "initial state to its end time with fish_advance_to (device CFL steps, the "
                               "last one clamped to the end time, graph replays), FP32 with FP64 pressure "
                               "recovery", "problems": per},
        "roofline": roof,
    }
    if not args.no_cpu:
        st, s = _problem_state(fi, "magnetic_explosion")
        log(f"CPU oracle baseline: {args.cpu_steps} step(s) of the magnetic explosion")
        out["cpu_baseline"] = cpu_baseline(st, s["shape"], s["cfl"], args.cpu_steps, limiter=s["limiter"], bc=s["bc"])
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ counter summaries
# The rocprofv3 counter passes each workload's committed summary comes from
# (REPO = the repository root, OUT = the output directory; each pass is its own run).
PMC_PASSES = (
    ("rd", "TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum"),
    ("wr", "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_HIT_sum TCC_MISS_sum"),
    ("sq1", "SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES "
            "SQ_ACTIVE_INST_VALU GRBM_GUI_ACTIVE"),
    ("sq2", "SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_INST_CYCLES_VMEM_RD SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU_TRANS_F32 "
            "SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_MUL_F32 GRBM_GUI_ACTIVE"),
)
PROFILED = {
    # workload: (summary tag, bench arguments of the profiled run, description, fluid bytes per cell)
    "box": ("256", "--no-cpu --no-fp64 --steps 2 --warmup 0 --segment 2",
            "256^3 FP32 random-Fourier box (Mach 1, beta 1, |k|<=16), van Leer, autotuned shapes", 13 * 4),
    "sphere": ("512_sphere", "--workload sphere --no-cpu --steps 2 --warmup 0",
               "512^3 FP32 stratified sphere, outflow, unsplit gravity + HSE, autotuned shapes", 14 * 4),
    "batch": ("batch", "--workload batch --no-cpu --steps 2 --warmup 0 --single-sample 0",
              "batch of 2048 FP32 boxes (edges 16-64), autotuned shapes, the eager double steps", 13 * 4),
}
COPY_PROBE = "--copy-probe 1024"
TRACED = {
    # tag: (bench arguments of the traced run, description, double steps summarised, later steps skipped)
    "256": ("--no-cpu --no-fp64 --steps 5 --warmup 1 --segment 5",
            "256^3 periodic random-Fourier box (Mach 1, beta 1, |k|<=16), van Leer, CFL 0.5, FP32 with FP64 pressure "
            "recovery, autotuned work shapes; the 5 headline double steps (the bench then repeats them with its "
            "launch-timing hook, which is not in these figures)", 5, 5),
    "256_fp64": ("--no-cpu --steps 5 --warmup 1 --segment 5",
                 "the same box in FP64 (the second half of the same run), autotuned work shapes; its 5 headline double "
                 "steps", 5, 5),
    "256_x_strided": ("--no-cpu --no-fp64 --steps 5 --warmup 1 --segment 5 --x-strided 128",
                      "the same FP32 box with the x fluid sweep on the strided policy (lanes along y, segments of 128, "
                      "XCD-grouped blocks) instead of the lanes policy, the CFL speed then from the check kernel; the "
                      "5 headline double steps", 5, 5),
    "512_sphere": ("--workload sphere --no-cpu --steps 5 --warmup 1",
                   "512^3 stratified sphere, outflow, unsplit gravity + HSE, FP32 with FP64 pressure recovery, "
                   "autotuned shapes; the 5 headline double steps (2 hooked steps follow)", 5, 2),
    "batch": ("--workload batch --no-cpu --steps 5 --warmup 1 --single-sample 0",
              "batch of 2048 periodic FP32 boxes (edges 16-64), autotuned shapes; the 5 timed double steps, replays "
              "of the captured graph (5 eager and 2 hooked steps follow)", 5, 7),
}


def _pmc_dispatches(path, nsteps):
    """Counter values per dispatch of the last nsteps double steps (from the
    nsteps-th last begin_step_kernel on) of one rocprofv3 --pmc csv."""
    import csv
    import collections

    disp = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            d = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"], "c": {},
                                                        "t": (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))})
            d["c"][r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(disp)
    starts = [i for i in ids if "begin_step_kernel" in disp[i]["name"]]
    return [disp[i] for i in ids if i >= starts[-nsteps]]


def _fetch_bytes(a):
    return 32 * a.get("TCC_EA0_RDREQ_32B_sum", 0) + 64 * a.get("TCC_EA0_RDREQ_64B_sum", 0) + \
        128 * a.get("TCC_EA0_RDREQ_128B_sum", 0)


def _write_bytes(a):
    return 64 * a.get("TCC_EA0_WRREQ_64B_sum", 0) + 32 * (a.get("TCC_EA0_WRREQ_sum", 0) -
                                                           a.get("TCC_EA0_WRREQ_64B_sum", 0))


def summarize_counters(workload, outdir, cells, nsteps=2):
    """Write profiles/fluid_sweep_traffic_<tag>.json and profiles/counters_<tag>.txt
    from the counter passes of PMC_PASSES in outdir/pmc_<tag>_<pass> (and the
    copy probe in outdir/pmccopy_rd, outdir/pmccopy_wr when present).  HBM
    bytes are the L2's read and write requests weighted by their size."""
    import collections

    tag, bargs, desc, fluid_bpc = PROFILED[workload]
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    cnt = collections.Counter()
    dur = collections.defaultdict(float)
    for sub, _ in PMC_PASSES:
        path = os.path.join(outdir, f"pmc_{tag}_{sub}", "run_counter_collection.csv")
        if not os.path.exists(path):
            continue
        for d in _pmc_dispatches(path, nsteps):
            n = d["name"].split("(")[0].replace("void ", "")
            if sub == "rd":
                cnt[n] += 1
            if sub == "sq1":
                dur[n] += (d["t"][1] - d["t"][0]) / 1e3
            for k, v in d["c"].items():
                agg[n][k] += v
    calib = None
    crd, cwr = os.path.join(outdir, "pmccopy_rd", "run_counter_collection.csv"), \
        os.path.join(outdir, "pmccopy_wr", "run_counter_collection.csv")
    if os.path.exists(crd) and os.path.exists(cwr):
        import csv

        c = collections.defaultdict(float)
        for path in (crd, cwr):
            with open(path) as f:
                for r in csv.DictReader(f):
                    if "copyBuffer" in r["Kernel_Name"]:
                        c[r["Counter_Name"]] += float(r["Counter_Value"])
        calib = {"probe": f"bench.py {COPY_PROBE}: three 1 GiB device-to-device copies",
                 "read_GiB_per_copy": _fetch_bytes(c) / 3 / 2 ** 30, "write_GiB_per_copy": _write_bytes(c) / 3 / 2 ** 30}
    ran = [(sub, c) for sub, c in PMC_PASSES
           if os.path.exists(os.path.join(outdir, f"pmc_{tag}_{sub}", "run_counter_collection.csv"))]
    cmds = ["cd /tmp && export TMPDIR=/tmp"] + [
        f"rocprofv3 --pmc {c} --output-format csv -d $OUT/pmc_{tag}_{sub} -o run -- "
        f"python3 $REPO/bench.py {bargs}" for sub, c in ran] + [
        f"rocprofv3 --pmc {PMC_PASSES[i][1]} --output-format csv -d $OUT/pmccopy_{PMC_PASSES[i][0]} -o run "
        f"-- python3 $REPO/bench.py {COPY_PROBE}" for i in (0, 1)] + [
        f"python3 $REPO/bench.py --summarize {workload} --counters-dir $OUT"]
    fluid = [n for n in cnt if "fluid_" in n]
    nl = sum(cnt[n] for n in fluid)
    tot_f = sum(_fetch_bytes(agg[n]) for n in fluid)
    tot_w = sum(_write_bytes(agg[n]) for n in fluid)
    algo = fluid_bpc * cells
    rec = {
        "kernel": f"fluid sweep class, {desc}: the launches of the last {nsteps} double steps of the profiled run",
        "kernel_hash": kernel_source_hash(), "cells": cells, "esize": 4,
        "bytes_per_launch": (tot_f + tot_w) / nl, "fetch_bytes_per_launch": tot_f / nl,
        "write_bytes_per_launch": tot_w / nl, "algorithmic_bytes_per_launch": algo,
        "traffic_over_algorithmic": (tot_f + tot_w) / nl / algo,
        "byte_counts": "HBM reads as the L2's read requests by size (32 x TCC_EA0_RDREQ_32B + 64 x TCC_EA0_RDREQ_64B "
                       "+ 128 x TCC_EA0_RDREQ_128B), writes as 64 x TCC_EA0_WRREQ_64B + 32 x the other write "
                       "requests; no calibration factor (the copy probe checks the counting)",
        "calibration_check": calib, "launches": nl,
        "per_kernel": [{"kernel": n, "dispatches": cnt[n], "fetch_bytes": _fetch_bytes(agg[n]) / cnt[n],
                        "write_bytes": _write_bytes(agg[n]) / cnt[n]} for n in fluid],
        "commands": cmds,
        "valu_wave_insts_per_launch": (sum(agg[n].get("SQ_INSTS_VALU", 0) for n in fluid) / nl) or None,
    }
    with open(os.path.join(ROOT, "profiles", f"fluid_sweep_traffic_{tag}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"Counters per launch of every sweep kernel: {desc}; the last {nsteps} double steps of each counter run",
             "(dispatches from the matching begin_step_kernel on).  HBM bytes from the L2's read and write requests",
             "by size" + (f" (a 1 GiB device copy reads {calib['read_GiB_per_copy']:.3f} GiB and writes "
                          f"{calib['write_GiB_per_copy']:.3f} GiB per copy in the same counting)" if calib else "") +
             ".  VALU busy: the kernel's VALU wave-instructions at one per 4 cycles per SIMD (1024 SIMDs, 2.4 GHz)",
             "over its duration in the sq1 pass.", "",
             "commands (REPO = the repository root, OUT = the directory the runs write to):"] + \
        ["  " + c for c in cmds] + ["", f"{'kernel':58s} {'n':>3s} {'dur us':>7s} {'fetch MB':>9s} {'write MB':>9s} "
                                        f"{'algo MB':>8s} {'x algo':>6s} {'TB/s':>5s} {'VALU/cell':>9s} "
                                        f"{'INT32/cell':>10s} {'VALU busy':>9s}"]
    for n in sorted(cnt, key=lambda n: -agg[n].get("SQ_INSTS_VALU", 0)):
        kind = "fluid" if "fluid_" in n else ("field" if "field_" in n else ("check" if "check_" in n else None))
        if kind is None:
            continue
        a, k = agg[n], cnt[n]
        d = dur[n] / k if dur[n] else 0.0
        f, w = _fetch_bytes(a) / k, _write_bytes(a) / k
        al = {"fluid": fluid_bpc, "field": 8 * 4, "check": 8 * 4}[kind] * cells
        valu = a.get("SQ_INSTS_VALU", 0)
        int32 = (f"{a['SQ_INSTS_VALU_INT32'] * 64 / k / cells:10.1f}" if "SQ_INSTS_VALU_INT32" in a
                 else f"{'n/a':>10s}")
        lines.append(f"{n.replace('fish::', '')[:58]:58s} {k:3d} {d:7.1f} {f / 1e6:9.1f} {w / 1e6:9.1f} {al / 1e6:8.1f} "
                     f"{(f + w) / al:6.2f} {((f + w) / d / 1e6) if d else 0:5.2f} {valu * 64 / k / cells:9.1f} "
                     f"{int32} {(valu / k * 4 / 1024 / (d * 1e-6 * 2.4e9)) if d else 0:9.2f}")
    with open(os.path.join(ROOT, "profiles", f"counters_{tag}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[-12:]))
    print(json.dumps({k: rec[k] for k in ("bytes_per_launch", "traffic_over_algorithmic", "launches")}))


def summarize_trace(tag, outdir):
    """Write profiles/kernels_<tag>.txt from the rocprofv3 kernel trace in
    outdir/pk_<tag>: per kernel the calls, average, minimum and maximum
    duration over the summarised double steps."""
    import csv
    import collections

    bargs, desc, nsteps, skip = TRACED[tag]
    with open(os.path.join(outdir, f"pk_{tag}", "run_kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "begin_step_kernel" in r["Kernel_Name"]]
    lo = starts[-(skip + nsteps)]
    hi = starts[-skip] if skip else len(rows)
    # not the next segment's state upload and its check
    nxt = [i for i in range(lo, hi) if "set_scalars_kernel" in rows[i]["Kernel_Name"] or
           "copyBuffer" in rows[i]["Kernel_Name"]]
    win = rows[lo:nxt[0] if nxt else hi]
    agg = collections.OrderedDict()
    for r in win:
        n = r["Kernel_Name"].split("(")[0].replace("void ", "")
        agg.setdefault(n, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in agg.values())
    span = (int(win[-1]["End_Timestamp"]) - int(win[0]["Start_Timestamp"])) / 1e3
    lines = ["rocprofv3 kernel statistics: " + desc + ".", "",
             "command (REPO = the repository root, OUT = the directory the run writes to):",
             "  cd /tmp && export TMPDIR=/tmp",
             f"  rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/pk_{tag} -o run -- "
             f"python3 $REPO/bench.py {bargs}",
             f"  python3 $REPO/bench.py --summarize-trace {tag} --counters-dir $OUT", "",
             f"{'kernel':66s} {'calls':>5s} {'avg us':>8s} {'min us':>8s} {'max us':>8s} {'%':>6s}"]
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{n[:66]:66s} {len(v):5d} {sum(v) / len(v):8.1f} {min(v):8.1f} {max(v):8.1f} "
                     f"{100 * sum(v) / tot:6.2f}")
    fl = [d for n, v in agg.items() if "fluid_" in n for d in v]
    lines += ["", f"fluid sweep class: {len(fl)} launches, average {sum(fl) / max(1, len(fl)):.1f} us",
              f"sum of kernel time per double step: {tot / nsteps:.1f} us; first dispatch to last, per double step: "
              f"{span / nsteps:.1f} us", "",
              "Template arguments: fluid_lanes_kernel<T, GRAV, HSE, LIM, CFL, NU> (x sweep, DPP lane streaming; CFL = "
              "the last L_x of a step with the fused CFL reduction); fluid_strided_kernel<T, D, GRAV, HSE, LIM, NU> "
              "(y, z sweeps, and the x sweep on the strided policy); field_lanes_kernel<T, LIM, NU> (B_x); "
              "field_strided_kernel<T, D, LIM, NU> (B_y, B_z)."]
    with open(os.path.join(ROOT, "profiles", f"kernels_{tag}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[7:]))


def batch_cells(nboxes=2048):
    import fish_inputs as fi

    return sum(s["edge"] ** 3 for s in fi.batch_box_specs(nboxes))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default work shapes")
    ap.add_argument("--segment", type=int, default=5,
                    help="timed steps per segment before the initial state is restored (the 256^3 Mach 1, beta 1 "
                         "box loses positivity after 6 steps, in the oracle as well)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    ap.add_argument("--workload", choices=("box", "batch", "serve", "sphere", "problems"), default="box",
                    help="box: the 256^3 box (default); batch: 2048 boxes of uneven size; serve: request loop; "
                         "sphere: 512^3 sphere with gravity + HSE; problems: the validation problems of Sect. 4.2-4.6")
    ap.add_argument("--limiter", choices=tuple(LIMITERS), default="vanleer",
                    help="box workload: van Leer (default), minmod, or the Mach switch of Sect. 2.2")
    ap.add_argument("--gravity", choices=("unsplit", "split"), default="unsplit",
                    help="sphere workload: unsplit source (default) or split kicks, Sect. 2.3")
    ap.add_argument("--stretch", type=float, default=0.0,
                    help="box workload on an irregular mesh: widths 1 + STRETCH sin(2 pi x + axis) (Sect. 2.5)")
    ap.add_argument("--x-strided", type=int, default=0, metavar="SEG",
                    help="box workload: run the x fluid sweep with the strided policy (lanes along y, segments "
                         "of SEG cells) instead of the lanes policy, to measure that alternative")
    ap.add_argument("--boxes", type=int, default=2048)
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--single-sample", type=int, default=8, help="boxes per size for the single-box comparison")
    ap.add_argument("--serve-pool-gb", type=float, default=200.0)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-skip", type=int, default=20)
    ap.add_argument("--serve-sat", type=int, default=48)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[0.25, 0.5, 0.75, 1.0, 1.25])
    ap.add_argument("--chunk", type=int, default=5)
    ap.add_argument("--summarize", choices=tuple(PROFILED), default=None,
                    help="no run: write the committed counter summary of a workload from its rocprofv3 passes")
    ap.add_argument("--summarize-trace", choices=tuple(TRACED), default=None,
                    help="no run: write the committed kernel-trace summary of a traced run")
    ap.add_argument("--counters-dir", default=os.path.join(ROOT, "rocprof_out"),
                    help="the directory the rocprofv3 runs of --summarize / --summarize-trace wrote to")
    args = ap.parse_args()
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace, args.counters_dir)
    if args.summarize:
        cells = {"box": args.n ** 3, "sphere": 512 ** 3, "batch": batch_cells(args.boxes)}[args.summarize]
        return summarize_counters(args.summarize, args.counters_dir, cells)
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
    if args.workload == "batch":
        return bench_batch(args, torch, fish, fi)
    if args.workload == "serve":
        return bench_serve(args, torch, fish, fi)
    if args.workload == "sphere":
        return bench_sphere(args, torch, fish, fi)
    if args.workload == "problems":
        return bench_problems(args, torch, fish, fi)
    n = (args.n,) * 3
    ncell = n[0] * n[1] * n[2]
    cfl = 0.5
    log(f"generating {n} random-Fourier state (Mach 1, beta 1, k<=16)")
    t0 = time.perf_counter()
    st = fi.random_fourier_state(n, seed=0, mach=1.0, beta=1.0, kmax=16)
    log(f"  {time.perf_counter() - t0:.1f} s")

    copy_gbs = copy_bandwidth(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s")
    res = {}
    for prec in ("fp32",) + (() if args.no_fp64 else ("fp64",)):
        log(f"GPU {prec}: {args.warmup} warmup + {args.steps} timed steps")
        res[prec] = run_gpu(fish, torch, st, n, prec, args.steps, args.warmup, cfl, args.segment,
                            autotune=not args.no_autotune, limiter=LIMITERS[args.limiter], stretch=args.stretch,
                            x_strided=args.x_strided)
        r = res[prec]
        log(f"  {r['wall'] * 1e3 / args.steps:.3f} ms/step, fluid launch avg "
            f"{r['fluid_ms'] / max(1, r['fluid_launches']):.3f} ms, state_ok={r['state_ok']}")

    r = res["fp32"]
    value = ncell * args.steps / r["wall"]
    esize = 4
    fluid_avg_s = r["fluid_ms"] / max(1, r["fluid_launches"]) * 1e-3
    bytes_fluid = ncell * 13 * esize  # reads rho, m, E and the three face fields; writes rho, m, E
    achieved = bytes_fluid / fluid_avg_s / 1e9
    # the counters were taken on the default configuration's kernels only
    default_kernels = args.limiter == "vanleer" and not args.stretch and not args.x_strided
    traffic, valu_insts = (load_counters("fluid_sweep_traffic_256.json", esize, ncell) if default_kernels
                           else (None, None))
    # the same launches against the VALU issue peak: the step is bound by
    # instruction issue, not by HBM (the counters' instructions over the live
    # launch time)
    alu = None
    if valu_insts:
        lane_insts = valu_insts * 64 / fluid_avg_s
        alu = {"achieved": lane_insts / 1e12, "peak": VALU_PEAK_LANE_INSTS / 1e12,
               "unit": "T VALU lane-instructions/s", "frac": lane_insts / VALU_PEAK_LANE_INSTS,
               "valu_per_cell": valu_insts * 64 / ncell}
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
            "limiter": {"vanleer": "van Leer", "minmod": "minmod",
                        "switch": "van Leer where subsonic, minmod where supersonic"}[args.limiter],
            "autotuned": r["tuned"],
            "mesh": "uniform" if not args.stretch else f"irregular: widths 1 + {args.stretch} sin(2 pi x + axis), Sect. 2.5",
            "x_fluid_layout": "lanes policy (rows streamed through the wavefront)" if not args.x_strided else
                              f"strided policy, lanes along y, segments of {args.x_strided} (CFL by the check kernel)",
        },
        "latency_ms": {"p50": pct(r["step_ms"], 50), "p99": pct(r["step_ms"], 99)},
        "step_roofline": {"bytes_per_cell": 384, "achieved_GBs": value * 384 / 1e9, "peak_GBs": HBM_PEAK_GBS,
                          "frac": value * 384 / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fluid sweep class: fluid_lanes_kernel (L_x) and fluid_strided_kernel (L_y, L_z), "
                               "average over its launches; the whole step is step_roofline",
                     "avg_launch_ms": fluid_avg_s * 1e3, "launches": r["fluid_launches"],
                     "timed_with": "the same steps run again with a hipEvent before and after every fluid launch "
                                   f"({r['wall_hooked'] * 1e3 / args.steps:.3f} ms/step with the events)",
                     "algorithmic_bytes_per_launch": bytes_fluid,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "valu_issue": alu},
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
        out["cpu_baseline"] = cpu_baseline(st, n, cfl, args.cpu_steps, per_core_state=(st, n, 1),
                                           limiter=LIMITERS[args.limiter])
        log(f"  {out['cpu_baseline']['value']:.3e} cell-updates/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
