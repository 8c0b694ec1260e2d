"""Full-size parity of the benchmark's box: 256^3 periodic, the random-Fourier
initialiser (rms Mach 1, beta 1, |k| <= 16, seed 0), CFL 0.5, run in the
launch configuration the benchmark times: autotuned work shapes and double
steps with dt = 0, i.e. the device CFL step, the reduction fused into the
last x sweep of the previous step.  The five double steps are one timed
segment of the benchmark (each segment restarts from the initial state,
since this box loses positivity in the seventh; the oracle test
test_oracle_c2_positivity.py shows it), so every timed step is covered.

The oracle steps the whole box in FP64 on the host threads (a few seconds
per double step), from the state rounded to the storage precision.  Both
sides take their own CFL step, so the comparison covers the reduction too.
Tolerances as for the small boxes: per-field relative L1 <= 1e-5 with FP32
storage, <= 1e-10 in FP64; the time steps agree to 1e-6 (FP32: the field's
cell means are formed in FP32) and 1e-12 (FP64).
"""
import os

import numpy as np
import pytest

try:  # first torch import on a fresh machine is slow: keep it out of the timed tests
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import Oracle

pytestmark = pytest.mark.gpu

N = (256, 256, 256)
STEPS = 5  # one timed segment of the benchmark


def _rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


@pytest.fixture(scope="module")
def initial():
    print("fullsize: random-Fourier 256^3 state", flush=True)
    return fi.random_fourier_state(N, seed=0, mach=1.0, beta=1.0, kmax=16)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol,dt_tol", [("fp32", 1e-5, 1e-6), ("fp64", 1e-10, 1e-12)])
def test_benchmark_box_steps_match_oracle(initial, prec, tol, dt_tol):
    import paper_0910_2854_amd as fish

    st = initial
    if prec == "fp32":
        st = {k: (None if v is None else v.astype(np.float32).astype(np.float64)) for k, v in st.items()}
    print(f"fullsize 256^3 {prec}: GPU, autotuned shapes, {STEPS} device-CFL steps", flush=True)
    g = fish.Box(*N, precision=prec, cfl=0.5)
    g.set_state(st)
    g.autotune(reps=2)
    g.set_state(st)
    dts_g = []
    for _ in range(STEPS):
        dts_g.append(g.cfl_dt())
        g.strang_step(0.0)
    out = g.get_state()
    g.close()

    print(f"fullsize 256^3 {prec}: oracle", flush=True)
    o = Oracle(*N, cfl=0.5, nthreads=len(os.sched_getaffinity(0)))
    o.set_state(st)
    dts_o = []
    for _ in range(STEPS):
        dts_o.append(o.cfl_dt())
        o.strang_step(0.0)
    ref = o.get_state()
    o.close()

    for a, b in zip(dts_g, dts_o):
        assert abs(a - b) <= dt_tol * b, (dts_g, dts_o)
    errs = {name: _rel_l1(out["cell"][k], ref["cell"][k]) for k, name in enumerate(("rho", "mx", "my", "mz", "E"))}
    for k in ("bx", "by", "bz"):
        errs[k] = _rel_l1(out[k], ref[k])
    print(prec, dts_g, errs, flush=True)
    assert max(errs.values()) <= tol, errs
