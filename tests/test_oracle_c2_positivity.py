"""Why the benchmark times its 256^3 box in segments of five double steps:
under the FP64 oracle the box (random-Fourier initialiser, rms Mach 1, beta
1, |k| <= 16, seed 0, CFL 0.5) keeps a positive pressure through six double
steps (p_min 0.43, 0.35, 0.24, 0.16, 0.11, 0.085) and loses it in the
seventh (p_min -0.033).  The scheme has no floors (a run stops on a negative
pressure, Sect. 4.4), so the benchmark restarts each five-step segment from
the initial state and every timed step advances a valid state.
"""
import os

import pytest

import fish_inputs as fi
from oracle import Oracle, OracleError

N = (256, 256, 256)
GAMMA = 5.0 / 3.0


def min_pressure(x):
    c = x["cell"]
    bx, by, bz = x["bx"], x["by"], x["bz"]
    bcx = 0.5 * (bx[:, :, :-1] + bx[:, :, 1:])
    bcy = 0.5 * (by[:, :-1, :] + by[:, 1:, :])
    bcz = 0.5 * (bz[:-1] + bz[1:])
    p = (GAMMA - 1.0) * (c[4] - 0.5 * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0] - 0.5 * (bcx ** 2 + bcy ** 2 + bcz ** 2))
    return float(p.min())


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_benchmark_box_keeps_positive_pressure_for_six_double_steps_only():
    st = fi.random_fourier_state(N, seed=0, mach=1.0, beta=1.0, kmax=16)
    assert min_pressure(st) > 0.0
    o = Oracle(*N, gamma=GAMMA, cfl=0.5, nthreads=len(os.sched_getaffinity(0)))
    o.set_state(st)
    pmin = []
    for _ in range(6):
        o.strang_step(o.cfl_dt())
        pmin.append(min_pressure(o.get_state(check=False)))
    print("p_min after double steps 1-6:", pmin, flush=True)
    assert all(p > 0.0 for p in pmin), pmin
    # the seventh double step leaves a negative pressure; the oracle then
    # refuses a further CFL step
    o.strang_step(o.cfl_dt())
    p7 = min_pressure(o.get_state(check=False))
    print("p_min after double step 7:", p7, flush=True)
    assert p7 < 0.0
    with pytest.raises(OracleError):
        o.cfl_dt()
    o.close()
