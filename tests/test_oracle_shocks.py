"""Oracle pins: discontinuous solutions fixed by conservation (CPU only).

* Sod's tube along each axis against the exact Riemann solution of the Euler
  equations (b = 0): the TVD relaxed-flux scheme (Sect. 2.2) must capture the
  star states;
* an isolated hydrodynamic shock and a perpendicular fast MHD shock whose
  downstream states are found by root finding of the Rankine-Hugoniot jump
  conditions: the shock must move at the prescribed speed, stay a few cells
  wide, and leave the plateaus at the jump values.
"""
import math

import numpy as np
import pytest

import analytic as an
from oracle import OUTFLOW, Oracle

GAMMA = 1.4


def run_1d(axis, st, n, T, cfl=0.8, limiter=1):
    shape = [1, 1, 1]
    shape[axis] = n
    o = Oracle(*shape, cfl=cfl, gamma=GAMMA, bc=(OUTFLOW,) * 3, limiter=limiter)
    o.set_state(st)
    t = 0.0
    while t < T - 1e-14:
        dt = min(o.cfl_dt(), 0.5 * (T - t))
        o.strang_step(dt)
        t += 2 * dt
    return o.get_state()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sod_tube_matches_exact_riemann_solution(axis):
    n, T = 800, 0.2
    x = an.centres(n)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    zero = np.zeros(n)
    st = an.state_1d(axis, n, rho, [zero, zero, zero], p, [zero, zero], GAMMA)
    out = run_1d(axis, st, n, T)
    prof = an.profile_1d(out, axis)
    pnum = an.pressure(out, GAMMA).reshape(-1)
    exact, star = an.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA, (x - 0.5) / T)
    # left star region: between the rarefaction tail and the contact
    aL = math.sqrt(GAMMA)
    asL = aL * (star["pstar"]) ** ((GAMMA - 1) / (2 * GAMMA))
    tail = 0.5 + (star["ustar"] - asL) * T
    contact = 0.5 + star["ustar"] * T
    i_ls = np.where((x > tail + 0.02) & (x < contact - 0.02))[0]
    # right star region: between the contact and the shock
    rR, pR = 0.125, 0.1
    aR = math.sqrt(GAMMA * pR / rR)
    shock = 0.5 + (aR * math.sqrt((GAMMA + 1) / (2 * GAMMA) * star["pstar"] / pR + (GAMMA - 1) / (2 * GAMMA))) * T
    i_rs = np.where((x > contact + 0.02) & (x < shock - 0.02))[0]
    assert len(i_ls) > 10 and len(i_rs) > 10
    for idx, rho_star in ((i_ls, star["rho_star_L"]), (i_rs, star["rho_star_R"])):
        assert np.all(np.abs(prof["rho"][idx] - rho_star) <= 0.01 * rho_star)
        assert np.all(np.abs(pnum[idx] - star["pstar"]) <= 0.01 * star["pstar"])
        assert np.all(np.abs(prof["v"][0][idx] - star["ustar"]) <= 0.01 * star["ustar"])
    # L1 agreement with the exact profile overall, and it improves with resolution
    e_fine = np.mean(np.abs(prof["rho"] - exact[0]))
    xc = an.centres(n // 4)
    st_c = an.state_1d(axis, n // 4, np.where(xc < 0.5, 1.0, 0.125), [np.zeros(n // 4)] * 3,
                       np.where(xc < 0.5, 1.0, 0.1), [np.zeros(n // 4)] * 2, GAMMA)
    out_c = run_1d(axis, st_c, n // 4, T)
    ex_c, _ = an.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA, (xc - 0.5) / T)
    e_coarse = np.mean(np.abs(an.profile_1d(out_c, axis)["rho"] - ex_c[0]))
    assert e_fine < 0.5 * e_coarse
    assert e_fine < 2e-3


def _shock_run(WR, WL, s, n=800, T=0.25, x0=0.3):
    x = an.centres(n)
    left = x < x0
    rho = np.where(left, WL[0], WR[0])
    u = np.where(left, WL[1], WR[1])
    p = np.where(left, WL[2], WR[2])
    by = np.where(left, WL[3], WR[3])
    zero = np.zeros(n)
    st = an.state_1d(0, n, rho, [u, zero, zero], p, [by, zero], GAMMA)
    out = run_1d(0, st, n, T)
    return x, an.profile_1d(out, 0), an.pressure(out, GAMMA).reshape(-1)


@pytest.mark.parametrize("byR,label", [(0.0, "hydro"), (0.8, "mhd-perpendicular")])
def test_rankine_hugoniot_shock(byR, label):
    WR = np.array([1.0, 0.0, 0.6, byR])  # upstream at rest
    aR = math.sqrt(GAMMA * WR[2] / WR[0])
    cf = math.sqrt(aR ** 2 + byR ** 2 / WR[0])
    s = 2.2 * cf  # fast-Mach 2.2 shock moving right
    guess = np.array([2.5, 1.2 * cf, 3.0, 2.5 * byR])
    WL, resid = an.rh_downstream(WR, s, GAMMA, guess)
    assert resid < 1e-11 and WL[0] > WR[0] and WL[2] > WR[2]  # compressive root
    x0, T = 0.3, 0.25
    x, prof, p = _shock_run(WR, WL, s, x0=x0, T=T)
    # shock position: where rho crosses the mid value
    mid = 0.5 * (WL[0] + WR[0])
    i = np.where(prof["rho"] < mid)[0][0]
    xs = x[i - 1] + (mid - prof["rho"][i - 1]) / (prof["rho"][i] - prof["rho"][i - 1]) * (x[i] - x[i - 1])
    speed = (xs - x0) / T
    assert abs(speed - s) <= 0.005 * s, (speed, s)
    # width: cells strictly between 10% and 90% of the jump
    frac = (prof["rho"] - WR[0]) / (WL[0] - WR[0])
    width = np.sum((frac > 0.1) & (frac < 0.9))
    assert width <= 4, width
    # plateaus (the start-up error of the initial jump is carried with the flow)
    post = (x > x0 + WL[1] * T + 0.04) & (x < xs - 0.04)
    assert post.sum() > 20
    pre = x > xs + 0.05
    for arr, (a, b) in ((prof["rho"], (WL[0], WR[0])), (p, (WL[2], WR[2])), (prof["v"][0], (WL[1], WR[1])),
                        (prof["b"][1], (WL[3], WR[3]))):
        assert np.all(np.abs(arr[post] - a) <= 1e-3 * max(abs(a), 1.0)), label
        assert np.all(np.abs(arr[pre] - b) <= 1e-12 + 1e-3 * abs(b)), label
