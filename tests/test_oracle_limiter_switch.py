"""Oracle pins for the Mach-dependent limiter switch (Sect. 2.2: van Leer in
subsonic, minmod in supersonic flow), limiter 2 (CPU only).

A cell is supersonic when |v| > c_S on the half-step state its limited flux
differences come from.  The corrected state of cell i reads the limiters of
cells i-1, i and i+1 only, and the predictor uses no limiter, so wherever those
three cells lie in one regime the switch gives bitwise the pure limiter's
result there; a box entirely in one regime gives it everywhere.  The field
advection keeps van Leer under the switch (a reading: the paper states the
switch for the fluid update).
"""
import numpy as np
import pytest

import analytic as an
import fish_inputs as fi
from oracle import MACH_SWITCH, MINMOD, VANLEER, Oracle

GAMMA = 5.0 / 3.0


def step(st, n, limiter, dt):
    o = Oracle(*n, limiter=limiter)
    o.set_state(st)
    o.strang_step(dt)
    return o.get_state(check=False)


def sweep(st, n, limiter, op, d, dt):
    o = Oracle(*n, limiter=limiter)
    o.set_state(st)
    o.apply(op, d, dt)
    return o.get_state(check=False)


def mach(st):
    c = st["cell"]
    p = an.pressure(st, GAMMA)
    v2 = (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0] ** 2
    return np.sqrt(v2 / (GAMMA * p / c[0]))


@pytest.mark.parametrize("regime,limiter", [("subsonic", VANLEER), ("supersonic", MINMOD)])
def test_switch_in_one_regime_is_that_limiter(regime, limiter):
    n = (16, 12, 10)
    st = fi.random_fourier_state(n, seed=31, mach=0.3, beta=5.0, kmax=2)
    if regime == "supersonic":  # a uniform drift at Mach 3 on top
        c = st["cell"]
        cs = np.sqrt(GAMMA * an.pressure(st, GAMMA) / c[0])
        u = 3.0 * float(np.max(cs))
        E_kin_old = 0.5 * (c[1] ** 2) / c[0]
        c[1] += c[0] * u
        c[4] += 0.5 * c[1] ** 2 / c[0] - E_kin_old
    M = mach(st)
    assert (M.max() < 0.8) if regime == "subsonic" else (M.min() > 1.5)
    o = Oracle(*n)
    o.set_state(st)
    dt = 0.4 * o.cfl_dt()
    for d in range(3):  # fluid sub-operators: the field advection keeps van Leer
        a = sweep(st, n, MACH_SWITCH, "L", d, dt)
        b = sweep(st, n, limiter, "L", d, dt)
        np.testing.assert_array_equal(a["cell"], b["cell"])
    if regime == "subsonic":  # van Leer everywhere, field included: whole steps agree
        a = step(st, n, MACH_SWITCH, dt)
        b = step(st, n, VANLEER, dt)
        for k in ("cell", "bx", "by", "bz"):
            np.testing.assert_array_equal(a[k], b[k])


def two_regime_pencil(n):
    """x pencil: Mach 1.8 in 0.1 < x < 0.5, 0.35 elsewhere, joined by
    steps; density and transverse field vary smoothly so the limiters act."""
    x = an.centres(n)
    sup = (x > 0.1) & (x < 0.5)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) + 0.1 * np.cos(6 * np.pi * x)
    p = np.full(n, 1.0)
    cs = np.sqrt(GAMMA * p / rho)
    vx = np.where(sup, 1.8, 0.35) * cs
    z = np.zeros(n)
    st = an.state_1d(0, n, rho, [vx, 0.1 * np.sin(4 * np.pi * x), z], p,
                     [0.2 + 0.05 * np.cos(2 * np.pi * x), z], GAMMA, b_normal=0.3)
    return st, sup


def test_switch_selects_per_cell():
    n = 128
    st, sup = two_regime_pencil(n)
    o = Oracle(n, 1, 1)
    o.set_state(st)
    dt = 0.5 * o.cfl_dt()
    res = {lim: Oracle(n, 1, 1, limiter=lim) for lim in (MACH_SWITCH, MINMOD, VANLEER)}
    out = {}
    for lim, oo in res.items():
        oo.set_state(st)
        oo.apply("L", 0, dt)  # one fluid sweep: the stencil statement is exact for it
        out[lim] = oo.get_state(check=False)["cell"][:, 0, 0, :]
    idx = np.arange(n)
    # cells whose neighbours (and their half-step states, a cell further)
    # lie in one regime
    inner_sup = np.array([sup[(idx[i] + np.arange(-2, 3)) % n].all() for i in idx])
    inner_sub = np.array([(~sup)[(idx[i] + np.arange(-2, 3)) % n].all() for i in idx])
    assert inner_sup.sum() > 30 and inner_sub.sum() > 50
    np.testing.assert_array_equal(out[MACH_SWITCH][:, inner_sup], out[MINMOD][:, inner_sup])
    np.testing.assert_array_equal(out[MACH_SWITCH][:, inner_sub], out[VANLEER][:, inner_sub])
    # and the two limiters do differ there (the test has teeth)
    assert np.max(np.abs(out[MINMOD][:, inner_sup] - out[VANLEER][:, inner_sup])) > 1e-6
    assert np.max(np.abs(out[MINMOD][:, inner_sub] - out[VANLEER][:, inner_sub])) > 1e-6
