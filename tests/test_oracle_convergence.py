"""Oracle pins: second-order convergence against analytic solutions (CPU only).

Linear Alfven, fast and entropy waves are translated exactly by ideal MHD;
the L1 error after a fixed time must fall by ~4x per grid doubling (the
second-order claims of Sect. 2.1, 2.2 and 2.4).  The circularly polarised
Alfven wave of Sect. 4.1 is the paper's own convergence test.  The symmetric
ordering of the sub-operators matters: a first-order (non-palindromic)
ordering would fail these rates on the Alfven wave.
"""
import math

import numpy as np
import pytest

import analytic as an
import fish_inputs as fi
from oracle import Oracle

GAMMA = 5.0 / 3.0


def evolve_to(o, T):
    """Strang steps of the CFL size, the last one shortened to land on T."""
    t = 0.0
    while t < T - 1e-14:
        dt = o.cfl_dt()
        dt = min(dt, 0.5 * (T - t))
        o.strang_step(dt)
        t += 2 * dt
    return t


def l1(a, b):
    return float(np.mean(np.abs(a - b)))


def wave_error(maker, axis, n, T, **kw):
    st0, c = maker(axis, n, 0.0, **kw)
    shape = [1, 1, 1]
    shape[axis] = n
    o = Oracle(*shape, cfl=0.8, gamma=kw.get("gamma", GAMMA))
    o.set_state(st0)
    evolve_to(o, T)
    out = o.get_state()
    ref, _ = maker(axis, n, T, **kw)
    err = sum(l1(out["cell"][k], ref["cell"][k]) for k in range(5))
    err += l1(out["bx"], ref["bx"]) + l1(out["by"], ref["by"]) + l1(out["bz"], ref["bz"])
    return err


def orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_alfven_wave_second_order(axis):
    errs = [wave_error(an.alfven_wave_1d, axis, n, 1.0) for n in (32, 64, 128)]
    assert min(orders(errs)) >= 1.9, errs


@pytest.mark.parametrize("axis", [0, 2])
def test_linear_fast_wave_second_order(axis):
    errs = [wave_error(lambda a, n, t: an.fast_wave_1d(a, n, t), axis, n, 0.7) for n in (32, 64, 128)]
    assert min(orders(errs)) >= 1.9, errs


def test_entropy_wave_second_order():
    errs = [wave_error(lambda a, n, t: (an.entropy_wave_1d(a, n, t), 1.0), 0, n, 1.0) for n in (32, 64, 128)]
    assert min(orders(errs)) >= 1.8, errs


def _oblique_alfven(N, t, eps=1e-6):
    """Alfven wave along k = (1, 1) in a unit 2-D box, b0 along k, db and dv along z."""
    x = an.centres(N)
    X, Y = np.meshgrid(x, x, indexing="xy")
    b0 = 1.0
    s = 1.0 / math.sqrt(2.0)
    kdotx = X + Y  # wave vector 2 pi (1, 1): wavelength along k is 1/sqrt(2)
    vA = b0
    # phase speed along k-hat is vA; k = 2 pi sqrt(2) -> phase = 2 pi (x + y - sqrt(2) vA t)
    db = eps * np.cos(2 * np.pi * (kdotx - math.sqrt(2.0) * vA * t))
    dv = -db
    one = np.ones((1, N, N))
    bx = np.full((1, N, N + 1), b0 * s)
    by = np.full((1, N + 1, N), b0 * s)
    bz = np.stack([db, db])
    return fi.conserved_from_primitive(one, 0 * one, 0 * one, dv[None], 0.6 * one, bx, by, bz, GAMMA)


def test_oblique_alfven_wave_2d_converges():
    """Oblique wave: both relaxed flux halves carry it (the freezing speed is the
    fast speed, not the Alfven speed), so limiter clipping at its extrema costs
    accuracy; the mean order over three doublings must still be near two."""
    errs = []
    T = 1.0 / math.sqrt(2.0)
    for N in (16, 32, 64, 128):
        o = Oracle(N, N, 1, cfl=0.8)
        o.set_state(_oblique_alfven(N, 0.0))
        evolve_to(o, T)
        out = o.get_state()
        ref = _oblique_alfven(N, T)
        errs.append(sum(l1(out["cell"][k], ref["cell"][k]) for k in range(5)) + l1(out["bz"], ref["bz"]))
    assert math.log2(errs[0] / errs[-1]) / 3 >= 1.7, errs
    assert all(e1 < e0 / 2.5 for e0, e1 in zip(errs, errs[1:])), errs


def test_circularly_polarised_alfven_wave_converges_at_second_order():
    """Sect. 4.1: L1 error (summed over components) after t = 1, slope ~2."""
    errs = []
    for N in (16, 32, 64):
        st0, (Lx, Ly) = an.cpaw_state(N)
        o = Oracle(N, N, 1, dx=Lx / N, dy=Ly / N, dz=1.0, cfl=0.8, gamma=GAMMA)
        o.set_state(st0)
        evolve_to(o, 1.0)
        out = o.get_state()
        err = sum(np.sum(np.abs(out["cell"][k] - st0["cell"][k])) for k in range(5)) / N ** 2
        bc_out = fi.cell_centred_b(out["bx"], out["by"], out["bz"])
        bc_0 = fi.cell_centred_b(st0["bx"], st0["by"], st0["bz"])
        err += sum(np.sum(np.abs(a - b)) for a, b in zip(bc_out, bc_0)) / N ** 2
        errs.append(err)
    assert orders(errs)[-1] >= 1.8, errs


def test_field_advection_second_order_and_tvd():
    """B_x alone with uniform v_x > 0 is scalar upwind TVD advection of b_y, b_z (Sect. 2.4)."""
    errs = []
    for n in (32, 64, 128):
        x = an.centres(n)
        prof = 1.0 + 0.3 * np.sin(2 * np.pi * x)
        u = 0.7
        zero = np.zeros(n)
        st = an.state_1d(0, n, np.ones(n), [u * np.ones(n), zero, zero], np.ones(n), [prof, 0.5 * prof], GAMMA)
        o = Oracle(n, 1, 1, cfl=0.8)
        o.set_state(st)
        dt = 0.4 / n / u
        T = 0.5
        steps = int(round(T / dt))
        for _ in range(steps):
            o.apply("B", 0, dt)
        out = o.get_state()
        exact = 1.0 + 0.3 * np.sin(2 * np.pi * (x - u * steps * dt))
        errs.append(l1(out["by"][0, 0], exact) + l1(out["bz"][0, 0], 0.5 * exact))
    assert min(orders(errs)) >= 1.8, errs

    # total variation of a step profile does not grow; no new extrema
    n = 64
    x = an.centres(n)
    step = np.where((x > 0.25) & (x < 0.55), 2.0, 0.5)
    zero = np.zeros(n)
    for u in (0.6, -0.6):
        # total energy is held fixed by B_d, so keep p large enough to absorb
        # the change of magnetic energy
        st = an.state_1d(0, n, np.ones(n), [u * np.ones(n), zero, zero], 10.0 * np.ones(n), [step, zero], GAMMA)
        o = Oracle(n, 1, 1)
        o.set_state(st)
        tv0 = np.sum(np.abs(np.diff(np.r_[step, step[0]])))
        for _ in range(40):
            o.apply("B", 0, 0.45 / n / abs(u))
            b = o.get_state(check=False)["by"][0, 0, :n]
            tv = np.sum(np.abs(np.diff(np.r_[b, b[0]])))
            assert tv <= tv0 * (1 + 1e-12)
            assert b.min() >= 0.5 - 1e-12 and b.max() <= 2.0 + 1e-12
            tv0 = tv
