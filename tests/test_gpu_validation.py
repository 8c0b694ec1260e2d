"""The HIP library against analytic solutions (not against the oracle):
second-order convergence of linear Alfven waves along every axis (which
exercises the x lanes kernels and the y/z strided kernels), the circularly
polarised Alfven wave of Sect. 4.1 in FP64 and FP32, and Sod's tube against
the exact Riemann solution."""
import math

import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import analytic as an
import fish_inputs as fi

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def _box(shape, **kw):
    import paper_0910_2854_amd as fish
    return fish.Box(*shape, **kw)


def evolve_to(g, T):
    """Device CFL steps, the last one shortened to land on T."""
    t = 0.0
    while t < T - 1e-14:
        dt = min(g.cfl_dt(), 0.5 * (T - t))
        g.strang_step(dt)
        t += 2 * dt
    return t


def l1(a, b):
    return float(np.mean(np.abs(a - b)))


def orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gpu_linear_alfven_wave_second_order(axis):
    print(f"Alfven wave axis {axis}", flush=True)
    errs = []
    for n in (32, 64, 128):
        st0, _ = an.alfven_wave_1d(axis, n, 0.0)
        shape = [1, 1, 1]
        shape[axis] = n
        g = _box(shape, cfl=0.8, precision="fp64")
        g.set_state(st0)
        evolve_to(g, 1.0)
        out = g.get_state()
        g.close()
        ref, _ = an.alfven_wave_1d(axis, n, 1.0)
        err = sum(l1(out["cell"][k], ref["cell"][k]) for k in range(5))
        err += l1(out["bx"], ref["bx"]) + l1(out["by"], ref["by"]) + l1(out["bz"], ref["bz"])
        errs.append(err)
    assert min(orders(errs)) >= 1.9, errs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gpu_circularly_polarised_alfven_wave(prec):
    """Sect. 4.1 on a 2-D box with dx != dy: L1 error after t = 1, slope ~2."""
    print(f"CPAW {prec}", flush=True)
    errs = []
    for N in (16, 32, 64):
        st0, (Lx, Ly) = an.cpaw_state(N)
        g = _box((N, N, 1), dx=Lx / N, dy=Ly / N, dz=1.0, cfl=0.8, gamma=GAMMA, precision=prec)
        g.set_state(st0)
        evolve_to(g, 1.0)
        out = g.get_state()
        g.close()
        err = sum(np.sum(np.abs(out["cell"][k] - st0["cell"][k])) for k in range(5)) / N ** 2
        bc_out = fi.cell_centred_b(out["bx"], out["by"], out["bz"])
        bc_0 = fi.cell_centred_b(st0["bx"], st0["by"], st0["bz"])
        err += sum(np.sum(np.abs(a - b)) for a, b in zip(bc_out, bc_0)) / N ** 2
        errs.append(err)
    assert orders(errs)[-1] >= 1.8, errs


@pytest.mark.parametrize("axis", [0, 2])
def test_gpu_sod_tube_plateaus(axis):
    """Sod's tube (b = 0) along x and z, outflow ends: the star states between
    the rarefaction tail, the contact and the shock match the exact Riemann
    solution within 1%."""
    from oracle import OUTFLOW
    print(f"Sod axis {axis}", flush=True)
    n, T = 800, 0.2
    x = an.centres(n)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    zero = np.zeros(n)
    st = an.state_1d(axis, n, rho, [zero, zero, zero], p, [zero, zero], GAMMA)
    shape = [1, 1, 1]
    shape[axis] = n
    bc = [OUTFLOW if a == axis else 0 for a in range(3)]
    g = _box(shape, cfl=0.8, gamma=GAMMA, bc=bc, precision="fp64")
    g.set_state(st)
    evolve_to(g, T)
    out = g.get_state()
    g.close()
    prof = an.profile_1d(out, axis)
    pnum = an.pressure(out, GAMMA).reshape(-1)
    _, star = an.exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), GAMMA, (x - 0.5) / T)
    aL = math.sqrt(GAMMA)
    asL = aL * (star["pstar"]) ** ((GAMMA - 1) / (2 * GAMMA))
    tail = 0.5 + (star["ustar"] - asL) * T
    contact = 0.5 + star["ustar"] * T
    aR = math.sqrt(GAMMA * 0.1 / 0.125)
    shock = 0.5 + aR * math.sqrt((GAMMA + 1) / (2 * GAMMA) * star["pstar"] / 0.1 + (GAMMA - 1) / (2 * GAMMA)) * T
    i_ls = np.where((x > tail + 0.02) & (x < contact - 0.02))[0]
    i_rs = np.where((x > contact + 0.02) & (x < shock - 0.02))[0]
    assert len(i_ls) > 10 and len(i_rs) > 10
    for idx, rho_star in ((i_ls, star["rho_star_L"]), (i_rs, star["rho_star_R"])):
        assert np.all(np.abs(prof["rho"][idx] - rho_star) <= 0.01 * rho_star)
        assert np.all(np.abs(pnum[idx] - star["pstar"]) <= 0.01 * star["pstar"])
        assert np.all(np.abs(prof["v"][0][idx] - star["ustar"]) <= 0.01 * star["ustar"])
