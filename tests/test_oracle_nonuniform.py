"""Oracle pins for irregular Cartesian meshes (Sect. 2.5: dx replaced by the
width dx_i of each cell, per axis) -- CPU only.

* a uniform state stays unchanged on a stretched mesh;
* periodic conservation of the volume-weighted totals and of the face
  fluxes (b times face area), and the discrete divergence with per-cell widths
  held by the constrained transport;
* widths all equal to the uniform dx reproduce the uniform-mesh step to
  rounding (the irregular formulas reduce to Sects. 2.2-2.4);
* second-order convergence of an entropy wave and a linear Alfven wave on
  smoothly stretched periodic meshes along each axis.
"""
import math

import numpy as np
import pytest

import analytic as an
import fish_inputs as fi
from oracle import Oracle

GAMMA = 5.0 / 3.0


def stretched_widths(n, amp=0.3, phase=0.0, L=1.0):
    xi = (np.arange(n) + 0.5) / n
    w = 1.0 + amp * np.sin(2 * np.pi * xi + phase)
    return w * (L / w.sum())


def centres_of(w):
    return np.cumsum(w) - 0.5 * w


def nonuniform_oracle(n, widths, **kw):
    o = Oracle(*n, **kw)
    for a, w in enumerate(widths):
        if w is not None:
            o.set_spacing(a, w)
    return o


def test_uniform_state_unchanged_on_a_stretched_mesh():
    n = (12, 10, 8)
    st = fi.uniform_state(n, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, b=(0.4, 0.2, -0.3), gamma=GAMMA)
    o = nonuniform_oracle(n, [stretched_widths(12), stretched_widths(10, 0.2, 1.0), stretched_widths(8, 0.25, 2.0)])
    o.set_state(st)
    for _ in range(2):
        o.strang_step(o.cfl_dt())
    out = o.get_state()
    for k in ("cell", "bx", "by", "bz"):
        np.testing.assert_allclose(out[k], st[k], rtol=1e-13, atol=1e-14)


def test_diagnostics_of_a_uniform_state_on_a_stretched_mesh():
    """Closed form: the totals are the state times the box volume (the product
    of the width sums), the face sums b times the face areas summed over the
    real faces (n per periodic axis, n + 1 per outflow axis), and a uniform
    field has no divergence."""
    from oracle import OUTFLOW, PERIODIC

    n = (12, 10, 8)
    ws = [stretched_widths(12, 0.3, 0.0, L=1.3), stretched_widths(10, 0.2, 1.0, L=0.7), stretched_widths(8, 0.25, 2.0)]
    rho, v, p, bv = 1.3, (0.3, -0.2, 0.1), 0.7, (0.4, 0.2, -0.3)
    st = fi.uniform_state(n, rho=rho, v=v, p=p, b=bv, gamma=GAMMA)
    L = [float(np.sum(w)) for w in ws]
    vol = L[0] * L[1] * L[2]
    for bc in ((PERIODIC,) * 3, (OUTFLOW, PERIODIC, OUTFLOW)):
        o = nonuniform_oracle(n, ws, bc=bc)
        o.set_state(st)
        d = o.diagnostics()
        o.close()
        assert abs(d["mass"] - rho * vol) <= 1e-14 * rho * vol
        E = st["cell"][4, 0, 0, 0]
        assert abs(d["energy"] - E * vol) <= 1e-14 * E * vol
        np.testing.assert_allclose(d["mom"], rho * np.array(v) * vol, rtol=1e-14, atol=1e-15)
        for a in range(3):
            nfaces = n[a] + (1 if bc[a] == OUTFLOW else 0)
            area = vol / L[a]
            assert abs(d["flux"][a] - bv[a] * nfaces * area) <= 1e-14 * abs(bv[a] * nfaces * area)
        assert d["divb_max"] <= 1e-13
        assert d["bmax"] == max(abs(x) for x in bv)


def test_conservation_and_divergence_on_a_stretched_mesh():
    n = (14, 12, 10)
    st = fi.random_fourier_state(n, seed=41, mach=0.5, beta=2.0, kmax=2)
    ws = [stretched_widths(14), stretched_widths(12, 0.2, 1.0), stretched_widths(10, 0.25, 2.0)]
    o = nonuniform_oracle(n, ws)
    o.set_state(st)
    d0 = o.diagnostics()
    for _ in range(3):
        o.strang_step(o.cfl_dt())
    d1 = o.diagnostics()
    assert abs(d1["mass"] / d0["mass"] - 1.0) < 1e-13
    assert abs(d1["energy"] / d0["energy"] - 1.0) < 1e-13
    assert np.max(np.abs(d1["mom"] - d0["mom"])) < 1e-13 * d0["mass"]
    assert np.max(np.abs(d1["flux"] - d0["flux"])) < 1e-13
    # the state's own divergence (a curl on the uniform index grid is not
    # divergence-free with per-cell widths) is carried unchanged
    assert abs(d1["divb_max"] - d0["divb_max"]) <= 1e-12 * max(1.0, d0["divb_max"])


def divergence(st, ws):
    hx, hy, hz = ws
    return (np.diff(st["bx"], axis=2) / hx[None, None, :] + np.diff(st["by"], axis=1) / hy[None, :, None] +
            np.diff(st["bz"], axis=0) / hz[:, None, None])


def test_constrained_transport_keeps_the_per_cell_divergence():
    n = (14, 12, 10)
    st = fi.random_fourier_state(n, seed=43, mach=0.5, beta=3.0, kmax=2)
    ws = [stretched_widths(14), stretched_widths(12, 0.2, 1.0), stretched_widths(10, 0.25, 2.0)]
    o = nonuniform_oracle(n, ws)
    o.set_state(st)
    div0 = divergence(st, ws)
    for _ in range(3):
        o.strang_step(o.cfl_dt())
    div1 = divergence(o.get_state(), ws)
    bscale = max(np.max(np.abs(st[k])) for k in ("bx", "by", "bz")) / min(w.min() for w in ws)
    assert np.max(np.abs(div1 - div0)) <= 1e-12 * bscale


def test_equal_widths_reproduce_the_uniform_step():
    n = (12, 10, 8)
    st = fi.random_fourier_state(n, seed=45, mach=0.7, beta=2.0, kmax=2)
    ref = Oracle(*n)
    ref.set_state(st)
    dt = ref.cfl_dt()
    ref.strang_step(dt)
    o = nonuniform_oracle(n, [np.full(12, 1 / 12), np.full(10, 1 / 10), np.full(8, 1 / 8)])
    o.set_state(st)
    assert abs(o.cfl_dt() / dt - 1.0) < 1e-14
    o.strang_step(dt)
    a, b = o.get_state(), ref.get_state()
    for k in ("cell", "bx", "by", "bz"):
        scale = np.max(np.abs(b[k]))
        assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * scale, k


def wave_state(axis, x, t, kind, eps=1e-6):
    """Along `axis` at cell centres x: an entropy wave (rho = 1 + 0.2 sin,
    v = 1, p = 1, b = 0) or a linear Alfven wave (rho = 1, p = 0.6, b_n = 1,
    b_t = eps sin, v_t = -b_t), translated by the exact speed (1 and v_A = 1)."""
    n = len(x)
    s = np.sin(2 * np.pi * (x - t))
    z = np.zeros(n)
    if kind == "entropy":
        return an.state_1d(axis, n, 1.0 + 0.2 * s, [np.ones(n), z, z], np.ones(n), [z, z], GAMMA)
    return an.state_1d(axis, n, np.ones(n), [z, -eps * s, z], 0.6 * np.ones(n), [eps * s, z], GAMMA, b_normal=1.0)


@pytest.mark.parametrize("kind", ["entropy", "alfven"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_second_order_on_a_stretched_mesh(kind, axis):
    errs = []
    for n in (32, 64, 128):
        w = stretched_widths(n)
        x = centres_of(w)
        nn = [1, 1, 1]
        nn[axis] = n
        o = Oracle(*nn, cfl=0.8)
        o.set_spacing(axis, w)
        o.set_state(wave_state(axis, x, 0.0, kind))
        t = 0.0
        while t < 0.5 - 1e-14:
            dt = min(o.cfl_dt(), 0.5 * (0.5 - t))
            o.strang_step(dt)
            t += 2 * dt
        out = an.profile_1d(o.get_state(), axis)
        ref = an.profile_1d(wave_state(axis, x, 0.5, kind), axis)
        if kind == "entropy":
            errs.append(float(np.sum(np.abs(out["rho"] - ref["rho"]) * w)))
        else:
            errs.append(float(np.sum((np.abs(out["b"][1] - ref["b"][1]) + np.abs(out["v"][1] - ref["v"][1])) * w)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.8, (errs, orders)


def test_face_velocity_interpolates_a_linear_shear_exactly():
    """Uniform rho and b_y = B, v_x = a + s y on a stretched y mesh (outflow
    in y): one B_x sweep leaves b_y alone (nothing varies along x) and moves
    b_x by dt (E_j+1/2 - E_j-1/2)/dy_j with E = v_x b_y at the y-faces.  With
    v_x interpolated linearly to each face (Sect. 2.5) that is exactly
    dt B s in every row away from the y boundaries; swapped or equal weights
    leave a row-to-row error of order s dy."""
    from oracle import OUTFLOW, PERIODIC
    nx, ny, nz = 8, 24, 1
    wy = stretched_widths(ny, amp=0.4)
    y = centres_of(wy)
    a, s, B, dt = 0.3, 0.8, 0.7, 0.01
    one = np.ones((nz, ny, nx))
    vx = (a + s * y)[None, :, None] * one
    st = fi.conserved_from_primitive(one, vx, 0 * one, 0 * one, one, np.zeros((nz, ny, nx + 1)),
                                     np.full((nz, ny + 1, nx), B), np.zeros((nz + 1, ny, nx)), GAMMA)
    o = Oracle(nx, ny, nz, bc=(PERIODIC, OUTFLOW, PERIODIC))
    o.set_spacing(1, wy)
    o.set_state(st)
    o.apply("B", 0, dt)
    out = o.get_state(check=False)
    np.testing.assert_array_equal(out["by"], st["by"])
    inner = out["bx"][:, 2:-2, :]
    np.testing.assert_allclose(inner, dt * B * s, rtol=1e-12)
