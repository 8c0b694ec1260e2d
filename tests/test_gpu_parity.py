"""GPU parity: the HIP library (through its C interface) against the FP64 oracle.

Every case prints what it runs before touching the GPU.  Tolerances:
FP64 per-sub-operator max relative error <= 1e-12; FP64 full steps per-field
relative L1 <= 1e-10 after 10 steps; FP32 storage with FP64 pressure
recovery per-field relative L1 <= 1e-5 after 10 steps on smooth data.
"""
import numpy as np
import pytest

try:  # first torch import on a fresh machine is slow: keep it out of the timed tests
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC, Oracle

pytestmark = pytest.mark.gpu

FIELDS = ("cell", "bx", "by", "bz")


def _box(n, **kw):
    import paper_0910_2854_amd as fish
    return fish.Box(*n, **kw)


def rel_l1(a, b):
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / den) if den > 0 else float(np.sum(np.abs(a - b)))


def per_field_rel_l1(sg, so):
    out = {}
    for k in range(5):
        out[("rho", "mx", "my", "mz", "E")[k]] = rel_l1(sg["cell"][k], so["cell"][k])
    for k in ("bx", "by", "bz"):
        out[k] = rel_l1(sg[k], so[k])
    return out


def max_rel(sg, so):
    worst = 0.0
    for k in FIELDS:
        scale = np.max(np.abs(so[k])) + 1e-300
        worst = max(worst, float(np.max(np.abs(sg[k] - so[k])) / scale))
    return worst


CASES = [
    # (shape, bc, gravity, hse, seed)
    ((12, 10, 8), (PERIODIC,) * 3, False, False, 1),
    ((9, 70, 5), (PERIODIC,) * 3, False, False, 2),       # two segments + ragged tail along y
    ((6, 5, 131), (PERIODIC,) * 3, False, False, 3),       # three segments along z
    ((11, 7, 6), (OUTFLOW,) * 3, False, False, 4),
    ((10, 9, 8), (OUTFLOW, PERIODIC, OUTFLOW), True, False, 5),
    ((10, 9, 8), (OUTFLOW,) * 3, True, True, 6),
    ((16, 1, 1), (PERIODIC,) * 3, False, False, 7),        # inactive axes
    ((1, 13, 3), (PERIODIC, OUTFLOW, PERIODIC), False, False, 8),
    ((2, 3, 2), (PERIODIC,) * 3, False, False, 9),          # wrap more than once
    ((150, 3, 2), (PERIODIC,) * 3, False, False, 10),       # x rows spanning several 64-lane iterations
    ((131, 4, 3), (OUTFLOW,) * 3, True, True, 11),          # same with outflow, gravity and HSE
]


def _state(n, bc, gravity, seed):
    if gravity:
        st = fi.sphere_state(n, seed)
        if any(b == PERIODIC for b in bc):
            # keep the sphere, periodic face n = face 0 is ignored on input
            pass
        return st
    return fi.random_fourier_state(n, seed=seed, mach=0.8, beta=2.0, kmax=2)


def test_lane_shift_primitive():
    """The x sweeps stream through the wavefront with a one-lane shift; check
    its lane layout directly (lane i takes lane i - 1, lane 0 takes 0)."""
    import paper_0910_2854_amd as fish
    print("lane-shift self-test", flush=True)
    out = fish.selftest_lane_shift(0)
    expect = np.empty(128, dtype=np.float32)
    for it in range(2):
        for lane in range(64):
            expect[64 * it + lane] = (100 * it + lane - 1) if lane > 0 else 0
    np.testing.assert_array_equal(out, expect)


def _ulps(a, b):
    """Distance in units in the last place between float64 arrays of one sign."""
    ia = a.view(np.int64).astype(object)
    ib = b.view(np.int64).astype(object)
    return np.array([abs(p - q) for p, q in zip(ia, ib)], dtype=np.float64)


def test_fp64_reciprocal_and_square_root():
    """The FP64 sweeps form 1/x and sqrt(x) from the hardware estimates with
    Newton and Goldschmidt steps instead of the IEEE sequences.  Against
    numpy's IEEE division and square root: within one ulp (in practice equal)
    wherever the argument and the result are normal numbers, and for the roots
    of subnormal numbers; sqrt(0) = 0 with its sign, NaN for a negative root;
    the special inputs the sweeps never pass (0, infinity and subnormal x for
    1/x, infinity for the root) give NaN."""
    import paper_0910_2854_amd as fish
    print("FP64 reciprocal / square-root self-test", flush=True)
    rng = np.random.default_rng(11)
    n = 1 << 18
    e = rng.integers(-1021, 1021, n)
    x = np.ldexp(rng.uniform(1.0, 2.0, n), e) * np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0)
    x[:8] = [1.0, -1.0, 3.0, 0.1, 1e-300, 1e300, 2.0 ** -1021, 1.5 * 2.0 ** 1020]
    r, s = fish.selftest_math(x)
    with np.errstate(invalid="ignore"):
        ref_r = 1.0 / x
        pos = x > 0
        ref_s = np.sqrt(np.where(pos, x, 1.0))
    ur = _ulps(r, ref_r)
    us = _ulps(s[pos], ref_s[pos])
    print(f"  1/x: max {ur.max():.0f} ulp, {int(np.count_nonzero(ur))} of {n} differ; "
          f"sqrt: max {us.max():.0f} ulp, {int(np.count_nonzero(us))} of {int(pos.sum())} differ", flush=True)
    assert ur.max() <= 1 and us.max() <= 1
    assert np.all(np.isnan(s[~pos]))
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 2.0 ** -1074, 2.0 ** -1030, 2.0 ** 1023])
    r, s = fish.selftest_math(special)
    print("  special x:", special.tolist(), flush=True)
    print("  1/x:", r.tolist(), flush=True)
    print("  sqrt:", s.tolist(), flush=True)
    assert s[0] == 0.0 and not np.signbit(s[0]) and s[1] == 0.0 and np.signbit(s[1])
    assert np.isnan(r[0]) and np.isnan(r[1]) and np.isnan(r[2]) and np.isnan(r[3]) and np.isnan(r[4])
    assert np.isnan(s[2]) and np.isnan(s[3]) and np.isnan(s[4])
    # subnormal arguments: their reciprocals overflow (NaN here, IEEE infinity);
    # their roots, and both results for the largest binade, are right
    assert np.isnan(r[5]) and np.isnan(r[6]) and r[7] == 1.0 / special[7]
    assert _ulps(s[5:], np.sqrt(special[5:])).max() <= 1


# van Leer and the Mach switch on every shape, minmod on a subset
LIMITER_CASES = [(c, lim) for lim in (1, 2) for c in range(len(CASES))] + [(c, 0) for c in (0, 3, 5, 10)]


@pytest.mark.parametrize("case,limiter", LIMITER_CASES)
@pytest.mark.parametrize("op", ["L", "B"])
def test_suboperator_parity_fp64(case, op, limiter):
    n, bc, grav, hse, seed = CASES[case]
    st = _state(n, bc, grav, seed)
    kw = dict(bc=bc, gravity=grav, hse=hse, limiter=limiter)
    o = Oracle(*n, **kw)
    o.set_state(st)
    dt = 0.4 * o.cfl_dt()
    for d in range(3):
        print(f"sub-operator {op}{d} case {case} shape {n} bc {bc} grav {grav} hse {hse} lim {limiter}", flush=True)
        o2 = Oracle(*n, **kw)
        o2.set_state(st)
        o2.apply(op, d, dt)
        ref = o2.get_state(check=False)
        g = _box(n, precision="fp64", **kw)
        g.set_state(st)
        g.sweep(op, d, dt)
        out = g.get_state(check=False)
        g.close()
        err = max_rel(out, ref)
        assert err <= 1e-12, (op, d, err)


def _run_pair(n, st, steps, precision, **kw):
    o = Oracle(*n, **kw)
    o.set_state(st)
    g = _box(n, precision=precision, **kw)
    g.set_state(st)
    for _ in range(steps):
        dt = o.cfl_dt()
        o.strang_step(dt)
        g.strang_step(dt)
    return g, o


def test_c1_ten_steps_fp64():
    """32^3 periodic random-Fourier box (rms Mach 0.5, beta 10), 10 steps."""
    print("C1 32^3 fp64 10 steps", flush=True)
    st = fi.random_fourier_state(32, seed=0, mach=0.5, beta=10.0, kmax=4)
    g, o = _run_pair((32, 32, 32), st, 10, "fp64", cfl=0.5)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= 1e-10, errs


def _sound_momentum_scale(st, gamma=5.0 / 3.0):
    """sum of rho c_s over the box: the momentum scale of a state at rest."""
    import analytic as an
    p = an.pressure(st, gamma)
    return float(np.sum(np.sqrt(gamma * np.abs(p) * st["cell"][0])))


@pytest.mark.parametrize("case", [0, 3, 5, 9, 10])
def test_suboperator_parity_fp32(case):
    """FP32 storage/arithmetic with FP64 pressure: one sub-operator at a time.

    Relative L1 per field; a momentum component that starts at rest (the
    stratified sphere) is measured against the sound-speed momentum scale,
    since its first kick is a residual of pressure and gravity forces that
    cancel to a few parts in 10^3 in FP32."""
    n, bc, grav, hse, seed = CASES[case]
    st = _state(n, bc, grav, seed)
    kw = dict(bc=bc, gravity=grav, hse=hse)
    o = Oracle(*n, **kw)
    o.set_state(st)
    dt = 0.4 * o.cfl_dt()
    for op in ("L", "B"):
        for d in range(3):
            print(f"fp32 sub-operator {op}{d} case {case} shape {n}", flush=True)
            o2 = Oracle(*n, **kw)
            o2.set_state(st)
            o2.apply(op, d, dt)
            ref = o2.get_state(check=False)
            g = _box(n, precision="fp32", **kw)
            g.set_state(st)
            g.sweep(op, d, dt)
            out = g.get_state(check=False)
            g.close()
            errs = per_field_rel_l1(out, ref)
            if grav:
                ms = _sound_momentum_scale(st)
                for k, name in ((1, "mx"), (2, "my"), (3, "mz")):
                    errs[name] = float(np.sum(np.abs(out["cell"][k] - ref["cell"][k]))) / max(
                        ms, float(np.sum(np.abs(ref["cell"][k]))))
            assert max(errs.values()) <= 2e-6, (op, d, errs)


def test_c1_ten_steps_fp32():
    print("C1 32^3 fp32 10 steps", flush=True)
    st = fi.random_fourier_state(32, seed=0, mach=0.5, beta=10.0, kmax=4)
    g, o = _run_pair((32, 32, 32), st, 10, "fp32", cfl=0.5)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= 1e-5, errs


def test_sphere_outflow_hse_fp64_steps():
    print("sphere 24^3 outflow gravity hse fp64 3 steps", flush=True)
    n = (24, 24, 24)
    st = fi.sphere_state(n, 0)
    kw = dict(bc=(OUTFLOW,) * 3, gravity=True, hse=True, cfl=0.5)
    g, o = _run_pair(n, st, 3, "fp64", **kw)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= 1e-10, errs


def test_device_cfl_matches_oracle():
    print("CFL 20^3 fp64 and fp32", flush=True)
    st = fi.random_fourier_state((20, 18, 16), seed=11, mach=1.0, beta=1.0, kmax=3)
    o = Oracle(20, 18, 16)
    o.set_state(st)
    ref = o.cfl_dt()
    for prec, tol in (("fp64", 1e-14), ("fp32", 1e-6)):
        g = _box((20, 18, 16), precision=prec)
        g.set_state(st)
        assert abs(g.cfl_dt() - ref) <= tol * ref, prec
        g.close()


def test_device_resident_dt_step_matches_oracle():
    """fish_strang_step(0): the device takes the CFL step itself."""
    print("dt==0 steps 16^3 fp64", flush=True)
    st = fi.random_fourier_state(16, seed=12, mach=0.5, beta=5.0, kmax=3)
    o = Oracle(16, 16, 16)
    o.set_state(st)
    g = _box((16, 16, 16), precision="fp64")
    g.set_state(st)
    for _ in range(3):
        o.strang_step(0.0)
        g.strang_step(0.0)
    so, sg = o.get_state(), g.get_state()
    assert abs(sg["t"] - so["t"]) <= 1e-13 * so["t"]
    assert max(per_field_rel_l1(sg, so).values()) <= 1e-11


def test_gpu_conservation_and_divergence():
    print("conservation 24^3 fp64", flush=True)
    st = fi.random_fourier_state(24, seed=13, mach=0.5, beta=10.0, kmax=3)
    g = _box((24, 24, 24), precision="fp64")
    g.set_state(st)
    d0 = g.diagnostics()
    for _ in range(5):
        g.strang_step(0.0)
    d1 = g.diagnostics()
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * d0["energy"]
    assert d1["divb_max"] * (1 / 24) / d1["bmax"] <= 1e-12
    o = Oracle(24, 24, 24)
    o.set_state(st)
    od = o.diagnostics()
    assert abs(od["mass"] - d0["mass"]) <= 1e-14 * od["mass"]
    assert np.allclose(od["flux"], d0["flux"], rtol=0, atol=1e-14)


def test_gpu_determinism_bitwise():
    print("determinism 20^3 fp32", flush=True)
    st = fi.random_fourier_state(20, seed=14, mach=0.5, beta=3.0, kmax=3)
    outs = []
    for _ in range(2):
        g = _box((20, 20, 20), precision="fp32")
        g.set_state(st)
        for _ in range(3):
            g.strang_step(0.0)
        outs.append(g.get_state())
        g.close()
    for k in FIELDS:
        assert np.array_equal(outs[0][k], outs[1][k])


def test_gpu_uniform_state_bitwise():
    print("uniform 9x7x5 outflow fp32/fp64", flush=True)
    n = (9, 7, 5)
    st = fi.uniform_state(n, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, b=(0.4, -0.5, 0.25))
    for prec in ("fp64", "fp32"):
        for bc in ((PERIODIC,) * 3, (OUTFLOW,) * 3):
            g = _box(n, precision=prec, bc=bc)
            g.set_state(st)
            ref = g.get_state()
            for _ in range(2):
                g.strang_step(0.0)
            out = g.get_state()
            for k in FIELDS:
                assert np.array_equal(out[k], ref[k]), (prec, bc, k)
            g.close()


def test_gpu_rejects_bad_state():
    import paper_0910_2854_amd as fish
    print("bad state 4^3", flush=True)
    st = fi.uniform_state((4, 4, 4), p=0.5)
    st["cell"][4, 1, 2, 3] = -1.0
    g = _box((4, 4, 4))
    with pytest.raises(fish.FishError) as e:
        g.set_state(st)
    assert e.value.code == fish.FISH_ERR_STATE


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_fused_cfl_matches_standalone_reduction(prec, tol):
    """The last x sweep of a step reduces the next CFL step; it must agree with
    the standalone reduction of the same state (and with the oracle)."""
    print(f"fused CFL {prec} 24x20x16", flush=True)
    n = (24, 20, 16)
    st = fi.random_fourier_state(n, seed=21, mach=0.7, beta=2.0, kmax=3)
    g = _box(n, precision=prec)
    g.set_state(st)
    g.strang_step(0.0)
    fused = g.cfl_dt()
    out = g.get_state()          # runs the standalone check/reduction
    standalone = g.cfl_dt()
    assert fused == standalone   # the same per-cell function and an order-free max
    o = Oracle(*n)
    o.set_state(out)
    assert abs(o.cfl_dt() - standalone) <= max(tol, 1e-14) * standalone


GRAVITY_CASES = [i for i, c in enumerate(CASES) if c[2]]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
@pytest.mark.parametrize("case", GRAVITY_CASES)
def test_split_gravity_fluid_sweep_parity(case, prec, tol):
    """Split gravity (Eqs. 38-40): each fluid sub-operator G_d(dt/2) L_d
    G_d(dt/2), kicks fused into the sweep, against the oracle's three separate
    steps.  FP32 momenta of the sphere at rest are measured against the
    sound-speed momentum scale (as for the unsplit form)."""
    n, bc, _, hse, seed = CASES[case]
    st = _state(n, bc, True, seed)
    kw = dict(bc=bc, gravity="split", hse=hse)
    o = Oracle(*n, **kw)
    o.set_state(st)
    dt = 0.4 * o.cfl_dt()
    for d in range(3):
        print(f"split gravity L{d} case {case} shape {n} {prec}", flush=True)
        o2 = Oracle(*n, **kw)
        o2.set_state(st)
        o2.apply("L", d, dt)
        ref = o2.get_state(check=False)
        g = _box(n, precision=prec, **kw)
        g.set_state(st)
        g.sweep("L", d, dt)
        out = g.get_state(check=False)
        g.close()
        if prec == "fp64":
            assert max_rel(out, ref) <= tol, (d, max_rel(out, ref))
        else:
            errs = per_field_rel_l1(out, ref)
            ms = _sound_momentum_scale(st)
            for k, name in ((1, "mx"), (2, "my"), (3, "mz")):
                errs[name] = float(np.sum(np.abs(out["cell"][k] - ref["cell"][k]))) / max(
                    ms, float(np.sum(np.abs(ref["cell"][k]))))
            assert max(errs.values()) <= tol, (d, errs)


@pytest.mark.parametrize("hse", [False, True])
def test_split_gravity_sphere_steps_fp64(hse):
    print(f"split gravity sphere 24^3 outflow hse {hse} fp64 3 steps", flush=True)
    n = (24, 24, 24)
    st = fi.sphere_state(n, 0)
    kw = dict(bc=(OUTFLOW,) * 3, gravity="split", hse=hse, cfl=0.5)
    g, o = _run_pair(n, st, 3, "fp64", **kw)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= 1e-10, errs


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("bcz", [PERIODIC, OUTFLOW])
@pytest.mark.parametrize("gravity,hse", [("none", False), ("unsplit", True), ("split", False)])
def test_flat_box_steps_with_and_without_gravity(bcz, gravity, hse, prec, tol):
    """A box with one cell along z (its z fluid sweeps are left out as the
    identity) against the oracle, which runs them: 3 double steps, relative
    L1 <= 1e-10 in FP64 and <= 1e-5 in FP32, and L_z alone returns the state
    bitwise."""
    n = (40, 36, 1)
    print(f"flat box {n} bc_z {bcz} gravity {gravity} hse {hse} {prec} 3 steps", flush=True)
    st = fi.random_fourier_state(n, seed=7, mach=0.8, beta=2.0, kmax=2)
    if gravity != "none":
        st["phi"] = 0.1 * np.random.default_rng(8).standard_normal((n[2], n[1], n[0]))
    kw = dict(bc=(PERIODIC, OUTFLOW, bcz), gravity=gravity, hse=hse)
    g, o = _run_pair(n, st, 3, prec, **kw)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= tol, errs
    before = g.get_state()
    g.sweep("L", 2, 0.5 * o.cfl_dt())
    after = g.get_state()
    g.close()
    for k in FIELDS:
        assert np.array_equal(after[k], before[k]), k


def test_split_gravity_constant_potential_is_the_plain_step():
    """A constant potential: the fused kicks change nothing, bitwise."""
    import paper_0910_2854_amd as fish  # noqa: F401
    print("split gravity constant phi 20^3 fp32", flush=True)
    n = (20, 20, 20)
    st = fi.random_fourier_state(n, seed=5, mach=0.6, beta=3.0, kmax=2)
    ref = _box(n, precision="fp32")
    ref.set_state(st)
    ref.strang_step(0.0)
    a = ref.get_state()
    ref.close()
    st["phi"] = np.full((n[2], n[1], n[0]), 1.75)
    g = _box(n, precision="fp32", gravity="split")
    g.set_state(st)
    g.strang_step(0.0)
    b = g.get_state()
    g.close()
    for k in FIELDS:
        np.testing.assert_array_equal(a[k], b[k])



def two_regime_box(n):
    """v_x = 1.8 c_S on 0.1 < x < 0.5 and 0.35 c_S elsewhere, density and
    field varying in all three directions: the limiter switch (limiter 2)
    picks minmod in one slab and van Leer in the other, with no cell near
    Mach 1 (FP32 rounding cannot move a cell across)."""
    import analytic as an
    nx, ny, nz = n
    x = an.centres(nx)[None, None, :]
    y = an.centres(ny)[None, :, None]
    z = an.centres(nz)[:, None, None]
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) + 0.1 * np.cos(2 * np.pi * (y + z)) + 0.05 * np.sin(6 * np.pi * x)
    rho = rho * np.ones((nz, ny, nx))
    p = np.ones_like(rho)
    cs = np.sqrt(GAMMA * p / rho)
    vx = np.where((x > 0.1) & (x < 0.5), 1.8, 0.35) * cs
    vy = 0.1 * np.sin(2 * np.pi * (x + z)) * np.ones_like(rho)
    vz = 0.05 * np.cos(2 * np.pi * y) * np.ones_like(rho)
    bx = np.full((nz, ny, nx + 1), 0.3)
    by = np.full((nz, ny + 1, nx), 0.2)
    bz = np.full((nz + 1, ny, nx), 0.1)
    return fi.conserved_from_primitive(rho, vx, vy, vz, p, bx, by, bz, GAMMA)


GAMMA = 5.0 / 3.0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_limiter_switch_steps(prec, tol):
    from oracle import MACH_SWITCH
    n = (70, 12, 10)
    print(f"limiter switch {n} {prec} 3 steps", flush=True)
    st = two_regime_box(n)
    g, o = _run_pair(n, st, 3, prec, limiter=MACH_SWITCH)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    print(errs)
    assert max(errs.values()) <= tol, errs
