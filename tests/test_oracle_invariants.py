"""Oracle pins: invariants the scheme is built to keep (CPU only).

* uniform states stay bitwise unchanged (every flux difference is zero), for
  periodic and outflow boundaries and single-cell axes;
* the fluid sweep along a single-cell axis is the identity on any state (the
  field sweep there is not);
* periodic conservation of mass, momentum, total energy (flux form, Eq. 18)
  and of the face-flux sums (constraint update, Eq. 64);
* the discrete divergence of Eq. (62) is left unchanged by the field update;
* cyclic axis equivariance of every sub-operator (checks the direction and
  index bookkeeping, including the sign of the constraint update);
* closed forms of the fast speed through the CFL step of Eq. (14);
* determinism and the state check of the C interface.
"""
import numpy as np
import pytest

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC, Oracle, OracleError, ERR_STATE

GAMMA = 5.0 / 3.0


def run(st, n, steps=1, dt=None, **kw):
    o = Oracle(*n, **kw)
    o.set_state(st)
    for _ in range(steps):
        o.strang_step(dt if dt is not None else o.cfl_dt())
    return o


@pytest.mark.parametrize("n,bc", [
    ((8, 6, 5), (PERIODIC,) * 3),
    ((8, 6, 5), (OUTFLOW,) * 3),
    ((7, 1, 1), (PERIODIC,) * 3),
    ((1, 5, 1), (OUTFLOW, OUTFLOW, PERIODIC)),
    ((6, 1, 4), (PERIODIC, OUTFLOW, OUTFLOW)),
])
def test_uniform_state_bitwise_unchanged(n, bc):
    st = fi.uniform_state(n, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, b=(0.4, -0.5, 0.25), gamma=GAMMA)
    o = run(st, n, steps=3, bc=bc, gamma=GAMMA)
    out = o.get_state()
    assert np.array_equal(out["cell"], st["cell"])
    for k in ("bx", "by", "bz"):
        assert np.array_equal(out[k], st[k]), k


def test_uniform_state_with_constant_potential_and_hse():
    n = (6, 5, 4)
    st = fi.uniform_state(n, rho=1.0, v=(0.1, 0.2, -0.3), p=0.5, b=(0.1, 0.2, 0.3), gamma=GAMMA)
    st["phi"] = np.full((n[2], n[1], n[0]), 2.5)
    o = run(st, n, steps=2, bc=(OUTFLOW,) * 3, gamma=GAMMA, gravity=True, hse=True)
    out = o.get_state()
    assert np.array_equal(out["cell"], st["cell"])


@pytest.mark.parametrize("bcz", [PERIODIC, OUTFLOW])
@pytest.mark.parametrize("gravity,hse", [("none", False), ("unsplit", True), ("split", False)])
def test_fluid_sweep_along_a_single_cell_axis_is_the_identity(bcz, gravity, hse):
    """Along an axis with one cell every ghost is the cell itself (and phi
    wraps or copies), so L_z of a flat box returns its input bitwise, which
    lets the library leave that sweep out; B_z is not the identity there: it
    leaves b_x and b_y but moves b_z by the transverse differences of the
    edge fluxes v_z b_t."""
    n = (12, 10, 1)
    st = fi.random_fourier_state(n, seed=5, mach=0.8, beta=2.0, kmax=2)
    if gravity != "none":
        rng = np.random.default_rng(6)
        st["phi"] = 0.1 * rng.standard_normal((n[2], n[1], n[0]))
    bc = (PERIODIC, OUTFLOW, bcz)
    o = Oracle(*n, bc=bc, gamma=GAMMA, gravity=gravity, hse=hse)
    o.set_state(st)
    dt = 0.5 * o.cfl_dt()
    before = o.get_state()
    o.apply("L", 2, dt)
    after = o.get_state()
    for k in ("cell", "bx", "by", "bz"):
        assert np.array_equal(after[k], before[k]), k
    o.apply("L", 0, dt)  # the sweep along x does change it
    assert not np.array_equal(o.get_state()["cell"], before["cell"])
    o.set_state(st)
    o.apply("B", 2, dt)
    after = o.get_state()
    assert np.array_equal(after["bx"], before["bx"]) and np.array_equal(after["by"], before["by"])
    assert np.max(np.abs(after["bz"] - before["bz"])) > 1e-6


@pytest.fixture(scope="module")
def c1_run():
    st = fi.random_fourier_state(32, seed=0, mach=0.5, beta=10.0, kmax=4)
    o = Oracle(32, 32, 32, cfl=0.5)
    o.set_state(st)
    diags = [o.diagnostics()]
    for _ in range(10):
        o.strang_step(o.cfl_dt())
        diags.append(o.diagnostics())
    return st, o, diags


def test_conservation_periodic(c1_run):
    st, o, diags = c1_run
    d0, d1 = diags[0], diags[-1]
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * abs(d0["energy"])
    cell = st["cell"]
    mscale = np.abs(cell[1:4]).sum() / cell[0].size
    assert np.all(np.abs(d1["mom"] - d0["mom"]) <= 1e-13 * mscale)
    bscale = max(d0["bmax"], 1e-300)
    assert np.all(np.abs(d1["flux"] - d0["flux"]) <= 1e-13 * bscale)


def test_divergence_stays_at_roundoff(c1_run):
    st, o, diags = c1_run
    h = 1.0 / 32
    for d in diags:
        assert d["divb_max"] * h / d["bmax"] <= 1e-12


def test_state_actually_evolves(c1_run):
    st, o, diags = c1_run
    out = o.get_state()
    assert np.max(np.abs(out["cell"] - st["cell"])) > 1e-3
    assert out["t"] > 0


def _rotate(st):
    """Cyclic relabelling x->y, y->z, z->x of a state (arrays are [z][y][x])."""
    cell = st["cell"]
    new = np.empty((5,) + tuple(np.transpose(cell[0], (1, 2, 0)).shape))
    new[0] = np.transpose(cell[0], (1, 2, 0))
    new[4] = np.transpose(cell[4], (1, 2, 0))
    new[2] = np.transpose(cell[1], (1, 2, 0))   # m_y' = m_x
    new[3] = np.transpose(cell[2], (1, 2, 0))   # m_z' = m_y
    new[1] = np.transpose(cell[3], (1, 2, 0))   # m_x' = m_z
    out = {"cell": new,
           "by": np.ascontiguousarray(np.transpose(st["bx"], (1, 2, 0))),
           "bz": np.ascontiguousarray(np.transpose(st["by"], (1, 2, 0))),
           "bx": np.ascontiguousarray(np.transpose(st["bz"], (1, 2, 0))),
           "phi": None if st.get("phi") is None else np.ascontiguousarray(np.transpose(st["phi"], (1, 2, 0)))}
    return out


@pytest.mark.parametrize("op", ["L", "B"])
@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("bc", [PERIODIC, OUTFLOW])
def test_cyclic_equivariance_per_suboperator(op, d, bc):
    n = (10, 8, 6)
    st = fi.random_fourier_state(n, seed=3, mach=1.0, beta=1.0, kmax=2)
    rot = _rotate(st)
    nr = (n[2], n[0], n[1])
    kw = dict(bc=(bc,) * 3, gamma=GAMMA)
    a = Oracle(*n, dx=0.1, dy=0.125, dz=1 / 6, **kw)
    a.set_state(st)
    dt = 0.3 * a.cfl_dt()
    a.apply(op, d, dt)
    b = Oracle(*nr, dx=1 / 6, dy=0.1, dz=0.125, **kw)
    b.set_state(rot)
    b.apply(op, (d + 1) % 3, dt)
    ra = _rotate(a.get_state())
    rb = b.get_state()
    for k in ("cell", "bx", "by", "bz"):
        scale = np.max(np.abs(ra[k])) + 1e-300
        assert np.max(np.abs(ra[k] - rb[k])) <= 1e-14 * scale, k
    # the sub-operator did something
    assert np.max(np.abs(a.get_state()["cell"] - st["cell"])) > 0 or op == "B"


@pytest.mark.parametrize("op", ["L", "B"])
def test_reflection_y_z_commutes(op):
    """Mirroring y <-> z swaps the two transverse directions of an x sweep."""
    n = (8, 6, 6)
    st = fi.random_fourier_state(n, seed=5, mach=0.8, beta=2.0, kmax=2)
    mir = {"cell": np.transpose(st["cell"], (0, 2, 1, 3))[[0, 1, 3, 2, 4]].copy(),
           "bx": np.ascontiguousarray(np.transpose(st["bx"], (1, 0, 2))),
           "by": np.ascontiguousarray(np.transpose(st["bz"], (1, 0, 2))),
           "bz": np.ascontiguousarray(np.transpose(st["by"], (1, 0, 2))), "phi": None}
    a = Oracle(*n)
    a.set_state(st)
    dt = 0.3 * a.cfl_dt()
    a.apply(op, 0, dt)
    b = Oracle(*n)
    b.set_state(mir)
    b.apply(op, 0, dt)
    sa, sb = a.get_state(), b.get_state()
    ma = np.transpose(sa["cell"], (0, 2, 1, 3))[[0, 1, 3, 2, 4]]
    assert np.max(np.abs(ma - sb["cell"])) <= 1e-14 * np.max(np.abs(ma))
    assert np.max(np.abs(np.transpose(sa["bx"], (1, 0, 2)) - sb["bx"])) <= 1e-14 * np.max(np.abs(sb["bx"]))
    assert np.max(np.abs(np.transpose(sa["by"], (1, 0, 2)) - sb["bz"])) <= 1e-14 * np.max(np.abs(sb["bz"]))


@pytest.mark.parametrize("b,expect", [
    ((0.0, 0.0, 0.0), "a"),
    ((0.9, 0.0, 0.0), "max"),
    ((0.3, 0.0, 0.0), "max"),
    ((0.0, 0.7, 0.2), "perp"),
])
def test_fast_speed_closed_forms_via_cfl(b, expect):
    """b = 0 -> c_F = a; b along the sweep -> max(a, v_A); b across it -> sqrt(a^2 + v_A^2)."""
    n = (16, 1, 1)
    rho, p, v = 1.7, 0.45, (-0.3, 0.2, 0.1)
    st = fi.uniform_state(n, rho=rho, v=v, p=p, b=b, gamma=GAMMA)
    o = Oracle(*n, cfl=0.8, gamma=GAMMA)
    o.set_state(st)
    a2 = GAMMA * p / rho
    vA2 = (b[0] ** 2 + b[1] ** 2 + b[2] ** 2) / rho
    cf = {"a": np.sqrt(a2), "max": np.sqrt(max(a2, vA2)), "perp": np.sqrt(a2 + vA2)}[expect]
    expected = 0.8 * (1.0 / 16) / (abs(v[0]) + cf)
    assert abs(o.cfl_dt() - expected) <= 1e-14 * expected


def test_cfl_uses_absolute_velocity():
    n = (16, 1, 1)
    dts = []
    for vx in (0.4, -0.4):
        o = Oracle(*n)
        o.set_state(fi.uniform_state(n, v=(vx, 0, 0), p=0.6, b=(0.2, 0.3, 0.0)))
        dts.append(o.cfl_dt())
    assert dts[0] == dts[1]


def test_determinism_bitwise():
    st = fi.random_fourier_state(16, seed=2, mach=0.5, beta=2.0, kmax=3)
    outs = []
    for threads in (1, 4):
        o = Oracle(16, 16, 16, nthreads=threads)
        o.set_state(st)
        for _ in range(2):
            o.strang_step(o.cfl_dt())
        outs.append(o.get_state())
    for k in ("cell", "bx", "by", "bz"):
        assert np.array_equal(outs[0][k], outs[1][k])


def test_bad_state_is_rejected():
    n = (4, 4, 4)
    st = fi.uniform_state(n, p=0.5)
    st["cell"][4, 1, 2, 3] = 0.1 * st["cell"][4, 1, 2, 3] - 10.0  # negative pressure
    o = Oracle(*n)
    with pytest.raises(OracleError) as e:
        o.set_state(st)
    assert e.value.code == ERR_STATE
    st = fi.uniform_state(n, p=0.5)
    st["cell"][0, 0, 0, 0] = np.nan
    with pytest.raises(OracleError):
        o.set_state(st)


def test_periodic_face_n_is_written_as_face_0(c1_run):
    st, o, diags = c1_run
    out = o.get_state()
    assert np.array_equal(out["bx"][:, :, -1], out["bx"][:, :, 0])
    assert np.array_equal(out["by"][:, -1, :], out["by"][:, 0, :])
    assert np.array_equal(out["bz"][-1], out["bz"][0])
