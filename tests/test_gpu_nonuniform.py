"""Irregular Cartesian meshes (Sect. 2.5) through the HIP library against the
oracle: every sub-operator and whole steps on stretched meshes along all
three axes (periodic and outflow, ragged rows, rows longer than one
wavefront), with and without gravity; the device CFL step; equal widths give
the uniform path's result; the diagnostics weight each cell and face by its
own volume and area.

Tolerances as for uniform meshes: sub-operators 1e-12 max relative (FP64),
2e-6 relative L1 per field (FP32); whole steps 1e-10 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC, Oracle
from test_gpu_parity import max_rel, per_field_rel_l1
from test_oracle_nonuniform import stretched_widths

pytestmark = pytest.mark.gpu

CASES = [
    # (shape, bc, gravity, hse, seed)
    ((20, 14, 10), (PERIODIC,) * 3, False, False, 1),
    ((11, 9, 13), (OUTFLOW,) * 3, False, False, 2),
    ((150, 5, 4), (PERIODIC, OUTFLOW, PERIODIC), False, False, 3),
    ((16, 12, 10), (OUTFLOW,) * 3, "unsplit", True, 4),
    ((16, 12, 10), (OUTFLOW, PERIODIC, OUTFLOW), "split", False, 5),
]


def widths_for(n):
    return [stretched_widths(n[0], 0.3, 0.0), stretched_widths(n[1], 0.25, 1.0), stretched_widths(n[2], 0.2, 2.0)]


def state_for(n, gravity, seed):
    if gravity:
        return fi.sphere_state(n, seed)
    return fi.random_fourier_state(n, seed=seed, mach=0.6, beta=2.0, kmax=2)


def pair(n, kw, prec, ws):
    import paper_0910_2854_amd as fish
    o = Oracle(*n, **kw)
    g = fish.Box(*n, precision=prec, **kw)
    for a in range(3):
        o.set_spacing(a, ws[a])
        g.set_spacing(a, ws[a])
    return o, g


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_nonuniform_suboperators(case, prec):
    n, bc, grav, hse, seed = CASES[case]
    kw = dict(bc=bc, gravity=grav or False, hse=hse)
    ws = widths_for(n)
    st = state_for(n, grav, seed)
    o0, _ = None, None
    for op in ("L", "B"):
        for d in range(3):
            print(f"irregular mesh {op}{d} case {case} {n} {prec}", flush=True)
            o, g = pair(n, kw, prec, ws)
            o.set_state(st)
            g.set_state(st)
            dt = 0.4 * o.cfl_dt()
            o.apply(op, d, dt)
            g.sweep(op, d, dt)
            ref, out = o.get_state(check=False), g.get_state(check=False)
            g.close()
            if prec == "fp64":
                assert max_rel(out, ref) <= 1e-12, (op, d, max_rel(out, ref))
            else:
                errs = per_field_rel_l1(out, ref)
                if grav:  # momenta of the sphere at rest: against the momentum scale of the others
                    for name in ("mx", "my", "mz"):
                        errs.pop(name)
                assert max(errs.values()) <= 2e-6, (op, d, errs)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("case", [0, 1, 3, 4])
def test_nonuniform_steps(case, prec, tol):
    n, bc, grav, hse, seed = CASES[case]
    kw = dict(bc=bc, gravity=grav or False, hse=hse, cfl=0.5)
    print(f"irregular mesh steps case {case} {n} {prec}", flush=True)
    ws = widths_for(n)
    st = state_for(n, grav, seed)
    o, g = pair(n, kw, prec, ws)
    o.set_state(st)
    g.set_state(st)
    for _ in range(3):
        dt = o.cfl_dt()
        assert abs(g.cfl_dt() / dt - 1.0) <= (1e-12 if prec == "fp64" else 1e-5)
        o.strang_step(dt)
        g.strang_step(dt)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    g.close()
    if grav and prec == "fp32":
        for name in ("mx", "my", "mz"):
            errs.pop(name)
    print(errs)
    assert max(errs.values()) <= tol, errs


def test_equal_widths_match_the_uniform_path():
    import paper_0910_2854_amd as fish
    print("irregular mesh with equal widths 24x16x12 fp64", flush=True)
    n = (24, 16, 12)
    st = fi.random_fourier_state(n, seed=8, mach=0.6, beta=2.0, kmax=2)
    a = fish.Box(*n, precision="fp64")
    a.set_state(st)
    b = fish.Box(*n, precision="fp64")
    for ax in range(3):
        b.set_spacing(ax, np.full(n[ax], 1.0 / n[ax]))
    b.set_state(st)
    for _ in range(2):
        dt = a.cfl_dt()
        assert abs(b.cfl_dt() / dt - 1.0) < 1e-14
        a.strang_step(dt)
        b.strang_step(dt)
    assert max_rel(b.get_state(), a.get_state()) <= 1e-13
    a.close()
    with pytest.raises(fish.FishError):
        b.set_spacing(0, np.full(n[0], -1.0))
    b.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
@pytest.mark.parametrize("case", [0, 1])
def test_nonuniform_diagnostics_match_oracle(case, prec, tol):
    """Volume-weighted totals, area-weighted face sums and the per-cell
    divergence on a stretched mesh, before and after two steps, against the
    oracle's diagnostics of the state the GPU holds (FP32: the device keeps
    the widths rounded to the storage precision, the oracle in FP64).  Each
    sum is compared on the scale of the sum of its absolute terms."""
    n, bc, grav, hse, seed = CASES[case]
    kw = dict(bc=bc, gravity=grav or False, hse=hse)
    ws = widths_for(n)
    st = state_for(n, grav, seed)
    print(f"irregular diagnostics case {case} {n} {prec}", flush=True)
    o, g = pair(n, kw, prec, ws)
    o.set_state(st)
    g.set_state(st)
    dv = ws[2][:, None, None] * ws[1][None, :, None] * ws[0][None, None, :]
    # face areas: x faces (z, y), y faces (z, x), z faces (y, x)
    area = [ws[2][:, None] * ws[1][None, :], ws[2][:, None] * ws[0][None, :], ws[1][:, None] * ws[0][None, :]]
    for step in range(3):
        sg = g.get_state()
        ref = Oracle(*n, **kw)
        for a in range(3):
            ref.set_spacing(a, ws[a])
        ref.set_state(sg)
        do = ref.diagnostics()
        ref.close()
        dg = g.diagnostics()
        scale = [float(np.sum(np.abs(sg["cell"][k]) * dv)) for k in range(5)]
        assert abs(dg["mass"] - do["mass"]) <= tol * scale[0], (step, dg["mass"], do["mass"])
        assert abs(dg["energy"] - do["energy"]) <= tol * scale[4], (step, dg["energy"], do["energy"])
        for c in range(3):
            assert abs(dg["mom"][c] - do["mom"][c]) <= tol * scale[1 + c], (step, c, dg["mom"], do["mom"])
        fsc = [float(np.sum(np.abs(sg["bx"]).sum(axis=2) * area[0])),
               float(np.sum(np.abs(sg["by"]).sum(axis=1) * area[1])),
               float(np.sum(np.abs(sg["bz"]).sum(axis=0) * area[2]))]
        for c in range(3):
            assert abs(dg["flux"][c] - do["flux"][c]) <= tol * fsc[c], (step, c, dg["flux"], do["flux"])
        assert dg["bmax"] == do["bmax"]
        assert abs(dg["divb_max"] - do["divb_max"]) <= 10 * tol * max(do["divb_max"], do["bmax"] / min(map(min, ws))), \
            (step, dg["divb_max"], do["divb_max"])
        if step < 2:
            dt = o.cfl_dt()
            o.strang_step(dt)
            g.strang_step(dt)
    o.close()
    g.close()


def _mild(n, seed):
    # every box stays valid for 8 steps on the oracle, on its mesh
    return fi.random_fourier_state(n, seed=seed, mach=0.4, beta=4.0, kmax=2)


def _alone(n, bc, seed, prec, steps, nu):
    import paper_0910_2854_amd as fish
    g = fish.Box(*n, precision=prec, bc=bc)
    if nu:
        for a, w in enumerate(widths_for(n)):
            g.set_spacing(a, w)
    g.set_state(_mild(n, seed))
    for _ in range(steps):
        g.strang_step(0.0)
    out = g.get_state()
    g.close()
    return out


def _close_to(got, ref, prec, n):
    if prec == "fp64":
        assert max_rel(got, ref) <= 1e-12, n
        assert abs(got["t"] - ref["t"]) <= 1e-13 * ref["t"]
    else:
        assert max(per_field_rel_l1(got, ref).values()) <= 1e-5, n
        assert abs(got["t"] - ref["t"]) <= 1e-6 * ref["t"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_with_irregular_and_uniform_boxes(prec):
    """A batch mixing boxes on stretched meshes with uniform ones, stepped
    with per-box CFL steps: an irregular box gives bitwise its result alone;
    a uniform box runs the irregular formulas with its own spacing, equal to
    its uniform result alone to rounding; the irregular boxes match the
    oracle (FP64).  Once the irregular boxes leave, the uniform kernels take
    over again."""
    import paper_0910_2854_amd as fish
    boxes = [((20, 14, 10), (PERIODIC,) * 3, 21, True), ((16, 12, 10), (PERIODIC,) * 3, 22, False),
             ((11, 9, 13), (OUTFLOW,) * 3, 23, True), ((150, 5, 4), (PERIODIC, OUTFLOW, PERIODIC), 24, False)]
    steps = 3
    print(f"batch of irregular and uniform boxes, {prec}", flush=True)
    b = fish.Batch(256 << 20, max_boxes=16, precision=prec)
    ids = []
    for n, bc, seed, nu in boxes:
        i = b.add(_mild(n, seed), bc=bc)
        if nu:
            for a, w in enumerate(widths_for(n)):
                b.set_spacing(i, a, w)
        ids.append(i)
    b.step(steps)
    for (n, bc, seed, nu), i in zip(boxes, ids):
        print(f"  box {n} irregular={nu}", flush=True)
        got = b.get(i)
        ref = _alone(n, bc, seed, prec, steps, nu)
        if not nu:
            _close_to(got, ref, prec, n)
            continue
        for k in ("cell", "bx", "by", "bz"):
            assert np.array_equal(got[k], ref[k]), (n, k)
        assert got["t"] == ref["t"]
        if prec == "fp64":
            o = Oracle(*n, bc=bc)
            for a, w in enumerate(widths_for(n)):
                o.set_spacing(a, w)
            o.set_state(_mild(n, seed))
            for _ in range(steps):
                o.strang_step(0.0)
            so = o.get_state()
            o.close()
            assert max(per_field_rel_l1(got, so).values()) <= 1e-10
            assert abs(got["t"] - so["t"]) <= 1e-12 * so["t"]
    for (n, bc, seed, nu), i in zip(boxes, ids):
        if nu:
            b.remove(i)
    b.step(1)
    for (n, bc, seed, nu), i in zip(boxes, ids):
        if not nu:
            print(f"  box {n} after the irregular boxes left", flush=True)
            _close_to(b.get(i), _alone(n, bc, seed, prec, steps + 1, False), prec, n)
    b.close()


def test_server_serves_requests_on_irregular_meshes():
    """Requests that carry cell widths beside uniform ones (FP64): an
    irregular request's result is bitwise its box stepped alone, a uniform
    one's equal to its result alone to rounding."""
    import paper_0910_2854_amd as fish
    reqs = [((20, 14, 10), (PERIODIC,) * 3, 4, 31, True), ((16, 12, 10), (PERIODIC,) * 3, 3, 32, False),
            ((11, 9, 13), (OUTFLOW,) * 3, 5, 33, True), ((12, 10, 8), (PERIODIC,) * 3, 2, 34, False)]
    print(f"server with {len(reqs)} requests, irregular and uniform", flush=True)
    srv = fish.Server(512 << 20, chunk_steps=2, precision="fp64")
    for tag, (n, bc, k, seed, nu) in enumerate(reqs):
        srv.submit(tag, _mild(n, seed), k, bc=bc, widths=widths_for(n) if nu else None)
    done = {}
    for _ in range(100):
        for tag, status, out in srv.pump():
            assert status == fish.FISH_OK, tag
            done[tag] = out
        if len(done) == len(reqs):
            break
    assert len(done) == len(reqs)
    for tag, (n, bc, k, seed, nu) in enumerate(reqs):
        ref = _alone(n, bc, seed, "fp64", k, nu)
        if nu:
            for f in ("cell", "bx", "by", "bz"):
                assert np.array_equal(done[tag][f], ref[f]), (n, f)
        else:
            assert max_rel(done[tag], ref) <= 1e-12, n
    with pytest.raises(fish.FishError):
        srv.submit(99, _mild((8, 8, 8), 1), 1, widths=[np.full(8, -1.0), None, None])
    srv.close()
