"""The allocation-free double step (fish_strang_step_noalloc) against the
context's fish_strang_step on the same state: both run the same kernels on
the same inputs, so the states after the step, the step size and the CFL
step of the new state must agree bitwise.  Three calls in a row on one GPU
per precision, each on a smaller box than the one before, so that each runs
on the scratch the previous call left behind: in FP64 and FP32, with the CFL
step (dt = 0) and a given dt, without gravity, with unsplit gravity and the
hydrostatic correction, with split gravity (FP64) and on a flat box, whose
z fluid sweeps both leave out (FP32).  Device arrays come from torch and the
work is enqueued on torch's current stream."""

import numpy as np
import pytest

try:  # first torch import on a fresh machine is slow: keep it out of the timed tests
    import torch
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi

pytestmark = pytest.mark.gpu

P, O = 0, 1


def _state(n, bc, gravity, seed):
    if gravity:
        return fi.sphere_state(n, seed)
    return fi.random_fourier_state(n, seed=seed, mach=0.8, beta=2.0, kmax=2)


def _context_step(fish, n, bc, st, precision, dt_mode, **kw):
    """The existing entry point: state, CFL step before, state after, CFL step after."""
    g = fish.Box(*n, bc=bc, precision=precision, **kw)
    g.set_state(st)
    dt0 = g.cfl_dt()
    dt = 0.0 if dt_mode == "cfl" else 0.5 * dt0
    g.strang_step(dt)
    out = g.get_state(check=False)
    dt_next = g.cfl_dt()
    g.close()
    return out, (dt0 if dt_mode == "cfl" else dt), dt_next, dt


GUARD = 4096  # NaN elements before and after every array


def _guarded(values, tdt, dev):
    """A device array with NaN guards on both sides: a write outside the
    array shows in the guards, a read of one would put NaN into the result."""
    ne = int(np.prod(values.shape))
    buf = torch.full((ne + 2 * GUARD,), float("nan"), dtype=tdt, device=dev)
    view = buf[GUARD:GUARD + ne]
    if values is not None:
        view.copy_(torch.from_numpy(np.ascontiguousarray(values).reshape(-1)).to(dev))
    return buf, view


def _noalloc_step(fish, n, bc, st, precision, dt, **kw):
    dtype = np.float64 if precision == "fp64" else np.float32
    tdt = torch.float64 if precision == "fp64" else torch.float32
    arrays, phi = fish.to_storage(st, n, bc, dtype)
    dev = torch.device("cuda", 0)
    state = [_guarded(a, tdt, dev) for a in arrays]
    # the work arrays start as NaN: the step must write before it reads them
    work = [_guarded(np.full(a.shape, np.nan, dtype=dtype), tdt, dev) for a in arrays]
    phid = _guarded(phi, tdt, dev) if phi is not None else None
    report = torch.zeros(3, dtype=torch.float64, device=dev)  # one fish_step_report (24 bytes)
    p = fish.make_params(*n, bc=bc, precision=precision, stream=torch.cuda.current_stream(dev).cuda_stream, **kw)
    fish.strang_step_noalloc(p, [v.data_ptr() for _, v in state], [v.data_ptr() for _, v in work],
                             phid[1].data_ptr() if phid is not None else None, dt, report.data_ptr())
    torch.cuda.synchronize(dev)
    for buf, _ in state + work + ([phid] if phid is not None else []):
        assert bool(torch.isnan(buf[:GUARD]).all()) and bool(torch.isnan(buf[-GUARD:]).all()), "write outside an array"
    shape = fish.storage_shape(n, bc)
    out = fish.from_storage([v.cpu().numpy().reshape(shape) for _, v in state], n, bc)
    rep = fish.StepReport.from_buffer_copy(report.cpu().numpy().tobytes())
    return out, rep


# (shape, bc, gravity, hse, dt mode, seed): successive calls, each on a smaller box
CALLS = {
    "fp64": [((40, 36, 44), (P, P, P), False, False, "cfl", 11),
             ((20, 12, 16), (O, P, O), True, True, "given", 12),
             ((16, 14, 12), (O, O, O), "split", True, "cfl", 13)],
    "fp32": [((48, 32, 40), (O, O, O), True, False, "given", 21),
             ((12, 10, 8), (P, P, P), False, False, "cfl", 22),
             ((24, 20, 1), (P, P, P), False, False, "cfl", 23)],
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_step_equals_the_context_step_on_successive_calls(precision):
    import paper_0910_2854_amd as fish
    for n, bc, grav, hse, mode, seed in CALLS[precision]:
        print(f"noalloc {precision} shape {n} bc {bc} gravity {grav} hse {hse} dt {mode} seed {seed}", flush=True)
        st = _state(n, bc, grav, seed)
        kw = dict(gravity=grav, hse=hse)
        ref, dt_ref, dt_next_ref, dt = _context_step(fish, n, bc, st, precision, mode, **kw)
        out, rep = _noalloc_step(fish, n, bc, st, precision, dt, **kw)
        assert rep.status == fish.FISH_OK
        assert rep.dt == dt_ref, (rep.dt, dt_ref)
        assert rep.dt_next == dt_next_ref, (rep.dt_next, dt_next_ref)
        for k in ("cell", "bx", "by", "bz"):
            np.testing.assert_array_equal(out[k], ref[k], err_msg=k)
        # the step did change the state
        assert np.max(np.abs(out["cell"][1:4] - st["cell"][1:4])) > 0.0


def test_noalloc_step_reports_a_bad_state():
    """A cell with rho < 0: the CFL step refuses the state (dt = 0, status
    FISH_ERR_STATE), as fish_cfl_dt does for the context."""
    import paper_0910_2854_amd as fish
    n, bc = (16, 12, 10), (P, P, P)
    print(f"noalloc bad state shape {n}", flush=True)
    st = _state(n, bc, False, 31)
    st["cell"][0, 3, 4, 5] = -1.0
    out, rep = _noalloc_step(fish, n, bc, st, "fp64", 0.0)
    assert rep.status == fish.FISH_ERR_STATE
    assert rep.dt == 0.0 and rep.dt_next == 0.0
