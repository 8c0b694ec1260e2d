"""GPU batches: many boxes of different shapes advanced by one launch per
sub-operator, each with its own CFL step.

A box must give bitwise the same result in a batch as alone (same
precision): boxes never interact and every cell is computed by the same
operations whatever wavefront computes it.  In FP64 the batch also matches the
oracle stepped with the same per-box CFL steps (per-field relative L1 1e-10).
"""
import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC, Oracle

pytestmark = pytest.mark.gpu

FIELDS = ("cell", "bx", "by", "bz")

# (shape, bc, seed): ragged shapes, single-segment and multi-segment pencils,
# outflow and periodic axes, inactive axes
BOXES = [
    ((16, 16, 16), (PERIODIC,) * 3, 1),
    ((24, 20, 12), (PERIODIC,) * 3, 2),
    ((9, 70, 5), (PERIODIC,) * 3, 3),
    ((11, 7, 6), (OUTFLOW,) * 3, 4),
    ((33, 1, 1), (PERIODIC,) * 3, 5),
    ((6, 5, 131), (PERIODIC, OUTFLOW, PERIODIC), 6),
    ((130, 3, 4), (PERIODIC,) * 3, 7),
]


def _state(n, seed):
    return fi.random_fourier_state(n, seed=seed, mach=0.8, beta=2.0, kmax=2)


def _batch(prec, nbox_bytes=256 << 20, **kw):
    import paper_0910_2854_amd as fish
    return fish.Batch(nbox_bytes, max_boxes=64, precision=prec, **kw)


def _alone(n, bc, st, prec, steps):
    import paper_0910_2854_amd as fish
    g = fish.Box(*n, precision=prec, bc=bc)
    g.set_state(st)
    for _ in range(steps):
        g.strang_step(0.0)
    out = g.get_state()
    g.close()
    return out


def rel_l1(a, b):
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / den) if den > 0 else float(np.sum(np.abs(a - b)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_each_box_alone_bitwise(prec):
    print(f"batch of {len(BOXES)} boxes vs alone, {prec}", flush=True)
    steps = 4
    b = _batch(prec)
    ids = []
    for n, bc, seed in BOXES:
        ids.append(b.add(_state(n, seed), bc=bc))
    b.step(steps)
    for (n, bc, seed), i in zip(BOXES, ids):
        got = b.get(i)
        ref = _alone(n, bc, _state(n, seed), prec, steps)
        for k in FIELDS:
            assert np.array_equal(got[k], ref[k]), (n, k)
        assert got["t"] == ref["t"]
    b.close()


def test_batch_fp64_matches_oracle_with_per_box_cfl():
    print("batch fp64 vs oracle, 3 boxes x 5 steps", flush=True)
    steps = 5
    sel = [BOXES[1], BOXES[3], BOXES[5]]
    b = _batch("fp64")
    ids = [b.add(_state(n, seed), bc=bc) for n, bc, seed in sel]
    b.step(steps)
    for (n, bc, seed), i in zip(sel, ids):
        o = Oracle(*n, bc=bc)
        o.set_state(_state(n, seed))
        for _ in range(steps):
            o.strang_step(0.0)
        ref = o.get_state()
        got = b.get(i)
        for k in FIELDS:
            assert rel_l1(got[k], ref[k]) <= 1e-10, (n, k)
        assert abs(got["t"] - ref["t"]) <= 1e-12 * ref["t"]
    b.close()


def test_batch_per_box_dt_differs_and_matches_the_cfl_step():
    print("per-box dt", flush=True)
    b = _batch("fp64")
    n = (16, 12, 10)
    slow = fi.random_fourier_state(n, seed=3, mach=0.3, beta=10.0, kmax=2)
    fast = fi.random_fourier_state(n, seed=4, mach=2.0, beta=0.5, kmax=2)
    i0, i1 = b.add(slow), b.add(fast)
    b.step(1)
    d0, d1 = b.info(i0)["dt"], b.info(i1)["dt"]
    o0, o1 = Oracle(*n), Oracle(*n)
    o0.set_state(slow)
    o1.set_state(fast)
    assert abs(d0 - o0.cfl_dt()) <= 1e-13 * d0
    assert abs(d1 - o1.cfl_dt()) <= 1e-13 * d1
    assert d0 > 1.5 * d1
    b.close()


def test_batch_graph_replays_match_eager_steps():
    """Replays of the captured step, with eager work and synchronisation
    between them, give the eager result after every replay."""
    print("graph vs eager, fp32, 3 boxes x 4 steps", flush=True)
    sel = BOXES[:3]
    be, bg = _batch("fp32"), _batch("fp32")
    ie = [be.add(_state(n, seed), bc=bc) for n, bc, seed in sel]
    ig = [bg.add(_state(n, seed), bc=bc) for n, bc, seed in sel]
    bg.use_graph(True)
    for s in range(4):
        be.step(1)
        bg.step(1)
        bg.sync()
        _ = torch.zeros(1024, device="cuda").sum().item()  # unrelated eager work in between
        for a, c in zip(ie, ig):
            ge, gg = be.get(a), bg.get(c)
            for k in FIELDS:
                assert np.array_equal(ge[k], gg[k]), (s, k)
    be.close()
    bg.close()


def test_batch_remove_and_add_keep_other_boxes_exact():
    print("remove/add mid-run", flush=True)
    prec = "fp32"
    b = _batch(prec)
    (n0, bc0, s0), (n1, bc1, s1), (n2, bc2, s2) = BOXES[0], BOXES[1], BOXES[3]
    i0 = b.add(_state(n0, s0), bc=bc0)
    i1 = b.add(_state(n1, s1), bc=bc1)
    b.step(2)
    b.remove(i1)
    i2 = b.add(_state(n2, s2), bc=bc2)   # reuses the freed range
    b.step(3)
    ref0 = _alone(n0, bc0, _state(n0, s0), prec, 5)
    ref2 = _alone(n2, bc2, _state(n2, s2), prec, 3)
    g0, g2 = b.get(i0), b.get(i2)
    for k in FIELDS:
        assert np.array_equal(g0[k], ref0[k]), k
        assert np.array_equal(g2[k], ref2[k]), k
    assert len(b) == 2
    b.close()


def test_batch_autotune_keeps_results_bitwise():
    print("autotune", flush=True)
    prec = "fp32"
    sel = BOXES[:4]
    b = _batch(prec)
    ids = [b.add(_state(n, seed), bc=bc) for n, bc, seed in sel]
    chosen = b.autotune(reps=2)
    assert set(chosen) >= {"fluid_x", "field_z"}
    b.step(3)
    for (n, bc, seed), i in zip(sel, ids):
        ref = _alone(n, bc, _state(n, seed), prec, 3)
        got = b.get(i)
        for k in FIELDS:
            assert np.array_equal(got[k], ref[k]), (n, k)
    b.close()


def test_batch_admission_refuses_when_pool_is_full():
    import paper_0910_2854_amd as fish
    print("pool admission", flush=True)
    n = (16, 16, 16)
    need = fish.box_pool_bytes(n, "fp32")
    b = _batch("fp32", nbox_bytes=3 * need + need // 2)
    ids = [b.add(_state(n, k)) for k in range(3)]
    with pytest.raises(fish.FishError) as e:
        b.add(_state(n, 9))
    assert e.value.code == fish.FISH_ERR_NOMEM
    assert len(b) == 3
    b.remove(ids[1])
    ids[1] = b.add(_state(n, 9))
    assert len(b) == 3
    b.close()


def test_batch_rejects_a_bad_box_and_keeps_the_rest():
    import paper_0910_2854_amd as fish
    print("bad box", flush=True)
    b = _batch("fp64")
    n = (12, 12, 12)
    good = fi.random_fourier_state(n, seed=1, mach=0.5, beta=10.0, kmax=2)
    i0 = b.add(good)
    bad = fi.uniform_state(n, p=0.5)
    bad["cell"][4, 1, 2, 3] = -1.0
    with pytest.raises(fish.FishError) as e:
        b.add(bad)
    assert e.value.code == fish.FISH_ERR_STATE
    assert len(b) == 1
    b.step(2)
    ref = _alone(n, (PERIODIC,) * 3, good, "fp64", 2)
    got = b.get(i0)
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    b.close()


def test_empty_batch_and_server():
    import paper_0910_2854_amd as fish
    print("empty batch and server", flush=True)
    b = _batch("fp32")
    b.step(3)  # no boxes: nothing to do
    b.sync()
    assert len(b) == 0
    with pytest.raises(fish.FishError):
        b.autotune(reps=1)  # nothing to tune on
    b.close()
    srv = fish.Server(16 << 20, precision="fp32")
    assert srv.pump() == []
    assert srv.stats()["resident"] == 0
    srv.close()


@pytest.mark.parametrize("mode", ["split_gravity_hse", "limiter_switch"])
def test_batch_modes_match_each_box_alone_bitwise(mode):
    """The gravity forms and the limiter switch run through the batch engine
    too: each box of a batch gives bitwise what it gives alone (FP32)."""
    import paper_0910_2854_amd as fish
    print(f"batch {mode} vs alone fp32", flush=True)
    if mode == "split_gravity_hse":
        kw = dict(gravity="split", hse=True)
        boxes = [((16, 16, 16), (OUTFLOW,) * 3, 11), ((20, 12, 10), (OUTFLOW,) * 3, 12),
                 ((9, 30, 7), (OUTFLOW, PERIODIC, OUTFLOW), 13)]
        make = lambda n, seed: fi.sphere_state(n, seed)  # noqa: E731
    else:
        kw = dict(limiter=fish.MACH_SWITCH)
        boxes = [((16, 16, 16), (PERIODIC,) * 3, 14), ((24, 10, 12), (OUTFLOW,) * 3, 15)]
        make = lambda n, seed: fi.random_fourier_state(n, seed=seed, mach=1.0, beta=2.0, kmax=2)  # noqa: E731
    steps = 3
    b = _batch("fp32", **kw)
    ids = [b.add(make(n, seed), bc=bc) for n, bc, seed in boxes]
    b.step(steps)
    for (n, bc, seed), i in zip(boxes, ids):
        got = b.get(i)
        g = fish.Box(*n, precision="fp32", bc=bc, **kw)
        g.set_state(make(n, seed))
        for _ in range(steps):
            g.strang_step(0.0)
        ref = g.get_state()
        g.close()
        for k in FIELDS:
            assert np.array_equal(got[k], ref[k]), (mode, n, k)
    b.close()
