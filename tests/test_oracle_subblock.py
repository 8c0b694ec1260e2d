"""The sub-block method of the full-size sphere check, on the oracle alone:
a block cut out of a box, stepped with outflow edges and the box's dt, equals
the whole box's step on the block's core (cells farther than the double
step's dependency radius from every cut side)."""
import numpy as np

import fish_inputs as fi
from oracle import OUTFLOW, Oracle

from test_gpu_sphere512 import RADIUS, _block


def test_block_core_equals_full_box_step():
    n, blk = 80, 56
    st = fi.sphere_state(n, seed=3)
    full = Oracle(n, n, n, bc=(OUTFLOW,) * 3, gravity=True, hse=True)
    full.set_state(st)
    dt = full.cfl_dt()
    full.strang_step(dt)
    ref = full.get_state()
    for lo in ((12, 12, 12), (0, 24, 0), (n - blk, n - blk, 10)):
        hi = tuple(o + blk for o in lo)
        o = Oracle(blk, blk, blk, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n, bc=(OUTFLOW,) * 3, gravity=True, hse=True)
        o.set_state(_block(st, lo, hi))
        o.strang_step(dt)
        got = o.get_state()
        want = _block(ref, lo, hi)
        core = [slice(0 if lo[a] == 0 else RADIUS, blk if hi[a] == n else blk - RADIUS) for a in range(3)]
        sx, sy, sz = core
        assert np.array_equal(got["cell"][:, sz, sy, sx], want["cell"][:, sz, sy, sx]), lo
        assert np.array_equal(got["bx"][sz, sy, sx], want["bx"][sz, sy, sx]), lo
        assert np.array_equal(got["by"][sz, sy, sx], want["by"][sz, sy, sx]), lo
        assert np.array_equal(got["bz"][sz, sy, sx], want["bz"][sz, sy, sx]), lo
        # the cut is felt within ten cells (the structural radius is a bound;
        # here the reach is 12 cells), so the comparison is not vacuous
        shrunk = [slice(0 if lo[a] == 0 else 10, blk if hi[a] == n else blk - 10) for a in range(3)]
        tx, ty, tz = shrunk
        assert not np.array_equal(got["cell"][:, tz, ty, tx], want["cell"][:, tz, ty, tx]), lo
