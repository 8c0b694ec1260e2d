"""Work shapes change how cells are dealt to wavefronts, never what a cell
computes: every shape (positions per wave, segment length, block order, the
alternative layouts) gives bitwise the result of the default shapes."""
import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC

pytestmark = pytest.mark.gpu

FIELDS = ("cell", "bx", "by", "bz")

BOXES = [((40, 24, 20), (PERIODIC,) * 3, 1), ((33, 17, 9), (OUTFLOW,) * 3, 2), ((150, 6, 5), (PERIODIC,) * 3, 3),
         ((70, 66, 9), (PERIODIC, OUTFLOW, PERIODIC), 4),
         # rows long enough for the x field sweep's patches (sides 2 and 4, partial at the box edges)
         ((160, 14, 11), (PERIODIC, OUTFLOW, OUTFLOW), 5), ((200, 9, 7), (OUTFLOW, PERIODIC, PERIODIC), 6)]

# (x kinds: positions per wave, y/z kinds: segment length, xcd block order, alternative layout)
VARIANTS = [(256, 8, 1, 1), (3072, 256, 0, 1), (768, 24, 1, 0), (384, 64, 0, 1)]


def _run(n, bc, st, prec, variant, **kw):
    import paper_0910_2854_amd as fish
    g = fish.Box(*n, precision=prec, bc=bc, **kw)
    g.set_state(st)
    if variant is not None:
        xt, seg, remap, alt = variant
        # alt: the strided x fluid layout with the y/z segment length
        g.set_shape("fluid_x", seg if alt else xt, remap, alt)
        g.set_shape("field_x", xt, remap, alt)
        for kind in ("fluid_y", "fluid_z", "field_y", "field_z"):
            g.set_shape(kind, seg, remap, alt)
        g.set_shape("check", 16 if alt else 4, remap, alt)  # alt: CFL in the check kernel, not the last sweep
    for _ in range(2):
        g.strang_step(0.0)
    out = g.get_state()
    g.close()
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("box", BOXES, ids=lambda b: "x".join(map(str, b[0])))
def test_every_work_shape_gives_the_default_result_bitwise(prec, box):
    n, bc, seed = box
    print(f"shapes {n} {prec}", flush=True)
    st = fi.random_fourier_state(n, seed=seed, mach=0.7, beta=3.0, kmax=2)
    ref = _run(n, bc, st, prec, None)
    bad = []
    for v in VARIANTS:
        got = _run(n, bc, st, prec, v)
        for k in FIELDS:
            if not np.array_equal(got[k], ref[k]):
                bad.append((v, k, float(np.max(np.abs(got[k] - ref[k]))), int(np.sum(got[k] != ref[k]))))
    assert not bad, bad


def test_set_shape_rejects_bad_values():
    import paper_0910_2854_amd as fish
    print("set_shape arguments", flush=True)
    g = fish.Box(8, 8, 8)
    with pytest.raises(fish.FishError):
        g.set_shape("fluid_x", 0)
    with pytest.raises(fish.FishError):
        g.set_shape("fluid_x", 768, 0, 2)  # outside the encoding
    g.close()


@pytest.mark.parametrize("gravity", ["unsplit", "split"])
def test_strided_x_layout_with_gravity_and_hse_gives_the_default_result_bitwise(gravity):
    """The strided x fluid layout under both gravity forms with the
    hydrostatic correction, outflow boundaries, FP64 and FP32."""
    n, bc = (37, 22, 18), (OUTFLOW,) * 3
    st = fi.sphere_state(n, 5)
    for prec in ("fp64", "fp32"):
        print(f"strided x {gravity} {prec}", flush=True)
        ref = _run(n, bc, st, prec, None, gravity=gravity, hse=True)
        for v in VARIANTS:
            if not v[3]:
                continue
            got = _run(n, bc, st, prec, v, gravity=gravity, hse=True)
            for k in FIELDS:
                assert np.array_equal(got[k], ref[k]), (prec, v, k)
