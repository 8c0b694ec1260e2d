"""The largest boxes a context accepts: every array just below 4 GiB, so the
kernels' 32-bit byte offsets run up to their limit.  A box of 1024 x 1024 x
1023 cells in FP32 (and 1024 x 1024 x 511 in FP64) holds a uniform
magnetised state with a Gaussian blob near its far corner, where the
offsets are largest; a 128^3 box holds the same blob at its centre.  After
one double step of the same dt the blob's neighbourhood (half-width 40, wider
than the 16 cells a double step can reach from the blob's 12) must agree
bitwise between the two boxes: every cell is computed by the same operations
whatever its offset, and the uniform state elsewhere stays uniform.

The states are built on the device with torch and stepped through
fish_strang_step_noalloc, so no host copy of the 64 GiB of arrays is made."""
import numpy as np
import pytest

try:  # first torch import on a fresh machine is slow: keep it out of the timed tests
    import torch
except Exception:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0
B0 = (0.5, 0.3, 0.2)
R = 12          # half-width of the blob's cube
HALF = 40       # half-width of the compared region


def _state(shape, centre, dtype, dev):
    """Eight arrays (storage layout of a periodic box: shape (nz, ny, nx)) of
    a uniform state (rho 1, p 1, v 0, b = B0) with a Gaussian blob in rho, p
    and v_x (sigma 3 cells) inside the cube of half-width R at centre."""
    arrays = [torch.empty(shape, dtype=dtype, device=dev) for _ in range(8)]
    rho, mx, my, mz, E, bx, by, bz = arrays
    b2 = sum(b * b for b in B0)
    rho.fill_(1.0)
    for m in (mx, my, mz):
        m.fill_(0.0)
    E.fill_(1.0 / (GAMMA - 1.0) + 0.5 * b2)
    for f, b in zip((bx, by, bz), B0):
        f.fill_(b)
    r = torch.arange(-R, R + 1, dtype=torch.float64, device=dev)
    zz, yy, xx = torch.meshgrid(r, r, r, indexing="ij")
    g = torch.exp(-(xx * xx + yy * yy + zz * zz) / 18.0)
    rb = 1.0 + 0.5 * g
    pb = 1.0 + 2.0 * g
    vx = 0.3 * g
    cz, cy, cx = centre
    sl = (slice(cz - R, cz + R + 1), slice(cy - R, cy + R + 1), slice(cx - R, cx + R + 1))
    rho[sl] = rb.to(dtype)
    mx[sl] = (rb * vx).to(dtype)
    E[sl] = (pb / (GAMMA - 1.0) + 0.5 * rb * vx * vx + 0.5 * b2).to(dtype)
    return arrays


def _step(fish, shape, centre, precision, dt):
    dtype = torch.float32 if precision == "fp32" else torch.float64
    dev = torch.device("cuda", 0)
    nz, ny, nx = shape
    state = _state(shape, centre, dtype, dev)
    work = [torch.empty(shape, dtype=dtype, device=dev) for _ in range(8)]
    report = torch.zeros(3, dtype=torch.float64, device=dev)
    p = fish.make_params(nx, ny, nz, dx=1.0 / 128, dy=1.0 / 128, dz=1.0 / 128, precision=precision,
                         stream=torch.cuda.current_stream(dev).cuda_stream)
    fish.strang_step_noalloc(p, [t.data_ptr() for t in state], [t.data_ptr() for t in work], None, dt,
                             report.data_ptr())
    torch.cuda.synchronize(dev)
    rep = fish.StepReport.from_buffer_copy(report.cpu().numpy().tobytes())
    cz, cy, cx = centre
    sl = (slice(cz - HALF, cz + HALF + 1), slice(cy - HALF, cy + HALF + 1), slice(cx - HALF, cx + HALF + 1))
    region = [t[sl].cpu().numpy() for t in state]
    # far from the blob the state stays exactly uniform
    far = [float(t[0:4, 0:4, 0:4].max() - t[0:4, 0:4, 0:4].min()) for t in state]
    del state, work
    torch.cuda.empty_cache()
    return region, rep, far


@pytest.mark.parametrize("precision,shape", [("fp32", (1023, 1024, 1024)), ("fp64", (511, 1024, 1024))])
def test_largest_box_agrees_bitwise_with_a_small_box(precision, shape):
    import paper_0910_2854_amd as fish
    esize = 4 if precision == "fp32" else 8
    nz, ny, nx = shape
    assert nz * ny * nx * esize < 2 ** 32 <= (nz + 1) * ny * nx * esize  # the largest such box
    dt = 2e-3
    print(f"max-size box {shape} {precision}: far corner", flush=True)
    big, rep_big, far = _step(fish, shape, (nz - 60, ny - 60, nx - 60), precision, dt)
    print(f"  128^3 box with the same blob", flush=True)
    small, rep_small, _ = _step(fish, (128, 128, 128), (64, 64, 64), precision, dt)
    assert rep_big.status == fish.FISH_OK and rep_small.status == fish.FISH_OK
    assert rep_big.dt == rep_small.dt == dt
    assert rep_big.dt_next == rep_small.dt_next  # the same cells set the CFL speed
    assert all(f == 0.0 for f in far), far
    for k, (a, b) in enumerate(zip(big, small)):
        np.testing.assert_array_equal(a, b, err_msg=f"array {k}")
    # the step moved the blob
    assert float(np.max(np.abs(small[1]))) > 0.0
