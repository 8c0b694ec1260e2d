"""Python binding of libfish.so, the MI355X (gfx950) FISH split-MHD step.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``csrc/``.  There is no CPU fallback -- importing the binding
without the built library raises.  PyTorch supplies device memory (its
caching allocator, through the allocator callbacks of ``fish_params``) and
the stream the work is enqueued on.

State dictionaries use the layout of ``include/fish.h`` (FP64 host arrays):
``cell`` (5, nz, ny, nx), ``bx`` (nz, ny, nx+1), ``by`` (nz, ny+1, nx),
``bz`` (nz+1, ny, nx), ``phi`` (nz, ny, nx) or None.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfish.so")

FISH_OK, FISH_ERR_ARG, FISH_ERR_NOMEM, FISH_ERR_DEVICE, FISH_ERR_STATE, FISH_ERR_UNSUPPORTED = range(6)
PERIODIC, OUTFLOW = 0, 1
MINMOD, VANLEER, MACH_SWITCH = 0, 1, 2
FP64, FP32 = 0, 1

_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("predictor_alpha", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32),
        ("gravity", ctypes.c_int32), ("hse", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("alloc", _ALLOC), ("free", _FREE),
        ("alloc_user", ctypes.c_void_p),
    ]


class StepReport(ctypes.Structure):
    """fish_step_report: what fish_strang_step_noalloc writes to device memory."""
    _fields_ = [("dt", ctypes.c_double), ("dt_next", ctypes.c_double),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


NOALLOC_MAX_WAVES = 1 << 20


class FishError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fish error {code}: {msg}")
        self.code = code


class BatchParams(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("predictor_alpha", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("gravity", ctypes.c_int32), ("hse", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("pool_bytes", ctypes.c_size_t),
        ("max_boxes", ctypes.c_int32),
        ("alloc", _ALLOC), ("free", _FREE),
        ("alloc_user", ctypes.c_void_p),
    ]


class BoxGeom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("box", BoxGeom),
        ("nsteps", ctypes.c_int32),
        ("cell5", ctypes.POINTER(ctypes.c_double)), ("bx", ctypes.POINTER(ctypes.c_double)),
        ("by", ctypes.POINTER(ctypes.c_double)), ("bz", ctypes.POINTER(ctypes.c_double)),
        ("phi", ctypes.POINTER(ctypes.c_double)),
        ("out_cell5", ctypes.POINTER(ctypes.c_double)), ("out_bx", ctypes.POINTER(ctypes.c_double)),
        ("out_by", ctypes.POINTER(ctypes.c_double)), ("out_bz", ctypes.POINTER(ctypes.c_double)),
        ("tag", ctypes.c_int64),
        ("widths", ctypes.POINTER(ctypes.c_double) * 3),
    ]


EXPORTS = ("fish_create", "fish_destroy", "fish_last_error", "fish_set_state", "fish_get_state",
           "fish_cfl_dt", "fish_strang_step", "fish_sweep", "fish_diagnostics", "fish_device_bytes",
           "fish_timing_enable", "fish_timing_read", "fish_selftest_lane_shift", "fish_selftest_math", "fish_autotune",
           "fish_box_pool_bytes", "fish_batch_create", "fish_batch_destroy", "fish_batch_last_error",
           "fish_batch_device_bytes", "fish_batch_free_bytes", "fish_batch_count", "fish_batch_add",
           "fish_batch_remove", "fish_batch_get", "fish_batch_box_info", "fish_batch_box_steps", "fish_batch_step",
           "fish_batch_use_graph", "fish_batch_autotune", "fish_batch_sync", "fish_batch_timing_enable",
           "fish_batch_timing_read", "fish_set_shape", "fish_batch_set_shape", "fish_server_create", "fish_server_destroy", "fish_server_last_error",
           "fish_server_batch", "fish_server_submit", "fish_server_pump", "fish_server_stats", "fish_set_spacing",
           "fish_advance_to", "fish_batch_set_spacing", "fish_strang_step_noalloc")
KERNEL_FLUID, KERNEL_FIELD, KERNEL_CHECK = 1, 2, 8
KINDS = ("fluid_x", "fluid_y", "fluid_z", "field_x", "field_y", "field_z", "check")

GRAVITY_MODES = {"none": 0, "unsplit": 1, "split": 2}


def gravity_mode(gravity):
    """False/"none": 0; True/"unsplit": 1 (Eqs. 41-43); "split": 2 (Eqs. 38-40)."""
    if isinstance(gravity, str):
        return GRAVITY_MODES[gravity]
    return int(gravity)


_lib = None


def hip_runtimes_loaded():
    """Resolved paths of the HIP runtimes (libamdhip64) mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                    paths.add(os.path.realpath(parts[-1]))
    except OSError:  # pragma: no cover - not Linux
        pass
    return sorted(paths)


def load_library(path: str = LIB_PATH):
    """Load libfish.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch first.  Its wheel ships a HIP runtime of its own (torch/lib/
    # libamdhip64.so, SONAME libamdhip64.so.7, which its libraries request
    # under the unversioned name through their RPATH).  The library requests
    # the SONAME libamdhip64.so.7, so with PyTorch loaded the dynamic linker
    # binds it to PyTorch's runtime, the one that owns the caching allocator's
    # memory and the streams handed to it.  Loaded before PyTorch, it would
    # bind the system runtime and PyTorch would then map a second copy.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - the library still runs with hipMalloc and raw streams
        pass
    lib = ctypes.CDLL(path)
    runtimes = hip_runtimes_loaded()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are loaded in this process (" + ", ".join(runtimes) + "); "
                          "libfish.so was loaded before PyTorch: import torch (or this package) first")
    P, d, vp = ctypes.POINTER, ctypes.c_double, ctypes.c_void_p
    lib.fish_create.argtypes = [P(Params), P(vp)]
    lib.fish_destroy.argtypes = [vp]
    lib.fish_destroy.restype = None
    lib.fish_last_error.argtypes = [vp]
    lib.fish_last_error.restype = ctypes.c_char_p
    lib.fish_set_state.argtypes = [vp, P(d), P(d), P(d), P(d), P(d)]
    lib.fish_get_state.argtypes = [vp, P(d), P(d), P(d), P(d), P(d)]
    lib.fish_cfl_dt.argtypes = [vp, P(d)]
    lib.fish_strang_step.argtypes = [vp, d]
    lib.fish_sweep.argtypes = [vp, ctypes.c_int, ctypes.c_int, d]
    lib.fish_diagnostics.argtypes = [vp, P(d)]
    lib.fish_device_bytes.argtypes = [vp]
    lib.fish_device_bytes.restype = ctypes.c_size_t
    lib.fish_timing_enable.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.fish_timing_read.argtypes = [vp, P(ctypes.c_int), P(d)]
    lib.fish_selftest_lane_shift.argtypes = [ctypes.c_int, P(ctypes.c_float)]
    lib.fish_selftest_lane_shift.restype = ctypes.c_int
    lib.fish_selftest_math.argtypes = [ctypes.c_int, ctypes.c_int, P(d), P(d), P(d)]
    lib.fish_selftest_math.restype = ctypes.c_int
    i32p = P(ctypes.c_int32)
    lib.fish_autotune.argtypes = [vp, ctypes.c_int, i32p]
    lib.fish_box_pool_bytes.argtypes = [P(BoxGeom), ctypes.c_int, ctypes.c_int]
    lib.fish_box_pool_bytes.restype = ctypes.c_size_t
    lib.fish_batch_create.argtypes = [P(BatchParams), P(vp)]
    lib.fish_batch_destroy.argtypes = [vp]
    lib.fish_batch_destroy.restype = None
    lib.fish_batch_last_error.argtypes = [vp]
    lib.fish_batch_last_error.restype = ctypes.c_char_p
    lib.fish_batch_device_bytes.argtypes = [vp]
    lib.fish_batch_device_bytes.restype = ctypes.c_size_t
    lib.fish_batch_free_bytes.argtypes = [vp]
    lib.fish_batch_free_bytes.restype = ctypes.c_size_t
    lib.fish_batch_count.argtypes = [vp]
    lib.fish_batch_add.argtypes = [vp, P(BoxGeom), P(d), P(d), P(d), P(d), P(d), P(ctypes.c_int)]
    lib.fish_batch_remove.argtypes = [vp, ctypes.c_int]
    lib.fish_batch_get.argtypes = [vp, ctypes.c_int, P(d), P(d), P(d), P(d), P(d)]
    lib.fish_batch_box_info.argtypes = [vp, ctypes.c_int, P(d), P(d), P(ctypes.c_int)]
    lib.fish_batch_box_steps.argtypes = [vp, ctypes.c_int, P(ctypes.c_int)]
    lib.fish_batch_step.argtypes = [vp, ctypes.c_int]
    lib.fish_batch_use_graph.argtypes = [vp, ctypes.c_int]
    lib.fish_batch_autotune.argtypes = [vp, ctypes.c_int, i32p]
    lib.fish_batch_sync.argtypes = [vp]
    lib.fish_batch_timing_enable.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.fish_batch_timing_read.argtypes = [vp, P(ctypes.c_int), P(d)]
    lib.fish_set_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int32]
    lib.fish_set_spacing.argtypes = [vp, ctypes.c_int, P(ctypes.c_double)]
    lib.fish_advance_to.argtypes = [vp, d, ctypes.c_int, P(ctypes.c_int), P(d)]
    lib.fish_strang_step_noalloc.argtypes = [P(Params), P(vp), P(vp), vp, d, vp]
    lib.fish_strang_step_noalloc.restype = ctypes.c_int
    lib.fish_set_spacing.restype = ctypes.c_int
    lib.fish_batch_set_spacing.argtypes = [vp, ctypes.c_int, ctypes.c_int, P(ctypes.c_double)]
    lib.fish_batch_set_spacing.restype = ctypes.c_int
    lib.fish_batch_set_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int32]
    lib.fish_set_shape.restype = ctypes.c_int
    lib.fish_batch_set_shape.restype = ctypes.c_int
    lib.fish_server_create.argtypes = [P(BatchParams), ctypes.c_int, P(vp)]
    lib.fish_server_destroy.argtypes = [vp]
    lib.fish_server_destroy.restype = None
    lib.fish_server_last_error.argtypes = [vp]
    lib.fish_server_last_error.restype = ctypes.c_char_p
    lib.fish_server_batch.argtypes = [vp]
    lib.fish_server_batch.restype = vp
    lib.fish_server_submit.argtypes = [vp, P(Request)]
    lib.fish_server_pump.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int32), ctypes.c_int, P(ctypes.c_int)]
    lib.fish_server_stats.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_size_t), P(ctypes.c_int64)]
    for name in ("fish_server_create", "fish_server_submit", "fish_server_pump", "fish_server_stats"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("fish_create", "fish_set_state", "fish_get_state", "fish_cfl_dt", "fish_strang_step",
                 "fish_sweep", "fish_diagnostics", "fish_timing_enable", "fish_timing_read", "fish_autotune",
                 "fish_batch_create", "fish_batch_count", "fish_batch_add", "fish_batch_remove", "fish_batch_get",
                 "fish_batch_box_info", "fish_batch_box_steps", "fish_batch_step", "fish_batch_use_graph",
                 "fish_batch_autotune",
                 "fish_batch_sync", "fish_batch_timing_enable", "fish_batch_timing_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def storage_shape(n, bc):
    """(nz+oz, ny+oy, nx+ox): the shape of every array of a box in the storage
    layout (o_d = 1 on an outflow axis, 0 on a periodic one)."""
    nx, ny, nz = n
    return (nz + int(bc[2] == OUTFLOW), ny + int(bc[1] == OUTFLOW), nx + int(bc[0] == OUTFLOW))


def to_storage(st, n, bc, dtype):
    """The eight arrays rho, m_x, m_y, m_z, E, b_x, b_y, b_z (and phi, or
    None) of a state in the interface layout, in the storage layout and
    precision of fish_strang_step_noalloc (zeros outside each array's
    extent; face n of a periodic axis dropped)."""
    nx, ny, nz = n
    ox, oy, oz = (int(b == OUTFLOW) for b in bc)
    shape = storage_shape(n, bc)
    out = []
    for k in range(5):
        a = np.zeros(shape, dtype=dtype)
        a[:nz, :ny, :nx] = st["cell"][k]
        out.append(a)
    a = np.zeros(shape, dtype=dtype)
    a[:nz, :ny, :nx + ox] = st["bx"][:, :, :nx + ox]
    out.append(a)
    a = np.zeros(shape, dtype=dtype)
    a[:nz, :ny + oy, :nx] = st["by"][:, :ny + oy, :]
    out.append(a)
    a = np.zeros(shape, dtype=dtype)
    a[:nz + oz, :ny, :nx] = st["bz"][:nz + oz]
    out.append(a)
    phi = None
    if st.get("phi") is not None:
        phi = np.zeros(shape, dtype=dtype)
        phi[:nz, :ny, :nx] = st["phi"]
    return out, phi


def from_storage(arrays, n, bc):
    """The state (interface layout, FP64) of eight storage-layout arrays; on
    a periodic axis face n is written equal to face 0."""
    nx, ny, nz = n
    ox, oy, oz = (int(b == OUTFLOW) for b in bc)
    a = [np.asarray(x, dtype=np.float64) for x in arrays]
    cell = np.stack([a[k][:nz, :ny, :nx] for k in range(5)])
    bx = a[5][:nz, :ny, :nx + ox]
    by = a[6][:nz, :ny + oy, :nx]
    bz = a[7][:nz + oz, :ny, :nx]
    if not ox:
        bx = np.concatenate([bx, bx[:, :, :1]], axis=2)
    if not oy:
        by = np.concatenate([by, by[:, :1, :]], axis=1)
    if not oz:
        bz = np.concatenate([bz, bz[:1]], axis=0)
    return {"cell": np.ascontiguousarray(cell), "bx": np.ascontiguousarray(bx), "by": np.ascontiguousarray(by),
            "bz": np.ascontiguousarray(bz)}


def strang_step_noalloc(params, state, work, phi=None, dt=0.0, report=None):
    """fish_strang_step_noalloc: one double step on device arrays in the
    storage layout (params: a Params; state, work: 8 device addresses each;
    phi: a device address or None; report: the device address of a
    StepReport, or None).  Enqueued on params.stream; raises FishError."""
    lib = load_library()
    vp = ctypes.c_void_p
    st = (vp * 8)(*[int(a) for a in state])
    wk = (vp * 8)(*[int(a) for a in work])
    rc = lib.fish_strang_step_noalloc(ctypes.byref(params), st, wk, vp(int(phi)) if phi else None, float(dt),
                                      vp(int(report)) if report else None)
    if rc != FISH_OK:
        raise FishError(rc, lib.fish_last_error(None).decode())


def selftest_lane_shift(device=0):
    """Run the lane-shift self-test kernel; returns the 128 output values."""
    lib = load_library()
    out = np.zeros(128, dtype=np.float32)
    rc = lib.fish_selftest_lane_shift(int(device), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != FISH_OK:
        raise FishError(rc, "lane-shift self-test failed to run")
    return out


def selftest_math(x, device=0):
    """Run the FP64 reciprocal/square-root self-test kernel on the values x;
    returns (1/x, sqrt(x)) as the FP64 sweeps compute them."""
    lib = load_library()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    r = np.empty_like(x)
    s = np.empty_like(x)
    rc = lib.fish_selftest_math(int(device), int(x.size), _dptr(x), _dptr(r), _dptr(s))
    if rc != FISH_OK:
        raise FishError(rc, "FP64 math self-test failed to run")
    return r, s


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _TorchAllocator:
    """Device memory from torch's caching allocator, handed to libfish."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device

        def alloc(nbytes, stream, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream))
            except Exception:
                return None

        def free(ptr, nbytes, stream, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch is gone, the process frees the memory
                pass

        self.alloc = _ALLOC(alloc)
        self.free = _FREE(free)


def make_params(nx, ny, nz, dx=None, dy=None, dz=None, gamma=5.0 / 3.0, cfl=0.5, limiter=VANLEER,
                predictor_alpha=1.0, bc=(PERIODIC,) * 3, precision="fp64", gravity=False, hse=False, device=0,
                stream=None):
    """A fish_params (spacing 1/n per axis unless given; no allocator)."""
    p = Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.dx = 1.0 / nx if dx is None else float(dx)
    p.dy = 1.0 / ny if dy is None else float(dy)
    p.dz = 1.0 / nz if dz is None else float(dz)
    p.gamma, p.cfl = float(gamma), float(cfl)
    p.limiter = int(limiter)
    p.predictor_alpha = float(predictor_alpha)
    for a in range(3):
        p.bc[a] = int(bc[a])
    p.precision = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
    p.gravity, p.hse = gravity_mode(gravity), int(bool(hse))
    p.device = int(device)
    p.stream = ctypes.c_void_p(int(stream)) if stream else None
    return p


class Box:
    """One box advanced by the HIP library on one GPU stream."""

    def __init__(self, nx, ny, nz, dx=None, dy=None, dz=None, gamma=5.0 / 3.0, cfl=0.5, limiter=VANLEER,
                 predictor_alpha=1.0, bc=(PERIODIC,) * 3, precision="fp64", gravity=False, hse=False,
                 device=0, stream=None, use_torch_allocator=True):
        lib = load_library()
        self._lib = lib
        self.shape = (int(nz), int(ny), int(nx))
        p = make_params(nx, ny, nz, dx, dy, dz, gamma, cfl, limiter, predictor_alpha, bc, precision, gravity, hse,
                        device)
        self._allocator = None
        if stream is None or use_torch_allocator:
            import torch
            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
            if use_torch_allocator:
                self._allocator = _TorchAllocator(device)
                p.alloc, p.free = self._allocator.alloc, self._allocator.free
        p.stream = ctypes.c_void_p(int(stream)) if stream else None
        self.params = p
        h = ctypes.c_void_p()
        rc = lib.fish_create(ctypes.byref(p), ctypes.byref(h))
        if rc != FISH_OK:
            raise FishError(rc, "fish_create failed: " + lib.fish_last_error(None).decode())
        self._h = h

    # ---------------------------------------------------------------- helpers
    def _check(self, rc):
        if rc != FISH_OK:
            raise FishError(rc, self._lib.fish_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fish_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self):
        return int(self._lib.fish_device_bytes(self._h))

    # ------------------------------------------------------------------ calls
    def set_state(self, st):
        nz, ny, nx = self.shape
        cell = np.ascontiguousarray(st["cell"], dtype=np.float64)
        bx = np.ascontiguousarray(st["bx"], dtype=np.float64)
        by = np.ascontiguousarray(st["by"], dtype=np.float64)
        bz = np.ascontiguousarray(st["bz"], dtype=np.float64)
        if cell.shape != (5, nz, ny, nx) or bx.shape != (nz, ny, nx + 1) or by.shape != (nz, ny + 1, nx) \
                or bz.shape != (nz + 1, ny, nx):
            raise ValueError("state arrays do not match the box shape")
        phi = st.get("phi")
        if phi is not None:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
            if phi.shape != (nz, ny, nx):
                raise ValueError("phi does not match the box shape")
        self._check(self._lib.fish_set_state(self._h, _dptr(cell), _dptr(bx), _dptr(by), _dptr(bz), _dptr(phi)))

    def get_state(self, check=True):
        nz, ny, nx = self.shape
        cell = np.empty((5, nz, ny, nx))
        bx = np.empty((nz, ny, nx + 1))
        by = np.empty((nz, ny + 1, nx))
        bz = np.empty((nz + 1, ny, nx))
        t = ctypes.c_double()
        rc = self._lib.fish_get_state(self._h, _dptr(cell), _dptr(bx), _dptr(by), _dptr(bz), ctypes.byref(t))
        if check:
            self._check(rc)
        return {"cell": cell, "bx": bx, "by": by, "bz": bz, "t": t.value, "status": rc}

    def cfl_dt(self):
        dt = ctypes.c_double()
        self._check(self._lib.fish_cfl_dt(self._h, ctypes.byref(dt)))
        return dt.value

    def strang_step(self, dt=0.0):
        self._check(self._lib.fish_strang_step(self._h, float(dt)))

    def sweep(self, op, direction, dt):
        """One sub-operator: op 'L' (fluid) or 'B' (field), direction 0/1/2."""
        code = {"L": 0, "B": 1}[op] if isinstance(op, str) else int(op)
        self._check(self._lib.fish_sweep(self._h, code, int(direction), float(dt)))

    def timing_enable(self, mask, max_launches=4096):
        """Record hipEvents around launches of the kernel classes in mask."""
        self._check(self._lib.fish_timing_enable(self._h, int(mask), int(max_launches)))

    def timing_read(self):
        """(launches, total milliseconds) recorded since the last read."""
        n = ctypes.c_int()
        ms = ctypes.c_double()
        self._check(self._lib.fish_timing_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def diagnostics(self):
        out = np.zeros(10)
        self._check(self._lib.fish_diagnostics(self._h, _dptr(out)))
        return _diag_dict(out)

    def advance_to(self, t_end, max_steps=1 << 30):
        """CFL-stepped double steps to time t_end, device-resident; returns
        (double steps taken, time reached)."""
        n = ctypes.c_int()
        t = ctypes.c_double()
        self._check(self._lib.fish_advance_to(self._h, float(t_end), int(max_steps), ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value

    def set_spacing(self, axis, widths):
        """Irregular mesh (Sect. 2.5): the widths of the cells along axis."""
        w = np.ascontiguousarray(widths, dtype=np.float64)
        if w.shape != (self.shape[2 - axis],):
            raise ValueError("one width per cell along the axis")
        self._check(self._lib.fish_set_spacing(self._h, int(axis), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def set_shape(self, kind, target, xcd_remap=0, alt_layout=0):
        """Set one kind's work shape (kind: a name of KINDS)."""
        self._check(self._lib.fish_set_shape(self._h, KINDS.index(kind), shape_value(target, xcd_remap, alt_layout)))

    def autotune(self, reps=3):
        """Pick the fastest work shape of every sweep kind; returns {kind: target}."""
        t = (ctypes.c_int32 * 7)()
        self._check(self._lib.fish_autotune(self._h, int(reps), t))
        return _tuned(t)


def _tuned(t):
    """{kind: {"target": shape, "xcd_remap": 0/1, "alt_layout": 0/1}} from the autotuner's output."""
    return {k: {"target": int(v) & 0xFFFF, "xcd_remap": (int(v) >> 16) & 1, "alt_layout": (int(v) >> 17) & 1}
            for k, v in zip(KINDS, list(t))}


def shape_value(target, xcd_remap=0, alt_layout=0):
    """Encode a work shape for set_shape."""
    return int(target) | (int(xcd_remap) << 16) | (int(alt_layout) << 17)


def _diag_dict(out):
    return {"mass": out[0], "mom": out[1:4].copy(), "energy": out[4], "flux": out[5:8].copy(),
            "divb_max": out[8], "bmax": out[9]}


def _geom(n, h=None, cfl=0.5, bc=(PERIODIC,) * 3):
    nx, ny, nz = (int(v) for v in n)
    g = BoxGeom()
    g.nx, g.ny, g.nz = nx, ny, nz
    if h is None:
        h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    g.dx, g.dy, g.dz = (float(v) for v in h)
    g.cfl = float(cfl)
    for a in range(3):
        g.bc[a] = int(bc[a])
    return g


def box_pool_bytes(n, precision="fp32", gravity=False, bc=(PERIODIC,) * 3):
    """Device bytes one box (nx, ny, nz) takes in a batch."""
    lib = load_library()
    prec = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
    return int(lib.fish_box_pool_bytes(ctypes.byref(_geom(n, bc=bc)), prec, gravity_mode(gravity)))


def _batch_params(owner, pool_bytes, max_boxes, gamma, limiter, predictor_alpha, precision, gravity, hse, device,
                  stream, use_torch_allocator):
    p = BatchParams()
    p.gamma = float(gamma)
    p.limiter = int(limiter)
    p.predictor_alpha = float(predictor_alpha)
    p.precision = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
    p.gravity, p.hse = gravity_mode(gravity), int(bool(hse))
    p.device = int(device)
    p.pool_bytes = int(pool_bytes)
    p.max_boxes = int(max_boxes)
    owner._allocator = None
    if use_torch_allocator or stream is None:
        import torch
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        if use_torch_allocator:
            owner._allocator = _TorchAllocator(device)
            p.alloc, p.free = owner._allocator.alloc, owner._allocator.free
    p.stream = ctypes.c_void_p(int(stream)) if stream else None
    return p


class Batch:
    """Many independent boxes advanced together (one launch per sub-operator
    covers them all), each with its own CFL step."""

    def __init__(self, pool_bytes, max_boxes=4096, gamma=5.0 / 3.0, limiter=VANLEER, predictor_alpha=1.0,
                 precision="fp32", gravity=False, hse=False, device=0, stream=None, use_torch_allocator=True):
        lib = load_library()
        self._lib = lib
        p = _batch_params(self, pool_bytes, max_boxes, gamma, limiter, predictor_alpha, precision, gravity, hse,
                          device, stream, use_torch_allocator)
        self.params = p
        self.gravity = bool(gravity)
        self.shapes = {}
        h = ctypes.c_void_p()
        rc = lib.fish_batch_create(ctypes.byref(p), ctypes.byref(h))
        if rc != FISH_OK:
            raise FishError(rc, "fish_batch_create failed: " + lib.fish_last_error(None).decode())
        self._h = h

    def _check(self, rc):
        if rc != FISH_OK:
            raise FishError(rc, self._lib.fish_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fish_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self):
        return int(self._lib.fish_batch_device_bytes(self._h))

    @property
    def free_bytes(self):
        return int(self._lib.fish_batch_free_bytes(self._h))

    def __len__(self):
        return int(self._lib.fish_batch_count(self._h))

    def add(self, st, h=None, cfl=0.5, bc=(PERIODIC,) * 3):
        """Add a box with state dict st (layouts of Box.set_state); returns its id."""
        cell = np.ascontiguousarray(st["cell"], dtype=np.float64)
        _, nz, ny, nx = cell.shape
        bx = np.ascontiguousarray(st["bx"], dtype=np.float64)
        by = np.ascontiguousarray(st["by"], dtype=np.float64)
        bz = np.ascontiguousarray(st["bz"], dtype=np.float64)
        if bx.shape != (nz, ny, nx + 1) or by.shape != (nz, ny + 1, nx) or bz.shape != (nz + 1, ny, nx):
            raise ValueError("face arrays do not match the cell array")
        phi = st.get("phi") if self.gravity else None
        if phi is not None:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
        g = _geom((nx, ny, nz), h, cfl, bc)
        i = ctypes.c_int(-1)
        self._check(self._lib.fish_batch_add(self._h, ctypes.byref(g), _dptr(cell), _dptr(bx), _dptr(by), _dptr(bz),
                                             _dptr(phi), ctypes.byref(i)))
        self.shapes[i.value] = (nz, ny, nx)
        return i.value

    def remove(self, box_id):
        self._check(self._lib.fish_batch_remove(self._h, int(box_id)))
        self.shapes.pop(box_id, None)

    def set_spacing(self, box_id, axis, widths):
        """Irregular mesh (Sect. 2.5) of one box: the widths of its cells along axis."""
        w = np.ascontiguousarray(widths, dtype=np.float64)
        if w.shape != (self.shapes[box_id][2 - axis],):
            raise ValueError("one width per cell along the axis")
        self._check(self._lib.fish_batch_set_spacing(self._h, int(box_id), int(axis),
                                                     w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def get(self, box_id, check=True):
        nz, ny, nx = self.shapes[box_id]
        cell = np.empty((5, nz, ny, nx))
        bx = np.empty((nz, ny, nx + 1))
        by = np.empty((nz, ny + 1, nx))
        bz = np.empty((nz + 1, ny, nx))
        t = ctypes.c_double()
        rc = self._lib.fish_batch_get(self._h, int(box_id), _dptr(cell), _dptr(bx), _dptr(by), _dptr(bz),
                                      ctypes.byref(t))
        if check:
            self._check(rc)
        return {"cell": cell, "bx": bx, "by": by, "bz": bz, "t": t.value, "status": rc}

    def info(self, box_id):
        t, dt, bad = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self._check(self._lib.fish_batch_box_info(self._h, int(box_id), ctypes.byref(t), ctypes.byref(dt),
                                                  ctypes.byref(bad)))
        return {"t": t.value, "dt": dt.value, "bad": bool(bad.value)}

    def steps_taken(self, box_id):
        """Double steps the box took with dt > 0 since its state was set."""
        n = ctypes.c_int()
        self._check(self._lib.fish_batch_box_steps(self._h, int(box_id), ctypes.byref(n)))
        return n.value

    def step(self, nsteps=1):
        self._check(self._lib.fish_batch_step(self._h, int(nsteps)))

    def use_graph(self, on=True):
        self._check(self._lib.fish_batch_use_graph(self._h, int(bool(on))))

    def autotune(self, reps=3):
        t = (ctypes.c_int32 * 7)()
        self._check(self._lib.fish_batch_autotune(self._h, int(reps), t))
        return _tuned(t)

    def set_shape(self, kind, target, xcd_remap=0, alt_layout=0):
        self._check(self._lib.fish_batch_set_shape(self._h, KINDS.index(kind),
                                                   shape_value(target, xcd_remap, alt_layout)))

    def sync(self):
        self._check(self._lib.fish_batch_sync(self._h))

    def timing_enable(self, mask, max_launches=4096):
        self._check(self._lib.fish_batch_timing_enable(self._h, int(mask), int(max_launches)))

    def timing_read(self):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        self._check(self._lib.fish_batch_timing_read(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


class Server:
    """Request loop over a batch: FIFO admission while the pool (the HBM
    budget) has room, all resident boxes advanced together, finished boxes
    retired into their output arrays."""

    def __init__(self, pool_bytes, chunk_steps=8, max_boxes=4096, gamma=5.0 / 3.0, limiter=VANLEER,
                 predictor_alpha=1.0, precision="fp32", gravity=False, hse=False, device=0, stream=None,
                 use_torch_allocator=True):
        lib = load_library()
        self._lib = lib
        p = _batch_params(self, pool_bytes, max_boxes, gamma, limiter, predictor_alpha, precision, gravity, hse,
                          device, stream, use_torch_allocator)
        self.params = p
        self.gravity = bool(gravity)
        h = ctypes.c_void_p()
        rc = lib.fish_server_create(ctypes.byref(p), int(chunk_steps), ctypes.byref(h))
        if rc != FISH_OK:
            raise FishError(rc, "fish_server_create failed: " + lib.fish_last_error(None).decode())
        self._h = h
        self._live = {}   # tag -> (request, input arrays, phi, output dict, widths) kept alive until completion
        self._done = (ctypes.c_int64 * 4096)()
        self._status = (ctypes.c_int32 * 4096)()

    def _check(self, rc):
        if rc != FISH_OK:
            raise FishError(rc, self._lib.fish_server_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fish_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, tag, st, nsteps, h=None, cfl=0.5, bc=(PERIODIC,) * 3, widths=None):
        """Queue a request; widths: None, or per axis None or the cell widths
        of an irregular mesh (Sect. 2.5)."""
        cell = np.ascontiguousarray(st["cell"], dtype=np.float64)
        _, nz, ny, nx = cell.shape
        arrs = [cell] + [np.ascontiguousarray(st[k], dtype=np.float64) for k in ("bx", "by", "bz")]
        phi = np.ascontiguousarray(st["phi"], dtype=np.float64) if self.gravity else None
        out = {"cell": np.empty((5, nz, ny, nx)), "bx": np.empty((nz, ny, nx + 1)),
               "by": np.empty((nz, ny + 1, nx)), "bz": np.empty((nz + 1, ny, nx))}
        r = Request()
        r.box = _geom((nx, ny, nz), h, cfl, bc)
        r.nsteps = int(nsteps)
        r.cell5, r.bx, r.by, r.bz = (_dptr(a) for a in arrs)
        r.phi = _dptr(phi)
        r.out_cell5, r.out_bx, r.out_by, r.out_bz = (_dptr(out[k]) for k in ("cell", "bx", "by", "bz"))
        r.tag = int(tag)
        ws = [None, None, None]
        for a in range(3):
            if widths is not None and widths[a] is not None:
                ws[a] = np.ascontiguousarray(widths[a], dtype=np.float64)
                if ws[a].shape != ((nx, ny, nz)[a],):
                    raise ValueError("one width per cell along the axis")
            r.widths[a] = _dptr(ws[a])
        self._check(self._lib.fish_server_submit(self._h, ctypes.byref(r)))
        self._live[int(tag)] = (r, arrs, phi, out, ws)

    def pump(self):
        """One scheduling round; returns [(tag, status, output state)] of the
        requests that completed."""
        n = ctypes.c_int()
        self._check(self._lib.fish_server_pump(self._h, self._done, self._status, len(self._done), ctypes.byref(n)))
        res = []
        for i in range(n.value):
            tag = int(self._done[i])
            out = self._live.pop(tag)[3]
            res.append((tag, int(self._status[i]), out))
        return res

    def stats(self):
        q, r, f, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t(), ctypes.c_int64()
        self._check(self._lib.fish_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f),
                                                ctypes.byref(c)))
        return {"queued": q.value, "resident": r.value, "pool_free": f.value, "cell_steps": c.value}

    def batch_autotune(self, reps=3):
        b = self._lib.fish_server_batch(self._h)
        t = (ctypes.c_int32 * 7)()
        rc = self._lib.fish_batch_autotune(b, int(reps), t)
        if rc != FISH_OK:
            raise FishError(rc, self._lib.fish_batch_last_error(b).decode())
        return _tuned(t)

    def use_graph(self, on=True):
        b = self._lib.fish_server_batch(self._h)
        rc = self._lib.fish_batch_use_graph(b, int(bool(on)))
        if rc != FISH_OK:
            raise FishError(rc, self._lib.fish_batch_last_error(b).decode())
