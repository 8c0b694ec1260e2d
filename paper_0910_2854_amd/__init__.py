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
MINMOD, VANLEER = 0, 1
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


class FishError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fish error {code}: {msg}")
        self.code = code


EXPORTS = ("fish_create", "fish_destroy", "fish_last_error", "fish_set_state", "fish_get_state",
           "fish_cfl_dt", "fish_strang_step", "fish_sweep", "fish_diagnostics", "fish_device_bytes",
           "fish_timing_enable", "fish_timing_read", "fish_selftest_lane_shift")
KERNEL_FLUID, KERNEL_FIELD, KERNEL_CHECK = 1, 2, 8

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfish.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
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
    for name in ("fish_create", "fish_set_state", "fish_get_state", "fish_cfl_dt", "fish_strang_step",
                 "fish_sweep", "fish_diagnostics", "fish_timing_enable", "fish_timing_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def selftest_lane_shift(device=0):
    """Run the lane-shift self-test kernel; returns the 128 output values."""
    lib = load_library()
    out = np.zeros(128, dtype=np.float32)
    rc = lib.fish_selftest_lane_shift(int(device), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != FISH_OK:
        raise FishError(rc, "lane-shift self-test failed to run")
    return out


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
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = _ALLOC(alloc)
        self.free = _FREE(free)


class Box:
    """One box advanced by the HIP library on one GPU stream."""

    def __init__(self, nx, ny, nz, dx=None, dy=None, dz=None, gamma=5.0 / 3.0, cfl=0.5, limiter=VANLEER,
                 predictor_alpha=1.0, bc=(PERIODIC,) * 3, precision="fp64", gravity=False, hse=False,
                 device=0, stream=None, use_torch_allocator=True):
        lib = load_library()
        self._lib = lib
        self.shape = (int(nz), int(ny), int(nx))
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
        p.gravity, p.hse = int(bool(gravity)), int(bool(hse))
        p.device = int(device)
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
            raise FishError(rc, "fish_create failed")
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
        return {"mass": out[0], "mom": out[1:4].copy(), "energy": out[4], "flux": out[5:8].copy(),
                "divb_max": out[8], "bmax": out[9]}
