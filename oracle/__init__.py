"""FP64 CPU oracle of the FISH operator-split ideal-MHD step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It is a ctypes binding of
``oracle/libfishref.so`` (built from ``oracle/fishref.cpp`` by
``oracle/build.py``), a plain FP64 C++ implementation of Sect. 2 of the FISH
paper that shares no code with the HIP library.

State dictionaries use the layout of the C interface:

``cell`` (5, nz, ny, nx)   rho, m_x, m_y, m_z, E
``bx``   (nz, ny, nx+1)    face f between cells f-1 and f
``by``   (nz, ny+1, nx)
``bz``   (nz+1, ny, nx)
``phi``  (nz, ny, nx) or None

Parity pins (CPU tests under ``tests/test_oracle_*.py``): uniform states stay
bitwise unchanged; periodic conservation of mass, momentum, energy and face
flux to round-off; discrete div b unchanged; axis equivariance; second-order
convergence on linear Alfven, fast and entropy waves and on the circularly
polarised Alfven wave of Sect. 4.1; the exact Riemann solution of a Sod tube;
Rankine-Hugoniot jumps of a hydrodynamic and a perpendicular MHD shock; TVD of
the field advection; the closed forms of the fast speed; the HSE reductions;
split gravity (closed-form kick, hydrostatic atmosphere at second order); the
Mach limiter switch (reduces to either limiter per regime); irregular meshes
(conservation, per-cell divergence, second order on stretched meshes, exact
face interpolation of a linear shear, reduction to the uniform mesh, the
closed-form diagnostics of a uniform state: volume, face areas, zero
divergence).

Parity unpinned (readings the paper does not fix and no pin can separate):
the exact directional fast speed in the freezing speed, the interface-local
freezing speed inside the limited flux differences, the predictor dissipation
scale (default 1), the default limiter (van Leer), the details of the
second-order field-advection corrector, the form of the HSE corrector, the
slope form of the second-order fluxes on irregular meshes (differences over
centre distances, carried half a cell) and the width of ghost cells.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfishref.so")

OK, ERR_ARG, ERR_NOMEM, ERR_STATE, ERR_UNSUPPORTED = 0, 1, 2, 4, 5
PERIODIC, OUTFLOW = 0, 1
MINMOD, VANLEER, MACH_SWITCH = 0, 1, 2


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("predictor_alpha", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
        ("gravity", ctypes.c_int32), ("hse", ctypes.c_int32),
        ("nthreads", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    d = ctypes.c_double
    vp = ctypes.c_void_p
    lib.fishref_create.argtypes = [P(_Params), P(vp)]
    lib.fishref_destroy.argtypes = [vp]
    lib.fishref_destroy.restype = None
    lib.fishref_last_error.argtypes = [vp]
    lib.fishref_last_error.restype = ctypes.c_char_p
    lib.fishref_set_state.argtypes = [vp, P(d), P(d), P(d), P(d), P(d)]
    lib.fishref_get_state.argtypes = [vp, P(d), P(d), P(d), P(d), P(d)]
    lib.fishref_cfl_dt.argtypes = [vp, P(d)]
    lib.fishref_strang_step.argtypes = [vp, d]
    lib.fishref_apply.argtypes = [vp, ctypes.c_int, ctypes.c_int, d]
    lib.fishref_set_spacing.argtypes = [vp, ctypes.c_int, P(d)]
    lib.fishref_diagnostics.argtypes = [vp, P(d)]
    for name in ("fishref_create", "fishref_set_state", "fishref_get_state", "fishref_cfl_dt",
                 "fishref_strang_step", "fishref_apply", "fishref_diagnostics"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def gravity_mode(gravity):
    """False/0: none; True/1/"unsplit": Eqs. (41)-(43); 2/"split": Eqs. (38)-(40)."""
    if isinstance(gravity, str):
        return {"none": 0, "unsplit": 1, "split": 2}[gravity]
    return int(gravity) if not isinstance(gravity, bool) else int(gravity)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One box advanced by the FP64 CPU oracle."""

    def __init__(self, nx, ny, nz, dx=None, dy=None, dz=None, gamma=5.0 / 3.0, cfl=0.5,
                 limiter=VANLEER, predictor_alpha=1.0, bc=(PERIODIC,) * 3, gravity=False,
                 hse=False, nthreads=0):
        lib = _load()
        self.shape = (int(nz), int(ny), int(nx))
        p = _Params()
        p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
        p.dx = 1.0 / nx if dx is None else float(dx)
        p.dy = 1.0 / ny if dy is None else float(dy)
        p.dz = 1.0 / nz if dz is None else float(dz)
        p.gamma, p.cfl = float(gamma), float(cfl)
        p.limiter = int(limiter)
        p.predictor_alpha = float(predictor_alpha)
        for a in range(3):
            p.bc[a] = int(bc[a])
        p.gravity, p.hse = gravity_mode(gravity), int(bool(hse))
        p.nthreads = int(nthreads)
        self.params = p
        h = ctypes.c_void_p()
        rc = lib.fishref_create(ctypes.byref(p), ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "create failed")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fishref_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise OracleError(rc, self._lib.fishref_last_error(self._h).decode())

    def set_state(self, st):
        nz, ny, nx = self.shape
        cell = np.ascontiguousarray(st["cell"], dtype=np.float64)
        bx = np.ascontiguousarray(st["bx"], dtype=np.float64)
        by = np.ascontiguousarray(st["by"], dtype=np.float64)
        bz = np.ascontiguousarray(st["bz"], dtype=np.float64)
        assert cell.shape == (5, nz, ny, nx)
        assert bx.shape == (nz, ny, nx + 1) and by.shape == (nz, ny + 1, nx) and bz.shape == (nz + 1, ny, nx)
        phi = st.get("phi")
        if phi is not None:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
            assert phi.shape == (nz, ny, nx)
        self._check(self._lib.fishref_set_state(self._h, _ptr(cell), _ptr(bx), _ptr(by), _ptr(bz), _ptr(phi)))

    def get_state(self, check=True):
        nz, ny, nx = self.shape
        cell = np.empty((5, nz, ny, nx))
        bx = np.empty((nz, ny, nx + 1))
        by = np.empty((nz, ny + 1, nx))
        bz = np.empty((nz + 1, ny, nx))
        t = ctypes.c_double()
        rc = self._lib.fishref_get_state(self._h, _ptr(cell), _ptr(bx), _ptr(by), _ptr(bz), ctypes.byref(t))
        if check:
            self._check(rc)
        return {"cell": cell, "bx": bx, "by": by, "bz": bz, "t": t.value, "status": rc}

    def cfl_dt(self):
        dt = ctypes.c_double()
        self._check(self._lib.fishref_cfl_dt(self._h, ctypes.byref(dt)))
        return dt.value

    def strang_step(self, dt=0.0):
        self._check(self._lib.fishref_strang_step(self._h, float(dt)))

    def apply(self, op, direction, dt):
        """One sub-operator: op 'L' (fluid) or 'B' (field), direction 0/1/2."""
        code = {"L": 0, "B": 1}[op] if isinstance(op, str) else int(op)
        self._check(self._lib.fishref_apply(self._h, code, int(direction), float(dt)))

    def set_spacing(self, axis, widths):
        """Irregular mesh (Sect. 2.5): the widths of the cells along axis."""
        w = np.ascontiguousarray(widths, dtype=np.float64)
        if w.shape != (self.shape[2 - axis],):
            raise ValueError("one width per cell along the axis")
        self._check(self._lib.fishref_set_spacing(self._h, int(axis), _ptr(w)))

    def diagnostics(self):
        out = np.zeros(10)
        self._check(self._lib.fishref_diagnostics(self._h, _ptr(out)))
        return {"mass": out[0], "mom": out[1:4].copy(), "energy": out[4], "flux": out[5:8].copy(),
                "divb_max": out[8], "bmax": out[9]}
