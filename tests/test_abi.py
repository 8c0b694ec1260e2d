"""The C interface library builds, loads and exports every declared call (CPU only)."""
import ctypes
import os
import re

import paper_0910_2854_amd as fish

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(fish_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = fish.load_library()
    names = declared_symbols()
    assert {"fish_create", "fish_set_state", "fish_cfl_dt", "fish_strang_step", "fish_get_state",
            "fish_destroy"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_binding_names_match_header():
    assert set(fish.EXPORTS) <= declared_symbols()


def test_create_rejects_bad_arguments_without_touching_a_device():
    lib = fish.load_library()
    p = fish.Params()
    p.nx = p.ny = p.nz = 0  # invalid shape: rejected before any HIP call
    h = ctypes.c_void_p()
    assert lib.fish_create(ctypes.byref(p), ctypes.byref(h)) == fish.FISH_ERR_ARG
    assert not h.value
    assert lib.fish_create(None, ctypes.byref(h)) == fish.FISH_ERR_ARG
    lib.fish_destroy(None)


def _valid_params(n, precision):
    p = fish.Params()
    p.nx, p.ny, p.nz = n
    p.dx, p.dy, p.dz = (1.0 / v for v in n)
    p.gamma, p.cfl = 5.0 / 3.0, 0.5
    p.limiter = fish.VANLEER
    p.predictor_alpha = 1.0
    p.precision = precision
    return p


def test_create_rejects_arrays_beyond_32bit_offsets_without_touching_a_device():
    """Each array of a box must stay below 4 GiB (the kernels address it with
    32-bit byte offsets): 1100^3 in FP32 is refused before any HIP call."""
    lib = fish.load_library()
    h = ctypes.c_void_p()
    assert lib.fish_create(ctypes.byref(_valid_params((1100, 1100, 1100), fish.FP32)), ctypes.byref(h)) == \
        fish.FISH_ERR_UNSUPPORTED
    assert not h.value
    # FP64 doubles the bytes per array: refused as well
    assert lib.fish_create(ctypes.byref(_valid_params((1100, 1100, 1100), fish.FP64)), ctypes.byref(h)) == \
        fish.FISH_ERR_UNSUPPORTED


def test_batch_and_box_geometry_checks_without_a_device():
    lib = fish.load_library()
    g = fish.BoxGeom()
    g.nx, g.ny, g.nz = 16, 16, 16
    g.dx = g.dy = g.dz = 1.0 / 16
    g.cfl = 0.5
    # both buffers of 8 arrays, padded to 64 elements
    assert lib.fish_box_pool_bytes(ctypes.byref(g), fish.FP32, 0) == 16 * 4096 * 4
    assert lib.fish_box_pool_bytes(ctypes.byref(g), fish.FP64, 1) == 17 * 4096 * 8
    bp = fish.BatchParams()
    bp.gamma, bp.limiter, bp.predictor_alpha, bp.precision = 5.0 / 3.0, fish.VANLEER, 1.0, fish.FP32
    bp.max_boxes = 0  # invalid: rejected before any HIP call
    bp.pool_bytes = 1 << 20
    h = ctypes.c_void_p()
    assert lib.fish_batch_create(ctypes.byref(bp), ctypes.byref(h)) == fish.FISH_ERR_ARG
    assert not h.value


_TWO_RUNTIMES = r"""
import ctypes, os, sys
sys.path.insert(0, ROOT)
lib = ctypes.CDLL(os.path.join(ROOT, "paper_0910_2854_amd", "libfish.so"))  # binds the system HIP runtime
import torch  # noqa: F401  -- maps PyTorch's own copy next to it
import paper_0910_2854_amd as fish
p = fish.Params()
p.nx = p.ny = p.nz = 8
p.dx = p.dy = p.dz = 1.0 / 8
p.gamma, p.cfl, p.limiter, p.predictor_alpha, p.precision = 5.0 / 3.0, 0.5, fish.VANLEER, 1.0, fish.FP64
p.stream = 0x1000  # a stream handle of the caller: refused before any HIP call touches it
lib.fish_create.argtypes = [ctypes.POINTER(fish.Params), ctypes.POINTER(ctypes.c_void_p)]
lib.fish_last_error.argtypes = [ctypes.c_void_p]
lib.fish_last_error.restype = ctypes.c_char_p
h = ctypes.c_void_p()
rc = lib.fish_create(ctypes.byref(p), ctypes.byref(h))
print(rc, h.value)
print(lib.fish_last_error(None).decode())
print(len(fish.hip_runtimes_loaded()))
"""


def test_a_stream_of_another_hip_runtime_is_refused_with_a_message():
    """Loaded before PyTorch, the library binds the system HIP runtime and
    PyTorch maps its own copy; a caller's stream (or allocator) then belongs
    to the other copy, and fish_create refuses it, naming both runtimes,
    before any HIP call."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, "-c", "ROOT = %r\n" % ROOT + _TWO_RUNTIMES], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    rc_line, msg, nrt = r.stdout.strip().splitlines()[-3:]
    assert rc_line.split()[0] == str(fish.FISH_ERR_DEVICE) and rc_line.split()[1] == "None"
    assert int(nrt) == 2
    assert msg.count("libamdhip64") == 2 and "import torch first" in msg


def test_the_binding_maps_one_hip_runtime():
    """Through the binding, PyTorch is loaded first and the library binds its
    runtime: one copy of libamdhip64 in the process."""
    fish.load_library()
    assert len(fish.hip_runtimes_loaded()) == 1


def _fake_arrays(base):
    # addresses that are never dereferenced: every call below is refused by
    # the host checks before any HIP call
    return [base + 0x1000 * i for i in range(8)]


def test_noalloc_step_refuses_bad_calls_without_touching_a_device():
    lib = fish.load_library()
    vp = ctypes.c_void_p
    ok = _valid_params((8, 8, 8), fish.FP64)
    st, wk = (vp * 8)(*_fake_arrays(0x100000)), (vp * 8)(*_fake_arrays(0x900000))
    # a null array, a repeated array, no phi with gravity, a negative dt, a bad setting
    holes = (vp * 8)(*(_fake_arrays(0x100000)[:7] + [0]))
    assert lib.fish_strang_step_noalloc(ctypes.byref(ok), holes, wk, None, 0.0, None) == fish.FISH_ERR_ARG
    assert lib.fish_strang_step_noalloc(ctypes.byref(ok), st, st, None, 0.0, None) == fish.FISH_ERR_ARG
    assert lib.fish_strang_step_noalloc(None, st, wk, None, 0.0, None) == fish.FISH_ERR_ARG
    assert lib.fish_strang_step_noalloc(ctypes.byref(ok), st, wk, None, -1.0, None) == fish.FISH_ERR_ARG
    grav = _valid_params((8, 8, 8), fish.FP64)
    grav.gravity = 1
    assert lib.fish_strang_step_noalloc(ctypes.byref(grav), st, wk, None, 0.0, None) == fish.FISH_ERR_ARG
    bad = _valid_params((8, 8, 8), fish.FP64)
    bad.gamma = 1.0
    assert lib.fish_strang_step_noalloc(ctypes.byref(bad), st, wk, None, 0.0, None) == fish.FISH_ERR_ARG
    assert b"dt" in lib.fish_last_error(None) or b"invalid" in lib.fish_last_error(None)


def test_noalloc_step_refuses_a_box_beyond_its_scratch():
    """The scratch holds 2^20 work-list entries: a 16384 x 1 x 16384 FP32 box
    (1 GiB per array, accepted by fish_create) needs 2^22 wavefronts in its y
    sweep and is refused before any HIP call; 1024^3 FP32 (every wave count at
    most 2^20) is refused only for its 4 GiB arrays."""
    lib = fish.load_library()
    vp = ctypes.c_void_p
    st, wk = (vp * 8)(*_fake_arrays(0x100000)), (vp * 8)(*_fake_arrays(0x900000))
    flat = _valid_params((16384, 1, 16384), fish.FP32)
    assert lib.fish_strang_step_noalloc(ctypes.byref(flat), st, wk, None, 0.0, None) == fish.FISH_ERR_UNSUPPORTED
    msg = lib.fish_last_error(None).decode()
    assert "4194304 wavefronts" in msg and str(fish.NOALLOC_MAX_WAVES) in msg, msg
    big = _valid_params((1024, 1024, 1024), fish.FP32)
    assert lib.fish_strang_step_noalloc(ctypes.byref(big), st, wk, None, 0.0, None) == fish.FISH_ERR_UNSUPPORTED
    assert "4 GiB" in lib.fish_last_error(None).decode()


def test_storage_layout_round_trip():
    """to_storage / from_storage: the interface arrays come back unchanged
    (face n of a periodic axis is face 0), every other entry is zero."""
    import numpy as np
    import fish_inputs as fi
    n, bc = (7, 5, 6), (fish.PERIODIC, fish.OUTFLOW, fish.PERIODIC)
    st = fi.random_fourier_state(n, seed=3, mach=0.8, beta=2.0, kmax=2)
    arrays, phi = fish.to_storage(st, n, bc, np.float64)
    assert phi is None
    assert all(a.shape == fish.storage_shape(n, bc) == (6, 6, 7) for a in arrays)
    back = fish.from_storage(arrays, n, bc)
    for k in ("cell", "bx", "by", "bz"):
        np.testing.assert_array_equal(back[k], st[k])
    assert not arrays[0][:, 5, :].any()  # the outflow layer of a cell array
    assert arrays[6][:, 5, :].any()      # face n of b_y on the outflow axis
