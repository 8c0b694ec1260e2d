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
