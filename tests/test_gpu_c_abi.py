"""The C interface without PyTorch: a caller that never imports torch creates
a box with alloc = NULL (the library's hipMalloc/hipFree) on the null stream
and steps the 32^3 smooth box (rms Mach 0.5, beta 10, |k| <= 4) against the
FP64 oracle.  The child process loads only the library, the oracle and the
input generator, so the library binds the system HIP runtime (one copy in
the process) and owns every device allocation itself."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, json, os, sys
import numpy as np
sys.path.insert(0, ROOT)
import fish_inputs as fi
from oracle import Oracle

class Params(ctypes.Structure):  # struct fish_params of include/fish.h
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("limiter", ctypes.c_int32),
                ("predictor_alpha", ctypes.c_double), ("bc", ctypes.c_int32 * 3), ("precision", ctypes.c_int32),
                ("gravity", ctypes.c_int32), ("hse", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p)]

lib = ctypes.CDLL(os.path.join(ROOT, "paper_0910_2854_amd", "libfish.so"))
vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
lib.fish_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(vp)]
lib.fish_last_error.argtypes = [vp]
lib.fish_last_error.restype = ctypes.c_char_p
lib.fish_set_state.argtypes = [vp, dp, dp, dp, dp, dp]
lib.fish_get_state.argtypes = [vp, dp, dp, dp, dp, dp]
lib.fish_cfl_dt.argtypes = [vp, dp]
lib.fish_strang_step.argtypes = [vp, ctypes.c_double]
lib.fish_destroy.argtypes = [vp]
lib.fish_destroy.restype = None

def ptr(a):
    return a.ctypes.data_as(dp)

n = (32, 32, 32)
st = fi.random_fourier_state(n, seed=0, mach=0.5, beta=10.0, kmax=4)
ref = Oracle(*n)
ref.set_state(st)
out = {"steps": 10}
for prec in (0, 1):  # FISH_FP64, FISH_FP32
    p = Params(nx=n[0], ny=n[1], nz=n[2], dx=1.0 / n[0], dy=1.0 / n[1], dz=1.0 / n[2], gamma=5.0 / 3.0, cfl=0.5,
               limiter=1, predictor_alpha=1.0, precision=prec)  # stream, alloc, free all NULL
    h = vp()
    rc = lib.fish_create(ctypes.byref(p), ctypes.byref(h))
    assert rc == 0, (rc, lib.fish_last_error(None))
    cell = np.ascontiguousarray(st["cell"]); bx, by, bz = (np.ascontiguousarray(st[k]) for k in ("bx", "by", "bz"))
    assert lib.fish_set_state(h, ptr(cell), ptr(bx), ptr(by), ptr(bz), None) == 0, lib.fish_last_error(h)
    dts = []
    for _ in range(10):
        dt = ctypes.c_double()
        assert lib.fish_cfl_dt(h, ctypes.byref(dt)) == 0, lib.fish_last_error(h)
        assert lib.fish_strang_step(h, dt.value) == 0, lib.fish_last_error(h)
        dts.append(dt.value)
    res = {k: np.empty_like(v) for k, v in (("cell", cell), ("bx", bx), ("by", by), ("bz", bz))}
    t = ctypes.c_double()
    assert lib.fish_get_state(h, ptr(res["cell"]), ptr(res["bx"]), ptr(res["by"]), ptr(res["bz"]),
                              ctypes.byref(t)) == 0, lib.fish_last_error(h)
    lib.fish_destroy(h)
    out[str(prec)] = {"dts": dts, "t": t.value, "state": res}
# the oracle with the oracle's own CFL steps
odts = []
for _ in range(10):
    dt = ref.cfl_dt()
    ref.strang_step(dt)
    odts.append(dt)
r = ref.get_state()
report = {"torch_loaded": "torch" in sys.modules, "runtimes": sorted({os.path.realpath(l.split()[-1])
          for l in open("/proc/self/maps") if "libamdhip64" in l.split()[-1]}), "oracle_dts": odts}
for prec in ("0", "1"):
    o = out[prec]
    rel = {}
    for k in ("cell", "bx", "by", "bz"):
        if k == "cell":
            for f, name in enumerate(("rho", "mx", "my", "mz", "E")):
                rel[name] = float(np.abs(o["state"][k][f] - r[k][f]).sum() / np.abs(r[k][f]).sum())
        else:
            rel[k] = float(np.abs(o["state"][k] - r[k]).sum() / np.abs(r[k]).sum())
    report[prec] = {"rel_l1": rel, "dts": o["dts"], "t": o["t"]}
print(json.dumps(report))
"""


@pytest.mark.gpu
def test_torch_free_caller_with_hipmalloc_and_null_stream_matches_the_oracle():
    env = dict(os.environ)
    print("child: C interface without torch, 32^3 box, FP64 and FP32, 10 steps", flush=True)
    r = subprocess.run([sys.executable, "-c", "ROOT = %r\n" % ROOT + CHILD], capture_output=True, text=True,
                       timeout=600, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-4000:]
    rep = json.loads(r.stdout.strip().splitlines()[-1])
    assert not rep["torch_loaded"]
    # one HIP runtime in the process: the system one the library links
    assert len(rep["runtimes"]) == 1 and "torch" not in rep["runtimes"][0], rep["runtimes"]
    for prec, tol_state, tol_dt in (("0", 1e-10, 1e-12), ("1", 1e-5, 1e-6)):
        for k, v in rep[prec]["rel_l1"].items():
            assert v <= tol_state, (prec, k, v)
        for a, b in zip(rep[prec]["dts"], rep["oracle_dts"]):
            assert abs(a - b) <= tol_dt * b, (prec, a, b)
        assert abs(rep[prec]["t"] - 2.0 * sum(rep[prec]["dts"])) <= 1e-12 * rep[prec]["t"]
