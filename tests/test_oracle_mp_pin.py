"""Brute-force pin of the oracle's arithmetic: every sub-operator against an
independent 50-digit transcription (tests/mp_reference.py) on small random
boxes whose sweep axis has 8-12 cells, over periodic, outflow and mixed
boundaries, both limiters, and unsplit gravity with and without the
hydrostatic correction.  The transcription evaluates each quantity as a
memoised function of a (possibly ghost) position, so it shares neither code
nor structure with the oracle's pencil arrays; where the paper leaves a
reading open it takes the oracle's reading, so this pins arithmetic (a
dropped term, a wrong index, sign or operand), not the readings.

Tolerances: the FP64 result against the 50-digit one, per array, max abs
difference <= 1e-13 of the array's largest entry and <= 1e-11 of the largest
change the sub-operator makes (measured: about 2e-16 and 3e-15)."""
import numpy as np
import pytest

from mp_reference import MpBox
from oracle import Oracle

GAMMA = 5.0 / 3.0


def random_state(rng, n, bc, gravity):
    """Random state of a box n = (nx, ny, nz): rho in [0.8, 1.6], |v_i| <=
    0.6, p in [0.6, 1.4], face fields uniform in [-0.8, 0.8] (a single
    sub-operator needs no divergence-free field), a random potential."""
    nx, ny, nz = n
    rho = rng.uniform(0.8, 1.6, (nz, ny, nx))
    v = rng.uniform(-0.6, 0.6, (3, nz, ny, nx))
    p = rng.uniform(0.6, 1.4, (nz, ny, nx))
    b = [rng.uniform(-0.8, 0.8, (nz, ny, nx + 1)), rng.uniform(-0.8, 0.8, (nz, ny + 1, nx)),
         rng.uniform(-0.8, 0.8, (nz + 1, ny, nx))]
    for a in range(3):
        if bc[a] == 0:  # face n is face 0 on a periodic axis
            last = [slice(None)] * 3
            first = [slice(None)] * 3
            last[2 - a], first[2 - a] = -1, 0
            b[a][tuple(last)] = b[a][tuple(first)]
    bcx = 0.5 * (b[0][:, :, :-1] + b[0][:, :, 1:])
    bcy = 0.5 * (b[1][:, :-1, :] + b[1][:, 1:, :])
    bcz = 0.5 * (b[2][:-1] + b[2][1:])
    E = p / (GAMMA - 1.0) + 0.5 * rho * (v ** 2).sum(0) + 0.5 * (bcx ** 2 + bcy ** 2 + bcz ** 2)
    return {"cell": np.array([rho, rho * v[0], rho * v[1], rho * v[2], E]), "bx": b[0], "by": b[1], "bz": b[2],
            "phi": rng.uniform(-0.3, 0.3, (nz, ny, nx)) if gravity else None}


def shape_for(d, rng):
    n = [int(rng.integers(2, 4)), int(rng.integers(2, 4)), int(rng.integers(2, 4))]
    n[d] = int(rng.integers(8, 13))
    return tuple(n)


BCS = {"periodic": (0, 0, 0), "outflow": (1, 1, 1), "mixed": (1, 0, 1)}
CASES = []
for d in range(3):
    for bcname in BCS:
        for lim in (0, 1):
            CASES.append(("L", d, bcname, lim, "none"))
            CASES.append(("B", d, bcname, lim, "none"))
        CASES.append(("L", d, bcname, 1, "gravity"))
        CASES.append(("L", d, bcname, 0, "gravity+hse"))
        CASES.append(("L", d, bcname, 1, "gravity+hse"))


@pytest.mark.parametrize("op,d,bcname,lim,mode", CASES)
def test_oracle_sub_operator_matches_a_50_digit_transcription(op, d, bcname, lim, mode):
    seed = 1000 + 97 * CASES.index((op, d, bcname, lim, mode))
    rng = np.random.default_rng(seed)
    n = shape_for(d, rng)
    bc = BCS[bcname]
    gravity = mode != "none"
    hse = mode == "gravity+hse"
    st = random_state(rng, n, bc, gravity)
    h = [1.0 / x for x in n]
    dt = 0.02
    o = Oracle(*n, gamma=GAMMA, limiter=lim, bc=bc, gravity=gravity, hse=hse, nthreads=1)
    o.set_state(st)
    o.apply(op, d, dt)
    ref = o.get_state()
    o.close()
    mpv = MpBox(st, n, h, bc, gamma=GAMMA, limiter=lim, gravity=gravity, hse=hse).sweep(0 if op == "L" else 1, d, dt)
    changed = 0.0
    for k in ("cell", "bx", "by", "bz"):
        diff = float(np.max(np.abs(ref[k] - mpv[k])))
        scale = float(np.max(np.abs(mpv[k])))
        inc = float(np.max(np.abs(mpv[k] - st[k])))
        changed = max(changed, inc)
        assert diff <= 1e-13 * scale, (k, diff, scale)
        assert diff <= 1e-11 * max(inc, 1e-300) or diff == 0.0, (k, diff, inc)
    assert changed > 1e-3  # the sub-operator did change the state
