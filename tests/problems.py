"""Helpers for the validation problems of Sect. 4.2-4.6 (test infrastructure).

The initial states come from ``fish_inputs``; this module reads the printed
ranges under ``tests/golden/`` and measures a finished state (value ranges,
radial profiles).  It calls neither the oracle nor the HIP library.
"""
from __future__ import annotations

import os

import numpy as np

import fish_inputs as fi

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_ranges(name):
    """{quantity: (min, max)} from a golden range file."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = (float(line[1]), float(line[2]))
    return out


def read_values(name):
    """{quantity: value} from a golden file of two columns."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = float(line[1])
    return out


def energies(state, gamma):
    """Cell fields rho, p, b^2/2 (cell-centred b) and rho v^2/2."""
    c = state["cell"]
    bcx, bcy, bcz = fi.cell_centred_b(state["bx"], state["by"], state["bz"])
    e_kin = 0.5 * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2) / c[0]
    e_mag = 0.5 * (bcx ** 2 + bcy ** 2 + bcz ** 2)
    return {"rho": c[0], "p": (gamma - 1.0) * (c[4] - e_kin - e_mag), "e_mag": e_mag, "e_kin": e_kin}


def value_ranges(state, gamma, plane=None):
    """(min, max) of each quantity over the box, or over one z plane."""
    out = {}
    for k, v in energies(state, gamma).items():
        if plane is not None:
            v = v[plane]
        out[k] = (float(np.min(v)), float(np.max(v)))
    return out


def range_mismatches(got, ref, max_tol, min_factor, zero_floor):
    """Quantities whose maximum differs from the printed one by more than
    max_tol (relative), or whose minimum is off by more than a factor
    min_factor (a printed minimum of 0 asks for got <= zero_floor * max)."""
    bad = []
    for k, (lo, hi) in ref.items():
        glo, ghi = got[k]
        if abs(ghi - hi) > max_tol * hi:
            bad.append((k, "max", ghi, hi))
        if lo == 0.0:
            if glo > zero_floor * ghi:
                bad.append((k, "min", glo, lo))
        elif not (lo / min_factor <= glo <= lo * min_factor):
            bad.append((k, "min", glo, lo))
    return bad
