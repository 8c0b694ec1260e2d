"""A 50-digit transcription of one sub-operator of the FISH step -- TEST
INFRASTRUCTURE, used only by tests/test_oracle_mp_pin.py.

It is written independently of the oracle (oracle/fishref.cpp) and of the
HIP kernels, straight from the equations of Sect. 2 of the paper and the
readings the oracle documents, in a different form: every quantity is a
memoised function of a position (a cell index that may lie outside the box,
mapped by the boundary rule) instead of an array filled pencil by pencil.
Its purpose is to catch arithmetic slips in the oracle (a dropped term, a
wrong index or sign, a transposed operand), not to choose between readings:
where the paper leaves a choice, the same reading is taken.

Conventions (those of the C interface): cell arrays [nz][ny][nx], face arrays
with one more entry along their own normal, entry f lying between cells f-1
and f; on a periodic axis face n is face 0.  Values are mpmath numbers at 50
significant digits; inputs are FP64 arrays, converted exactly.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

mp.mp.dps = 50

RHO, MX, MY, MZ, EN = range(5)


def _mp(x):
    return mp.mpf(float(x))


def minmod(a, b):
    """Eq. (29): zero unless a and b share a sign, else the smaller modulus."""
    if a * b <= 0:
        return mp.mpf(0)
    return a if abs(a) < abs(b) else b


def vanleer(a, b):
    """Eq. (30) read as the harmonic mean 2ab/(a+b) of two slopes of one sign."""
    if a * b <= 0:
        return mp.mpf(0)
    return 2 * a * b / (a + b)


class MpBox:
    """One box at 50 digits; sweep(op, d, dt) applies L_d (op 0) or B_d (op 1)
    and returns the new state as FP64 arrays (rounded once, at the end)."""

    def __init__(self, state, n, h, bc, gamma=5.0 / 3.0, alpha=1.0, limiter=1, gravity=False, hse=False):
        self.n = tuple(n)            # (nx, ny, nz)
        self.h = tuple(_mp(v) for v in h)
        self.bc = tuple(bc)          # per axis: 0 periodic, 1 outflow
        self.gamma = _mp(gamma)
        self.alpha = _mp(alpha)
        self.lim = minmod if limiter == 0 else vanleer
        self.gravity = bool(gravity)
        self.hse = bool(hse)
        cell = np.asarray(state["cell"], dtype=np.float64)
        self.u = [[[[_mp(cell[q, k, j, i]) for i in range(n[0])] for j in range(n[1])] for k in range(n[2])]
                  for q in range(5)]
        self.b = []
        for a, key in enumerate(("bx", "by", "bz")):
            arr = np.asarray(state[key], dtype=np.float64)
            self.b.append([[[_mp(v) for v in row] for row in plane] for plane in arr])
        phi = state.get("phi")
        self.phi = None if phi is None else [[[_mp(v) for v in row] for row in plane] for plane in np.asarray(phi)]

    # ---------------------------------------------------------- index maps
    def cell_index(self, i, a):
        """Cell index along axis a: periodic wrap, or the nearest real cell
        (zeroth-order extrapolation) on an outflow axis."""
        n = self.n[a]
        if self.bc[a] == 0:
            return i % n
        return min(max(i, 0), n - 1)

    def face_index(self, f, a):
        """Face index along the face array's own normal a: faces 0..n-1 on a
        periodic axis (face n is face 0), 0..n on an outflow axis (a face
        beyond the last one copies it)."""
        n = self.n[a]
        if self.bc[a] == 0:
            return f % n
        return min(max(f, 0), n)

    def U(self, q, p):
        """Conserved quantity q at cell position p = (i, j, k), mapped."""
        i, j, k = (self.cell_index(p[a], a) for a in range(3))
        return self.u[q][k][j][i]

    def Bface(self, a, p):
        """Face array a at position p: face index along a, cell index across."""
        idx = [self.face_index(p[x], x) if x == a else self.cell_index(p[x], x) for x in range(3)]
        return self.b[a][idx[2]][idx[1]][idx[0]]

    def Bcentre(self, p):
        """Cell-centred field: the mean of the two faces of the cell (Sect. 2.2)."""
        out = []
        for a in range(3):
            hi = list(p)
            hi[a] += 1
            out.append((self.Bface(a, p) + self.Bface(a, hi)) / 2)
        return out

    def Phi(self, p, d):
        """Potential at position p, whose index along d may be a ghost: wrap on a
        periodic axis, linear extrapolation from the two nearest cells on an
        outflow axis (the transverse indices are real)."""
        i = p[d]
        n = self.n[d]

        def at(s):
            q = list(p)
            q[d] = s
            return self.phi[q[2]][q[1]][q[0]]

        if 0 <= i < n:
            return at(i)
        if self.bc[d] == 0 or n == 1:
            return at(i % n)
        if i < 0:
            return at(0) + i * (at(1) - at(0))
        return at(n - 1) + (i - (n - 1)) * (at(n - 1) - at(n - 2))

    # ---------------------------------------------------------- L_d
    def cell_state(self, u, bc, d):
        """Primitive and flux quantities of one cell (Sect. 2.1-2.2): velocity,
        the pressure of Eq. (5), the fast speed along d, the freezing speed
        |v_d| + c_F of Eq. (21), the flux of Eq. (17) along d, and for the
        hydrostatic correction the sound speed and xi of Eq. (50)."""
        rho = u[RHO]
        m = u[MX:MZ + 1]
        v = [mq / rho for mq in m]
        bb = sum(x * x for x in bc)
        kin = sum(mq * vq for mq, vq in zip(m, v)) / 2
        p = (self.gamma - 1) * (u[EN] - kin - bb / 2)
        ptot = p + bb / 2
        a2 = self.gamma * p / rho
        s = a2 + bb / rho
        disc = s * s - 4 * a2 * bc[d] * bc[d] / rho
        cf = mp.sqrt((s + mp.sqrt(max(disc, mp.mpf(0)))) / 2)
        flux = [m[d]]
        for k in range(3):
            flux.append(m[d] * v[k] - bc[d] * bc[k] + (ptot if k == d else 0))
        flux.append((u[EN] + ptot) * v[d] - bc[d] * sum(x * y for x, y in zip(bc, v)))
        xi = [-rho, -m[0], -m[1], -m[2], -(u[EN] + p)]
        return {"u": list(u), "F": flux, "vd": v[d], "cf": cf, "cs": mp.sqrt(a2), "dfreeze": abs(v[d]) + cf, "xi": xi}

    def dissipation(self, L, R, phiL, phiR):
        """Q_j such that the first-order flux is (F_L + F_R)/2 - Q_j/2: Eqs.
        (24)-(25), or with the hydrostatic correction Eqs. (51)-(57)."""
        du = [R["u"][q] - L["u"][q] for q in range(5)]
        if not self.hse:
            dmax = max(L["dfreeze"], R["dfreeze"])
            return [dmax * x for x in du]
        dadv = max(abs(L["vd"]), abs(R["vd"]))
        dac = max(L["cf"], R["cf"])
        out = []
        for q in range(5):
            g = (L["xi"][q] + R["xi"][q]) / 2 * (phiR - phiL) / (L["cs"] * R["cs"])
            out.append(dadv * du[q] + dac * minmod(du[q] - g, du[q]))
        return out

    def source(self, rho, md, p, d):
        """Unsplit gravity, Eq. (42) with the sign of Eq. (36)."""
        lo, hi = list(p), list(p)
        lo[d] -= 1
        hi[d] += 1
        grad = (self.Phi(hi, d) - self.Phi(lo, d)) / (2 * self.h[d])
        s = [mp.mpf(0)] * 5
        s[MX + d] = -rho * grad
        s[EN] = -md * grad
        return s

    def fluid(self, d, dt):
        dt = _mp(dt)
        h = self.h[d]
        gravity = self.gravity
        phi_on = gravity or self.hse

        def shifted(p, s):
            q = list(p)
            q[d] += s
            return tuple(q)

        @functools.lru_cache(maxsize=None)
        def q0(p):
            return self.cell_state([self.U(q, p) for q in range(5)], self.Bcentre(p), d)

        def phi(p):
            return self.Phi(p, d) if phi_on else mp.mpf(0)

        @functools.lru_cache(maxsize=None)
        def flux1(p):  # predictor flux at the interface between p and p + e_d (Eq. 24, scaled dissipation)
            L, R = q0(p), q0(shifted(p, 1))
            Q = self.dissipation(L, R, phi(p), phi(shifted(p, 1)))
            return [(L["F"][q] + R["F"][q]) / 2 - self.alpha * Q[q] / 2 for q in range(5)]

        @functools.lru_cache(maxsize=None)
        def half(p):  # predictor half step, Eq. (41)
            c = q0(p)
            fr, fl = flux1(p), flux1(shifted(p, -1))
            s = self.source(c["u"][RHO], c["u"][MX + d], p, d) if gravity else [0] * 5
            u = [c["u"][q] - dt / (2 * h) * (fr[q] - fl[q]) + dt / 2 * s[q] for q in range(5)]
            return self.cell_state(u, self.Bcentre(p), d)

        @functools.lru_cache(maxsize=None)
        def diffs(p):  # a+-_j = (dF +- Q)/2 across the interface p | p + e_d, on the half-step state
            L, R = half(p), half(shifted(p, 1))
            Q = self.dissipation(L, R, phi(p), phi(shifted(p, 1)))
            dF = [R["F"][q] - L["F"][q] for q in range(5)]
            return ([(dF[q] + Q[q]) / 2 for q in range(5)], [(dF[q] - Q[q]) / 2 for q in range(5)], Q)

        @functools.lru_cache(maxsize=None)
        def flux2(p):  # second-order flux, Eq. (34), at the interface p | p + e_d
            L, R = half(p), half(shifted(p, 1))
            apl, _, _ = diffs(shifted(p, -1))
            ap, am, Q = diffs(p)
            _, amr, _ = diffs(shifted(p, 1))
            return [(L["F"][q] + R["F"][q]) / 2 - Q[q] / 2 + (self.lim(apl[q], ap[q]) - self.lim(am[q], amr[q])) / 2
                    for q in range(5)]

        new = [[[[None] * self.n[0] for _ in range(self.n[1])] for _ in range(self.n[2])] for _ in range(5)]
        for k in range(self.n[2]):
            for j in range(self.n[1]):
                for i in range(self.n[0]):
                    p = (i, j, k)
                    fr, fl = flux2(p), flux2(shifted(p, -1))
                    hq = half(p)
                    s = self.source(hq["u"][RHO], hq["u"][MX + d], p, d) if gravity else [0] * 5
                    for q in range(5):  # corrector, Eq. (43)
                        new[q][k][j][i] = self.u[q][k][j][i] - dt / h * (fr[q] - fl[q]) + dt * s[q]
        self.u = new

    # ---------------------------------------------------------- B_d
    def field(self, d, dt):
        """Transverse advection of b_t1, b_t2 along d and the constraint update
        of b_d from the same edge fluxes (Sect. 2.4, Eqs. 62-68), physical
        signs; the fluid state is held fixed."""
        dt = _mp(dt)
        h = self.h[d]
        n = self.n

        def vd(p):
            return self.U(MX + d, p) / self.U(RHO, p)

        def pos(base, axis, value):
            q = list(base)
            q[axis] = value
            return tuple(q)

        edge = {}  # (t, row position with d index = face f_d) -> Phi2 at d-face f_d

        def row(t, start):
            """One face row of b_t: start holds the t-face index along t and a
            cell index along the other transverse axis; the d index runs."""

            @functools.lru_cache(maxsize=None)
            def w(i):  # Eq. (65): v_d on the t-face, mean of the two cells sharing it
                p = pos(start, d, i)
                return (vd(pos(p, t, p[t] - 1)) + vd(p)) / 2

            @functools.lru_cache(maxsize=None)
            def vbar(i):  # Eq. (66), outer neighbours summed first
                return ((w(i - 1) + w(i + 1)) + 2 * w(i)) / 4

            def V(i):  # Eq. (68): the velocity at the interface i | i+1
                return (vbar(i) + vbar(i + 1)) / 2

            def bt(i):
                return self.Bface(t, pos(start, d, i))

            def f(i):
                return vbar(i) * bt(i)

            def phi1(i):  # Eq. (67): upwind flux at i | i+1, the right cell when V <= 0
                return f(i) if V(i) > 0 else f(i + 1)

            @functools.lru_cache(maxsize=None)
            def fhalf(i):  # v-bar times the half-step b'
                return vbar(i) * (bt(i) - dt / (2 * h) * (phi1(i) - phi1(i - 1)))

            @functools.lru_cache(maxsize=None)
            def phi2(i):  # limited upwind flux of the half-step state at i | i+1
                if V(i) > 0:
                    return fhalf(i) + self.lim(fhalf(i) - fhalf(i - 1), fhalf(i + 1) - fhalf(i)) / 2
                return fhalf(i + 1) - self.lim(fhalf(i + 1) - fhalf(i), fhalf(i + 2) - fhalf(i + 1)) / 2

            return bt, phi2

        t1, t2 = (d + 1) % 3, (d + 2) % 3
        newb = [[[[x for x in r] for r in pl] for pl in arr] for arr in self.b]
        for t, o in ((t1, t2), (t2, t1)):
            nf = n[t] + (1 if self.bc[t] else 0)   # real t-face rows
            for ft in range(nf):
                for co in range(n[o]):
                    start = pos(pos((0, 0, 0), t, ft), o, co)
                    bt, phi2 = row(t, start)
                    for fd in range(-1, n[d] + 2):
                        edge[(t, pos(start, d, fd))] = phi2(fd - 1)
                    for i in range(n[d]):
                        p = pos(start, d, i)
                        newb[t][p[2]][p[1]][p[0]] = bt(i) - dt / h * (phi2(i) - phi2(i - 1))

        def E(t, p):
            """Edge flux of b_t at p: t index a face (mapped), d index a face."""
            q = list(p)
            q[t] = self.face_index(q[t], t)
            return edge[(t, tuple(q))]

        nd = n[d] + (1 if self.bc[d] else 0)       # real d-faces
        for fd in range(nd):
            for c1 in range(n[t1]):
                for c2 in range(n[t2]):
                    p = pos(pos(pos((0, 0, 0), d, fd), t1, c1), t2, c2)
                    e1 = (E(t1, pos(p, t1, c1 + 1)) - E(t1, p)) / self.h[t1]
                    e2 = (E(t2, pos(p, t2, c2 + 1)) - E(t2, p)) / self.h[t2]
                    newb[d][p[2]][p[1]][p[0]] = self.b[d][p[2]][p[1]][p[0]] + dt * (e1 + e2)
        # periodic axes: face n of a face array along its normal is face 0
        self.b = newb

    def sweep(self, op, d, dt):
        if op == 0:
            self.fluid(d, dt)
        else:
            self.field(d, dt)
        return self.state()

    def state(self):
        cell = np.array([[[[float(x) for x in r] for r in pl] for pl in arr] for arr in self.u])
        out = {"cell": cell}
        for a, key in enumerate(("bx", "by", "bz")):
            arr = np.array([[[float(x) for x in r] for r in pl] for pl in self.b[a]])
            if self.bc[a] == 0:  # the interface writes face n equal to face 0
                sl = [slice(None)] * 3
                sl[2 - a] = -1
                s0 = [slice(None)] * 3
                s0[2 - a] = 0
                arr[tuple(sl)] = arr[tuple(s0)]
            out[key] = arr
        return out
