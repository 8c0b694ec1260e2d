"""Seeded synthetic initial states shared by the oracle tests and the HIP path.

This module builds inputs only: it holds none of the arithmetic of the
operator-split scheme (no fluxes, limiters, sweeps or time steps).  Every
state is returned as a dict in the layout of the C interface, FP64:

``cell`` (5, nz, ny, nx)   rho, m_x, m_y, m_z, E
``bx``   (nz, ny, nx+1)    face f between cells f-1 and f along x
``by``   (nz, ny+1, nx)
``bz``   (nz+1, ny, nx)
``phi``  (nz, ny, nx) or None

The magnetic field is always the discrete curl of an edge-centred vector
potential, so its discrete divergence vanishes up to round-off.  Total energy
is E = p/(gamma-1) + rho v^2/2 + b_c^2/2 with b_c the mean of the two faces of
a cell (the energy definition of Sect. 2.1 of the FISH paper).

Recipes (unit box unless stated; x_i = (i + 1/2) dx):

* random-Fourier box: rho = 1 + 0.1 sum_{m=1..8} cos(2 pi k_m.x + theta_m),
  k_m integer vectors drawn uniformly from 1 <= |k| <= kmax; each velocity
  component a sum of 8 such modes with N(0,1) amplitudes, scaled to the rms
  Mach number sqrt(<v^2/c_s^2>); p = 1/gamma uniform; b from a vector
  potential of 8 modes per component scaled to <b_c^2> = 2 p / beta.
* stratified sphere: rho = rho_c/(1 + (r/r_c)^2) (1 + 0.01 eta), eta ~ U[-1,1],
  the matching potential and hydrostatic pressure in closed form (G = 1),
  v = 0, weak random-potential b with <b_c^2> = 2 <p>/beta; outflow boundaries.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "empty_state", "conserved_from_primitive", "cell_centred_b", "curl_of_potential",
    "random_fourier_state", "sphere_state", "uniform_state", "kvectors", "batch_box_specs",
    "serving_requests", "sedov_state", "spherical_riemann_state", "magnetic_explosion_state", "rotor_state",
    "mhd_riemann_2d_state",
]


def empty_state(nx, ny, nz, with_phi=False):
    return {
        "cell": np.zeros((5, nz, ny, nx)),
        "bx": np.zeros((nz, ny, nx + 1)),
        "by": np.zeros((nz, ny + 1, nx)),
        "bz": np.zeros((nz + 1, ny, nx)),
        "phi": np.zeros((nz, ny, nx)) if with_phi else None,
    }


def cell_centred_b(bx, by, bz):
    """Mean of the two faces of each cell, per component."""
    return (0.5 * (bx[:, :, :-1] + bx[:, :, 1:]),
            0.5 * (by[:, :-1, :] + by[:, 1:, :]),
            0.5 * (bz[:-1, :, :] + bz[1:, :, :]))


def conserved_from_primitive(rho, vx, vy, vz, p, bx, by, bz, gamma, phi=None):
    """Assemble a state dict from primitive cell fields and face fields."""
    bcx, bcy, bcz = cell_centred_b(bx, by, bz)
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz)
    cell = np.stack([rho, rho * vx, rho * vy, rho * vz, E]).astype(np.float64)
    return {"cell": np.ascontiguousarray(cell), "bx": np.ascontiguousarray(bx, dtype=np.float64),
            "by": np.ascontiguousarray(by, dtype=np.float64), "bz": np.ascontiguousarray(bz, dtype=np.float64),
            "phi": None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)}


def kvectors(kmax, dims=3):
    """All integer wave vectors with 1 <= |k| <= kmax (Euclidean norm)."""
    r = np.arange(-kmax, kmax + 1)
    if dims == 3:
        kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    else:
        kx, ky = np.meshgrid(r, r, indexing="ij")
        kz = np.zeros_like(kx)
    k = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    n2 = (k * k).sum(axis=1)
    return k[(n2 >= 1) & (n2 <= kmax * kmax)]


def _modes(coords, ks, thetas, amps):
    """sum_m amp_m cos(2 pi k_m . x + theta_m) on the grid given by 1-D coords.

    coords = (x, y, z) 1-D position arrays; result shape (len z, len y, len x).
    Uses separable complex exponentials (exact up to round-off).
    """
    x, y, z = coords
    ks = np.asarray(ks, dtype=np.float64)
    ph = np.asarray(amps, dtype=np.float64) * np.exp(1j * np.asarray(thetas, dtype=np.float64))
    ex = np.exp(2j * np.pi * np.outer(ks[:, 0], x))                      # (m, nx)
    ey = np.exp(2j * np.pi * np.outer(ks[:, 1], y))                      # (m, ny)
    ez = np.exp(2j * np.pi * np.outer(ks[:, 2], z)) * ph[:, None]        # (m, nz)
    t = (ez[:, :, None] * ey[:, None, :]).reshape(len(ks), -1)           # (m, nz*ny)
    # real part of the sum over modes as two real products over the mode index
    out = t.real.T @ ex.real - t.imag.T @ ex.imag
    return out.reshape(len(z), len(y), len(x))


def curl_of_potential(Ax, Ay, Az, dx, dy, dz):
    """Face fields b = curl A from edge-centred potentials.

    Ax[k, j, i] sits on the x-edge at (x_i, y_{j-1/2}, z_{k-1/2}), shape
    (nz+1, ny+1, nx); Ay[k, j, i] on (x_{i-1/2}, y_j, z_{k-1/2}), shape
    (nz+1, ny, nx+1); Az[k, j, i] on (x_{i-1/2}, y_{j-1/2}, z_k), shape
    (nz, ny+1, nx+1).  Returns bx (nz, ny, nx+1), by (nz, ny+1, nx),
    bz (nz+1, ny, nx), whose discrete divergence is zero up to round-off.
    """
    bx = (Az[:, 1:, :] - Az[:, :-1, :]) / dy - (Ay[1:, :, :] - Ay[:-1, :, :]) / dz
    by = (Ax[1:, :, :] - Ax[:-1, :, :]) / dz - (Az[:, :, 1:] - Az[:, :, :-1]) / dx
    bz = (Ay[:, :, 1:] - Ay[:, :, :-1]) / dx - (Ax[:, 1:, :] - Ax[:, :-1, :]) / dy
    return bx, by, bz


def _potential_field(rng, n, L, kmax, nmodes, periodic):
    """Random edge-centred vector potential -> face field (unscaled)."""
    nx, ny, nz = n
    Lx, Ly, Lz = L
    dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
    kset = kvectors(kmax)
    cen = [(np.arange(m) + 0.5) * d for m, d in zip(n, (dx, dy, dz))]       # cell centres
    lo = [np.arange(m + 1) * d for m, d in zip(n, (dx, dy, dz))]            # low faces 0..n
    comps = []
    for _ in range(3):
        idx = rng.integers(0, len(kset), size=nmodes)
        th = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        amp = rng.standard_normal(nmodes)
        # wave vectors in units of the box: k / L per axis
        comps.append((kset[idx], th, amp))

    def evaluate(comp, coords):
        ks, th, amp = comp
        kk = ks.astype(np.float64) / np.array([Lx, Ly, Lz])
        return _modes(coords, kk, th, amp)

    Ax = evaluate(comps[0], (cen[0], lo[1], lo[2]))
    Ay = evaluate(comps[1], (lo[0], cen[1], lo[2]))
    Az = evaluate(comps[2], (lo[0], lo[1], cen[2]))
    if periodic:
        # exact periodic images: index n along a face axis equals index 0
        Ax[:, -1, :] = Ax[:, 0, :]
        Ax[-1, :, :] = Ax[0, :, :]
        Ay[:, :, -1] = Ay[:, :, 0]
        Ay[-1, :, :] = Ay[0, :, :]
        Az[:, :, -1] = Az[:, :, 0]
        Az[:, -1, :] = Az[:, 0, :]
    return curl_of_potential(Ax, Ay, Az, dx, dy, dz)


def random_fourier_state(n, seed, mach=0.5, beta=10.0, kmax=4, gamma=5.0 / 3.0, nmodes=8, L=(1.0, 1.0, 1.0)):
    """Periodic random-Fourier box (smooth, shock-forming at high Mach)."""
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = n
    rng = np.random.Generator(np.random.PCG64(seed))
    kset = kvectors(kmax)
    cen = [(np.arange(m) + 0.5) * (l / m) for m, l in zip(n, L)]
    scale = np.array(L, dtype=np.float64)

    idx = rng.integers(0, len(kset), size=nmodes)
    th = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    rho = 1.0 + 0.1 * _modes(cen, kset[idx] / scale, th, np.ones(nmodes))

    vel = []
    for _ in range(3):
        idx = rng.integers(0, len(kset), size=nmodes)
        th = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        amp = rng.standard_normal(nmodes)
        vel.append(_modes(cen, kset[idx] / scale, th, amp))
    p0 = 1.0 / gamma
    p = np.full((nz, ny, nx), p0)
    cs2 = gamma * p / rho
    msq = np.mean((vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2) / cs2)
    vs = mach / math.sqrt(msq) if msq > 0 else 0.0
    vx, vy, vz = (v * vs for v in vel)

    bx, by, bz = _potential_field(rng, n, L, kmax, nmodes, periodic=True)
    bcx, bcy, bcz = cell_centred_b(bx, by, bz)
    b2 = np.mean(bcx ** 2 + bcy ** 2 + bcz ** 2)
    bs = math.sqrt(2.0 * p0 / beta / b2) if (beta > 0 and b2 > 0) else 0.0
    return conserved_from_primitive(rho, vx, vy, vz, p, bx * bs, by * bs, bz * bs, gamma)


def sphere_state(n, seed, gamma=5.0 / 3.0, rho_c=1.0, r_c=0.1, beta=100.0, kmax=4, nmodes=8, noise=0.01):
    """Stratified sphere in a fixed potential, for outflow boundaries (G = 1).

    rho = rho_c/(1+x^2), x = r/r_c; enclosed-mass potential
    phi = 4 pi rho_c r_c^2 (atan(x)/x + ln(1+x^2)/2) solves lap phi = 4 pi rho;
    p = 4 pi rho_c^2 r_c^2 (pi^2/8 - atan(x)/x - atan(x)^2/2) solves
    dp/dr = -rho dphi/dr with p -> 0 at infinity.
    """
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = n
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(nx) + 0.5) / nx - 0.5
    y = (np.arange(ny) + 0.5) / ny - 0.5
    z = (np.arange(nz) + 0.5) / nz - 0.5
    r = np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2)
    s = r / r_c
    small = s < 1e-6
    s_safe = np.where(small, 1.0, s)
    atan_over = np.where(small, 1.0 - s * s / 3.0, np.arctan(s_safe) / s_safe)
    K = 4.0 * math.pi * rho_c * r_c * r_c
    phi = K * (atan_over + 0.5 * np.log1p(s * s))
    p = K * rho_c * (math.pi ** 2 / 8.0 - atan_over - 0.5 * np.arctan(s) ** 2)
    eta = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    rho = rho_c / (1.0 + s * s) * (1.0 + noise * eta)
    zero = np.zeros_like(rho)
    bx, by, bz = _potential_field(rng, n, (1.0, 1.0, 1.0), kmax, nmodes, periodic=False)
    bcx, bcy, bcz = cell_centred_b(bx, by, bz)
    b2 = np.mean(bcx ** 2 + bcy ** 2 + bcz ** 2)
    bs = math.sqrt(2.0 * float(np.mean(p)) / beta / b2)
    return conserved_from_primitive(rho, zero, zero, zero, p, bx * bs, by * bs, bz * bs, gamma, phi=phi)


def uniform_state(n, rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, b=(0.0, 0.0, 0.0), gamma=5.0 / 3.0):
    nx, ny, nz = n
    one = np.ones((nz, ny, nx))
    bx = np.full((nz, ny, nx + 1), float(b[0]))
    by = np.full((nz, ny + 1, nx), float(b[1]))
    bz = np.full((nz + 1, ny, nx), float(b[2]))
    return conserved_from_primitive(rho * one, v[0] * one, v[1] * one, v[2] * one, p * one, bx, by, bz, gamma)


# Edge lengths of the batched many-box workload (geometric set 16..64).
BATCH_EDGES = (16, 24, 32, 48, 64)


def batch_box_specs(nboxes, base_seed=1000, edges=BATCH_EDGES, seed=0):
    """Per-box (edge, seed, mach, beta) of the batched workload.

    Edge drawn uniformly from the geometric set (log-uniform), Mach from
    U[0.3, 2], beta log-uniform on [0.5, 50]; box b uses seed base_seed + b.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(nboxes):
        e = int(edges[rng.integers(0, len(edges))])
        mach = float(rng.uniform(0.3, 2.0))
        beta = float(math.exp(rng.uniform(math.log(0.5), math.log(50.0))))
        out.append({"edge": e, "seed": base_seed + b, "mach": mach, "beta": beta})
    return out


def serving_requests(nreq, rate, seed=7, edge_range=(32, 192), step_range=(10, 200)):
    """Poisson-arrival request stream: (arrival time, edge, steps, seed).

    Inter-arrival times are exponential with the given rate (requests per
    second); edges log-uniform on edge_range (rounded to an integer), step
    counts uniform on step_range (inclusive).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    lo, hi = math.log(edge_range[0]), math.log(edge_range[1])
    for r in range(nreq):
        t += float(rng.exponential(1.0 / rate))
        edge = int(round(math.exp(rng.uniform(lo, hi))))
        steps = int(rng.integers(step_range[0], step_range[1] + 1))
        out.append({"arrival": t, "edge": edge, "steps": steps, "seed": 100000 + r})
    return out


# ---------------------------------------------------------------------------
# Initial states of the paper's validation problems (Sect. 4.2-4.6).  Every
# field is sampled at cell centres (faces for b); a cell belongs to a region
# when its centre does.  Each builder returns (state, setup) where setup holds
# the box shape, spacings, gamma, boundaries, limiter, CFL number and end time
# that the section states (or the reading taken where it states none).

PERIODIC_BC, OUTFLOW_BC = 0, 1
MINMOD_LIMITER, VANLEER_LIMITER = 0, 1


def _centres(n, L=1.0):
    return (np.arange(n) + 0.5) * (L / n)


def _radius_from_centre(n, L=(1.0, 1.0, 1.0)):
    nx, ny, nz = n
    x = _centres(nx, L[0]) - 0.5 * L[0]
    y = _centres(ny, L[1]) - 0.5 * L[1]
    z = _centres(nz, L[2]) - 0.5 * L[2]
    return np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2)


def _setup(n, L, gamma, bc, limiter, cfl, t_end):
    return {"shape": tuple(int(v) for v in n), "h": tuple(L[a] / n[a] for a in range(3)), "L": tuple(L),
            "gamma": gamma, "bc": tuple(bc), "limiter": limiter, "cfl": cfl, "t_end": t_end}


def sedov_state(n=256, e_in=3.0e3, e_out=1.0e-3, r_dep=0.01, gamma=5.0 / 3.0):
    """Sedov-Taylor blast (Sect. 4.2): unit cube, rho = 1, v = 0, internal
    energy per volume e_in inside r < r_dep around the centre and e_out outside,
    b = 0.  The end time is left to the caller (the section's stop time and
    shock radius do not agree with each other)."""
    N = (n, n, n)
    r = _radius_from_centre(N)
    e = np.where(r < r_dep, e_in, e_out)
    one = np.ones_like(r)
    zero = 0.0 * one
    st = conserved_from_primitive(one, zero, zero, zero, (gamma - 1.0) * e, np.zeros((n, n, n + 1)),
                                  np.zeros((n, n + 1, n)), np.zeros((n + 1, n, n)), gamma)
    return st, _setup(N, (1.0,) * 3, gamma, (PERIODIC_BC,) * 3, VANLEER_LIMITER, 0.5, None)


def spherical_riemann_state(n=256, gamma=5.0 / 3.0):
    """Spherical Riemann problem (Sect. 4.3): unit cube, v = 0, b = 0;
    rho = 0.125, p = 0.1 inside r < 0.25 around the centre, rho = 1, p = 1
    outside; t = 0.09."""
    N = (n, n, n)
    r = _radius_from_centre(N)
    inside = r < 0.25
    rho = np.where(inside, 0.125, 1.0)
    p = np.where(inside, 0.1, 1.0)
    zero = 0.0 * rho
    st = conserved_from_primitive(rho, zero, zero, zero, p, np.zeros((n, n, n + 1)), np.zeros((n, n + 1, n)),
                                  np.zeros((n + 1, n, n)), gamma)
    return st, _setup(N, (1.0,) * 3, gamma, (OUTFLOW_BC,) * 3, VANLEER_LIMITER, 0.5, 0.09)


def magnetic_explosion_state(n=256, gamma=5.0 / 3.0):
    """Magnetic explosion (Sect. 4.4): unit cube, rho = 1, v = 0; p = 100 for
    r < 0.1, p = 1 for r > 0.125, linear in r between; b = (7, 7, 0)/sqrt(2);
    minmod limiter, CFL 0.5, t = 0.03."""
    N = (n, n, n)
    r = _radius_from_centre(N)
    p = np.where(r < 0.1, 100.0, np.where(r < 0.125, 100.0 + (1.0 - 100.0) * (r - 0.1) / 0.025, 1.0))
    one = np.ones_like(r)
    zero = 0.0 * one
    b0 = 7.0 / math.sqrt(2.0)
    st = conserved_from_primitive(one, zero, zero, zero, p, np.full((n, n, n + 1), b0), np.full((n, n + 1, n), b0),
                                  np.zeros((n + 1, n, n)), gamma)
    return st, _setup(N, (1.0,) * 3, gamma, (OUTFLOW_BC,) * 3, MINMOD_LIMITER, 0.5, 0.03)


def rotor_state(n=256, gamma=1.4):
    """Rotor (Sect. 4.5): unit square, one cell along z.  rho = 10 spinning
    at angular speed 2/r0 inside r0 = 0.1, resting rho = 1 beyond r1 = 0.115,
    the taper f = (r1 - r)/(r1 - r0) between; p = 1, b = (5/sqrt(4 pi), 0, 0),
    gamma = 1.4, t = 0.15."""
    x = _centres(n)
    X = x[None, None, :] - 0.5
    Y = x[None, :, None] - 0.5
    r = np.sqrt(X * X + Y * Y)
    r0, r1 = 0.1, 0.115
    f = (r1 - r) / (r1 - r0)
    rho = np.where(r < r0, 10.0, np.where(r < r1, 1.0 + 9.0 * f, 1.0))
    w = np.where(r < r0, 2.0 / r0, np.where(r < r1, 2.0 * f / np.maximum(r, 1e-300), 0.0))
    vx = -w * Y
    vy = w * X
    one = np.ones((1, n, n))
    st = conserved_from_primitive(rho * one, vx * one, vy * one, 0.0 * one, one,
                                  np.full((1, n, n + 1), 5.0 / math.sqrt(4.0 * math.pi)), np.zeros((1, n + 1, n)),
                                  np.zeros((2, n, n)), gamma)
    return st, _setup((n, n, 1), (1.0, 1.0, 1.0 / n), gamma, (OUTFLOW_BC, OUTFLOW_BC, PERIODIC_BC),
                      VANLEER_LIMITER, 0.5, 0.15)


def mhd_riemann_2d_state(n=512, gamma=5.0 / 3.0, L=0.8):
    """Two-dimensional MHD Riemann problem (Sect. 4.6): [0, 0.8]^2, one cell
    along z, four constant quadrants (rho, v_x, v_y) = (1, -0.75, 0.5) lower
    left, (3, -0.75, -0.5) lower right, (2, 0.75, 0.5) upper left,
    (1, 0.75, -0.5) upper right, v_z = 0, p = 1; b = (2, 0, 1)/sqrt(4 pi);
    zeroth-order extrapolation (outflow) boundaries; t = 0.8."""
    x = _centres(n, L)
    lx = (x <= 0.5 * L)[None, None, :]
    ly = (x <= 0.5 * L)[None, :, None]
    rho = np.where(ly, np.where(lx, 1.0, 3.0), np.where(lx, 2.0, 1.0))
    vx = np.where(ly, -0.75, 0.75) * np.ones_like(rho)
    vy = np.where(ly, np.where(lx, 0.5, -0.5), np.where(lx, 0.5, -0.5))
    one = np.ones((1, n, n))
    s4 = math.sqrt(4.0 * math.pi)
    st = conserved_from_primitive(rho * one, vx * one, vy * one, 0.0 * one, one, np.full((1, n, n + 1), 2.0 / s4),
                                  np.zeros((1, n + 1, n)), np.full((2, n, n), 1.0 / s4), gamma)
    return st, _setup((n, n, 1), (L, L, L / n), gamma, (OUTFLOW_BC, OUTFLOW_BC, PERIODIC_BC), VANLEER_LIMITER, 0.5,
                      0.8)


def lane_emden(n_index=3.0, xi_max=20.0):
    """Lane-Emden solution theta(xi) of index n: theta'' + 2 theta'/xi +
    theta^n = 0, theta(0) = 1, theta'(0) = 0, integrated (from a series start
    at xi = 1e-4) to its first zero xi1.  Returns (theta, xi1, dtheta_xi1) with
    theta a callable that is 0 beyond xi1."""
    from scipy.integrate import solve_ivp

    n = float(n_index)
    x0 = 1e-4
    y0 = [1.0 - x0 ** 2 / 6.0 + n * x0 ** 4 / 120.0, -x0 / 3.0 + n * x0 ** 3 / 30.0]

    def rhs(x, y):
        th = max(y[0], 0.0)
        return [y[1], -th ** n - 2.0 * y[1] / x]

    def surface(x, y):
        return y[0]
    surface.terminal = True
    surface.direction = -1
    sol = solve_ivp(rhs, (x0, xi_max), y0, events=surface, dense_output=True, rtol=1e-12, atol=1e-14,
                    method="DOP853")
    xi1 = float(sol.t_events[0][0])
    dth1 = float(sol.y_events[0][0][1])

    def theta(xi):
        xi = np.asarray(xi, dtype=np.float64)
        out = np.zeros_like(xi)
        inner = xi < x0
        mid = (~inner) & (xi < xi1)
        out[inner] = 1.0 - xi[inner] ** 2 / 6.0
        if np.any(mid):
            out[mid] = np.maximum(sol.sol(xi[mid])[0], 0.0)
        return out

    return theta, xi1, dth1


def polytrope_model(M=1.0, R=1.0, G=1.0, n_index=3.0):
    """Polytropic star p = kappa rho^(1+1/n) of mass M and radius R
    (Sect. 4.7): central density, kappa, mean density, the length scale alpha
    = R/xi1, and the hydrostatic time scale (rho_mean G)^(-1/2)/2."""
    theta, xi1, dth1 = lane_emden(n_index)
    alpha = R / xi1
    rho_c = M * xi1 / (4.0 * math.pi * R ** 3 * (-dth1))
    kappa = 4.0 * math.pi * G * alpha ** 2 * rho_c ** (1.0 - 1.0 / n_index) / (n_index + 1.0)
    rho_mean = M / (4.0 / 3.0 * math.pi * R ** 3)
    return {"theta": theta, "xi1": xi1, "dtheta_xi1": dth1, "alpha": alpha, "rho_c": rho_c, "kappa": kappa,
            "rho_mean": rho_mean, "tau_hse": 0.5 / math.sqrt(rho_mean * G), "n": n_index, "M": M, "R": R, "G": G}


def polytrope_state(n=64, L=2.9, atmosphere=1e-6, gamma=4.0 / 3.0, virial_atmosphere=True):
    """Steady polytrope (Sect. 4.7) in units G = M = R = 1: an n = 3 star
    centred in [0, L]^3; rho = rho_c theta^3 inside R, a resting atmosphere of
    rho_atm = atmosphere * rho_c outside; p = kappa rho^(4/3), but at least
    rho_atm G M / R (the atmosphere at the virial temperature, not in
    equilibrium; a colder one falls in supersonically and a total-energy
    scheme then recovers negative pressures within half a tau_HSE); the fixed
    potential -M/R - 4 kappa rho_c^(1/3) theta inside and -M/r outside; v = 0,
    b = 0; gas gamma 4/3; outflow boundaries."""
    mod = polytrope_model()
    N = (n, n, n)
    r = _radius_from_centre(N, (L, L, L))
    th = mod["theta"](r / mod["alpha"])
    inside = r < mod["R"]
    rho = np.where(inside, mod["rho_c"] * th ** 3, atmosphere * mod["rho_c"])
    rho = np.maximum(rho, atmosphere * mod["rho_c"])
    p = mod["kappa"] * rho ** (4.0 / 3.0)
    if virial_atmosphere:
        p = np.maximum(p, atmosphere * mod["rho_c"] * mod["G"] * mod["M"] / mod["R"])
    phi = np.where(inside, -mod["M"] / mod["R"] - 4.0 * mod["kappa"] * mod["rho_c"] ** (1.0 / 3.0) * th,
                   -mod["M"] / np.maximum(r, 1e-300))
    zero = np.zeros_like(rho)
    st = conserved_from_primitive(rho, zero, zero, zero, p, np.zeros((n, n, n + 1)), np.zeros((n, n + 1, n)),
                                  np.zeros((n + 1, n, n)), gamma, phi=phi)
    s = _setup(N, (L,) * 3, gamma, (OUTFLOW_BC,) * 3, VANLEER_LIMITER, 0.5, 20.0 * mod["tau_hse"])
    s["model"] = mod
    return st, s
