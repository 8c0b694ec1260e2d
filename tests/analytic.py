"""Closed-form and textbook solutions the oracle is pinned against.

Nothing here calls the oracle or the HIP library; these are independent
statements of what ideal MHD (Sect. 2.1 of the FISH paper, Eqs. 1-5) fixes:
linear eigenmodes, the circularly polarised Alfven wave of Sect. 4.1, the
exact Riemann solution of the Euler equations (Toro's textbook method,
pressure-function iteration and wave sampling), and Rankine-Hugoniot jump
states found by root finding.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize

import fish_inputs as fi


def centres(n, L=1.0):
    return (np.arange(n) + 0.5) * (L / n)


def faces(n, L=1.0):
    return np.arange(n + 1) * (L / n)


# ----------------------------------------------------------------- 1-D states
def state_1d(axis, n, rho, v, p, b_t, gamma, b_normal=0.0, L=1.0):
    """A 1-D profile along `axis` (0, 1, 2) in a box with the other axes inactive.

    rho, p: arrays (n,); v: (3, n) in the local frame (normal, t1, t2);
    b_t: (2, n) cell-centred tangential field in the local frame; b_normal a
    constant.  The local frame is cyclic: x:(y,z), y:(z,x), z:(x,y).
    Tangential faces carry the profile; the normal face field is constant.
    """
    shape = [1, 1, 1]
    shape[axis] = n
    nx, ny, nz = shape
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3

    def cellarr(a):
        out = np.asarray(a, dtype=np.float64).reshape(n)
        s = [1, 1, 1]
        s[2 - axis] = n
        return out.reshape(s)

    vel = [None, None, None]
    vel[axis], vel[t1], vel[t2] = cellarr(v[0]), cellarr(v[1]), cellarr(v[2])
    st = fi.empty_state(nx, ny, nz)
    B = [st["bx"], st["by"], st["bz"]]
    B[axis][...] = b_normal
    for comp, arr in ((t1, b_t[0]), (t2, b_t[1])):
        # tangential face field: faces of axis `comp` (inactive, 2 entries) both = profile
        B[comp][...] = cellarr(arr)
    rhoa, pa = cellarr(rho), cellarr(p)
    return fi.conserved_from_primitive(rhoa * np.ones((nz, ny, nx)), vel[0] * np.ones((nz, ny, nx)),
                                       vel[1] * np.ones((nz, ny, nx)), vel[2] * np.ones((nz, ny, nx)),
                                       pa * np.ones((nz, ny, nx)), B[0], B[1], B[2], gamma)


def profile_1d(state, axis):
    """Primitive profile (rho, v_local(3), p, b_t_local(2)) of a 1-D state."""
    cell = state["cell"]
    n = cell.shape[3 - axis]
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    rho = cell[0].reshape(-1)
    m = [cell[1].reshape(-1), cell[2].reshape(-1), cell[3].reshape(-1)]
    bcx, bcy, bcz = fi.cell_centred_b(state["bx"], state["by"], state["bz"])
    bc = [bcx.reshape(-1), bcy.reshape(-1), bcz.reshape(-1)]
    return {"rho": rho, "v": [m[axis] / rho, m[t1] / rho, m[t2] / rho], "E": cell[4].reshape(-1),
            "b": [bc[axis], bc[t1], bc[t2]], "n": n}


def pressure(state, gamma):
    cell = state["cell"]
    bcx, bcy, bcz = fi.cell_centred_b(state["bx"], state["by"], state["bz"])
    rho = cell[0]
    ke = 0.5 * (cell[1] ** 2 + cell[2] ** 2 + cell[3] ** 2) / rho
    return (gamma - 1.0) * (cell[4] - ke - 0.5 * (bcx ** 2 + bcy ** 2 + bcz ** 2))


# ------------------------------------------------------- linear MHD eigenmodes
def fast_speed(rho, p, bn, bt, gamma):
    """Fast magnetosonic speed for propagation along the normal (closed form)."""
    a2 = gamma * p / rho
    b2 = (bn * bn + bt * bt) / rho
    return math.sqrt(0.5 * (a2 + b2 + math.sqrt((a2 + b2) ** 2 - 4.0 * a2 * bn * bn / rho)))


def fast_wave_1d(axis, n, t, eps=1e-6, rho0=1.0, p0=0.6, bn=0.8, bt=0.6, gamma=5.0 / 3.0, k=1):
    """Right-going linear fast wave along `axis`, field in the (normal, t1) plane.

    Linearising Eqs. (1)-(4) for a profile f(x - c t): dv_n = eps f,
    drho = rho0 dv_n / c, dp = gamma p0 dv_n / c,
    db_t1 = bt c dv_n / (c^2 - bn^2/rho0), dv_t1 = -bn db_t1 / (rho0 c),
    with c the fast root of rho0 c^2 - gamma p0 - bt^2 c^2/(c^2 - bn^2/rho0) = 0.
    Returns the state at time t (analytic translation).
    """
    c = fast_speed(rho0, p0, bn, bt, gamma)
    x = centres(n)
    f = np.cos(2 * np.pi * k * (x - c * t))
    dvn = eps * f
    drho = rho0 * dvn / c
    dp = gamma * p0 * dvn / c
    dbt = bt * c * dvn / (c * c - bn * bn / rho0)
    dvt = -bn * dbt / (rho0 * c)
    zero = np.zeros(n)
    return state_1d(axis, n, rho0 + drho, [dvn, dvt, zero], p0 + dp, [bt + dbt, zero], gamma, b_normal=bn), c


def alfven_wave_1d(axis, n, t, eps=1e-6, rho0=1.0, p0=0.6, bn=1.0, gamma=5.0 / 3.0, k=1):
    """Right-going linear Alfven wave along `axis`: db_t2 = eps f, dv_t2 = -db_t2/sqrt(rho0)."""
    vA = bn / math.sqrt(rho0)
    x = centres(n)
    db = eps * np.cos(2 * np.pi * k * (x - vA * t))
    dv = -db / math.sqrt(rho0)
    zero = np.zeros(n)
    one = np.ones(n)
    return state_1d(axis, n, rho0 * one, [zero, zero, dv], p0 * one, [zero, db], gamma, b_normal=bn), vA


def entropy_wave_1d(axis, n, t, amp=0.1, u=1.0, p0=1.0, gamma=5.0 / 3.0):
    x = centres(n)
    rho = 1.0 + amp * np.sin(2 * np.pi * (x - u * t))
    zero = np.zeros(n)
    return state_1d(axis, n, rho, [u * np.ones(n), zero, zero], p0 * np.ones(n), [zero, zero], gamma)


def cpaw_state(N, t=0.0, alpha_deg=30.0, A=0.1, gamma=5.0 / 3.0, p0=0.1):
    """Circularly polarised Alfven wave of Sect. 4.1 on [0, 1/cos a] x [0, 1/sin a].

    rho = 1, v_par = 0, p = 0.1, b_par = 1, v_perp = b_perp = A sin(2 pi xi),
    v_z = b_z = A cos(2 pi xi), xi = x cos a + y sin a (- t for t > 0, the
    Alfven speed being b_par/sqrt(rho) = 1).  The face field is the discrete
    curl of the vector potential of the wave, so div b = 0 to round-off.
    With the field aligned with v (v = +b, rho = 1) the wave moves in -xi
    unless v = -b; here v = b and the wave travels backwards: the exact
    solution at time t is the profile evaluated at xi + t.
    """
    a = math.radians(alpha_deg)
    ca, sa = math.cos(a), math.sin(a)
    Lx, Ly = 1.0 / ca, 1.0 / sa
    nx = ny = N
    dx, dy = Lx / nx, Ly / ny
    xc, yc = centres(nx, Lx), centres(ny, Ly)
    xf, yf = faces(nx, Lx), faces(ny, Ly)
    # vector potential of b = b_par e_par + A sin(2 pi xi) e_perp + A cos(2 pi xi) e_z
    # with e_par = (ca, sa, 0), e_perp = (-sa, ca, 0):
    # A_z(x, y) = b_par (x sa - y ca)... chosen so that curl gives the uniform part,
    # plus the wave part A_par (along e_par direction is not needed):
    # b_perp = -d(psi)/dxi with psi = A cos(2 pi xi)/(2 pi)  -> A_z = psi + uniform part
    # b_z comes from A_perp = A sin(2 pi xi)/(2 pi) e_perp (curl_z = d/dxi A_perp).
    def xi(X, Y):
        return X * ca + Y * sa + t

    # edges: Ax at (x_i, y_{j-1/2}), Ay at (x_{i-1/2}, y_j), Az at (x_{i-1/2}, y_{j-1/2}); nz = 1
    Xa, Ya = np.meshgrid(xc, yf, indexing="xy")  # (ny+1, nx)
    Xb, Yb = np.meshgrid(xf, yc, indexing="xy")  # (ny, nx+1)
    Xc, Yc = np.meshgrid(xf, yf, indexing="xy")  # (ny+1, nx+1)
    k2 = 2 * np.pi
    # uniform field b_par (ca, sa, 0) = curl(A_z e_z) with A_z = y ca - x sa
    Az = (Yc * ca - Xc * sa) + A * np.cos(k2 * xi(Xc, Yc)) / k2
    # perpendicular in-plane potential for b_z: A_perp e_perp, A_perp = A sin(2 pi xi)/(2 pi)
    Ap_a = A * np.sin(k2 * xi(Xa, Ya)) / k2
    Ap_b = A * np.sin(k2 * xi(Xb, Yb)) / k2
    Ax = (-sa) * Ap_a
    Ay = ca * Ap_b
    # periodicity: the uniform part of Az is not periodic, but its differences are
    Ax3 = np.stack([Ax, Ax])  # (nz+1=2, ny+1, nx)
    Ay3 = np.stack([Ay, Ay])  # (2, ny, nx+1)
    Az3 = Az[None]            # (1, ny+1, nx+1)
    bx, by, bz = fi.curl_of_potential(Ax3, Ay3, Az3, dx, dy, 1.0)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    s = np.sin(k2 * xi(X, Y))
    c = np.cos(k2 * xi(X, Y))
    vpar = 0.0
    vperp = A * s
    vx = vpar * ca - vperp * sa
    vy = vpar * sa + vperp * ca
    vz = A * c
    one = np.ones((1, ny, nx))
    st = fi.conserved_from_primitive(one, vx[None] * one, vy[None] * one, vz[None] * one, p0 * one,
                                     bx, by, bz, gamma)
    return st, (Lx, Ly)


# ------------------------------------------------ exact Riemann solver (Euler)
def exact_riemann(WL, WR, gamma, xi):
    """Exact solution of the Euler Riemann problem sampled at xi = x/t.

    W = (rho, u, p).  Star pressure from the pressure function
    f_L(p) + f_R(p) + u_R - u_L = 0 (shock: Rankine-Hugoniot, rarefaction:
    isentropic), solved with a bracketing root finder; then each xi is
    classified into left state / left fan / left star / right star / right fan
    / right state.
    """
    rL, uL, pL = WL
    rR, uR, pR = WR
    g = gamma
    aL, aR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)

    def fK(p, rK, pK, aK):
        if p > pK:
            A = 2.0 / ((g + 1.0) * rK)
            B = (g - 1.0) / (g + 1.0) * pK
            return (p - pK) * math.sqrt(A / (p + B))
        return 2.0 * aK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    fun = lambda p: fK(p, rL, pL, aL) + fK(p, rR, pR, aR) + uR - uL
    pstar = optimize.brentq(fun, 1e-12, 100.0 * max(pL, pR), xtol=1e-15, rtol=1e-15, maxiter=500)
    ustar = 0.5 * (uL + uR) + 0.5 * (fK(pstar, rR, pR, aR) - fK(pstar, rL, pL, aL))

    def star_rho(rK, pK):
        if pstar > pK:
            q = pstar / pK
            gm = (g - 1.0) / (g + 1.0)
            return rK * (q + gm) / (gm * q + 1.0)
        return rK * (pstar / pK) ** (1.0 / g)

    rsL, rsR = star_rho(rL, pL), star_rho(rR, pR)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(xi):
        if s <= ustar:  # left of contact
            if pstar > pL:
                SL = uL - aL * math.sqrt((g + 1) / (2 * g) * pstar / pL + (g - 1) / (2 * g))
                W = (rL, uL, pL) if s <= SL else (rsL, ustar, pstar)
            else:
                asL = aL * (pstar / pL) ** ((g - 1) / (2 * g))
                SHL, STL = uL - aL, ustar - asL
                if s <= SHL:
                    W = (rL, uL, pL)
                elif s >= STL:
                    W = (rsL, ustar, pstar)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * aL) * (uL - s)
                    W = (rL * c ** (2 / (g - 1)), 2 / (g + 1) * (aL + (g - 1) / 2 * uL + s),
                         pL * c ** (2 * g / (g - 1)))
        else:
            if pstar > pR:
                SR = uR + aR * math.sqrt((g + 1) / (2 * g) * pstar / pR + (g - 1) / (2 * g))
                W = (rR, uR, pR) if s >= SR else (rsR, ustar, pstar)
            else:
                asR = aR * (pstar / pR) ** ((g - 1) / (2 * g))
                SHR, STR = uR + aR, ustar + asR
                if s >= SHR:
                    W = (rR, uR, pR)
                elif s <= STR:
                    W = (rsR, ustar, pstar)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * aR) * (uR - s)
                    W = (rR * c ** (2 / (g - 1)), 2 / (g + 1) * (-aR + (g - 1) / 2 * uR + s),
                         pR * c ** (2 * g / (g - 1)))
        out[:, n] = W
    return out, {"pstar": pstar, "ustar": ustar, "rho_star_L": rsL, "rho_star_R": rsR}


# -------------------------------------------- Rankine-Hugoniot by root finding
def mhd_flux_1d(W, gamma):
    """Conserved vector and x-flux of 1-D MHD with b_x = 0, b = (0, by, 0), v = (u, 0, 0).

    W = (rho, u, p, by).  U = (rho, rho u, E, by); F = (rho u, rho u^2 + p + by^2/2,
    (E + p + by^2/2) u, u by).  (Eqs. 1-4 restricted to this geometry.)
    """
    rho, u, p, by = W
    E = p / (gamma - 1) + 0.5 * rho * u * u + 0.5 * by * by
    U = np.array([rho, rho * u, E, by])
    ptot = p + 0.5 * by * by
    F = np.array([rho * u, rho * u * u + ptot, (E + ptot) * u, u * by])
    return U, F


def rh_downstream(WR, s, gamma, guess):
    """Left (post-shock) state W_L with F(W_L) - F(W_R) = s (U(W_L) - U(W_R))."""
    UR, FR = mhd_flux_1d(WR, gamma)

    def res(x):
        UL, FL = mhd_flux_1d(x, gamma)
        r = FL - FR - s * (UL - UR)
        return r / np.array([1.0, 1.0, 1.0, 1.0])

    sol, info, ier, msg = optimize.fsolve(res, guess, full_output=True, xtol=1e-14)
    if ier != 1:
        raise RuntimeError(msg)
    return sol, float(np.max(np.abs(res(sol))))


# ------------------------------------ radial Euler reference (1-D, spherical)
def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _hlle_flux(WL, WR, gamma):
    def cons_flux(W):
        rho, u, p = W
        E = p / (gamma - 1.0) + 0.5 * rho * u * u
        return np.stack([rho, rho * u, E]), np.stack([rho * u, rho * u * u + p, (E + p) * u])

    UL, FL = cons_flux(WL)
    UR, FR = cons_flux(WR)
    cL = np.sqrt(gamma * WL[2] / WL[0])
    cR = np.sqrt(gamma * WR[2] / WR[0])
    SL = np.minimum(np.minimum(WL[1] - cL, WR[1] - cR), 0.0)
    SR = np.maximum(np.maximum(WL[1] + cL, WR[1] + cR), 0.0)
    return (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)


def euler_radial(rho, u, p, dr, gamma, t_end, geometry=2, cfl=0.4, inner="reflect"):
    """Euler equations in one radial coordinate, a textbook finite-volume
    scheme of its own (not the FISH scheme): MUSCL reconstruction of the
    primitive variables with minmod slopes, the HLLE flux, Heun (RK2) steps.

    geometry 0 is planar, 2 spherical: faces r_f = f dr carry the area
    r_f^geometry, cells the volume (r_{i+1}^(g+1) - r_i^(g+1))/(g+1), and the
    momentum gains p_i (A_{i+1} - A_i)/V_i, the pressure on the side walls of
    the cone, so that a uniform pressure at rest stays at rest.  The inner end
    reflects (r = 0, or a wall) or lets waves out; the outer end lets them out
    (zeroth-order extrapolation).  Returns (rho, u, p) at the cell centres."""
    g = gamma
    n = len(rho)
    rf = np.arange(n + 1) * dr
    A = rf ** geometry
    V = (rf[1:] ** (geometry + 1) - rf[:-1] ** (geometry + 1)) / (geometry + 1)
    dA = A[1:] - A[:-1]

    def prim(U):
        r = U[0]
        v = U[1] / r
        return np.stack([r, v, (g - 1.0) * (U[2] - 0.5 * r * v * v)])

    def rhs(U):
        W = prim(U)
        Wg = np.empty((3, n + 4))
        Wg[:, 2:-2] = W
        if inner == "reflect":
            Wg[:, 1], Wg[:, 0] = W[:, 0], W[:, 1]
            Wg[1, :2] *= -1.0
        else:
            Wg[:, 0] = Wg[:, 1] = W[:, 0]
        Wg[:, -2] = Wg[:, -1] = W[:, -1]
        d = np.diff(Wg, axis=1)
        slope = _minmod(d[:, :-1], d[:, 1:])
        F = _hlle_flux(Wg[:, 1:-2] + 0.5 * slope[:, :-1], Wg[:, 2:-1] - 0.5 * slope[:, 1:], g)
        dU = -(A[1:] * F[:, 1:] - A[:-1] * F[:, :-1]) / V
        dU[1] += W[2] * dA / V
        return dU, W

    U = np.stack([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u]).astype(np.float64)
    t = 0.0
    while t < t_end * (1.0 - 1e-12):
        dU, W = rhs(U)
        smax = float(np.max(np.abs(W[1]) + np.sqrt(g * W[2] / W[0])))
        dt = min(cfl * dr / smax, t_end - t)
        U1 = U + dt * dU
        U = 0.5 * (U + U1 + dt * rhs(U1)[0])
        t += dt
    return tuple(prim(U))


# ------------------------------------------------ Sedov-Taylor similarity law
# Radius of a strong point blast of energy E in gas of density rho:
# R = xi0 (E t^2 / rho)^(1/5) (dimensional analysis fixes the exponent);
# xi0 = 1.152 for gamma = 5/3 from the similarity solution (Sedov; Landau &
# Lifshitz, Fluid Mechanics, Sect. 106).
SEDOV_XI0_GAMMA_5_3 = 1.152


def sedov_radius(E, t, rho=1.0, xi0=SEDOV_XI0_GAMMA_5_3):
    return xi0 * (E * t * t / rho) ** 0.2


def radial_bins(field, r, h, rmax):
    """Mean of a cell field in radial shells of width h (shell k: k h <= r < (k+1) h)."""
    k = np.floor(r / h).astype(np.int64).ravel()
    nb = int(rmax / h)
    sel = k < nb
    s = np.bincount(k[sel], weights=field.ravel()[sel], minlength=nb)
    c = np.bincount(k[sel], minlength=nb)
    centres = (np.arange(nb) + 0.5) * h
    return centres[c > 0], s[c > 0] / c[c > 0]


def shock_radius(rc, prof, ambient):
    """Outermost radius where a radial profile falls through the midpoint
    between its peak and the ambient value (linear between shells)."""
    level = ambient + 0.5 * (float(np.max(prof)) - ambient)
    above = np.where(prof > level)[0]
    i = int(above[-1])
    if i + 1 >= len(prof):
        return float(rc[i])
    f = (prof[i] - level) / (prof[i] - prof[i + 1])
    return float(rc[i] + f * (rc[i + 1] - rc[i]))
