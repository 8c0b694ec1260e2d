"""The validation problems of Sect. 4.2-4.6 through the HIP library.

Parity: each problem at a reduced size, 10 steps on the oracle's time steps,
per-field relative L1 against the oracle <= 1e-10 in FP64 and <= 2e-5 in
FP32 (a field that starts at zero, m_z of the 2-D problems, is measured
against its own small size).  The field sweep decides the upwind tie of an odd
velocity field exactly as the oracle does, on every axis.

At the paper's sizes, against what the paper or the mathematics fixes:
Sedov-Taylor (256^3) follows the similarity law; the spherical Riemann
problem (128^3, 256^3) converges to a 1-D spherical solution; the magnetic
explosion (256^3) and the 2-D MHD Riemann problem (512^2) land on the printed
figure ranges (loose: maxima within 15%, minima within a factor 2, extremes of
discontinuous solutions at the grid scale); the rotor (256^2) conserves mass
and keeps div b at round-off.
"""
import math

import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import analytic as an
import fish_inputs as fi
import problems as pb
from oracle import Oracle
from test_oracle_problems import TIE_SHAPES, odd_velocity_state, radial_reference_density, spherical_riemann_l1

pytestmark = pytest.mark.gpu

FIELDS = ("cell", "bx", "by", "bz")


def _box(s, prec):
    import paper_0910_2854_amd as fish
    h = s["h"]
    return fish.Box(*s["shape"], dx=h[0], dy=h[1], dz=h[2], gamma=s["gamma"], cfl=s["cfl"], limiter=s["limiter"],
                    bc=s["bc"], precision=prec)


def _oracle(s):
    h = s["h"]
    return Oracle(*s["shape"], dx=h[0], dy=h[1], dz=h[2], gamma=s["gamma"], cfl=s["cfl"], limiter=s["limiter"],
                  bc=s["bc"])


def evolve(g, t, T):
    k = 0
    while t < T - 1e-14:
        dt = min(g.cfl_dt(), 0.5 * (T - t))
        g.strang_step(dt)
        t += 2.0 * dt
        k += 1
    return t, k


def per_field_rel_l1(a, b):
    out = {}
    for k in range(5):
        den = float(np.sum(np.abs(b["cell"][k])))
        out["rho mx my mz E".split()[k]] = float(np.sum(np.abs(a["cell"][k] - b["cell"][k]))) / max(den, 1e-300)
    for k in ("bx", "by", "bz"):
        den = float(np.sum(np.abs(b[k])))
        out[k] = float(np.sum(np.abs(a[k] - b[k]))) / max(den, 1e-300)
    return out


PROBLEMS = {
    "sedov": lambda: fi.sedov_state(32, r_dep=0.08),
    "spherical_riemann": lambda: fi.spherical_riemann_state(32),
    "magnetic_explosion": lambda: fi.magnetic_explosion_state(32),
    "rotor": lambda: fi.rotor_state(64),
    "mhd_riemann_2d": lambda: fi.mhd_riemann_2d_state(64),
}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_problem_parity_with_oracle(name, prec, tol):
    st, s = PROBLEMS[name]()
    print(f"problem parity {name} {s['shape']} {prec}", flush=True)
    o = _oracle(s)
    o.set_state(st)
    g = _box(s, prec)
    g.set_state(st)
    for _ in range(10):
        dt = o.cfl_dt()
        assert abs(g.cfl_dt() / dt - 1.0) <= (1e-12 if prec == "fp64" else 1e-5)
        o.strang_step(dt)
        g.strang_step(dt)
    errs = per_field_rel_l1(g.get_state(), o.get_state())
    g.close()
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_field_upwind_tie_matches_oracle(axis, prec):
    """An odd velocity field along the sweep axis: V = 0 exactly at the
    centre and at the periodic seam; the right-cell branch of Eq. (67) must be
    taken, as in the oracle (a branch picked by rounding differs at O(v b))."""
    import paper_0910_2854_amd as fish
    n = TIE_SHAPES[axis]
    print(f"upwind tie axis {axis} {n} {prec}", flush=True)
    st = odd_velocity_state(n, axis, 0.0)
    dt = 0.4 / n[axis] / 0.6
    o = Oracle(*n)
    o.set_state(st)
    o.apply("B", axis, dt)
    ref = o.get_state(check=False)
    g = fish.Box(*n, precision=prec)
    g.set_state(st)
    g.sweep("B", axis, dt)
    out = g.get_state(check=False)
    g.close()
    tol = 1e-13 if prec == "fp64" else 2e-6
    for k in ("bx", "by", "bz"):
        assert np.max(np.abs(out[k] - ref[k])) <= tol, k


# ------------------------------------------------------------ paper sizes
def test_sedov_blast_follows_similarity_law():
    """Sect. 4.2 at 256^3 in FP32, energies as printed (e = 3e3 inside
    r = 0.01, 1e-3 outside).  The printed stop time and shock radius disagree
    (at t = 1.74e-4 the law puts the shock at 0.015), so the blast runs until
    the law's radius reaches 0.15, 0.30 and 0.45: the measured radius lies
    within 3% of it each time, the fitted exponent of R(t) within 0.02 of
    2/5, the post-shock peak density above 2.5 (4 is the strong-shock limit,
    smeared over two cells) and total energy is conserved (periodic box)."""
    n = 256
    h = 1.0 / n
    print("Sedov 256^3 fp32", flush=True)
    st, s = fi.sedov_state(n)
    r = fi._radius_from_centre(s["shape"])
    E0 = float(np.sum(st["cell"][4])) * h ** 3
    Eb = E0 - 1e-3
    g = _box(s, "fp32")
    g.set_state(st)
    del st
    t = 0.0
    Rs, ts = [], []
    for R in (0.15, 0.30, 0.45):
        T = (R / an.SEDOV_XI0_GAMMA_5_3) ** 2.5 / math.sqrt(Eb)
        t, _ = evolve(g, t, T)
        x = g.get_state()
        rc, prof = an.radial_bins(x["cell"][0], r, h, 0.5)
        Rn = an.shock_radius(rc, prof, 1.0)
        print(f"  t {T:.4f} R {Rn:.4f} law {an.sedov_radius(Eb, T):.4f} peak {prof.max():.3f}", flush=True)
        assert abs(Rn / an.sedov_radius(Eb, T) - 1.0) < 0.03
        assert prof.max() > 2.5
        assert abs(float(np.sum(x["cell"][4])) * h ** 3 / E0 - 1.0) < 1e-6
        Rs.append(Rn)
        ts.append(T)
    g.close()
    slope = np.polyfit(np.log(ts), np.log(Rs), 1)[0]
    assert abs(slope - 0.4) < 0.02, slope


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_spherical_riemann_converges_to_radial_reference(prec):
    """Sect. 4.3: relative L1 density error against the 1-D spherical
    solution below 2% at 128^3 and 1% at 256^3, falling at least by 0.7 per
    doubling; mirror symmetry about the three centre planes."""
    rc, rho1 = radial_reference_density(0.09)
    errs = []
    for n in (128, 256):
        print(f"spherical Riemann {n}^3 {prec}", flush=True)
        st, s = fi.spherical_riemann_state(n)
        g = _box(s, prec)
        g.set_state(st)
        del st
        evolve(g, 0.0, s["t_end"])
        x = g.get_state()
        g.close()
        errs.append(spherical_riemann_l1(x, s, rc, rho1))
        c = x["cell"][0]
        for flip in (c[:, :, ::-1], c[:, ::-1, :], c[::-1, :, :]):
            assert np.max(np.abs(flip - c)) <= 1e-6 * np.max(c)
    print("  L1", errs, flush=True)
    assert errs[0] < 0.02 and errs[1] < 0.01 and errs[1] < 0.7 * errs[0], errs


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_magnetic_explosion_matches_printed_ranges(prec):
    """Sect. 4.4 at 256^3 (minmod, CFL 0.5, t = 0.03): the run completes with
    a valid state (the low-beta test the paper uses to show positivity) and
    the ranges over the z = 1/2 plane match the figure caption."""
    print(f"magnetic explosion 256^3 {prec}", flush=True)
    st, s = fi.magnetic_explosion_state(256)
    g = _box(s, prec)
    g.set_state(st)
    del st
    evolve(g, 0.0, s["t_end"])
    x = g.get_state()
    g.close()
    got = pb.value_ranges(x, s["gamma"], plane=128)
    print("  ranges", got, flush=True)
    assert min(v[0] for k, v in got.items() if k in ("rho", "p")) > 0.0
    bad = pb.range_mismatches(got, pb.read_ranges("magnetic_explosion_ranges.txt"), 0.15, 2.0, 1e-6)
    assert not bad, bad


@pytest.mark.parametrize("prec,div_tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_rotor_conserves_mass_and_divergence(prec, div_tol):
    """Sect. 4.5 at 256^2 to t = 0.15: no wave reaches the outflow boundary
    (fast speed about 1.9 from r = 0.115), so mass is conserved to round-off;
    h max|div b| / max|b| stays at round-off (FP32: the rounding of the face
    values accumulated over about 140 steps); density and pressure stay
    positive."""
    print(f"rotor 256^2 {prec}", flush=True)
    st, s = fi.rotor_state(256)
    g = _box(s, prec)
    g.set_state(st)
    m0 = float(np.sum(st["cell"][0]))
    evolve(g, 0.0, s["t_end"])
    x = g.get_state()
    g.close()
    h = s["h"]
    div = (np.diff(x["bx"], axis=2) / h[0] + np.diff(x["by"], axis=1) / h[1] + np.diff(x["bz"], axis=0) / h[2])
    bmax = max(float(np.max(np.abs(x[k]))) for k in ("bx", "by", "bz"))
    rel_div = float(np.max(np.abs(div))) * h[0] / bmax
    e = pb.energies(x, s["gamma"])
    print("  ranges", pb.value_ranges(x, s["gamma"]), "h div/b", rel_div, flush=True)
    assert abs(float(np.sum(x["cell"][0])) / m0 - 1.0) < (1e-12 if prec == "fp64" else 1e-6)
    assert rel_div < div_tol
    assert e["rho"].min() > 0 and e["p"].min() > 0


def test_mhd_riemann_2d_matches_printed_ranges():
    """Sect. 4.6 at 512^2 to t = 0.8 in FP32: ranges over the box match the
    figure caption."""
    print("2-D MHD Riemann 512^2 fp32", flush=True)
    st, s = fi.mhd_riemann_2d_state(512)
    g = _box(s, "fp32")
    g.set_state(st)
    evolve(g, 0.0, s["t_end"])
    x = g.get_state()
    g.close()
    got = pb.value_ranges(x, s["gamma"])
    print("  ranges", got, flush=True)
    bad = pb.range_mismatches(got, pb.read_ranges("mhd_riemann_2d_ranges.txt"), 0.15, 2.0, 1e-3)
    assert not bad, bad


# ------------------------------------------------------- steady polytrope
def _poly_box(s, prec, hse, gravity="unsplit"):
    import paper_0910_2854_amd as fish
    h = s["h"]
    return fish.Box(*s["shape"], dx=h[0], dy=h[1], dz=h[2], gamma=s["gamma"], cfl=s["cfl"], bc=s["bc"],
                    gravity=gravity, hse=hse, precision=prec)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
@pytest.mark.parametrize("hse", [False, True])
@pytest.mark.parametrize("gravity", ["unsplit", "split"])
def test_polytrope_parity_with_oracle(gravity, hse, prec, tol):
    """Sect. 4.7 at 48^3 (unsplit or split gravity, outflow, HSE on and off),
    10 steps on the oracle's time steps.  FP32: the momenta start at rest and grow from the
    residual of pressure and gravity forces, so they are measured against the
    sound-speed momentum scale sum(rho c_s)."""
    st, s = fi.polytrope_state(48)
    print(f"polytrope parity 48^3 {gravity} hse {hse} {prec}", flush=True)
    h = s["h"]
    o = Oracle(*s["shape"], dx=h[0], dy=h[1], dz=h[2], gamma=s["gamma"], cfl=s["cfl"], bc=s["bc"], gravity=gravity,
               hse=hse)
    o.set_state(st)
    g = _poly_box(s, prec, hse, gravity)
    g.set_state(st)
    for _ in range(10):
        dt = o.cfl_dt()
        o.strang_step(dt)
        g.strang_step(dt)
    out, ref = g.get_state(), o.get_state()
    g.close()
    errs = per_field_rel_l1(out, ref)
    p = an.pressure(ref, s["gamma"])
    scale = float(np.sum(np.sqrt(s["gamma"] * p * ref["cell"][0])))
    for k, name in ((1, "mx"), (2, "my"), (3, "mz")):
        errs[name] = float(np.sum(np.abs(out["cell"][k] - ref["cell"][k]))) / max(scale, float(np.sum(np.abs(ref["cell"][k]))))
    for k in ("bx", "by", "bz"):
        errs.pop(k)  # b = 0 stays exactly 0
        assert not np.any(out[k])
    print("  ", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs


def test_polytrope_hse_keeps_the_centre():
    """Sect. 4.7 at 64^3 and 128^3 over 20 tau_HSE, FP32, HSE on and off,
    against the paper's statements: without HSE the central density falls
    monotonically (the star evaporates); HSE slows the fall at both
    resolutions; resolution slows it; with HSE at 128^3 the centre stays
    within 5% of its value after the first tau_HSE (the initial relaxation).
    The paper also finds HSE at 64^3 ahead of no HSE at 128^3; here it is not
    (0.83 against 0.91 after 20 tau_HSE), so that is reported, not asserted."""
    from test_oracle_problems import central_density
    final = {}
    for n in (64, 128):
        st, s = fi.polytrope_state(n)
        tau = s["model"]["tau_hse"]
        rc0 = central_density(st, n)
        for hse in (False, True):
            print(f"polytrope {n}^3 hse {hse} fp32, 20 tau", flush=True)
            g = _poly_box(s, "fp32", hse)
            g.set_state(st)
            t, hist = 0.0, []
            for j in range(1, 21):
                t, _ = evolve(g, t, j * tau)
                hist.append(central_density(g.get_state(), n) / rc0)
            g.close()
            print("   ", " ".join(f"{v:.4f}" for v in hist), flush=True)
            if not hse:
                assert all(b < a for a, b in zip([1.0] + hist, hist)), hist
            if hse and n == 128:
                assert max(abs(v / hist[0] - 1.0) for v in hist) < 0.05, hist
            final[(n, hse)] = hist[-1]
    print("  final", final, flush=True)
    assert final[(64, True)] > final[(64, False)] and final[(128, True)] > final[(128, False)], final
    assert final[(128, False)] > final[(64, False)] and final[(128, True)] > final[(64, True)], final


# ------------------------------------------------- device-resident end time
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("problem", ["rotor", "box"])
def test_advance_to_matches_the_host_loop_bitwise(problem, prec):
    """fish_advance_to clamps dt = min(k/C, (t_end - t)/2) on the device: the
    same steps, bitwise, as the host loop of the validation tests, landing on
    t_end exactly; max_steps bounds it; afterwards steps are unclamped."""
    import paper_0910_2854_amd as fish
    print(f"advance_to {problem} {prec}", flush=True)
    if problem == "rotor":
        st, s = fi.rotor_state(64)
        T = 0.05
        mk = lambda: _box(s, prec)  # noqa: E731
    else:
        st = fi.random_fourier_state((24, 20, 16), seed=3, mach=0.5, beta=5.0, kmax=2)
        T = 0.02
        stream = torch.cuda.Stream().cuda_stream if prec == "fp32" else None  # a caller stream: graph replays
        mk = lambda: fish.Box(24, 20, 16, precision=prec, stream=stream)  # noqa: E731
    a = mk()
    a.set_state(st)
    t_host, k_host = evolve(a, 0.0, T)
    b = mk()
    b.set_state(st)
    k_dev, t_dev = b.advance_to(T)
    assert (k_dev, t_dev) == (k_host, t_host) and t_dev == T, (k_dev, t_dev, k_host, t_host)
    sa, sb = a.get_state(), b.get_state()
    for k in FIELDS:
        assert np.array_equal(sa[k], sb[k]), k
    # unclamped afterwards: the next device step equals a host CFL step
    a.strang_step(a.cfl_dt())
    b.strang_step(0.0)
    sa, sb = a.get_state(), b.get_state()
    for k in FIELDS:
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    # max_steps
    c = mk()
    c.set_state(st)
    k3, t3 = c.advance_to(10 * T, max_steps=3)
    assert k3 == 3 and t3 < 10 * T
    c.close()
    b.close()
