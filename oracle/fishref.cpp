// fishref.cpp -- plain FP64 CPU oracle of the FISH operator-split MHD step.
//
// TEST INFRASTRUCTURE ONLY (see fishref.h).  Written from Sect. 2 of the FISH
// paper, one pencil at a time, on ghost-padded arrays, in the order and
// notation of the paper.  No blocking, no fusion, no streaming: every
// intermediate quantity of a pencil is held in its own plain array.
//
// Readings of passages the paper leaves open are marked "reading:".  The
// matching list (with the reasons) is kept with the design notes.
//
// Parity pins: every function below is exercised by the CPU tests against
// closed forms, invariants, textbook solutions or brute force, except for the
// reading-level choices listed as "parity unpinned" in the file header of the
// Python binding (oracle/__init__.py).

#include "fishref.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Ghost depth.  The fluid operator has a 7-cell stencil (3 per side, Sect. 3),
// the field operator smooths the edge velocity once more (Eq. 66): 4 per side.
constexpr int G = 4;

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4 };
enum { PERIODIC = 0, OUTFLOW = 1 };

struct Ctx {
  fishref_params p{};
  int n[3]{};
  double h[3]{};
  int N[3]{};  // padded extent n + 2G
  std::vector<double> u[5];
  std::vector<double> b[3];  // face f along the normal stored at padded cell f
  std::vector<double> phi;
  // Irregular Cartesian mesh (Sect. 2.5): the width of every padded cell
  // along each axis (ghosts take the width of the cell they copy or wrap to).
  // Uniform meshes keep the formulas of Sects. 2.2-2.4 exactly.
  bool nonuniform = false;
  std::vector<double> hs[3];
  bool have_state = false;
  double t = 0.0;
  int status = FISHREF_OK;
  std::string err;

  size_t at(int i, int j, int k) const {
    return (size_t)(i + G) + (size_t)N[0] * ((size_t)(j + G) + (size_t)N[1] * (size_t)(k + G));
  }
  size_t ncell_padded() const { return (size_t)N[0] * N[1] * N[2]; }
  // number of real faces of b[a] along its normal
  int nface(int a) const { return p.bc[a] == OUTFLOW ? n[a] + 1 : n[a]; }
};

// Widths of the padded cells along axis a from the real widths w[0..n-1]:
// a periodic ghost takes the width of the cell it wraps to, an outflow ghost
// that of the nearest real cell (the cell it copies).
void fill_spacing(Ctx* c, int a, const double* w) {
  const int n = c->n[a];
  c->hs[a].assign(n + 2 * G, 0.0);
  for (int m = 0; m < n + 2 * G; ++m) {
    int i = m - G;
    if (i < 0 || i >= n) i = (c->p.bc[a] == PERIODIC || n == 1) ? ((i % n) + n) % n : (i < 0 ? 0 : n - 1);
    c->hs[a][m] = w[i];
  }
}

int fail(Ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

// ---------------------------------------------------------------- boundaries
// Sect. 4 (periodic boundaries unless stated), Sect. 4.6 (zeroth-order
// extrapolation), Sect. 4.7 ("continuous" boundaries for the polytrope).
// reading: outflow = zeroth-order extrapolation: a ghost copies the nearest
// real entry; for a face array along its own normal the last real face is
// face n.
int source_index(int i, int n, int bc, bool normal_face) {
  if (bc == PERIODIC) return ((i % n) + n) % n;
  const int hi = normal_face ? n : n - 1;
  return std::min(std::max(i, 0), hi);
}

// Fill the ghosts of one padded array along one axis, over the full padded
// range of the two other axes.  Done for x, then y, then z, so corners hold
// the value of the corner of the real domain they fold onto.
void fill_axis(Ctx* c, std::vector<double>& a, int axis, bool normal_face) {
  const int n = c->n[axis];
  const int bc = c->p.bc[axis];
  const int hi_real = (normal_face && bc == OUTFLOW) ? n : n - 1;
  const int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
#pragma omp parallel for collapse(2) schedule(static)
  for (int s2 = -G; s2 < c->n[o2] + G; ++s2)
    for (int s1 = -G; s1 < c->n[o1] + G; ++s1)
      for (int s = -G; s < n + G; ++s) {
        if (s >= 0 && s <= hi_real) continue;
        int q[3], r[3];
        q[axis] = s;
        q[o1] = s1;
        q[o2] = s2;
        r[axis] = source_index(s, n, bc, normal_face);
        r[o1] = s1;
        r[o2] = s2;
        a[c->at(q[0], q[1], q[2])] = a[c->at(r[0], r[1], r[2])];
      }
}

void fill_ghosts(Ctx* c) {
  for (int axis = 0; axis < 3; ++axis) {
    for (int f = 0; f < 5; ++f) fill_axis(c, c->u[f], axis, false);
    for (int a = 0; a < 3; ++a) fill_axis(c, c->b[a], axis, a == axis);
  }
}

// The potential is fixed in time (Sect. 2.3).  reading: on an outflow axis it
// is extrapolated linearly from the two nearest real cells, so that the
// centred gradient of Eq. (40) stays the same across the boundary.
void fill_phi_ghosts(Ctx* c) {
  for (int axis = 0; axis < 3; ++axis) {
    const int n = c->n[axis];
    const int bc = c->p.bc[axis];
    for (int k = -G; k < c->n[2] + G; ++k)
      for (int j = -G; j < c->n[1] + G; ++j)
        for (int i = -G; i < c->n[0] + G; ++i) {
          int q[3] = {i, j, k};
          const int s = q[axis];
          if (s >= 0 && s < n) continue;
          int r0[3] = {i, j, k}, r1[3] = {i, j, k};
          double val;
          if (bc == PERIODIC || n == 1) {
            r0[axis] = ((s % n) + n) % n;
            val = c->phi[c->at(r0[0], r0[1], r0[2])];
          } else if (s < 0) {
            r0[axis] = 0;
            r1[axis] = 1;
            const double p0 = c->phi[c->at(r0[0], r0[1], r0[2])];
            const double p1 = c->phi[c->at(r1[0], r1[1], r1[2])];
            val = p0 + (double)s * (p1 - p0);
          } else {
            r0[axis] = n - 1;
            r1[axis] = n - 2;
            const double p0 = c->phi[c->at(r0[0], r0[1], r0[2])];
            const double p1 = c->phi[c->at(r1[0], r1[1], r1[2])];
            val = p0 + (double)(s - (n - 1)) * (p0 - p1);
          }
          c->phi[c->at(i, j, k)] = val;
        }
  }
}

// ------------------------------------------------------------ cell physics
// Quantities of one cell for a sweep along axis d, from the conserved state u
// and the cell-centred field b (Sect. 2.2: "held constant and interpolated to
// cell centers"; reading: the mean of the two faces of the cell).
struct CellQ {
  double u[5];
  double F[5];   // directional flux, Eq. (17) rotated to axis d
  double vd;     // v_d
  double cF;     // fast magnetosonic speed along d
  double cS;     // sound speed
  double p;      // gas pressure
  double d;      // freezing speed |v_d| + c_F, Eq. (21)
  double xi[5];  // hydrostatic gradient vector, Eq. (50)
  bool supersonic;  // |v| > c_S (the limiter switch of Sect. 2.2)
};

CellQ cell_quantities(const double* u, const double* b, int d, double gamma) {
  CellQ c;
  for (int k = 0; k < 5; ++k) c.u[k] = u[k];
  const double rho = u[RHO];
  const double v[3] = {u[MX] / rho, u[MY] / rho, u[MZ] / rho};
  const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const double m2 = u[MX] * u[MX] + u[MY] * u[MY] + u[MZ] * u[MZ];
  // E = rho e + rho v^2/2 + b^2/2 and p = rho e (gamma - 1): Sect. 2.1, Eq. (5).
  const double p = (gamma - 1.0) * (u[EN] - 0.5 * m2 / rho - 0.5 * b2);
  const double ptot = p + 0.5 * b2;  // P_tot = p + b^2/2
  const double bv = b[0] * v[0] + b[1] * v[1] + b[2] * v[2];
  // Fast magnetosonic speed along d (the speed named after Eq. 21):
  // c_F^2 = (a^2 + b^2/rho + sqrt((a^2 + b^2/rho)^2 - 4 a^2 b_d^2/rho)) / 2.
  // reading: the exact directional fast speed, not an isotropic bound.
  const double a2 = gamma * p / rho;
  const double q = a2 + b2 / rho;
  const double disc = q * q - 4.0 * a2 * b[d] * b[d] / rho;
  const double cf = std::sqrt(0.5 * (q + std::sqrt(std::max(disc, 0.0))));
  // Flux vector, Eq. (17), with x replaced by d.
  c.F[RHO] = u[MX + d];
  for (int k = 0; k < 3; ++k) {
    double f = u[MX + d] * v[k] - b[d] * b[k];
    if (k == d) f += ptot;
    c.F[MX + k] = f;
  }
  c.F[EN] = (u[EN] + ptot) * v[d] - b[d] * bv;
  c.vd = v[d];
  c.cF = cf;
  c.cS = std::sqrt(a2);
  c.p = p;
  c.supersonic = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > a2;
  c.d = std::fabs(v[d]) + cf;
  c.xi[RHO] = -u[RHO];
  c.xi[MX] = -u[MX];
  c.xi[MY] = -u[MY];
  c.xi[MZ] = -u[MZ];
  c.xi[EN] = -(u[EN] + p);
  return c;
}

// Flux limiters, Sect. 2.2.
// minmod, Eq. (29).
double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return a > 0.0 ? std::min(a, b) : std::max(a, b);
}
// van Leer, Eq. (30).  reading: the harmonic mean 2ab/(a+b) where a and b
// share a sign, 0 otherwise (the printed prefactor (sign a + sign b)/2 would
// flip the sign of the result for two negative slopes).
double vanleer(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return 2.0 * a * b / (a + b);
}

// ------------------------------------------------------- fluid operator L_d
// One pencil along d.  Position m = 0..M-1 holds padded cell m - G.
struct Pencil {
  int M;
  std::vector<double> u[5];
  std::vector<double> b[3];  // cell-centred field
  std::vector<double> phi;
};

// Interface dissipation term Q_j between cells i and i+1 (so that the
// first-order flux is (F_i + F_i+1)/2 - Q_j/2).
//   no HSE: Q = max(d_i, d_i+1) (u_i+1 - u_i), Eqs. (24)-(25);
//   HSE:    Q = D_adv du + D_ac delta_u with g of Eq. (51), delta_u of
//           Eqs. (52)-(53), D_adv of Eq. (55) and D_ac of Eq. (57).
// reading: D_adv = max(|v_i|, |v_i+1|) (Eq. 55 is printed without |.|).
void dissipation(const CellQ& L, const CellQ& R, double phiL, double phiR, bool hse, double* Q) {
  if (!hse) {
    const double dmax = std::max(L.d, R.d);
    for (int k = 0; k < 5; ++k) Q[k] = dmax * (R.u[k] - L.u[k]);
    return;
  }
  const double dadv = std::max(std::fabs(L.vd), std::fabs(R.vd));
  const double dac = std::max(L.cF, R.cF);
  const double scale = (phiR - phiL) / (L.cS * R.cS);
  for (int k = 0; k < 5; ++k) {
    const double du = R.u[k] - L.u[k];
    const double g = 0.5 * (L.xi[k] + R.xi[k]) * scale;
    const double delta = minmod(du - g, du);
    Q[k] = dadv * du + dac * delta;
  }
}

// Gravitational source of the unsplit scheme, Eq. (42), for cell i with the
// centred potential difference phi_i+1 - phi_i-1 over the distance span of
// the two cell centres (2 dx; on an irregular mesh dx_i-1/2 + dx_i +
// dx_i+1/2).  reading: the source is -(0, rho e_d, m_d) dphi/dx (the minus
// sign of Eq. 36, dropped in Eq. 42).
void gravity_source(const double* u, int d, double dphi2, double span, double* S) {
  const double g = dphi2 / span;
  for (int k = 0; k < 5; ++k) S[k] = 0.0;
  S[MX + d] = -u[RHO] * g;
  S[EN] = -u[MX + d] * g;
}

// L_d on one pencil; writes unew for the real cells G..G+n-1.
// centre distance of padded cells m-1 and m+1 along the pencil
double span_of(const double* hs, int m, double h) { return hs ? 0.5 * hs[m - 1] + hs[m] + 0.5 * hs[m + 1] : 2.0 * h; }

// hs: widths of the padded cells along d on an irregular mesh, else null.
void fluid_pencil(const Pencil& P, int n, int d, double dt, double h, const double* hs, const fishref_params& prm,
                  std::vector<double>* unew) {
  const int M = P.M;
  const bool grav = prm.gravity == 1;  // unsplit source inside the sweep
  const bool hse = prm.hse != 0;
  const double alpha = prm.predictor_alpha;
  // Limiter of cell c: minmod (Eq. 29), van Leer (Eq. 30), or, for the switch
  // used in core-collapse runs (Sect. 2.2), van Leer where the flow is
  // subsonic and minmod where it is supersonic.  reading: a cell is
  // supersonic when its speed |v| exceeds its sound speed c_S on the state the
  // limited differences are taken from (the half-step state).
  auto lim = [&](const CellQ& c, double a, double b) {
    const bool mm = prm.limiter == 0 || (prm.limiter == 2 && c.supersonic);
    return mm ? minmod(a, b) : vanleer(a, b);
  };

  // cell quantities of u^n, positions G-3 .. G+n+2
  std::vector<CellQ> C0(M);
  for (int m = G - 3; m < G + n + 3; ++m) {
    double u[5] = {P.u[0][m], P.u[1][m], P.u[2][m], P.u[3][m], P.u[4][m]};
    double b[3] = {P.b[0][m], P.b[1][m], P.b[2][m]};
    C0[m] = cell_quantities(u, b, d, prm.gamma);
  }
  // Predictor flux (first order, Eq. 24) at the interface m+1/2,
  // m = G-3 .. G+n+1.  The predictor freezing speed is a parameter between 0
  // and max(d_i, d_i+1) (Sect. 2.2); reading: alpha times the corrector's
  // dissipation.
  std::vector<double> F1[5];
  for (auto& v : F1) v.assign(M, 0.0);
  for (int m = G - 3; m < G + n + 2; ++m) {
    double Q[5];
    dissipation(C0[m], C0[m + 1], P.phi[m], P.phi[m + 1], hse, Q);
    for (int k = 0; k < 5; ++k) F1[k][m] = 0.5 * (C0[m].F[k] + C0[m + 1].F[k]) - 0.5 * alpha * Q[k];
  }
  // Predictor half step, Eq. (41), cells G-2 .. G+n+1.
  std::vector<double> up[5];
  for (auto& v : up) v.assign(M, 0.0);
  for (int m = G - 2; m < G + n + 2; ++m) {
    double S[5] = {0, 0, 0, 0, 0};
    if (grav) gravity_source(C0[m].u, d, P.phi[m + 1] - P.phi[m - 1], span_of(hs, m, h), S);
    const double hm = hs ? hs[m] : h;  // Eq. (69) on an irregular mesh
    for (int k = 0; k < 5; ++k)
      up[k][m] = P.u[k][m] - dt / (2.0 * hm) * (F1[k][m] - F1[k][m - 1]) + 0.5 * dt * S[k];
  }
  // Cell quantities of the half-step state u^n' (field unchanged).
  std::vector<CellQ> C1(M);
  for (int m = G - 2; m < G + n + 2; ++m) {
    double u[5] = {up[0][m], up[1][m], up[2][m], up[3][m], up[4][m]};
    double b[3] = {P.b[0][m], P.b[1][m], P.b[2][m]};
    C1[m] = cell_quantities(u, b, d, prm.gamma);
  }
  // Differences of the right- and left-moving relaxed fluxes F+- = (F +- d u)/2
  // (after Eq. 23) across interface m+1/2, m = G-2 .. G+n: a+-_j = (dF +- Q)/2.
  // reading: the freezing speed inside every difference is the interface-local
  // one of Eq. (25) (or the HSE split of Eqs. 54-57), so that the corrector flux
  // reduces to Eq. (24) where the limiters vanish.
  std::vector<double> ap[5], am[5], Qc[5];
  for (int k = 0; k < 5; ++k) {
    ap[k].assign(M, 0.0);
    am[k].assign(M, 0.0);
    Qc[k].assign(M, 0.0);
  }
  for (int m = G - 2; m < G + n + 1; ++m) {
    double Q[5];
    dissipation(C1[m], C1[m + 1], P.phi[m], P.phi[m + 1], hse, Q);
    for (int k = 0; k < 5; ++k) {
      const double dF = C1[m + 1].F[k] - C1[m].F[k];
      ap[k][m] = 0.5 * (dF + Q[k]);
      am[k][m] = 0.5 * (dF - Q[k]);
      Qc[k][m] = Q[k];
    }
  }
  // Second-order TVD flux, Eq. (34), at interface m+1/2, m = G-1 .. G+n-1:
  // F = F+_i + F-_i+1 + (phi(dF+_i-1/2, dF+_i+1/2) - phi(dF-_i+1/2, dF-_i+3/2))/2.
  // The limiters are homogeneous of degree one, so the 1/dx of Eq. (27) and
  // the dx/2 of Eq. (34) cancel.
  // On an irregular mesh (Sect. 2.5) the slopes of the piecewise-linear F+-
  // divide each difference by the distance of its two cell centres and are
  // carried half a cell width to the interface: a correction
  // (dx_i/2) phi(dF_i-1/2 / delta_i-1/2, dF_i+1/2 / delta_i+1/2), which is
  // phi(dF_i-1/2, dF_i+1/2)/2 on a uniform mesh.
  std::vector<double> F2[5];
  for (auto& v : F2) v.assign(M, 0.0);
  for (int m = G - 1; m < G + n; ++m)
    for (int k = 0; k < 5; ++k) {
      F2[k][m] = 0.5 * (C1[m].F[k] + C1[m + 1].F[k]) - 0.5 * Qc[k][m];
      if (!hs) {
        F2[k][m] += 0.5 * (lim(C1[m], ap[k][m - 1], ap[k][m]) - lim(C1[m + 1], am[k][m], am[k][m + 1]));
      } else {
        const double dl = 0.5 * (hs[m - 1] + hs[m]), dr = 0.5 * (hs[m] + hs[m + 1]);
        const double dr2 = 0.5 * (hs[m + 1] + hs[m + 2]);
        F2[k][m] += 0.5 * hs[m] * lim(C1[m], ap[k][m - 1] / dl, ap[k][m] / dr) -
                    0.5 * hs[m + 1] * lim(C1[m + 1], am[k][m] / dr, am[k][m + 1] / dr2);
      }
    }
  // Corrector full step, Eq. (43) (Eq. 35 without gravity), real cells.
  for (int m = G; m < G + n; ++m) {
    double S[5] = {0, 0, 0, 0, 0};
    if (grav) gravity_source(C1[m].u, d, P.phi[m + 1] - P.phi[m - 1], span_of(hs, m, h), S);
    const double hm = hs ? hs[m] : h;
    for (int k = 0; k < 5; ++k)
      unew[k][m - G] = P.u[k][m] - dt / hm * (F2[k][m] - F2[k][m - 1]) + dt * S[k];
  }
}

// Split gravity G_d(dt), Eqs. (39)-(40): on every real cell the momentum along
// d changes by -dt rho (phi_i+1 - phi_i-1)/(2 h); density and internal energy
// are left as they are, so the total energy changes by the change of the
// kinetic energy (Sect. 2.3: the code's variables are density, momentum and
// internal energy, and the total energy handed to L_d is their sum).
int q_of(int i, int j, int k, int d) { return d == 0 ? i : (d == 1 ? j : k); }

void gravity_kick(Ctx* c, int d, double dt) {
  const double h = c->h[d];
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < c->n[2]; ++k)
    for (int j = 0; j < c->n[1]; ++j)
      for (int i = 0; i < c->n[0]; ++i) {
        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
        lo[d] -= 1;
        hi[d] += 1;
        const size_t s = c->at(i, j, k);
        const double dphi = c->phi[c->at(hi[0], hi[1], hi[2])] - c->phi[c->at(lo[0], lo[1], lo[2])];
        const double rho = c->u[RHO][s];
        const double m_old = c->u[MX + d][s];
        const double span = c->nonuniform ? 0.5 * c->hs[d][lo[d] + G] + c->hs[d][q_of(i, j, k, d) + G] +
                                                0.5 * c->hs[d][hi[d] + G]
                                          : 2.0 * h;
        const double m_new = m_old - dt * rho * dphi / span;
        c->u[MX + d][s] = m_new;
        c->u[EN][s] += 0.5 * m_new * m_new / rho - 0.5 * m_old * m_old / rho;
      }
}

void apply_fluid_pencils(Ctx* c, int d, double dt);

// L_d, Eq. (35) or, with unsplit gravity, Eqs. (41)-(43); with split gravity
// G_d(dt/2) L_d(dt) G_d(dt/2), Eq. (38), L_d then without the source.
void apply_fluid(Ctx* c, int d, double dt) {
  if (c->p.gravity == 2) {
    gravity_kick(c, d, 0.5 * dt);
    apply_fluid_pencils(c, d, dt);
    gravity_kick(c, d, 0.5 * dt);
  } else {
    apply_fluid_pencils(c, d, dt);
  }
}

void apply_fluid_pencils(Ctx* c, int d, double dt) {
  fill_ghosts(c);
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const int n = c->n[d];
  const int n1 = c->n[t1], n2 = c->n[t2];
  const int M = n + 2 * G;
  const bool have_phi = !c->phi.empty();
#pragma omp parallel
  {
    Pencil P;
    P.M = M;
    for (auto& v : P.u) v.assign(M, 0.0);
    for (auto& v : P.b) v.assign(M, 0.0);
    P.phi.assign(M, 0.0);
    std::vector<double> unew[5];
    for (auto& v : unew) v.assign(n, 0.0);
#pragma omp for collapse(2) schedule(static)
    for (int c2 = 0; c2 < n2; ++c2)
      for (int c1 = 0; c1 < n1; ++c1) {
        for (int m = 0; m < M; ++m) {
          int q[3];
          q[d] = m - G;
          q[t1] = c1;
          q[t2] = c2;
          const size_t s = c->at(q[0], q[1], q[2]);
          for (int k = 0; k < 5; ++k) P.u[k][m] = c->u[k][s];
          // cell-centred field: mean of the low and high face of each component
          for (int a = 0; a < 3; ++a) {
            int r[3] = {q[0], q[1], q[2]};
            r[a] += 1;
            if (r[a] >= c->n[a] + G) {  // outermost ghost: outside every stencil
              P.b[a][m] = 0.0;
              continue;
            }
            P.b[a][m] = 0.5 * (c->b[a][s] + c->b[a][c->at(r[0], r[1], r[2])]);
          }
          P.phi[m] = have_phi ? c->phi[s] : 0.0;
        }
        fluid_pencil(P, n, d, dt, c->h[d], c->nonuniform ? c->hs[d].data() : nullptr, c->p, unew);
        for (int i = 0; i < n; ++i) {
          int q[3];
          q[d] = i;
          q[t1] = c1;
          q[t2] = c2;
          const size_t s = c->at(q[0], q[1], q[2]);
          for (int k = 0; k < 5; ++k) c->u[k][s] = unew[k][i];
        }
      }
  }
}

// ------------------------------------------------------- field operator B_d
// Transverse advection of one face row of b_t along d (Sect. 2.4).
// w[m]: v_d averaged onto the t-face (Eq. 65), positions 0..M-1;
// b[m]: the b_t face values along the row.  Outputs bnew for the real cells
// and the second-order edge flux (EMF) at d-faces f = 0..n (face f between
// cells f-1 and f).
// hs: widths of the padded cells along d on an irregular mesh, else null.
void field_row(const std::vector<double>& w, const std::vector<double>& b, int n, double dt, double h,
               const double* hs, int limiter, std::vector<double>& bnew, std::vector<double>& emf) {
  const int M = n + 2 * G;
  auto lim = [&](double a, double c) { return limiter == 0 ? minmod(a, c) : vanleer(a, c); };
  // 1-2-1 smoothing of the face velocity along d, Eq. (66).  reading: the two
  // outer neighbours are summed first, so that a face velocity odd about an
  // interface gives smoothed velocities that are exact negatives of each
  // other there and an interface velocity of exactly zero, which the <= 0
  // branch of Eq. (67) then decides (rounding cannot pick the branch).
  std::vector<double> vb(M, 0.0);
  for (int m = 1; m < M - 1; ++m) vb[m] = 0.25 * ((w[m - 1] + w[m + 1]) + 2.0 * w[m]);
  // Interface velocity, Eq. (68), and cell flux v b.
  std::vector<double> V(M, 0.0), f(M, 0.0);
  for (int m = 1; m < M - 2; ++m) V[m] = 0.5 * (vb[m] + vb[m + 1]);
  for (int m = 1; m < M - 1; ++m) f[m] = vb[m] * b[m];
  // First-order upwind flux, Eq. (67), interfaces m+1/2 for m = G-3 .. G+n+1.
  std::vector<double> phi1(M, 0.0);
  for (int m = G - 3; m < G + n + 2; ++m) phi1[m] = V[m] > 0.0 ? f[m] : f[m + 1];
  // Half-step predictor (Sect. 2.4: first-order predictor, as for the fluid).
  std::vector<double> bp(M, 0.0), fp(M, 0.0);
  for (int m = G - 2; m < G + n + 2; ++m) {
    bp[m] = b[m] - dt / (2.0 * (hs ? hs[m] : h)) * (phi1[m] - phi1[m - 1]);
    fp[m] = vb[m] * bp[m];
  }
  // Second-order corrector flux: piecewise-linear upwind reconstruction of the
  // half-step flux v b' with the TVD limiter (Sect. 2.4, last paragraph).
  // reading: the limited slope of v b' on the upwind cell, evaluated at the
  // interface.  Interfaces m+1/2 for m = G-1 .. G+n-1.  On an irregular mesh
  // the slope divides each difference by its centre distance and is carried
  // half the upwind cell's width (as for the fluid corrector).
  std::vector<double> phi2(M, 0.0);
  for (int m = G - 1; m < G + n; ++m) {
    if (!hs) {
      if (V[m] > 0.0)
        phi2[m] = fp[m] + 0.5 * lim(fp[m] - fp[m - 1], fp[m + 1] - fp[m]);
      else
        phi2[m] = fp[m + 1] - 0.5 * lim(fp[m + 1] - fp[m], fp[m + 2] - fp[m + 1]);
    } else {
      auto delta = [&](int a) { return 0.5 * (hs[a] + hs[a + 1]); };  // centres a, a+1
      if (V[m] > 0.0)
        phi2[m] = fp[m] + 0.5 * hs[m] * lim((fp[m] - fp[m - 1]) / delta(m - 1), (fp[m + 1] - fp[m]) / delta(m));
      else
        phi2[m] = fp[m + 1] - 0.5 * hs[m + 1] *
                                  lim((fp[m + 1] - fp[m]) / delta(m), (fp[m + 2] - fp[m + 1]) / delta(m + 1));
    }
  }
  // Advection update of b_t, Eq. (63) with the flux difference along d.
  for (int m = G; m < G + n; ++m) bnew[m - G] = b[m] - dt / (hs ? hs[m] : h) * (phi2[m] - phi2[m - 1]);
  // Edge flux at d-face f lies at interface (G + f - 1) + 1/2.
  for (int f = 0; f <= n; ++f) emf[f] = phi2[G + f - 1];
}

void apply_field(Ctx* c, int d, double dt) {
  fill_ghosts(c);
  const int nd = c->n[d];
  const int M = nd + 2 * G;
  const int tt[2] = {(d + 1) % 3, (d + 2) % 3};
  // Edge fluxes of the two transverse components: emf[s] for t = tt[s],
  // indexed [co][ft][f] with ft = 0..n_t (t-face), co = cell along the other
  // transverse axis, f = 0..n_d (d-face).
  std::vector<double> emf[2];
  // v_d of every padded cell of the current fluid state (held fixed, Sect. 2.4)
  std::vector<double> vd(c->ncell_padded());
  for (size_t s = 0; s < vd.size(); ++s) vd[s] = c->u[MX + d][s] / c->u[RHO][s];

  for (int s = 0; s < 2; ++s) {
    const int t = tt[s], o = tt[1 - s];
    const int nt = c->n[t], no = c->n[o];
    const int real_faces_t = c->nface(t);
    emf[s].assign((size_t)no * (nt + 1) * (nd + 1), 0.0);
    std::vector<double>& bt = c->b[t];
#pragma omp parallel
    {
      std::vector<double> w(M), b(M), bnew(nd), e(nd + 1);
#pragma omp for collapse(2) schedule(static)
      for (int co = 0; co < no; ++co)
        for (int ft = 0; ft <= nt; ++ft) {
          for (int m = 0; m < M; ++m) {
            int q[3];
            q[d] = m - G;
            q[t] = ft;
            q[o] = co;
            int r[3] = {q[0], q[1], q[2]};
            r[t] = ft - 1;
            // Eq. (65): v_d at the t-face, mean of the two cells sharing it;
            // on an irregular mesh the linear interpolation between their
            // centres (Sect. 2.5), in a form odd under mirroring.
            const double vlo = vd[c->at(r[0], r[1], r[2])], vhi = vd[c->at(q[0], q[1], q[2])];
            if (!c->nonuniform) {
              w[m] = 0.5 * (vlo + vhi);
            } else {
              const double hlo = c->hs[t][ft - 1 + G], hhi = c->hs[t][ft + G];
              w[m] = (vlo * hhi + vhi * hlo) / (hlo + hhi);
            }
            b[m] = bt[c->at(q[0], q[1], q[2])];
          }
          // the limiter switch is a fluid choice; the field advection keeps van Leer
          field_row(w, b, nd, dt, c->h[d], c->nonuniform ? c->hs[d].data() : nullptr, c->p.limiter == 0 ? 0 : 1,
                    bnew, e);
          std::copy(e.begin(), e.end(), emf[s].begin() + ((size_t)co * (nt + 1) + ft) * (nd + 1));
          if (ft < real_faces_t)
            for (int i = 0; i < nd; ++i) {
              int q[3];
              q[d] = i;
              q[t] = ft;
              q[o] = co;
              bt[c->at(q[0], q[1], q[2])] = bnew[i];
            }
        }
    }
  }
  // Constraint update of the normal component with the same edge fluxes,
  // Eq. (64); reading: the physical sign for both transverse components,
  //   d/dt b_d = + d/dt1 (v_d b_t1) + d/dt2 (v_d b_t2),
  // which keeps the discrete divergence of Eq. (62) unchanged.
  const int t1 = tt[0], t2 = tt[1];
  const int n1 = c->n[t1], n2 = c->n[t2];
  const int nfd = c->nface(d);
  std::vector<double>& bd = c->b[d];
#pragma omp parallel for collapse(2) schedule(static)
  for (int c2 = 0; c2 < n2; ++c2)
    for (int c1 = 0; c1 < n1; ++c1)
      for (int f = 0; f < nfd; ++f) {
        // emf[0]: t = t1, other = t2 -> index [c2][c1][f]
        const double e1lo = emf[0][((size_t)c2 * (n1 + 1) + c1) * (nd + 1) + f];
        const double e1hi = emf[0][((size_t)c2 * (n1 + 1) + c1 + 1) * (nd + 1) + f];
        // emf[1]: t = t2, other = t1 -> index [c1][c2][f]
        const double e2lo = emf[1][((size_t)c1 * (n2 + 1) + c2) * (nd + 1) + f];
        const double e2hi = emf[1][((size_t)c1 * (n2 + 1) + c2 + 1) * (nd + 1) + f];
        int q[3];
        q[d] = f;
        q[t1] = c1;
        q[t2] = c2;
        const size_t s = c->at(q[0], q[1], q[2]);
        // on an irregular mesh the widths of the face's cell across t1 and t2
        const double w1 = c->nonuniform ? c->hs[t1][c1 + G] : c->h[t1];
        const double w2 = c->nonuniform ? c->hs[t2][c2 + G] : c->h[t2];
        bd[s] = bd[s] + dt * ((e1hi - e1lo) / w1 + (e2hi - e2lo) / w2);
      }
}

// ------------------------------------------------------------------- CFL
// Eq. (14) with Eq. (15).  reading: the speed is |v_d| + c_F,d (the freezing
// speed of Eq. 21); axes with a single cell carry no wave and are skipped.
int cfl(Ctx* c, double* dt_out) {
  double cmax = 0.0;
  bool bad = false;
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
#pragma omp parallel for collapse(2) reduction(max : cmax) reduction(|| : bad) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t s = c->at(i, j, k);
        double u[5], b[3];
        for (int f = 0; f < 5; ++f) u[f] = c->u[f][s];
        b[0] = 0.5 * (c->b[0][s] + c->b[0][c->at(i + 1, j, k)]);
        b[1] = 0.5 * (c->b[1][s] + c->b[1][c->at(i, j + 1, k)]);
        b[2] = 0.5 * (c->b[2][s] + c->b[2][c->at(i, j, k + 1)]);
        for (int d = 0; d < 3; ++d) {
          if (c->n[d] == 1) continue;
          CellQ q = cell_quantities(u, b, d, c->p.gamma);
          if (!(q.p > 0.0) || !(u[RHO] > 0.0) || !std::isfinite(q.d)) bad = true;
          // Eq. (70) on an irregular mesh: the width of this cell along d
          const int idx[3] = {i, j, k};
          const double hd = c->nonuniform ? c->hs[d][idx[d] + G] : c->h[d];
          cmax = std::max(cmax, (std::fabs(q.vd) + q.cF) / hd);
        }
      }
  if (bad) return FISHREF_ERR_STATE;
  if (!(cmax > 0.0) || !std::isfinite(cmax)) return FISHREF_ERR_STATE;
  *dt_out = c->p.cfl / cmax;
  return FISHREF_OK;
}

// State check used by set_state / get_state: rho > 0, p > 0, all finite
// (negative internal energy stops a run, Sect. 4.4).  No floors.
bool state_ok(Ctx* c) {
  fill_ghosts(c);
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  bool bad = false;
#pragma omp parallel for collapse(2) reduction(|| : bad) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t s = c->at(i, j, k);
        double u[5], b[3];
        for (int f = 0; f < 5; ++f) {
          u[f] = c->u[f][s];
          if (!std::isfinite(u[f])) bad = true;
        }
        b[0] = 0.5 * (c->b[0][s] + c->b[0][c->at(i + 1, j, k)]);
        b[1] = 0.5 * (c->b[1][s] + c->b[1][c->at(i, j + 1, k)]);
        b[2] = 0.5 * (c->b[2][s] + c->b[2][c->at(i, j, k + 1)]);
        for (int a = 0; a < 3; ++a)
          if (!std::isfinite(b[a])) bad = true;
        CellQ q = cell_quantities(u, b, 0, c->p.gamma);
        if (!(u[RHO] > 0.0) || !(q.p > 0.0)) bad = true;
      }
  return !bad;
}

}  // namespace

struct fishref_ctx : Ctx {};

extern "C" {

int fishref_create(const fishref_params* p, fishref_ctx** out) {
  if (!out) return FISHREF_ERR_ARG;
  *out = nullptr;
  if (!p) return FISHREF_ERR_ARG;
  const int n[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->dx, p->dy, p->dz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > 4096) return FISHREF_ERR_ARG;
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) return FISHREF_ERR_ARG;
    if (p->bc[a] != PERIODIC && p->bc[a] != OUTFLOW) return FISHREF_ERR_ARG;
  }
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || p->cfl > 1.0) return FISHREF_ERR_ARG;
  if (p->limiter < 0 || p->limiter > 2) return FISHREF_ERR_ARG;
  if (!(p->predictor_alpha >= 0.0) || p->predictor_alpha > 1.0) return FISHREF_ERR_ARG;
  if (p->gravity < 0 || p->gravity > 2) return FISHREF_ERR_ARG;
  if (p->hse && !p->gravity) return FISHREF_ERR_ARG;
  fishref_ctx* c = new (std::nothrow) fishref_ctx();
  if (!c) return FISHREF_ERR_NOMEM;
  c->p = *p;
  for (int a = 0; a < 3; ++a) {
    c->n[a] = n[a];
    c->h[a] = h[a];
    c->N[a] = n[a] + 2 * G;
  }
  for (int a = 0; a < 3; ++a) {
    const std::vector<double> w(n[a], h[a]);
    fill_spacing(c, a, w.data());
  }
  try {
    for (auto& v : c->u) v.assign(c->ncell_padded(), 0.0);
    for (auto& v : c->b) v.assign(c->ncell_padded(), 0.0);
    if (p->gravity) c->phi.assign(c->ncell_padded(), 0.0);
  } catch (...) {
    delete c;
    return FISHREF_ERR_NOMEM;
  }
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  *out = c;
  return FISHREF_OK;
}

void fishref_destroy(fishref_ctx* c) { delete c; }

const char* fishref_last_error(const fishref_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fishref_set_state(fishref_ctx* c, const double* cell5, const double* bx, const double* by,
                      const double* bz, const double* phi) {
  if (!c || !cell5 || !bx || !by || !bz) return FISHREF_ERR_ARG;
  if (c->p.gravity && !phi) return fail(c, FISHREF_ERR_ARG, "gravity needs phi");
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  const size_t nc = (size_t)nx * ny * nz;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t src = (size_t)i + (size_t)nx * (j + (size_t)ny * k);
        for (int f = 0; f < 5; ++f) c->u[f][c->at(i, j, k)] = cell5[f * nc + src];
        if (c->p.gravity) c->phi[c->at(i, j, k)] = phi[src];
      }
  // faces: the input always carries n+1 entries along the normal
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < c->nface(0); ++i)
        c->b[0][c->at(i, j, k)] = bx[(size_t)i + (size_t)(nx + 1) * (j + (size_t)ny * k)];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < c->nface(1); ++j)
      for (int i = 0; i < nx; ++i)
        c->b[1][c->at(i, j, k)] = by[(size_t)i + (size_t)nx * (j + (size_t)(ny + 1) * k)];
  for (int k = 0; k < c->nface(2); ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        c->b[2][c->at(i, j, k)] = bz[(size_t)i + (size_t)nx * (j + (size_t)ny * k)];
  if (c->p.gravity) fill_phi_ghosts(c);
  c->t = 0.0;
  c->have_state = true;
  c->status = FISHREF_OK;
  if (!state_ok(c)) {
    c->status = FISHREF_ERR_STATE;
    return fail(c, FISHREF_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  }
  return FISHREF_OK;
}

int fishref_get_state(fishref_ctx* c, double* cell5, double* bx, double* by, double* bz, double* t_out) {
  if (!c) return FISHREF_ERR_ARG;
  if (!c->have_state) return fail(c, FISHREF_ERR_ARG, "no state");
  fill_ghosts(c);
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  const size_t nc = (size_t)nx * ny * nz;
  if (cell5)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const size_t dst = (size_t)i + (size_t)nx * (j + (size_t)ny * k);
          for (int f = 0; f < 5; ++f) cell5[f * nc + dst] = c->u[f][c->at(i, j, k)];
        }
  // face n on a periodic axis is the ghost copy of face 0
  if (bx)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i)
          bx[(size_t)i + (size_t)(nx + 1) * (j + (size_t)ny * k)] = c->b[0][c->at(i, j, k)];
  if (by)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i)
          by[(size_t)i + (size_t)nx * (j + (size_t)(ny + 1) * k)] = c->b[1][c->at(i, j, k)];
  if (bz)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          bz[(size_t)i + (size_t)nx * (j + (size_t)ny * k)] = c->b[2][c->at(i, j, k)];
  if (t_out) *t_out = c->t;
  if (c->status == FISHREF_OK && !state_ok(c)) c->status = FISHREF_ERR_STATE;
  return c->status;
}

int fishref_cfl_dt(fishref_ctx* c, double* dt_out) {
  if (!c || !dt_out) return FISHREF_ERR_ARG;
  if (!c->have_state) return fail(c, FISHREF_ERR_ARG, "no state");
  fill_ghosts(c);
  int rc = cfl(c, dt_out);
  if (rc != FISHREF_OK) {
    c->status = rc;
    return fail(c, rc, "CFL found rho <= 0, p <= 0 or a non-finite value");
  }
  return FISHREF_OK;
}

int fishref_apply(fishref_ctx* c, int op, int dir, double dt) {
  if (!c || dir < 0 || dir > 2 || (op != 0 && op != 1) || !(dt >= 0.0)) return FISHREF_ERR_ARG;
  if (!c->have_state) return fail(c, FISHREF_ERR_ARG, "no state");
  if (op == 0)
    apply_fluid(c, dir, dt);
  else
    apply_field(c, dir, dt);
  return FISHREF_OK;
}

int fishref_strang_step(fishref_ctx* c, double dt) {
  if (!c || !(dt >= 0.0) || !std::isfinite(dt)) return FISHREF_ERR_ARG;
  if (!c->have_state) return fail(c, FISHREF_ERR_ARG, "no state");
  if (dt == 0.0) {
    int rc = fishref_cfl_dt(c, &dt);
    if (rc != FISHREF_OK) return rc;
  }
  // Eqs. (12)-(13).  reading: the symmetric (palindromic) composition
  //   L_x B_x L_y B_y L_z B_z | B_z L_z B_y L_y B_x L_x
  // (operators applied left to right), which keeps the direction order of
  // Eq. (13) and is the symmetric product the second-order claim rests on.
  for (int d = 0; d < 3; ++d) {
    apply_fluid(c, d, dt);
    apply_field(c, d, dt);
  }
  for (int d = 2; d >= 0; --d) {
    apply_field(c, d, dt);
    apply_fluid(c, d, dt);
  }
  c->t += 2.0 * dt;
  return FISHREF_OK;
}

int fishref_set_spacing(fishref_ctx* c, int axis, const double* widths) {
  if (!c || !widths || axis < 0 || axis > 2) return FISHREF_ERR_ARG;
  for (int i = 0; i < c->n[axis]; ++i)
    if (!(widths[i] > 0.0) || !std::isfinite(widths[i])) return fail(c, FISHREF_ERR_ARG, "bad cell width");
  fill_spacing(c, axis, widths);
  c->nonuniform = true;
  return FISHREF_OK;
}

int fishref_diagnostics(fishref_ctx* c, double* out) {
  if (!c || !out) return FISHREF_ERR_ARG;
  if (!c->have_state) return fail(c, FISHREF_ERR_ARG, "no state");
  fill_ghosts(c);
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  const double vol = c->h[0] * c->h[1] * c->h[2];
  double tot[5] = {0, 0, 0, 0, 0};
  double divmax = 0.0, bmax = 0.0;
  // fixed-order serial sums (deterministic)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t s = c->at(i, j, k);
        const double hx = c->nonuniform ? c->hs[0][i + G] : c->h[0];
        const double hy = c->nonuniform ? c->hs[1][j + G] : c->h[1];
        const double hz = c->nonuniform ? c->hs[2][k + G] : c->h[2];
        const double cw = c->nonuniform ? hx * hy * hz / vol : 1.0;  // cell volume / vol
        for (int f = 0; f < 5; ++f) tot[f] += c->nonuniform ? c->u[f][s] * cw : c->u[f][s];
        // Eq. (62)
        const double div = (c->b[0][c->at(i + 1, j, k)] - c->b[0][s]) / hx +
                           (c->b[1][c->at(i, j + 1, k)] - c->b[1][s]) / hy +
                           (c->b[2][c->at(i, j, k + 1)] - c->b[2][s]) / hz;
        divmax = std::max(divmax, std::fabs(div));
      }
  for (int f = 0; f < 5; ++f) out[f] = tot[f] * vol;
  for (int a = 0; a < 3; ++a) {
    double sum = 0.0;
    int lim[3] = {nx, ny, nz};
    lim[a] = c->nface(a);
    for (int k = 0; k < lim[2]; ++k)
      for (int j = 0; j < lim[1]; ++j)
        for (int i = 0; i < lim[0]; ++i) {
          const double v = c->b[a][c->at(i, j, k)];
          if (c->nonuniform) {  // face area over the uniform one
            const int q[3] = {i, j, k};
            double area = 1.0;
            for (int e = 0; e < 3; ++e)
              if (e != a) area *= c->hs[e][q[e] + G] / c->h[e];
            sum += v * area;
          } else {
            sum += v;
          }
          bmax = std::max(bmax, std::fabs(v));
        }
    out[5 + a] = sum * vol / c->h[a];
  }
  out[8] = divmax;
  out[9] = bmax;
  return FISHREF_OK;
}

}  // extern "C"
