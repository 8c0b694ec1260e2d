// sweeps.h -- HIP kernels of the FISH directional sweeps for gfx950.
//
// Layout: eight SoA arrays (rho, m_x, m_y, m_z, E, b_x, b_y, b_z) of one
// element type, x fastest, all sharing the strides (1, sy, sz).  Along an
// outflow axis every array has one extra layer so that a face array along its
// own normal can hold its last real face n; on a periodic axis face n is face
// 0 and is never stored.  Ghost cells are never stored either: every load
// maps its index (periodic wrap, or clamp for zeroth-order extrapolation).
//
// Fluid sweep L_d (Sect. 2.2-2.3): one thread streams one pencil segment
// along d through a register window -- the predictor of cell c-1 and the
// corrector of cell c-3 are produced when cell c is loaded, so each cell is
// read from HBM once per pass plus a 3-cell halo per segment end (the 7-cell
// stencil of Sect. 3).  Lanes of a wave are adjacent along x for the y and z
// sweeps, so every load and store is coalesced across the wave.
//
// Field sweep B_d (Sect. 2.4): transverse advection of b_t1 and b_t2 along d
// by the same streaming scheme (4-cell halo: Eq. 66 smooths once more), which
// writes the edge fluxes (EMFs); then the constraint update of b_d from those
// EMFs (Eq. 64).
#pragma once

#include "physics.h"

namespace fish {

struct Geo {
  int n[3];
  int bc[3];          // 0 periodic, 1 outflow
  long long st[3];    // element strides, st[0] = 1
  double h[3];
};

// Device-resident step scalars.
struct Scalars {
  double dt;                    // step size of every sub-operator
  double t;                     // simulation time
  unsigned long long cmax_bits; // max CFL speed (FP64 bits; all values >= 0)
  int status;                   // sticky: 1 = bad state seen
  int pad;
};

template <typename T>
struct FluidArgs {
  const T* u[5];
  T* uo[5];
  const T* b[3];
  const T* phi;
  Geo g;
  double gamma, alpha;
  int limiter;
  int seg, nseg;
  const Scalars* sc;
};

template <typename T>
__device__ __forceinline__ T load_phi(const T* phi, long long base, long long st, int s, int n, int bc) {
  if (s >= 0 && s < n) return phi[base + (long long)s * st];
  if (bc == 0 || n == 1) return phi[base + (long long)wrap(s, n) * st];
  // outflow: linear extrapolation from the two nearest real cells
  if (s < 0) {
    const T p0 = phi[base], p1 = phi[base + st];
    return p0 + (T)s * (p1 - p0);
  }
  const T p0 = phi[base + (long long)(n - 1) * st], p1 = phi[base + (long long)(n - 2) * st];
  return p0 + (T)(s - (n - 1)) * (p0 - p1);
}

// ------------------------------------------------------------ L_d
template <typename T, int D, bool GRAV, bool HSE>
__global__ __launch_bounds__(256) void fluid_sweep_kernel(FluidArgs<T> a) {
  constexpr int A = (D == 0) ? 1 : 0;  // axis adjacent lanes walk along
  constexpr int O = 3 - D - A;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const Geo& g = a.g;
  const int nA = g.n[A], nO = g.n[O], nD = g.n[D];
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nA * nO * a.nseg;
  if (tid >= total) return;
  const int ia = (int)(tid % nA);
  const long long r = tid / nA;
  const int io = (int)(r % nO);
  const int sg = (int)(r / nO);
  const int s0 = sg * a.seg;
  const int s1 = min(nD, s0 + a.seg);

  int c[3];
  c[A] = ia;
  c[O] = io;
  c[D] = 0;
  const long long stD = g.st[D];
  const long long base = (long long)c[A] * g.st[A] + (long long)c[O] * g.st[O];
  // high transverse faces of the cell (Eq. 9-11 layout: face f+1 closes cell f)
  const long long hi1 = base + (long long)(map_face(c[T1] + 1, g.n[T1], g.bc[T1]) - c[T1]) * g.st[T1];
  const long long hi2 = base + (long long)(map_face(c[T2] + 1, g.n[T2], g.bc[T2]) - c[T2]) * g.st[T2];

  const double dt = a.sc->dt;
  const T k_half = (T)(dt / (2.0 * g.h[D]));
  const T k_full = (T)(dt / g.h[D]);
  const T half_dt = (T)(0.5 * dt);
  const T dtT = (T)dt;
  const T h = (T)g.h[D];
  const T alpha = (T)a.alpha;
  const T halfalpha = T(0.5) * alpha;
  const double gamma = a.gamma;
  const int lim = a.limiter;

  CellQ<T> q0p, q1p;
  T u2[5], u3[5], bcp[3], F1p[5], app[5], amp[5], basep[5], Lpp[5], F2p[5];
  T ph1 = T(0), ph2 = T(0), ph3 = T(0), ph4 = T(0);
  T rp2 = T(0), mp2 = T(0), rp3 = T(0), mp3 = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    q0p.u[k] = q0p.F[k] = q1p.u[k] = q1p.F[k] = T(0);
    u2[k] = u3[k] = F1p[k] = app[k] = amp[k] = basep[k] = Lpp[k] = F2p[k] = T(0);
  }
  q0p.vd = q0p.cF = q0p.d = q0p.cS = q0p.xiE = T(0);
  q1p.vd = q1p.cF = q1p.d = q1p.cS = q1p.xiE = T(0);
  bcp[0] = bcp[1] = bcp[2] = T(0);

  const int npos = (s1 - s0) + 6;
  for (int it = 0; it < npos; ++it) {
    const int s = s0 - 3 + it;  // cell c loaded at this position
    const int ms = map_cell(s, nD, g.bc[D]);
    const long long off = (long long)ms * stD;
    T uc[5], bc[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) uc[k] = a.u[k][base + off];
    {
      const long long f0 = (long long)map_face(s, nD, g.bc[D]) * stD;
      const long long f1 = (long long)map_face(s + 1, nD, g.bc[D]) * stD;
      bc[D] = T(0.5) * (a.b[D][base + f0] + a.b[D][base + f1]);
      bc[T1] = T(0.5) * (a.b[T1][base + off] + a.b[T1][hi1 + off]);
      bc[T2] = T(0.5) * (a.b[T2][base + off] + a.b[T2][hi2 + off]);
    }
    T phc = T(0);
    if (GRAV) phc = load_phi(a.phi, base, stD, s, nD, g.bc[D]);

    // cell quantities of u at c
    CellQ<T> q0;
    cell_quantities<T, D, HSE>(uc, bc, gamma, q0);
    // predictor flux at the interface c-1/2 (Eq. 24, dissipation scaled by alpha)
    T Q[5], F1[5];
    dissipation<T, HSE>(q0p, q0, ph1, phc, Q);
#pragma unroll
    for (int k = 0; k < 5; ++k) F1[k] = T(0.5) * (q0p.F[k] + q0.F[k]) - halfalpha * Q[k];
    // predictor half step of cell c-1 (Eq. 41)
    T up[5];
    if (GRAV) {
      T S[5];
      gravity_source<T, D>(q0p.u[RHO], q0p.u[MX + D], phc - ph2, h, S);
#pragma unroll
      for (int k = 0; k < 5; ++k) up[k] = q0p.u[k] - k_half * (F1[k] - F1p[k]) + half_dt * S[k];
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) up[k] = q0p.u[k] - k_half * (F1[k] - F1p[k]);
    }
    // cell quantities of the half-step state of cell c-1 (field unchanged)
    CellQ<T> q1;
    cell_quantities<T, D, HSE>(up, bcp, gamma, q1);
    // relaxed flux differences across interface c-3/2 (between c-2 and c-1)
    T Qc[5], ap[5], am[5], bs[5];
    dissipation<T, HSE>(q1p, q1, ph2, ph1, Qc);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T dF = q1.F[k] - q1p.F[k];
      ap[k] = T(0.5) * (dF + Qc[k]);
      am[k] = T(0.5) * (dF - Qc[k]);
      bs[k] = T(0.5) * (q1p.F[k] + q1.F[k]) - T(0.5) * Qc[k];
    }
    // limited second-order flux at interface c-5/2 (Eq. 34) and the
    // corrector of cell c-3 (Eq. 43)
    T Lp[5], F2[5], un[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Lp[k] = limit(app[k], ap[k], lim);
      const T Lm = limit(amp[k], am[k], lim);
      F2[k] = basep[k] + T(0.5) * (Lpp[k] - Lm);
    }
    if (GRAV) {
      T S[5];
      gravity_source<T, D>(rp3, mp3, ph2 - ph4, h, S);
#pragma unroll
      for (int k = 0; k < 5; ++k) un[k] = u3[k] - k_full * (F2[k] - F2p[k]) + dtT * S[k];
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) un[k] = u3[k] - k_full * (F2[k] - F2p[k]);
    }
    if (it >= 6) {
      const long long o = base + (long long)(s - 3) * stD;
#pragma unroll
      for (int k = 0; k < 5; ++k) a.uo[k][o] = un[k];
    }
    // shift the window
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      F2p[k] = F2[k];
      Lpp[k] = Lp[k];
      basep[k] = bs[k];
      app[k] = ap[k];
      amp[k] = am[k];
      F1p[k] = F1[k];
      u3[k] = u2[k];
      u2[k] = q0p.u[k];
    }
    q1p = q1;
    q0p = q0;
    rp3 = rp2;
    mp3 = mp2;
    rp2 = up[RHO];
    mp2 = up[MX + D];
    bcp[0] = bc[0];
    bcp[1] = bc[1];
    bcp[2] = bc[2];
    ph4 = ph3;
    ph3 = ph2;
    ph2 = ph1;
    ph1 = phc;
  }
}

// ------------------------------------------------------------ B_d, advection
template <typename T>
struct AdvectArgs {
  const T* rho;
  const T* md;    // momentum along d
  const T* bt;    // transverse face field b_t (input)
  T* bto;         // b_t output
  T* emf;         // edge flux output, layout of the fields
  Geo g;
  int t;          // transverse axis
  int limiter;
  int seg, nseg;
  const Scalars* sc;
};

// One face row of b_t along D: Eq. (65) face velocity, Eq. (66) smoothing,
// Eq. (68) interface velocity, Eq. (67) first-order upwind predictor flux,
// second-order limited upwind corrector flux (end of Sect. 2.4), Eq. (63).
template <typename T, int D>
__global__ __launch_bounds__(256) void field_advect_kernel(AdvectArgs<T> a) {
  constexpr int A = (D == 0) ? 1 : 0;
  constexpr int O = 3 - D - A;
  const Geo& g = a.g;
  const int t = a.t;
  const int nD = g.n[D];
  // face rows along t include face n_t on an outflow axis
  const int rA = g.n[A] + ((A == t && g.bc[A] == 1) ? 1 : 0);
  const int rO = g.n[O] + ((O == t && g.bc[O] == 1) ? 1 : 0);
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)rA * rO * a.nseg;
  if (tid >= total) return;
  const int ia = (int)(tid % rA);
  const long long r = tid / rA;
  const int io = (int)(r % rO);
  const int sg = (int)(r / rO);
  const int s0 = sg * a.seg;
  const int s1 = min(nD, s0 + a.seg);
  const bool last = (s1 == nD);
  const bool outD = g.bc[D] == 1;

  int c[3];
  c[A] = ia;
  c[O] = io;
  c[D] = 0;
  const long long stD = g.st[D];
  const long long base = (long long)c[A] * g.st[A] + (long long)c[O] * g.st[O];  // the face row
  // the two cells sharing the t-face: t-index ft-1 and ft (mapped)
  const int ft = c[t];
  const long long cell_lo = base + (long long)(map_cell(ft - 1, g.n[t], g.bc[t]) - ft) * g.st[t];
  const long long cell_hi = base + (long long)(map_cell(ft, g.n[t], g.bc[t]) - ft) * g.st[t];

  const double dt = a.sc->dt;
  const T k_half = (T)(dt / (2.0 * g.h[D]));
  const T k_full = (T)(dt / g.h[D]);
  const int lim = a.limiter;

  T w1 = T(0), w2 = T(0);                  // w at c-1, c-2
  T vb1 = T(0), vb2 = T(0), vb3 = T(0);  // v-bar at c-2, c-3, c-4
  T b1 = T(0), b2 = T(0), b3 = T(0), b4 = T(0);  // b_t at c-1 .. c-4
  T f2 = T(0);                              // f at c-2
  T p1 = T(0);                              // Phi1 at interface c-5/2
  T fp3 = T(0), fp4 = T(0), fp5 = T(0);     // f' at c-3, c-4, c-5
  T P2 = T(0);                              // Phi2 at interface c-9/2

  const int npos = (s1 - s0) + 8;
  for (int it = 0; it < npos; ++it) {
    const int s = s0 - 4 + it;
    const long long off = (long long)map_cell(s, nD, g.bc[D]) * stD;
    // Eq. (65): v_d at the t-face, mean of the two cells sharing it
    const T vlo = a.md[cell_lo + off] / a.rho[cell_lo + off];
    const T vhi = a.md[cell_hi + off] / a.rho[cell_hi + off];
    const T w0 = T(0.5) * (vlo + vhi);
    const T bb = a.bt[base + off];
    // Eq. (66) at c-1
    const T vbc = T(0.25) * (w2 + T(2) * w1 + w0);
    const T fc = vbc * b1;                 // f at c-1
    // Eq. (68), interface c-3/2 between c-2 and c-1; Eq. (67) upwind flux
    const T V = T(0.5) * (vb1 + vbc);
    const T P1 = V > T(0) ? f2 : fc;
    // half-step predictor of cell c-2 and its flux
    const T bp = b2 - k_half * (P1 - p1);
    const T fp2 = vb1 * bp;
    // corrector flux at interface c-7/2 (between c-4 and c-3), upwind by V there
    const T V7 = T(0.5) * (vb3 + vb2);
    T P2c;
    if (V7 > T(0))
      P2c = fp4 + T(0.5) * limit(fp4 - fp5, fp3 - fp4, lim);
    else
      P2c = fp3 - T(0.5) * limit(fp3 - fp4, fp2 - fp3, lim);
    // advection update of cell c-4 (Eq. 63 along d)
    const T bn = b4 - k_full * (P2c - P2);
    if (it >= 8) a.bto[base + (long long)(s - 4) * stD] = bn;
    // EMF at d-face c-3 (interface c-7/2)
    const int fd = s - 3;
    if (it >= 7 && (fd < s1 || (last && outD && fd == nD))) a.emf[base + (long long)fd * stD] = P2c;
    // shift
    P2 = P2c;
    fp5 = fp4;
    fp4 = fp3;
    fp3 = fp2;
    p1 = P1;
    f2 = fc;
    vb3 = vb2;
    vb2 = vb1;
    vb1 = vbc;
    b4 = b3;
    b3 = b2;
    b2 = b1;
    b1 = bb;
    w2 = w1;
    w1 = w0;
  }
}

// ------------------------------------------------------------ B_d, constraint
template <typename T>
struct ConstraintArgs {
  const T* bd;
  T* bdo;
  const T* e1;  // EMF of b_t1
  const T* e2;  // EMF of b_t2
  Geo g;
  const Scalars* sc;
};

// Eq. (64) with the physical signs: b_d += dt (d_t1 Phi^t1 + d_t2 Phi^t2).
template <typename T, int D>
__global__ __launch_bounds__(256) void field_constraint_kernel(ConstraintArgs<T> a) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const Geo& g = a.g;
  const int nfx = g.n[0] + ((D == 0 && g.bc[0] == 1) ? 1 : 0);
  const int nfy = g.n[1] + ((D == 1 && g.bc[1] == 1) ? 1 : 0);
  const int nfz = g.n[2] + ((D == 2 && g.bc[2] == 1) ? 1 : 0);
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nfx * nfy * nfz;
  if (tid >= total) return;
  int c[3];
  c[0] = (int)(tid % nfx);
  const long long r = tid / nfx;
  c[1] = (int)(r % nfy);
  c[2] = (int)(r / nfy);
  const long long idx = (long long)c[0] * g.st[0] + (long long)c[1] * g.st[1] + (long long)c[2] * g.st[2];
  const long long up1 = idx + (long long)(map_face(c[T1] + 1, g.n[T1], g.bc[T1]) - c[T1]) * g.st[T1];
  const long long up2 = idx + (long long)(map_face(c[T2] + 1, g.n[T2], g.bc[T2]) - c[T2]) * g.st[T2];
  const double dt = a.sc->dt;
  const T dtT = (T)dt;
  const T h1 = (T)g.h[T1], h2 = (T)g.h[T2];
  a.bdo[idx] = a.bd[idx] + dtT * ((a.e1[up1] - a.e1[idx]) / h1 + (a.e2[up2] - a.e2[idx]) / h2);
}

// ------------------------------------------------------------ CFL + state check
template <typename T>
struct CheckArgs {
  const T* u[5];
  const T* b[3];
  Geo g;
  double gamma;
  Scalars* sc;
};

// Eq. (14)-(15): max over cells and active axes of (|v_d| + c_F,d)/h_d in FP64,
// plus the state check (rho > 0, p > 0, every value finite).
template <typename T>
__global__ __launch_bounds__(256) void check_cfl_kernel(CheckArgs<T> a) {
  const Geo& g = a.g;
  const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
  double cmax = 0.0;
  int bad = 0;
  for (long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x; cidx < ncell;
       cidx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(cidx % g.n[0]);
    const long long r = cidx / g.n[0];
    const int j = (int)(r % g.n[1]);
    const int k = (int)(r / g.n[1]);
    const long long s = (long long)i * g.st[0] + (long long)j * g.st[1] + (long long)k * g.st[2];
    double u[5], b[3];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      u[f] = (double)a.u[f][s];
      if (!isfinite(u[f])) bad = 1;
    }
    const long long sx = s + (long long)(map_face(i + 1, g.n[0], g.bc[0]) - i) * g.st[0];
    const long long sy = s + (long long)(map_face(j + 1, g.n[1], g.bc[1]) - j) * g.st[1];
    const long long sz = s + (long long)(map_face(k + 1, g.n[2], g.bc[2]) - k) * g.st[2];
    b[0] = 0.5 * ((double)a.b[0][s] + (double)a.b[0][sx]);
    b[1] = 0.5 * ((double)a.b[1][s] + (double)a.b[1][sy]);
    b[2] = 0.5 * ((double)a.b[2][s] + (double)a.b[2][sz]);
    if (!isfinite(b[0]) || !isfinite(b[1]) || !isfinite(b[2])) bad = 1;
    CellQ<double> q;
    cell_quantities<double, 0, false>(u, b, a.gamma, q);
    double p2;
    const double p = pressure_fp64(u[0], u[1], u[2], u[3], u[4], b[0], b[1], b[2], a.gamma, &p2);
    if (!(u[0] > 0.0) || !(p > 0.0)) bad = 1;
    if (g.n[0] > 1) {
      if (!isfinite(q.d)) bad = 1;
      cmax = fmax(cmax, (fabs(q.vd) + q.cF) / g.h[0]);
    }
    if (g.n[1] > 1) {
      cell_quantities<double, 1, false>(u, b, a.gamma, q);
      if (!isfinite(q.d)) bad = 1;
      cmax = fmax(cmax, (fabs(q.vd) + q.cF) / g.h[1]);
    }
    if (g.n[2] > 1) {
      cell_quantities<double, 2, false>(u, b, a.gamma, q);
      if (!isfinite(q.d)) bad = 1;
      cmax = fmax(cmax, (fabs(q.vd) + q.cF) / g.h[2]);
    }
  }
  // wavefront reduction (64 lanes), then one atomic per wave
  unsigned long long bits = __double_as_longlong(cmax);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(bits, off, 64);
    bits = o > bits ? o : bits;
    bad |= __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&a.sc->cmax_bits, bits);
    if (bad) atomicOr(&a.sc->status, 1);
  }
}

__global__ void reset_cmax_kernel(Scalars* sc) { sc->cmax_bits = 0ull; }

// dt = k / cmax (Eq. 14); a bad reduction marks the state.
__global__ void finalize_dt_kernel(Scalars* sc, double cfl) {
  const double cmax = __longlong_as_double((long long)sc->cmax_bits);
  if (!(cmax > 0.0) || !isfinite(cmax)) {
    sc->status |= 1;
    sc->dt = 0.0;
    return;
  }
  sc->dt = cfl / cmax;
}

__global__ void set_dt_kernel(Scalars* sc, double dt) { sc->dt = dt; }
__global__ void advance_time_kernel(Scalars* sc) { sc->t += 2.0 * sc->dt; }
__global__ void set_scalars_kernel(Scalars* sc, double t, int status) {
  sc->t = t;
  sc->status = status;
  sc->cmax_bits = 0ull;
  sc->dt = 0.0;
}

// ------------------------------------------------------------ diagnostics
template <typename T>
struct DiagArgs {
  const T* u[5];
  const T* b[3];
  Geo g;
  double* partial;   // [nblocks][10]
};

// Per-block partial sums in a fixed order (deterministic): each block owns a
// fixed contiguous range of cells; a fixed tree inside the block.
template <typename T>
__global__ __launch_bounds__(256) void diag_partial_kernel(DiagArgs<T> a, long long per_block) {
  __shared__ double sh[10][256];
  const Geo& g = a.g;
  const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
  const long long c0 = (long long)blockIdx.x * per_block;
  const long long c1 = min(ncell, c0 + per_block);
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (long long cidx = c0 + threadIdx.x; cidx < c1; cidx += blockDim.x) {
    const int i = (int)(cidx % g.n[0]);
    const long long r = cidx / g.n[0];
    const int j = (int)(r % g.n[1]);
    const int k = (int)(r / g.n[1]);
    const long long s = (long long)i * g.st[0] + (long long)j * g.st[1] + (long long)k * g.st[2];
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[f] += (double)a.u[f][s];
    const long long sx = s + (long long)(map_face(i + 1, g.n[0], g.bc[0]) - i) * g.st[0];
    const long long sy = s + (long long)(map_face(j + 1, g.n[1], g.bc[1]) - j) * g.st[1];
    const long long sz = s + (long long)(map_face(k + 1, g.n[2], g.bc[2]) - k) * g.st[2];
    // Eq. (62)
    const double div = ((double)a.b[0][sx] - (double)a.b[0][s]) / g.h[0] +
                       ((double)a.b[1][sy] - (double)a.b[1][s]) / g.h[1] +
                       ((double)a.b[2][sz] - (double)a.b[2][s]) / g.h[2];
    acc[8] = fmax(acc[8], fabs(div));
    // face sums over real faces: the low face of every cell, plus face n on
    // outflow axes (owned by the last cell)
    const double bx = (double)a.b[0][s], by = (double)a.b[1][s], bz = (double)a.b[2][s];
    acc[5] += bx;
    acc[6] += by;
    acc[7] += bz;
    acc[9] = fmax(acc[9], fmax(fabs(bx), fmax(fabs(by), fabs(bz))));
    if (g.bc[0] == 1 && i == g.n[0] - 1) {
      const double v = (double)a.b[0][sx];
      acc[5] += v;
      acc[9] = fmax(acc[9], fabs(v));
    }
    if (g.bc[1] == 1 && j == g.n[1] - 1) {
      const double v = (double)a.b[1][sy];
      acc[6] += v;
      acc[9] = fmax(acc[9], fabs(v));
    }
    if (g.bc[2] == 1 && k == g.n[2] - 1) {
      const double v = (double)a.b[2][sz];
      acc[7] += v;
      acc[9] = fmax(acc[9], fabs(v));
    }
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        if (q == 8 || q == 9)
          sh[q][threadIdx.x] = fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + w]);
        else
          sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 10) a.partial[(long long)blockIdx.x * 10 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void diag_final_kernel(const double* partial, int nblocks, double* out, double vol, double ax, double ay,
                                  double az) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int b = 0; b < nblocks; ++b)
    for (int q = 0; q < 10; ++q) {
      const double v = partial[(long long)b * 10 + q];
      if (q == 8 || q == 9)
        acc[q] = fmax(acc[q], v);
      else
        acc[q] += v;
    }
  for (int q = 0; q < 5; ++q) out[q] = acc[q] * vol;
  out[5] = acc[5] * ax;
  out[6] = acc[6] * ay;
  out[7] = acc[7] * az;
  out[8] = acc[8];
  out[9] = acc[9];
}

}  // namespace fish
