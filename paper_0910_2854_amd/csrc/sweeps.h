// sweeps.h -- HIP kernels of the FISH directional sweeps for gfx950.
//
// Layout: eight SoA arrays (rho, m_x, m_y, m_z, E, b_x, b_y, b_z) of one
// element type, x fastest, all sharing the strides (1, sy, sz).  Along an
// outflow axis every array has one extra layer so that a face array along its
// own normal can hold its last real face n; on a periodic axis face n is face
// 0 and is never stored.  Ghost cells are never stored either: every load
// maps its index (periodic wrap, or clamp for zeroth-order extrapolation).
//
// Both sweeps are written once as a streaming pipeline over the positions of
// a pencil: when cell c is loaded, the predictor of cell c-1 and the
// corrector of cell c-3 are produced (the 7-cell stencil of Sect. 3), so each
// cell is read from HBM once per pass.  "The value one position back" comes
// from one of two policies:
//   Strided (y and z sweeps): a lane owns a pencil segment and walks it; the
//     previous position is the lane's own register from the last iteration.
//     Adjacent lanes are adjacent along x, so every access is coalesced.
//   Lanes (x sweep): the 64 lanes of a wave hold 64 consecutive positions of
//     a stream of whole x rows (each row padded by its 3-cell halos); the
//     previous position is the neighbour lane (DPP wave shift), lane 0 taking
//     lane 63 of the previous iteration.  Again every access is coalesced and
//     no row is transposed.
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

// ------------------------------------------------------------ position history
// prev(cur, h): the value this quantity had one stream position earlier.
struct StridedHist {
  template <typename V>
  __device__ __forceinline__ static V prev(const V& cur, V& h) {
    V p = h;
    h = cur;
    return p;
  }
};

__device__ __forceinline__ int lane_prev_bits(int cur, int& carry) {
  // wave_shr:1 -- lane i takes lane i-1; lane 0 keeps `old` = carry (whose
  // lane 0 holds lane 63 of the previous iteration); then carry = wave_ror:1.
  const int o = __builtin_amdgcn_update_dpp(carry, cur, 0x138, 0xf, 0xf, false);
  carry = __builtin_amdgcn_mov_dpp(cur, 0x13C, 0xf, 0xf, false);
  return o;
}
__device__ __forceinline__ float lane_prev(float cur, float& carry) {
  int c = __float_as_int(carry);
  const int o = lane_prev_bits(__float_as_int(cur), c);
  carry = __int_as_float(c);
  return __int_as_float(o);
}
__device__ __forceinline__ double lane_prev(double cur, double& carry) {
  const long long cb = __double_as_longlong(cur);
  long long kb = __double_as_longlong(carry);
  int klo = (int)(kb & 0xffffffffll), khi = (int)(kb >> 32);
  const int olo = lane_prev_bits((int)(cb & 0xffffffffll), klo);
  const int ohi = lane_prev_bits((int)(cb >> 32), khi);
  carry = __longlong_as_double(((long long)khi << 32) | (unsigned int)klo);
  return __longlong_as_double(((long long)ohi << 32) | (unsigned int)olo);
}

struct LaneHist {
  template <typename T>
  __device__ __forceinline__ static T prev(const T& cur, T& h) {
    return lane_prev(cur, h);
  }
  template <typename T, bool HSE>
  __device__ __forceinline__ static CellQ<T, HSE> prev(const CellQ<T, HSE>& cur, CellQ<T, HSE>& h) {
    CellQ<T, HSE> o;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      o.u[k] = lane_prev(cur.u[k], h.u[k]);
      o.F[k] = lane_prev(cur.F[k], h.F[k]);
    }
    o.d = lane_prev(cur.d, h.d);
    if (HSE) {
      o.vd = lane_prev(cur.vd, h.vd);
      o.cF = lane_prev(cur.cF, h.cF);
      o.cS = lane_prev(cur.cS, h.cS);
      o.xiE = lane_prev(cur.xiE, h.xiE);
    } else {
      o.vd = o.cF = o.cS = o.xiE = T(0);
    }
    return o;
  }
};

template <typename T, int N>
struct Vec {
  T v[N];
};
template <typename H, typename T, int N>
__device__ __forceinline__ Vec<T, N> prev_vec(const Vec<T, N>& cur, Vec<T, N>& h) {
  Vec<T, N> o;
#pragma unroll
  for (int k = 0; k < N; ++k) o.v[k] = H::prev(cur.v[k], h.v[k]);
  return o;
}

// ------------------------------------------------------------ L_d pipeline
template <typename T>
struct FluidArgs {
  const T* u[5];
  T* uo[5];
  const T* b[3];
  const T* phi;
  Geo g;
  double gamma, alpha;
  int seg, nseg;   // strided: segment length along D and segments per pencil
  int rows_per_wave; // lanes: whole rows per wave
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

template <typename T>
struct FluidConsts {
  T k_half, k_full, half_dt, dt, inv2h, halfalpha;
  double gamma;
};

template <typename T, bool HSE>
struct FluidHist {
  CellQ<T, HSE> q0, q1;
  Vec<T, 3> bc;
  Vec<T, 5> F1, ap, am, Lp, bs, F2, ua, ub;
  T ph1, ph2, ph3, ph4, rp1, rp2, mp1, mp2;
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      q0.u[k] = q0.F[k] = q1.u[k] = q1.F[k] = T(0);
      F1.v[k] = ap.v[k] = am.v[k] = Lp.v[k] = bs.v[k] = F2.v[k] = ua.v[k] = ub.v[k] = T(0);
    }
    q0.vd = q0.cF = q0.d = q0.cS = q0.xiE = T(0);
    q1.vd = q1.cF = q1.d = q1.cS = q1.xiE = T(0);
    bc.v[0] = bc.v[1] = bc.v[2] = T(0);
    ph1 = ph2 = ph3 = ph4 = rp1 = rp2 = mp1 = mp2 = T(0);
  }
};

// One stream position: loads of cell c in (uc, bc, phc); returns the
// corrected state of cell c-3 in un.  u3 is the state of cell c-3 when the
// caller reloads it (lanes policy); otherwise the history chain supplies it.
template <typename T, int D, bool GRAV, bool HSE, int LIM, typename H, bool RELOAD_U3>
__device__ __forceinline__ void fluid_position(const T* uc, const Vec<T, 3>& bcc, T phc, const T* u3_loaded,
                                               const FluidConsts<T>& k, FluidHist<T, HSE>& h, T* un) {
  // cell quantities of u at c and c-1
  CellQ<T, HSE> q0;
  cell_quantities<T, D, HSE>(uc, bcc.v, k.gamma, q0);
  const CellQ<T, HSE> q0m = H::prev(q0, h.q0);
  const Vec<T, 3> bcm = prev_vec<H>(bcc, h.bc);
  T phm1 = T(0), phm2 = T(0), phm3 = T(0), phm4 = T(0);
  if (GRAV || HSE) {
    phm1 = H::prev(phc, h.ph1);
    phm2 = H::prev(phm1, h.ph2);
    phm3 = H::prev(phm2, h.ph3);
    phm4 = H::prev(phm3, h.ph4);
  }
  // predictor flux at interface c-1/2 (Eq. 24, dissipation scaled by alpha)
  T Q[5];
  Vec<T, 5> F1;
  dissipation<T, HSE>(q0m, q0, phm1, phc, Q);
#pragma unroll
  for (int i = 0; i < 5; ++i) F1.v[i] = T(0.5) * (q0m.F[i] + q0.F[i]) - k.halfalpha * Q[i];
  const Vec<T, 5> F1m = prev_vec<H>(F1, h.F1);
  // predictor half step of cell c-1 (Eq. 41)
  T up[5];
  if (GRAV) {
    T S[5];
    gravity_source<T, D>(q0m.u[RHO], q0m.u[MX + D], phc - phm2, k.inv2h, S);
#pragma unroll
    for (int i = 0; i < 5; ++i) up[i] = q0m.u[i] - k.k_half * (F1.v[i] - F1m.v[i]) + k.half_dt * S[i];
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) up[i] = q0m.u[i] - k.k_half * (F1.v[i] - F1m.v[i]);
  }
  // cell quantities of the half-step state of c-1 (field unchanged), and of c-2
  CellQ<T, HSE> q1;
  cell_quantities<T, D, HSE>(up, bcm.v, k.gamma, q1);
  const CellQ<T, HSE> q1m = H::prev(q1, h.q1);
  // relaxed flux differences across interface c-3/2 (between c-2 and c-1)
  T Qc[5];
  Vec<T, 5> ap, am, bs;
  dissipation<T, HSE>(q1m, q1, phm2, phm1, Qc);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const T dF = q1.F[i] - q1m.F[i];
    ap.v[i] = T(0.5) * (dF + Qc[i]);
    am.v[i] = T(0.5) * (dF - Qc[i]);
    bs.v[i] = T(0.5) * (q1m.F[i] + q1.F[i]) - T(0.5) * Qc[i];
  }
  const Vec<T, 5> apm = prev_vec<H>(ap, h.ap);
  const Vec<T, 5> amm = prev_vec<H>(am, h.am);
  const Vec<T, 5> bsm = prev_vec<H>(bs, h.bs);
  // limited second-order flux at interface c-5/2 (Eq. 34)
  Vec<T, 5> Lp, F2;
#pragma unroll
  for (int i = 0; i < 5; ++i) Lp.v[i] = limit<T, LIM>(apm.v[i], ap.v[i]);
  const Vec<T, 5> Lpm = prev_vec<H>(Lp, h.Lp);
#pragma unroll
  for (int i = 0; i < 5; ++i) F2.v[i] = bsm.v[i] + T(0.5) * (Lpm.v[i] - limit<T, LIM>(amm.v[i], am.v[i]));
  const Vec<T, 5> F2m = prev_vec<H>(F2, h.F2);
  // state of cell c-3 before the sweep
  T u3[5];
  if (RELOAD_U3) {
#pragma unroll
    for (int i = 0; i < 5; ++i) u3[i] = u3_loaded[i];
  } else {
    Vec<T, 5> um1;
#pragma unroll
    for (int i = 0; i < 5; ++i) um1.v[i] = q0m.u[i];
    const Vec<T, 5> um2 = prev_vec<H>(um1, h.ua);
    const Vec<T, 5> um3 = prev_vec<H>(um2, h.ub);
#pragma unroll
    for (int i = 0; i < 5; ++i) u3[i] = um3.v[i];
  }
  // corrector of cell c-3 (Eq. 43)
  if (GRAV) {
    const T rpm2 = H::prev(up[RHO], h.rp1);   // rho' of c-2
    const T rpm3 = H::prev(rpm2, h.rp2);      // rho' of c-3
    const T mpm2 = H::prev(up[MX + D], h.mp1);
    const T mpm3 = H::prev(mpm2, h.mp2);
    T S[5];
    gravity_source<T, D>(rpm3, mpm3, phm2 - phm4, k.inv2h, S);
#pragma unroll
    for (int i = 0; i < 5; ++i) un[i] = u3[i] - k.k_full * (F2.v[i] - F2m.v[i]) + k.dt * S[i];
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) un[i] = u3[i] - k.k_full * (F2.v[i] - F2m.v[i]);
  }
  (void)phm3;
}

template <typename T>
__device__ __forceinline__ FluidConsts<T> fluid_consts(const FluidArgs<T>& a, int D) {
  const double dt = a.sc->dt;
  const double h = a.g.h[D];
  FluidConsts<T> k;
  k.k_half = (T)(dt / (2.0 * h));
  k.k_full = (T)(dt / h);
  k.half_dt = (T)(0.5 * dt);
  k.dt = (T)dt;
  k.inv2h = (T)(1.0 / (2.0 * h));
  k.halfalpha = (T)(0.5 * a.alpha);
  k.gamma = a.gamma;
  return k;
}

// Strided policy (D = y or z): one thread per pencil segment.
template <typename T, int D, bool GRAV, bool HSE, int LIM>
__global__ __launch_bounds__(256) void fluid_strided_kernel(FluidArgs<T> a) {
  static_assert(D != 0, "x sweeps use the lanes policy");
  constexpr int A = 0;  // lanes walk along x
  constexpr int O = 3 - D;
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
  const long long hi1 = base + (long long)(map_face(c[T1] + 1, g.n[T1], g.bc[T1]) - c[T1]) * g.st[T1];
  const long long hi2 = base + (long long)(map_face(c[T2] + 1, g.n[T2], g.bc[T2]) - c[T2]) * g.st[T2];
  const FluidConsts<T> k = fluid_consts(a, D);
  FluidHist<T, HSE> h;
  h.zero();
  const int npos = (s1 - s0) + 6;
#pragma unroll 2
  for (int it = 0; it < npos; ++it) {
    const int s = s0 - 3 + it;
    const long long off = (long long)map_cell(s, nD, g.bc[D]) * stD;
    T uc[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) uc[i] = a.u[i][base + off];
    Vec<T, 3> bcc;
    const long long f0 = (long long)map_face(s, nD, g.bc[D]) * stD;
    const long long f1 = (long long)map_face(s + 1, nD, g.bc[D]) * stD;
    bcc.v[D] = T(0.5) * (a.b[D][base + f0] + a.b[D][base + f1]);
    bcc.v[T1] = T(0.5) * (a.b[T1][base + off] + a.b[T1][hi1 + off]);
    bcc.v[T2] = T(0.5) * (a.b[T2][base + off] + a.b[T2][hi2 + off]);
    T phc = T(0);
    if (GRAV) phc = load_phi(a.phi, base, stD, s, nD, g.bc[D]);
    T un[5];
    fluid_position<T, D, GRAV, HSE, LIM, StridedHist, false>(uc, bcc, phc, nullptr, k, h, un);
    if (it >= 6) {
      const long long o = base + (long long)(s - 3) * stD;
#pragma unroll
      for (int i = 0; i < 5; ++i) a.uo[i][o] = un[i];
    }
  }
}

// Lanes policy (D = x): each wave streams rows_per_wave whole x rows.
template <typename T, bool GRAV, bool HSE, int LIM>
__global__ __launch_bounds__(256) void fluid_lanes_kernel(FluidArgs<T> a) {
  constexpr int D = 0;
  const Geo& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int L = nx + 6;                     // stream positions per row
  const long long nrows = (long long)ny * nz;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const long long r0 = wave * a.rows_per_wave;
  if (r0 >= nrows) return;  // whole wave exits together
  const int rows = (int)min((long long)a.rows_per_wave, nrows - r0);
  const int npos = rows * L;
  const int nit = (npos + 63) >> 6;
  const FluidConsts<T> k = fluid_consts(a, D);
  FluidHist<T, HSE> h;
  h.zero();
  for (int it = 0; it < nit; ++it) {
    const int q = (it << 6) + lane;
    const bool valid = q < npos;
    const int qq = valid ? q : npos - 1;
    const int rr = qq / L;
    const int cpos = qq - rr * L - 3;        // cell index along x (-3 .. nx+2)
    const long long row = r0 + rr;
    const int y = (int)(row % ny), z = (int)(row / ny);
    const long long base = (long long)y * g.st[1] + (long long)z * g.st[2];
    const long long yhi = base + (long long)(map_face(y + 1, ny, g.bc[1]) - y) * g.st[1];
    const long long zhi = base + (long long)(map_face(z + 1, nz, g.bc[2]) - z) * g.st[2];
    const int ms = map_cell(cpos, nx, g.bc[0]);
    T uc[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) uc[i] = a.u[i][base + ms];
    Vec<T, 3> bcc;
    bcc.v[0] = T(0.5) * (a.b[0][base + map_face(cpos, nx, g.bc[0])] + a.b[0][base + map_face(cpos + 1, nx, g.bc[0])]);
    bcc.v[1] = T(0.5) * (a.b[1][base + ms] + a.b[1][yhi + ms]);
    bcc.v[2] = T(0.5) * (a.b[2][base + ms] + a.b[2][zhi + ms]);
    T phc = T(0);
    if (GRAV) phc = load_phi(a.phi, base, 1, cpos, nx, g.bc[0]);
    const int m3 = map_cell(cpos - 3, nx, g.bc[0]);
    T u3[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) u3[i] = a.u[i][base + m3];
    T un[5];
    fluid_position<T, D, GRAV, HSE, LIM, LaneHist, true>(uc, bcc, phc, u3, k, h, un);
    const int co = cpos - 3;
    if (valid && co >= 0 && co < nx) {
#pragma unroll
      for (int i = 0; i < 5; ++i) a.uo[i][base + co] = un[i];
    }
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
  int seg, nseg;
  int rows_per_wave;
  const Scalars* sc;
};

template <typename T>
struct AdvectHist {
  T w1, w2, b1, b2, b3, b4, f2, p1, vb1, vb2, vb3, fp3, fp4, fp5, P2;
  __device__ void zero() { w1 = w2 = b1 = b2 = b3 = b4 = f2 = p1 = vb1 = vb2 = vb3 = fp3 = fp4 = fp5 = P2 = T(0); }
};

// One position of one face row of b_t along D: Eq. (65) face velocity w0 at
// cell c, Eq. (66) smoothing, Eq. (68) interface velocity, Eq. (67)
// first-order upwind predictor flux, second-order limited upwind corrector
// flux (end of Sect. 2.4), Eq. (63).  Outputs the new b_t of cell c-4 and
// the edge flux at d-face c-3 (the interface between c-4 and c-3).
template <typename T, int LIM, typename H, bool RELOAD_B4>
__device__ __forceinline__ void advect_position(T w0, T bb, T b4_loaded, T k_half, T k_full, AdvectHist<T>& h,
                                                T& bn, T& emf) {
  const T w1 = H::prev(w0, h.w1);
  const T w2 = H::prev(w1, h.w2);
  const T vbc = T(0.25) * (w2 + T(2) * w1 + w0);   // v-bar of c-1
  const T b1 = H::prev(bb, h.b1);                   // b of c-1
  const T fc = vbc * b1;                            // f of c-1
  const T vb1 = H::prev(vbc, h.vb1);                // v-bar of c-2
  const T V = T(0.5) * (vb1 + vbc);                 // interface c-3/2
  const T f2 = H::prev(fc, h.f2);                   // f of c-2
  const T P1 = V > T(0) ? f2 : fc;                  // Phi1 at c-3/2
  const T p1 = H::prev(P1, h.p1);                   // Phi1 at c-5/2
  const T b2 = H::prev(b1, h.b2);                   // b of c-2
  const T bp = b2 - k_half * (P1 - p1);             // b' of c-2
  const T fp2 = vb1 * bp;                           // f' of c-2
  const T vb2 = H::prev(vb1, h.vb2);                // v-bar of c-3
  const T vb3 = H::prev(vb2, h.vb3);                // v-bar of c-4
  const T V7 = T(0.5) * (vb3 + vb2);                // interface c-7/2
  const T fp3 = H::prev(fp2, h.fp3);
  const T fp4 = H::prev(fp3, h.fp4);
  const T fp5 = H::prev(fp4, h.fp5);
  T P2c;
  if (V7 > T(0))
    P2c = fp4 + T(0.5) * limit<T, LIM>(fp4 - fp5, fp3 - fp4);
  else
    P2c = fp3 - T(0.5) * limit<T, LIM>(fp3 - fp4, fp2 - fp3);
  const T P2 = H::prev(P2c, h.P2);                  // Phi2 at c-9/2
  T b4;
  if (RELOAD_B4) {
    b4 = b4_loaded;
  } else {
    const T b3 = H::prev(b2, h.b3);
    b4 = H::prev(b3, h.b4);
  }
  bn = b4 - k_full * (P2c - P2);
  emf = P2c;
}

template <typename T, int D, int LIM>
__global__ __launch_bounds__(256) void advect_strided_kernel(AdvectArgs<T> a) {
  static_assert(D != 0, "x sweeps use the lanes policy");
  constexpr int A = 0;
  constexpr int O = 3 - D;
  const Geo& g = a.g;
  const int t = a.t;
  const int nD = g.n[D];
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
  const long long base = (long long)c[A] * g.st[A] + (long long)c[O] * g.st[O];
  const int ft = c[t];
  const long long cell_lo = base + (long long)(map_cell(ft - 1, g.n[t], g.bc[t]) - ft) * g.st[t];
  const long long cell_hi = base + (long long)(map_cell(ft, g.n[t], g.bc[t]) - ft) * g.st[t];
  const double dt = a.sc->dt;
  const T k_half = (T)(dt / (2.0 * g.h[D]));
  const T k_full = (T)(dt / g.h[D]);
  AdvectHist<T> h;
  h.zero();
  const int npos = (s1 - s0) + 8;
#pragma unroll 2
  for (int it = 0; it < npos; ++it) {
    const int s = s0 - 4 + it;
    const long long off = (long long)map_cell(s, nD, g.bc[D]) * stD;
    const T vlo = a.md[cell_lo + off] * rcp(a.rho[cell_lo + off]);
    const T vhi = a.md[cell_hi + off] * rcp(a.rho[cell_hi + off]);
    const T w0 = T(0.5) * (vlo + vhi);
    const T bb = a.bt[base + off];
    T bn, e;
    advect_position<T, LIM, StridedHist, false>(w0, bb, T(0), k_half, k_full, h, bn, e);
    if (it >= 8) a.bto[base + (long long)(s - 4) * stD] = bn;
    const int fd = s - 3;
    if (it >= 7 && (fd < s1 || (last && outD && fd == nD))) a.emf[base + (long long)fd * stD] = e;
  }
}

// Lanes policy for B_x: each wave streams whole face rows along x, each row
// padded by 4 positions before and 4 after.
template <typename T, int LIM>
__global__ __launch_bounds__(256) void advect_lanes_kernel(AdvectArgs<T> a) {
  const Geo& g = a.g;
  const int t = a.t;  // 1 or 2
  const int nx = g.n[0];
  const bool outx = g.bc[0] == 1;
  const int L = nx + 8;
  const int ry = g.n[1] + ((t == 1 && g.bc[1] == 1) ? 1 : 0);
  const int rz = g.n[2] + ((t == 2 && g.bc[2] == 1) ? 1 : 0);
  const long long nrows = (long long)ry * rz;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const long long r0 = wave * a.rows_per_wave;
  if (r0 >= nrows) return;
  const int rows = (int)min((long long)a.rows_per_wave, nrows - r0);
  const int npos = rows * L;
  const int nit = (npos + 63) >> 6;
  const double dt = a.sc->dt;
  const T k_half = (T)(dt / (2.0 * g.h[0]));
  const T k_full = (T)(dt / g.h[0]);
  AdvectHist<T> h;
  h.zero();
  for (int it = 0; it < nit; ++it) {
    const int q = (it << 6) + lane;
    const bool valid = q < npos;
    const int qq = valid ? q : npos - 1;
    const int rr = qq / L;
    const int cpos = qq - rr * L - 4;  // cell index along x (-4 .. nx+3)
    const long long row = r0 + rr;
    const int y = (int)(row % ry), z = (int)(row / ry);
    const long long base = (long long)y * g.st[1] + (long long)z * g.st[2];
    const int ft = (t == 1) ? y : z;
    const long long st_t = g.st[t];
    const long long cell_lo = base + (long long)(map_cell(ft - 1, g.n[t], g.bc[t]) - ft) * st_t;
    const long long cell_hi = base + (long long)(map_cell(ft, g.n[t], g.bc[t]) - ft) * st_t;
    const int ms = map_cell(cpos, nx, g.bc[0]);
    const T vlo = a.md[cell_lo + ms] * rcp(a.rho[cell_lo + ms]);
    const T vhi = a.md[cell_hi + ms] * rcp(a.rho[cell_hi + ms]);
    const T w0 = T(0.5) * (vlo + vhi);
    const T bb = a.bt[base + ms];
    const T b4 = a.bt[base + map_cell(cpos - 4, nx, g.bc[0])];
    T bn, e;
    advect_position<T, LIM, LaneHist, true>(w0, bb, b4, k_half, k_full, h, bn, e);
    const int cb = cpos - 4;
    if (valid && cb >= 0 && cb < nx) a.bto[base + cb] = bn;
    const int fd = cpos - 3;
    if (valid && fd >= 0 && (fd < nx || (outx && fd == nx))) a.emf[base + fd] = e;
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
  const T ih1 = (T)(1.0 / g.h[T1]), ih2 = (T)(1.0 / g.h[T2]);
  a.bdo[idx] = a.bd[idx] + dtT * ((a.e1[up1] - a.e1[idx]) * ih1 + (a.e2[up2] - a.e2[idx]) * ih2);
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

__device__ __forceinline__ double fast_speed64(const double* u, const double* b, int d, double gamma, double p,
                                               double b2) {
  const double rho = u[0];
  const double a2 = gamma * p / rho;
  const double q = a2 + b2 / rho;
  const double disc = q * q - 4.0 * a2 * b[d] * b[d] / rho;
  return sqrt(0.5 * (q + sqrt(disc < 0.0 ? 0.0 : disc)));
}

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
    const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double m2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double p = (a.gamma - 1.0) * (u[4] - 0.5 * m2 / u[0] - 0.5 * b2);
    if (!(u[0] > 0.0) || !(p > 0.0)) bad = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (g.n[d] > 1) {
        const double cf = fast_speed64(u, b, d, a.gamma, p, b2);
        const double sp = (fabs(u[1 + d] / u[0]) + cf) / g.h[d];
        if (!isfinite(sp)) bad = 1;
        cmax = fmax(cmax, sp);
      }
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

// Self-test of the lane-shift primitive: out[64*it + lane] = previous
// position's value of (100*it + lane) over two iterations (128 entries).
__global__ void lane_shift_selftest_kernel(float* out) {
  const int lane = threadIdx.x & 63;
  float carry = -1.0f;
  for (int it = 0; it < 2; ++it) {
    const float cur = (float)(100 * it + lane);
    out[64 * it + lane] = lane_prev(cur, carry);
  }
}

}  // namespace fish
