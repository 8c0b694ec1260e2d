// physics.h -- per-cell and per-interface arithmetic of the FISH sweeps,
// as device functions for gfx950.  Templated on the storage/arithmetic type T
// (double, or float with FP64 pressure recovery) and on the sweep axis D so
// that every component index is a compile-time constant (no scratch).
//
// FP32 arithmetic uses the hardware reciprocal and square root (1 ulp) in
// place of the IEEE division/square-root sequences; FP64 arithmetic refines
// the hardware estimates by Newton (reciprocal) and Goldschmidt (square root)
// steps, without the IEEE sequences' range scaling and special-case fixups,
// and divides by multiplying with the reciprocal.
//
// Sect. 2.1-2.4 of the FISH paper; equation numbers are the printed ones.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Multiply-adds are fused only within one source expression (never across
// statements), so the rounding of every value is fixed by the source alone:
// the kernels that stream the same arithmetic in different layouts (lanes,
// pairs of positions, strided pencils, any work shape) give bitwise the same
// result.
#pragma clang fp contract(on)

namespace fish {

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4 };

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1/x in FP64: the hardware estimate (relative error about 5e-8) and two
// Newton steps r <- r + r (1 - x r), each squaring the relative error.  Equal
// to the IEEE quotient on every sampled x whose reciprocal is a finite
// nonzero number; 0, infinite x and an overflowing reciprocal give NaN (the
// sweeps take reciprocals of densities, cell widths and sums of same-signed
// slopes, which are positive and finite in any valid state).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) in FP64: Goldschmidt's iteration from the hardware estimate y of
// 1/sqrt(x), carrying s -> sqrt(x) and h -> 1/(2 sqrt(x)) (s = x y, h = y/2),
// one coupled step and two residual corrections s += h (x - s^2).  Within one
// ulp of the IEEE root for positive finite x, subnormals included (equal on
// nearly every sample); sqrt(0) = 0, negative x gives NaN, +inf gives NaN
// (IEEE: inf), so a non-finite or negative argument still leaves a
// non-finite result.
__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double e = fma(-h, s, 0.5);
  s = fma(s, e, s);
  h = fma(h, e, h);
  double d = fma(-s, s, x);
  s = fma(d, h, s);
  d = fma(-s, s, x);
  s = fma(d, h, s);
  return x == 0.0 ? x : s;
}

// 1/rho in FP64 for the pressure recovery: the FP64 reciprocal above in FP64
// mode (the same value as the sweep's 1/rho); in FP32 mode the hardware
// FP32 reciprocal refined by one Newton step in FP64 (relative error ~1e-14,
// far below the FP32 storage rounding of E).
__device__ __forceinline__ double rinv64(double rho, double) { return rcp(rho); }
__device__ __forceinline__ double rinv64(double rho, float rho32) {
  const double r0 = (double)__builtin_amdgcn_rcpf(rho32);
  return r0 * (2.0 - rho * r0);
}

// Quantities of one cell for a sweep along D (Sect. 2.2).  F is the flux of
// Eq. (17) with x replaced by D, d the freezing speed |v_D| + c_F of Eq. (21).
// cS and xiE (= -(E + p), the energy entry of Eq. 50) only for HSE.
template <typename T, bool HSE>
struct CellQ {
  T u[5];
  T F[5];
  T vd, cF, d;
  T cS, xiE;
  T sup;  // 1 where |v| > c_S (the limiter switch of Sect. 2.2), else 0
};

// E = rho e + m^2/(2 rho) + b^2/2 and p = (gamma-1) rho e (Sect. 2.1, Eq. 5):
// the cancellation step, always evaluated in FP64.
template <typename T>
__device__ __forceinline__ T pressure(const T* u, const T* b, double gm1, T* b2_out) {
  const double rho = (double)u[RHO];
  const double mx = (double)u[MX], my = (double)u[MY], mz = (double)u[MZ];
  const double bx = (double)b[0], by = (double)b[1], bz = (double)b[2];
  const double b2 = bx * bx + by * by + bz * bz;
  const double m2 = mx * mx + my * my + mz * mz;
  const double ri = rinv64(rho, u[RHO]);
  *b2_out = (T)b2;
  return (T)(gm1 * ((double)u[EN] - 0.5 * m2 * ri - 0.5 * b2));
}

template <typename T, int D, bool HSE>
__device__ __forceinline__ void cell_quantities(const T* u, const T* b, double gamma, CellQ<T, HSE>& c) {
#pragma unroll
  for (int k = 0; k < 5; ++k) c.u[k] = u[k];
  const T ri = rcp(u[RHO]);
  const T v[3] = {u[MX] * ri, u[MY] * ri, u[MZ] * ri};
  T b2;
  const T p = pressure<T>(u, b, gamma - 1.0, &b2);
  const T ptot = p + T(0.5) * b2;
  const T bv = b[0] * v[0] + b[1] * v[1] + b[2] * v[2];
  // Directional fast magnetosonic speed (named after Eq. 21).
  const T a2 = (T)gamma * p * ri;
  const T q = a2 + b2 * ri;
  const T disc = q * q - T(4) * a2 * b[D] * b[D] * ri;
  const T cf = fsqrt(T(0.5) * (q + fsqrt(disc < T(0) ? T(0) : disc)));
  const T md = u[MX + D];
  c.F[RHO] = md;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T f = md * v[k] - b[D] * b[k];
    if (k == D) f += ptot;
    c.F[MX + k] = f;
  }
  c.F[EN] = (u[EN] + ptot) * v[D] - b[D] * bv;
  c.vd = v[D];
  c.cF = cf;
  c.d = fabs(v[D]) + cf;
  c.sup = v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > a2 ? T(1) : T(0);
  if (HSE) {
    c.cS = fsqrt(a2);
    c.xiE = -(u[EN] + p);
  } else {
    c.cS = T(0);
    c.xiE = T(0);
  }
}

// Limiters, Eqs. (29)-(30).  van Leer as the harmonic mean 2ab/(a+b) where a
// and b share a sign (the printed sign prefactor would flip negative pairs).
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  if (a * b <= T(0)) return T(0);
  return a > T(0) ? (a < b ? a : b) : (a > b ? a : b);
}
template <typename T>
__device__ __forceinline__ T vanleer(T a, T b) {
  // the quotient is formed unconditionally and selected: as an arm of the
  // conditional, the FP64 reciprocal's length would keep it a branch
  const T ab = a * b;
  const T q = T(2) * ab * rcp(a + b);
  return ab > T(0) ? q : T(0);
}
template <typename T, int LIM>
__device__ __forceinline__ T limit(T a, T b) {
  return LIM == 0 ? minmod(a, b) : vanleer(a, b);
}
// Limiter of one cell: LIM 0 minmod, 1 van Leer, 2 the switch of Sect. 2.2
// (minmod where the cell is supersonic, sup = 1; van Leer elsewhere).
template <typename T, int LIM>
__device__ __forceinline__ T limit_cell(T sup, T a, T b) {
  if (LIM == 2) return sup != T(0) ? minmod(a, b) : vanleer(a, b);
  return limit<T, LIM>(a, b);
}

// Dissipation Q_j at the interface between cells L and R, so that the
// first-order relaxed flux is (F_L + F_R)/2 - Q_j/2:
//   no HSE: Q = max(d_L, d_R) (u_R - u_L), Eqs. (24)-(25);
//   HSE:    Q = max(|v_L|, |v_R|) du + max(cF_L, cF_R) minmod(du - g, du),
//           g = (xi_L + xi_R)/2 (phi_R - phi_L)/(cS_L cS_R), Eqs. (50)-(57).
template <typename T, bool HSE>
__device__ __forceinline__ void dissipation(const CellQ<T, HSE>& L, const CellQ<T, HSE>& R, T phiL, T phiR,
                                            T* Q) {
  if (!HSE) {
    const T dmax = L.d > R.d ? L.d : R.d;
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = dmax * (R.u[k] - L.u[k]);
  } else {
    const T avL = fabs(L.vd), avR = fabs(R.vd);
    const T dadv = avL > avR ? avL : avR;
    const T dac = L.cF > R.cF ? L.cF : R.cF;
    const T scale = (phiR - phiL) * rcp(L.cS * R.cS);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T du = R.u[k] - L.u[k];
      const T xiL = (k == EN) ? L.xiE : -L.u[k];
      const T xiR = (k == EN) ? R.xiE : -R.u[k];
      const T g = T(0.5) * (xiL + xiR) * scale;
      const T delta = minmod(du - g, du);
      Q[k] = dadv * du + dac * delta;
    }
  }
}

// Unsplit gravitational source of cell i, Eq. (42) with the sign of Eq. (36):
// S = -(0, rho e_D, m_D) (phi_i+1 - phi_i-1)/(2 h); inv2h = 1/(2 h).
template <typename T, int D>
__device__ __forceinline__ void gravity_source(T rho, T mD, T dphi2, T inv2h, T* S) {
  const T gr = dphi2 * inv2h;
#pragma unroll
  for (int k = 0; k < 5; ++k) S[k] = T(0);
  S[MX + D] = -rho * gr;
  S[EN] = -mD * gr;
}

// Split gravity G_D over half a step, Eqs. (39)-(40): m_D -= rho gh with
// gh = (dt/2)(phi_i+1 - phi_i-1)/(2 h).  Density and internal energy stay, so
// E changes by the kinetic energy, (m'^2 - m^2)/(2 rho) = -gh (m + m')/2.
template <typename T, int D>
__device__ __forceinline__ void gravity_kick(T* u, T gh) {
  const T m = u[MX + D];
  const T mn = m - u[RHO] * gh;
  u[MX + D] = mn;
  u[EN] = u[EN] - gh * (T(0.5) * (m + mn));
}

// ----------------------------------------------------------- index maps
// Periodic axes wrap; outflow axes copy the nearest real entry (zeroth-order
// extrapolation).  A face array along its own normal has n+1 real faces on
// an outflow axis (last real face n) and n on a periodic one.
__device__ __forceinline__ int wrap(int i, int n) {
  if (i >= 0 && i < n) return i;
  int r = i % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int map_cell(int i, int n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == 0) return wrap(i, n);
  return i < 0 ? 0 : n - 1;
}
__device__ __forceinline__ int map_face(int i, int n, int bc) {
  if (bc == 0) return wrap(i, n);
  return i < 0 ? 0 : (i > n ? n : i);
}

}  // namespace fish
