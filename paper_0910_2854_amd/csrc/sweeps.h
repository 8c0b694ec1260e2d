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
//     previous position is the neighbour lane (DPP wave shift).  The first
//     lanes of each iteration recompute the positions the previous one ended
//     on, so no value crosses iterations.  Again every access is coalesced
//     and no row is transposed.
#pragma once

#include "layout.h"
#include "physics.h"

// Multiply-adds are fused only within one source expression (never across
// statements), so the rounding of every value is fixed by the source alone:
// the kernels that stream the same arithmetic in different layouts (lanes,
// pairs of positions, strided pencils, any work shape) give bitwise the same
// result.
#pragma clang fp contract(on)

namespace fish {

// The wave's box and its wave index within the box; false past the list
// (the whole wave exits together).
// Blocks are dealt round-robin to the 8 XCDs, each with its own L2.  With
// xcd_remap the list's block order is re-dealt so that the blocks an XCD runs
// are consecutive in the list (neighbouring pencils and rows, whose shared
// halo rows then hit in that XCD's L2); the full rounds of 8 are permuted, a
// ragged tail keeps its order.
__device__ __forceinline__ int list_block(int xcd_remap) {
  int b = (int)blockIdx.x;
  if (xcd_remap) {
    const int q = (int)gridDim.x >> 3;
    if (b < (q << 3)) b = (b & 7) * q + (b >> 3);
  }
  return b;
}

template <int KIND>
__device__ __forceinline__ bool work_item(const WorkList& wl, const BoxDesc*& d, int& lw) {
  const int wave =
      __builtin_amdgcn_readfirstlane((int)((list_block(wl.xcd_remap) * blockDim.x + threadIdx.x) >> 6));
  if (wave >= wl.nwaves) return false;
  d = wl.boxes + wl.wave_box[wave];
  lw = wave - d->wave0[KIND];
  return true;
}

// ------------------------------------------------------------ addressing
// A pointer every lane of the wave holds (a stream position of the strided
// sweeps), pinned to scalar registers.  Without the pin the compiler folds the
// per-lane offset into the loop-invariant part of the address and pays a
// 64-bit vector add per load; pinned, the loads take the scalar base + 32-bit
// lane offset form.  The asm is empty: it only names the register class.
template <typename P>
__device__ __forceinline__ P in_sgpr(P p) {
  asm("" : "+s"(p));
  return p;
}

// Load/store at a wave-uniform base pointer plus a 32-bit per-lane byte
// offset (the scalar-base + vector-offset form of the global memory
// instructions: no 64-bit address arithmetic per lane).  The form needs the
// offset's zero extension in the block of the access; the empty asm on the
// offset keeps the compiler from extending a loop-invariant offset once before
// the loop, which would leave a 64-bit vector add per access inside it.  Every
// array the kernels touch is global memory: the address-space cast keeps the
// global form when the compiler cannot see where a pointer came from.
#define FISH_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ld(const T* p, unsigned off_bytes) {
  asm("" : "+v"(off_bytes));
  return *(const FISH_GLOBAL T*)((const FISH_GLOBAL char*)p + off_bytes);
}
template <typename T>
__device__ __forceinline__ void st(T* p, unsigned off_bytes, T v) {
  asm("" : "+v"(off_bytes));
  *(FISH_GLOBAL T*)((FISH_GLOBAL char*)p + off_bytes) = v;
}

// ------------------------------------------------------------ position history
// prev(cur, hin, hout): the value this quantity had one stream position
// earlier, read from the history hin; the history for the next position is
// written to hout.  The kernels alternate two history sets (hin/hout swap
// every position), so no register is copied to move the window.
struct StridedHist {
  template <typename V>
  __device__ __forceinline__ static V prev(const V& cur, const V& hin, V& hout) {
    hout = cur;
    return hin;
  }
};

// Lanes policy without a carry: lane i takes lane i-1 by one DPP shift and
// lane 0 takes zero.  The caller makes the wave's first lanes a halo that
// recomputes the positions the previous iteration ended on, so nothing has
// to cross from one iteration to the next and no history is kept.
__device__ __forceinline__ float lane_shr(float cur) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(cur), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_shr(double cur) {
  const long long cb = __double_as_longlong(cur);
  const int lo = __builtin_amdgcn_mov_dpp((int)(cb & 0xffffffffll), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(cb >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct LaneShift {
  template <typename T>
  __device__ __forceinline__ static T prev(const T& cur, const T&, T&) {
    return lane_shr(cur);
  }
  template <typename T, bool HSE>
  __device__ __forceinline__ static CellQ<T, HSE> prev(const CellQ<T, HSE>& cur, const CellQ<T, HSE>&,
                                                       CellQ<T, HSE>&) {
    CellQ<T, HSE> o;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      o.u[k] = lane_shr(cur.u[k]);
      o.F[k] = lane_shr(cur.F[k]);
    }
    o.d = lane_shr(cur.d);
    if (HSE) {
      o.vd = lane_shr(cur.vd);
      o.cF = lane_shr(cur.cF);
      o.cS = lane_shr(cur.cS);
      o.xiE = lane_shr(cur.xiE);
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
__device__ __forceinline__ Vec<T, N> prev_vec(const Vec<T, N>& cur, const Vec<T, N>& hin, Vec<T, N>& hout) {
  Vec<T, N> o;
#pragma unroll
  for (int k = 0; k < N; ++k) o.v[k] = H::prev(cur.v[k], hin.v[k], hout.v[k]);
  return o;
}

// ------------------------------------------------------------ lanes cursor
// Position of one lane in the stream of whole rows a wave walks (lanes
// policy): row rr of the wave's rows and position cp in [0, L) of that row,
// with the row's transverse indices (y, z) and its element offset base =
// y st1 + z st2.  Advancing by one iteration moves `step` positions (64, or
// 128 with two positions per lane); the row indices and the offset are
// stepped, never divided or multiplied, and stay on the wave's last row past
// its end (those lanes' positions are beyond the stream and write nothing).
// nrow is the number of rows per plane (cells, or face rows of the field
// sweep).
struct RowCursor {
  int cp, rr, y, z;
  unsigned base;
  bool moved;
  // r0 (the wave's first row) is uniform across the wave: one division per
  // wave, then the lane's own rows are stepped.  up: the element offset from
  // the last row of a plane to the first row of the next one, st2 - (nrow - 1) st1.
  __device__ void init(int pos, int L, int r0, int rows, int nrow, unsigned st1, unsigned st2, unsigned up) {
    const int z0 = r0 / nrow, y0 = r0 - z0 * nrow;
    cp = pos;
    rr = 0;
    y = y0;
    z = z0;
    base = (unsigned)y0 * st1 + (unsigned)z0 * st2;
    moved = true;
    while (cp >= L && rr < rows - 1) {
      cp -= L;
      ++rr;
      if (++y == nrow) {
        y = 0;
        ++z;
        base += up;
      } else {
        base += st1;
      }
    }
  }
  __device__ void advance(int L, int rows, int nrow, unsigned st1, unsigned up, int step = 64) {
    cp += step;
    moved = false;
    while (cp >= L && rr < rows - 1) {
      cp -= L;
      ++rr;
      if (++y == nrow) {
        y = 0;
        ++z;
        base += up;
      } else {
        base += st1;
      }
      moved = true;
    }
  }
};

// Branch-free maps for indices the stencils reach from a box row, i in
// [-8, n + 4): a clamp on outflow axes, at most one period added or removed
// on periodic ones (boxes thinner than 8 cells take the general wrap).  bc and
// n are uniform across the wave, so the choice of path is a scalar branch.
// The periodic map is the smallest of i, i + n and i - n as unsigned values
// (one of them lies in [0, n), the others are larger or negative), which is
// one three-way minimum.
__device__ __forceinline__ int map_cell_near(int i, int n, int bc) {
  if (bc) return min(max(i, 0), n - 1);
  if (n >= 8) {
    const unsigned a = (unsigned)i, b = (unsigned)(i + n), c = (unsigned)(i - n);
    return (int)min(a, min(b, c));
  }
  return wrap(i, n);
}
__device__ __forceinline__ int map_face_near(int i, int n, int bc) {
  if (bc) return min(max(i, 0), n);
  return map_cell_near(i, n, 0);
}

// ------------------------------------------------------------ L_d pipeline
template <typename T>
struct FluidArgs {
  const T* u[5];
  T* uo[5];
  const T* b[3];
  const T* phi;
  const T* wid[3];  // irregular mesh: cell widths per axis, else null
  Geo g;
  double gamma, alpha;
  int seg, nseg;   // strided: segment length along D and segments per pencil
  int rows_per_wave; // lanes: whole rows per wave
  const Scalars* sc;
  double i2h[3];     // 1 / (2 h_d)
};

// Kernel arguments of a fluid sweep over a batch: the pools and the list.
template <typename T>
struct FluidLaunch {
  const T* u[5];
  T* uo[5];
  const T* b[3];
  const T* phi;
  const T* wid[3];  // irregular meshes: every table box's cell widths per axis (at BoxDesc::woff), else null
  double gamma, alpha;
  WorkList wl;
  Scalars* sc;
};

// The per-box view of a launch (pointers at the box, its geometry and step
// scalars).
template <typename T, int KIND>
__device__ __forceinline__ FluidArgs<T> fluid_view(const FluidLaunch<T>& L, const BoxDesc& d) {
  FluidArgs<T> a;
  const long long off = d.off;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    a.u[i] = L.u[i] + off;
    a.uo[i] = L.uo[i] + off;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) a.b[i] = L.b[i] + off;
  a.phi = L.phi ? L.phi + off : nullptr;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.wid[i] = L.wid[i] ? L.wid[i] + d.woff[i] : nullptr;
  a.g = d.g;
  a.gamma = L.gamma;
  a.alpha = L.alpha;
  const int D = KIND - K_FLUID_X;
  a.seg = d.par[KIND];
  a.nseg = d.nseg[KIND];
  a.rows_per_wave = d.par[KIND];
  a.sc = L.sc + d.slot;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.i2h[i] = d.i2h[i];
  (void)D;
  return a;
}

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

// ------------------------------------------------ irregular meshes (Sect. 2.5)
// Width of the cell at stream index i along an axis, mapped as the cell is
// (a ghost takes the width of the cell it copies or wraps to).
template <typename T>
__device__ __forceinline__ T width_at(const T* w, int i, int n, int bc) {
  return w[map_cell(i, n, bc)];
}
// 1/(distance of the centres of the cells either side of a cell)
template <typename T>
__device__ __forceinline__ T inv_span(T wm, T w0, T wp) {
  return rcp(T(0.5) * wm + w0 + T(0.5) * wp);
}
// Per-position factors of the fluid sweep from the widths of cells c-4 .. c
// (w[0..4]): the predictor step of c-1 (dt/(2 dx)), the corrector step of c-3
// (dt/dx), the weights dx_i/(dx_i-1 + dx_i) and dx_i/(dx_i + dx_i+1) that put
// the limited slope of cell c-2 on its interfaces (the 1/2 of Eq. 34 on a
// uniform mesh), and the inverse centre spans of c-1 and c-3 for gravity.
template <typename T>
struct FluidNU {
  T kh1, kf3, wl2, wr2, isp1, isp3;
};
template <typename T>
__device__ __forceinline__ FluidNU<T> fluid_nu(const T* w, T dt) {
  FluidNU<T> n;
  n.kh1 = T(0.5) * dt * rcp(w[3]);
  n.kf3 = dt * rcp(w[1]);
  n.wl2 = w[2] * rcp(w[1] + w[2]);
  n.wr2 = w[2] * rcp(w[2] + w[3]);
  n.isp1 = inv_span(w[2], w[3], w[4]);
  n.isp3 = inv_span(w[0], w[1], w[2]);
  return n;
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
  T ph1, ph2, ph3, ph4, rp1, rp2, mp1, mp2, sp1;
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      q0.u[k] = q0.F[k] = q1.u[k] = q1.F[k] = T(0);
      F1.v[k] = ap.v[k] = am.v[k] = Lp.v[k] = bs.v[k] = F2.v[k] = ua.v[k] = ub.v[k] = T(0);
    }
    q0.vd = q0.cF = q0.d = q0.cS = q0.xiE = q0.sup = T(0);
    q1.vd = q1.cF = q1.d = q1.cS = q1.xiE = q1.sup = T(0);
    bc.v[0] = bc.v[1] = bc.v[2] = T(0);
    ph1 = ph2 = ph3 = ph4 = rp1 = rp2 = mp1 = mp2 = sp1 = T(0);
  }
};

// One stream position: loads of cell c in (uc, bc, phc); returns the
// corrected state of cell c-3 in un.  u3 is the state of cell c-3 when the
// caller reloads it (lanes policy); otherwise the history chain supplies it.
// GRAV: 0 none, 1 unsplit source in the predictor and corrector (Eqs. 41-43),
// 2 split kicks G(dt/2) L G(dt/2) (Eqs. 38-40): the entering cell is kicked
// by gh_c = (dt/2)(phi_c+1 - phi_c-1)/(2h), which the caller computes from
// its own loads for the cell the position maps to (the first positions of a
// stream have no history of phi; a ghost is then the exact copy of its kicked
// cell), before its first use; the output cell c-3 after its corrector, by
// the same factor formed from the history of phi.
// NU: irregular mesh, with the per-position factors in nu (uniform: k).
template <typename T, int D, int GRAV, bool HSE, int LIM, typename H, bool RELOAD_U3, bool NU = false>
__device__ __forceinline__ void fluid_position(const T* uc_in, const Vec<T, 3>& bcc, T phc, T gh_c,
                                               const T* u3_loaded, const FluidConsts<T>& k, const FluidNU<T>& nu,
                                               const FluidHist<T, HSE>& hi, FluidHist<T, HSE>& ho, T* un) {
  T phm1 = T(0), phm2 = T(0), phm3 = T(0), phm4 = T(0);
  if (GRAV != 0 || HSE) {
    phm1 = H::prev(phc, hi.ph1, ho.ph1);
    phm2 = H::prev(phm1, hi.ph2, ho.ph2);
    phm3 = H::prev(phm2, hi.ph3, ho.ph3);
    phm4 = H::prev(phm3, hi.ph4, ho.ph4);
  }
  T uc[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) uc[i] = uc_in[i];
  if (GRAV == 2) gravity_kick<T, D>(uc, gh_c);
  // cell quantities of u at c and c-1
  CellQ<T, HSE> q0;
  cell_quantities<T, D, HSE>(uc, bcc.v, k.gamma, q0);
  const CellQ<T, HSE> q0m = H::prev(q0, hi.q0, ho.q0);
  const Vec<T, 3> bcm = prev_vec<H>(bcc, hi.bc, ho.bc);
  // predictor flux at interface c-1/2 (Eq. 24, dissipation scaled by alpha)
  T Q[5];
  Vec<T, 5> F1;
  dissipation<T, HSE>(q0m, q0, phm1, phc, Q);
#pragma unroll
  for (int i = 0; i < 5; ++i) F1.v[i] = T(0.5) * (q0m.F[i] + q0.F[i]) - k.halfalpha * Q[i];
  const Vec<T, 5> F1m = prev_vec<H>(F1, hi.F1, ho.F1);
  // predictor half step of cell c-1 (Eq. 41; Eq. 69 on an irregular mesh)
  T up[5];
  const T khalf = NU ? nu.kh1 : k.k_half;
  if (GRAV == 1) {
    T S[5];
    gravity_source<T, D>(q0m.u[RHO], q0m.u[MX + D], phc - phm2, NU ? nu.isp1 : k.inv2h, S);
#pragma unroll
    for (int i = 0; i < 5; ++i) up[i] = q0m.u[i] - khalf * (F1.v[i] - F1m.v[i]) + k.half_dt * S[i];
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) up[i] = q0m.u[i] - khalf * (F1.v[i] - F1m.v[i]);
  }
  // cell quantities of the half-step state of c-1 (field unchanged), and of c-2
  CellQ<T, HSE> q1;
  cell_quantities<T, D, HSE>(up, bcm.v, k.gamma, q1);
  const CellQ<T, HSE> q1m = H::prev(q1, hi.q1, ho.q1);
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
  const Vec<T, 5> apm = prev_vec<H>(ap, hi.ap, ho.ap);
  const Vec<T, 5> amm = prev_vec<H>(am, hi.am, ho.am);
  const Vec<T, 5> bsm = prev_vec<H>(bs, hi.bs, ho.bs);
  // limited second-order flux at interface c-5/2 (Eq. 34); both limiters
  // taken here belong to cell c-2 (its half-step state decides the switch)
  const T sup2 = LIM == 2 ? H::prev(q1.sup, hi.sp1, ho.sp1) : T(0);
  // (irregular mesh: each difference weighted to put cell c-2's slope on its
  // interfaces, which absorbs the 1/2)
  Vec<T, 5> Lp, F2;
  if (!NU) {
#pragma unroll
    for (int i = 0; i < 5; ++i) Lp.v[i] = limit_cell<T, LIM>(sup2, apm.v[i], ap.v[i]);
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) Lp.v[i] = limit_cell<T, LIM>(sup2, nu.wl2 * apm.v[i], nu.wr2 * ap.v[i]);
  }
  const Vec<T, 5> Lpm = prev_vec<H>(Lp, hi.Lp, ho.Lp);
  if (!NU) {
#pragma unroll
    for (int i = 0; i < 5; ++i)
      F2.v[i] = bsm.v[i] + T(0.5) * (Lpm.v[i] - limit_cell<T, LIM>(sup2, amm.v[i], am.v[i]));
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i)
      F2.v[i] = bsm.v[i] + (Lpm.v[i] - limit_cell<T, LIM>(sup2, nu.wl2 * amm.v[i], nu.wr2 * am.v[i]));
  }
  const Vec<T, 5> F2m = prev_vec<H>(F2, hi.F2, ho.F2);
  // state of cell c-3 before the sweep
  T u3[5];
  // kick of c-3 (split gravity): phi of c-2 and c-4
  const T gh3 = GRAV == 2 ? k.half_dt * (phm2 - phm4) * (NU ? nu.isp3 : k.inv2h) : T(0);
  if (RELOAD_U3) {
#pragma unroll
    for (int i = 0; i < 5; ++i) u3[i] = u3_loaded[i];
    if (GRAV == 2) gravity_kick<T, D>(u3, gh3);  // bitwise the kick it had on entry
  } else {
    Vec<T, 5> um1;
#pragma unroll
    for (int i = 0; i < 5; ++i) um1.v[i] = q0m.u[i];
    const Vec<T, 5> um2 = prev_vec<H>(um1, hi.ua, ho.ua);
    const Vec<T, 5> um3 = prev_vec<H>(um2, hi.ub, ho.ub);
#pragma unroll
    for (int i = 0; i < 5; ++i) u3[i] = um3.v[i];
  }
  // corrector of cell c-3 (Eq. 43)
  const T kfull = NU ? nu.kf3 : k.k_full;
  if (GRAV == 1) {
    const T rpm2 = H::prev(up[RHO], hi.rp1, ho.rp1);   // rho' of c-2
    const T rpm3 = H::prev(rpm2, hi.rp2, ho.rp2);      // rho' of c-3
    const T mpm2 = H::prev(up[MX + D], hi.mp1, ho.mp1);
    const T mpm3 = H::prev(mpm2, hi.mp2, ho.mp2);
    T S[5];
    gravity_source<T, D>(rpm3, mpm3, phm2 - phm4, NU ? nu.isp3 : k.inv2h, S);
#pragma unroll
    for (int i = 0; i < 5; ++i) un[i] = u3[i] - kfull * (F2.v[i] - F2m.v[i]) + k.dt * S[i];
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) un[i] = u3[i] - kfull * (F2.v[i] - F2m.v[i]);
    if (GRAV == 2) gravity_kick<T, D>(un, gh3);
  }
  (void)phm3;
}

// The step factors of a sweep along D: dt / (2h) and dt / h from the box's
// step scalars (evaluated once per step with dt), 1 / (2h) from its table entry.
template <typename T>
__device__ __forceinline__ FluidConsts<T> fluid_consts(const FluidArgs<T>& a, int D) {
  const double dt = a.sc->dt;
  FluidConsts<T> k;
  k.k_half = (T)a.sc->kh[D];
  k.k_full = (T)a.sc->kf[D];
  k.half_dt = (T)(0.5 * dt);
  k.dt = (T)dt;
  k.inv2h = (T)a.i2h[D];
  k.halfalpha = (T)(0.5 * a.alpha);
  k.gamma = a.gamma;
  return k;
}

// Strided policy: wave w walks segment sg of 64 pencils.  The segment (hence
// every position and its boundary mapping along d) is uniform across the wave
// and lives in scalar registers; each lane only adds its pencil offset.
// Returns false for waves beyond the grid (the whole wave exits together).
// Two orders of the pencils (nA along x times nO along the other transverse
// axis, p = o * nA + a): contiguous (64 consecutive pencils per wave), or,
// with row_groups and nA >= 64, the four waves of a block on four
// consecutive rows o over the same 64 values of a, so that the neighbouring
// rows a sweep reads along o are mostly the block's own (L1/L2 hits).
__device__ __forceinline__ bool strided_map(int wave, int nA, int nO, int nseg, int row_groups, int& sg, int& p,
                                            bool& active) {
  const int lane = (int)(threadIdx.x & 63);
  if (row_groups && nA >= 64) {
    const int xc = (nA + 63) >> 6;
    const int per_seg = xc * ((nO + 3) >> 2) * 4;
    sg = wave / per_seg;
    if (sg >= nseg) return false;
    const int w = wave - sg * per_seg;
    const int g = w >> 2;
    const int o = (g / xc) * 4 + (w & 3);
    const int a = (g % xc) * 64 + lane;
    active = a < nA && o < nO;
    p = (o < nO ? o : nO - 1) * nA + (a < nA ? a : nA - 1);
    return true;
  }
  const int P = nA * nO;
  const int wps = (P + 63) >> 6;
  sg = wave / wps;
  if (sg >= nseg) return false;
  const int p0 = (wave - sg * wps) * 64 + lane;
  active = p0 < P;
  p = active ? p0 : P - 1;
  return true;
}

// Strided policy: one lane per pencil segment.  For D = y or z the lanes
// walk along x (each load of a wave is 64 consecutive values); for D = x (an
// alternative to the lanes policy) they walk along y, so that a wave's load
// touches 64 rows, one value of each.
template <typename T, int D, int GRAV, bool HSE, int LIM, bool NU>
__global__ __launch_bounds__(256) void fluid_strided_kernel(FluidLaunch<T> L) {
  constexpr int A = D == 0 ? 1 : 0;
  constexpr int O = D == 0 ? 2 : 3 - D;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const BoxDesc* d;
  int lw;
  if (!work_item<K_FLUID_X + D>(L.wl, d, lw)) return;
  const FluidArgs<T> a = fluid_view<T, K_FLUID_X + D>(L, *d);
  const Geo& g = a.g;
  const int nA = g.n[A], nO = g.n[O], nD = g.n[D];
  int sg, p;
  bool active;
  if (!strided_map(lw, nA, nO, a.nseg, L.wl.row_groups, sg, p, active)) return;
  const int s0 = sg * a.seg;
  const int s1 = min(nD, s0 + a.seg);
  int c[3];
  c[A] = p % nA;
  c[O] = p / nA;
  c[D] = 0;
  const long long stD = g.st[D];
  const int bcD = g.bc[D];
  // lane byte offsets (every array is below 4 GiB)
  const long long lbase = (long long)c[A] * g.st[A] + (long long)c[O] * g.st[O];
  const unsigned base = (unsigned)(lbase * (long long)sizeof(T));
  const unsigned hi1 = (unsigned)((lbase + (long long)(map_face(c[T1] + 1, g.n[T1], g.bc[T1]) - c[T1]) * g.st[T1]) *
                                  (long long)sizeof(T));
  const unsigned hi2 = (unsigned)((lbase + (long long)(map_face(c[T2] + 1, g.n[T2], g.bc[T2]) - c[T2]) * g.st[T2]) *
                                  (long long)sizeof(T));
  const FluidConsts<T> k = fluid_consts(a, D);
  FluidHist<T, HSE> hA, hB;
  hA.zero();
  hB.zero();
  struct In {
    T u[5];
    Vec<T, 3> bc;
    T phi, gh;
    T w[5];  // irregular mesh: widths of cells c-4 .. c
  };
  // inputs of position it (loads only: issued one position ahead of use)
  auto load = [&](int it) {
    In in;
    const int s = s0 - 3 + it;  // uniform
    const long long off = (long long)map_cell(s, nD, bcD) * stD;
#pragma unroll
    for (int i = 0; i < 5; ++i) in.u[i] = ld(in_sgpr(a.u[i] + off), base);
    const T* bD0 = in_sgpr(a.b[D] + (long long)map_face(s, nD, bcD) * stD);
    const T* bD1 = in_sgpr(a.b[D] + (long long)map_face(s + 1, nD, bcD) * stD);
    const T* b1 = in_sgpr(a.b[T1] + off);
    const T* b2 = in_sgpr(a.b[T2] + off);
    in.bc.v[D] = T(0.5) * (ld(bD0, base) + ld(bD1, base));
    in.bc.v[T1] = T(0.5) * (ld(b1, base) + ld(b1, hi1));
    in.bc.v[T2] = T(0.5) * (ld(b2, base) + ld(b2, hi2));
    in.phi = GRAV ? load_phi(a.phi, lbase, stD, s, nD, bcD) : T(0);
    if (NU) {
#pragma unroll
      for (int j = 0; j < 5; ++j) in.w[j] = width_at(a.wid[D], s - 4 + j, nD, bcD);
    }
    if (GRAV == 2) {
      // the kick of the cell this position maps to (a ghost is exactly the
      // copy of its kicked cell)
      const int sm = map_cell(s, nD, bcD);
      const T isp0 = NU ? inv_span(width_at(a.wid[D], sm - 1, nD, bcD), width_at(a.wid[D], sm, nD, bcD),
                                   width_at(a.wid[D], sm + 1, nD, bcD))
                        : k.inv2h;
      in.gh = k.half_dt * (load_phi(a.phi, lbase, stD, sm + 1, nD, bcD) -
                           load_phi(a.phi, lbase, stD, sm - 1, nD, bcD)) * isp0;
    } else {
      in.gh = T(0);
    }
    return in;
  };
  auto compute = [&](int it, const In& in, const FluidHist<T, HSE>& hi, FluidHist<T, HSE>& ho) {
    const int s = s0 - 3 + it;
    T un[5];
    const FluidNU<T> nu = NU ? fluid_nu(in.w, k.dt) : FluidNU<T>{};
    fluid_position<T, D, GRAV, HSE, LIM, StridedHist, false, NU>(in.u, in.bc, in.phi, in.gh, nullptr, k, nu, hi, ho,
                                                                  un);
    if (it >= 6 && s - 3 < s1 && active) {
      const long long o = (long long)(s - 3) * stD;
#pragma unroll
      for (int i = 0; i < 5; ++i) st(in_sgpr(a.uo[i] + o), base, un[i]);
    }
  };
  // positions s0-3 .. s1+2, padded to an even count (the pad writes nothing;
  // the prefetch reads at most two positions past the end, mapped in range)
  const int npos = (s1 - s0) + 6;
  if (sizeof(T) == 8 && (GRAV != 0 || HSE || NU || LIM == 2)) {
    // FP64 with gravity, HSE, an irregular mesh or the limiter switch: no
    // lookahead; its registers would halve the waves per SIMD (to one)
    for (int it = 0; it < npos; it += 2) {
      compute(it, load(it), hA, hB);
      compute(it + 1, load(it + 1), hB, hA);
    }
    return;
  }
  In cur = load(0);
  for (int it = 0; it < npos; it += 2) {
    const In nxt = load(it + 1);
    compute(it, cur, hA, hB);
    cur = load(it + 2);
    compute(it + 1, nxt, hB, hA);
  }
}

// Speeds of one cell for Eq. (14)-(15): sp[d] = |v_d| + c_F,d on the active
// axes (0 on an axis with one cell), in the storage precision, with the
// pressure recovered in FP64; also flags a bad state (rho <= 0, p <= 0 or a
// non-finite value).  The pressure takes every conserved value and the cell's
// field, so a non-finite one leaves rho or p non-finite or p <= 0, and a
// speed that is not finite leaves their sum non-finite: four tests instead of
// one per value.  The division by h_d is left to cfl_of: it is monotonic, so
// the maximum of the divided speeds is the divided maximum, bitwise.
template <typename T>
__device__ __forceinline__ void cell_cfl_speeds(const T* u, const T* b, double gamma, const Geo& g, T* sp, int& bad) {
  T b2;
  const T p = pressure<T>(u, b, gamma - 1.0, &b2);
  const T ri = rcp(u[RHO]);
  const T a2 = (T)gamma * p * ri;
  const T q = a2 + b2 * ri;
  T sum = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    sp[d] = T(0);
    if (g.n[d] > 1) {
      const T disc = q * q - T(4) * a2 * b[d] * b[d] * ri;
      const T cf = fsqrt(T(0.5) * (q + fsqrt(disc < T(0) ? T(0) : disc)));
      sp[d] = fabs(u[MX + d] * ri) + cf;
      sum += sp[d];
    }
  }
  const bool ok = u[RHO] > T(0) && p > T(0) && isfinite(u[RHO]) && isfinite(p) && isfinite(sum);
  if (!ok) bad = 1;
}

// max over the active axes of smax[d] / h_d (Eq. 15).
template <typename T>
__device__ __forceinline__ double cfl_of(const T* smax, const Geo& g) {
  double c = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.n[d] > 1) c = fmax(c, (double)smax[d] / g.h[d]);
  return c;
}

// Eq. (70), the CFL condition on an irregular mesh: max over the active axes
// of one cell's speed over its own width along that axis.
template <typename T>
__device__ __forceinline__ double cfl_of_cell(const T* sp, double wx, double wy, double wz, const Geo& g) {
  const double w[3] = {wx, wy, wz};
  double c = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.n[d] > 1) c = fmax(c, (double)sp[d] / w[d]);
  return c;
}

// Reduce (cmax, bad) over the wave and publish with one atomic per wave.
// Every lane of the wave must reach this call.
__device__ __forceinline__ void publish_cfl(double cmax, int bad, Scalars* sc) {
  unsigned long long bits = __double_as_longlong(cmax);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(bits, off, 64);
    bits = o > bits ? o : bits;
    bad |= __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&sc->cmax_bits, bits);
    if (bad) atomicOr(&sc->status, 1);
  }
}

// Lanes policy (D = x): each wave streams rows_per_wave whole x rows.  With
// CFL the sweep also reduces the CFL speed of the state it writes (the last
// sub-operator of a double step leaves the next step's time step ready).
template <typename T, int GRAV, bool HSE, int LIM, bool CFL, bool NU>
__global__ __launch_bounds__(256) void fluid_lanes_kernel(FluidLaunch<T> FL) {
  constexpr int D = 0;
  const BoxDesc* d;
  int lw;
  if (!work_item<K_FLUID_X>(FL.wl, d, lw)) return;
  const FluidArgs<T> a = fluid_view<T, K_FLUID_X>(FL, *d);
  const Geo& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int L = nx + 6;                     // stream positions per row
  const long long nrows = (long long)ny * nz;
  const long long wave = lw;
  const int lane = threadIdx.x & 63;
  const long long r0 = wave * a.rows_per_wave;
  if (r0 >= nrows) return;  // whole wave exits together
  const int rows = (int)min((long long)a.rows_per_wave, nrows - r0);
  const int npos = rows * L;
  // lanes 0..HALO-1 recompute the last positions of the previous iteration:
  // the output of lane i depends on lanes i-6 .. i (the corrector's flux
  // difference, the limited slopes, the relaxed differences, the predictor
  // and its fluxes each reach one position back), so lanes 6..63 are exact
  constexpr int HALO = 6, STEP = 64 - HALO;
  const int nit = (npos + STEP - 1) / STEP;
  const FluidConsts<T> k = fluid_consts(a, D);
  FluidHist<T, HSE> hA, hB;  // unused by the carry-free policy
  T smax[3] = {T(0), T(0), T(0)};  // per axis, the largest |v_d| + c_F,d of the lane's cells
  double cnu = 0.0;  // irregular mesh: the CFL speed over widths, per cell
  int bad = 0;
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];  // arrays < 2^32 bytes
  const unsigned up = st2 - (unsigned)(ny - 1) * st1;
  RowCursor rc;
  rc.init(lane - HALO, L, (int)r0, rows, ny, st1, st2, up);  // the halo lanes start before the stream (clamped to its start)
  constexpr unsigned z4 = sizeof(T);
  // byte offsets of the face above the row's cells along y and z: the next
  // row or plane, or on a periodic axis from the last one back to the first
  const unsigned dy_in = st1 * z4, dy_last = g.bc[1] ? dy_in : (unsigned)(1 - ny) * st1 * z4;
  const unsigned dz_in = st2 * z4, dz_last = g.bc[2] ? dz_in : (unsigned)(1 - nz) * st2 * z4;
  unsigned base = 0, dy = 0, dz = 0;  // the row's offset (elements) and face offsets (bytes)
  T wy = T(1), wz = T(1);             // irregular mesh: widths of the row's cell in y, z
  struct In {
    T u[5], u3[5];
    Vec<T, 3> bc;
    T phi, gh;
    T w[5], wy, wz;  // irregular mesh: widths of cells c-4 .. c along x; the row's y, z widths
    unsigned o3;  // byte offset of the output cell c-3
    int co;       // output cell index along x
    bool valid;
  };
  // inputs of the lane's next stream position (loads only, one iteration ahead)
  auto load = [&](int it) {
    if (rc.moved) {
      const int y = rc.y, z = rc.z;
      base = rc.base;
      dy = y + 1 < ny ? dy_in : dy_last;
      dz = z + 1 < nz ? dz_in : dz_last;
      if (NU) {
        wy = width_at(a.wid[1], y, ny, g.bc[1]);
        wz = width_at(a.wid[2], z, nz, g.bc[2]);
      }
    }
    In in;
    in.valid = lane >= HALO && it * STEP + lane - HALO < npos;
    // cell index along x (-3 .. nx+2); lanes past the end of the stream sit
    // on the wave's last row with cp >= L and are clamped into it, and the
    // halo lanes of the first iteration onto its start, so that every index
    // they map stays in the box (they store nothing)
    const int cpos = min(max(rc.cp, 0), L - 1) - 3;
    in.co = cpos - 3;
    const unsigned ms = (base + (unsigned)map_cell_near(cpos, nx, g.bc[0])) * z4;
#pragma unroll
    for (int i = 0; i < 5; ++i) in.u[i] = ld(a.u[i], ms);
    const unsigned f0 = (base + (unsigned)map_face_near(cpos, nx, g.bc[0])) * z4;
    const unsigned f1 = (base + (unsigned)map_face_near(cpos + 1, nx, g.bc[0])) * z4;
    in.bc.v[0] = T(0.5) * (ld(a.b[0], f0) + ld(a.b[0], f1));
    in.bc.v[1] = T(0.5) * (ld(a.b[1], ms) + ld(a.b[1], ms + dy));
    in.bc.v[2] = T(0.5) * (ld(a.b[2], ms) + ld(a.b[2], ms + dz));
    in.phi = GRAV ? load_phi(a.phi, (long long)base, 1, cpos, nx, g.bc[0]) : T(0);
    if (NU) {
#pragma unroll
      for (int j = 0; j < 5; ++j) in.w[j] = width_at(a.wid[0], cpos - 4 + j, nx, g.bc[0]);
      in.wy = wy;
      in.wz = wz;
    }
    if (GRAV == 2) {
      // the kick of the cell this position maps to (a ghost is exactly the
      // copy of its kicked cell)
      const int cm = map_cell(cpos, nx, g.bc[0]);
      const T isp0 = NU ? inv_span(width_at(a.wid[0], cm - 1, nx, g.bc[0]), width_at(a.wid[0], cm, nx, g.bc[0]),
                                   width_at(a.wid[0], cm + 1, nx, g.bc[0]))
                        : k.inv2h;
      in.gh = k.half_dt * (load_phi(a.phi, (long long)base, 1, cm + 1, nx, g.bc[0]) -
                           load_phi(a.phi, (long long)base, 1, cm - 1, nx, g.bc[0])) * isp0;
    } else {
      in.gh = T(0);
    }
    in.o3 = (base + (unsigned)map_cell_near(cpos - 3, nx, g.bc[0])) * z4;
#pragma unroll
    for (int i = 0; i < 5; ++i) in.u3[i] = ld(a.u[i], in.o3);
    rc.advance(L, rows, ny, st1, up, STEP);
    return in;
  };
  auto compute = [&](const In& in, const FluidHist<T, HSE>& hi, FluidHist<T, HSE>& ho) {
    T un[5];
    const FluidNU<T> nu = NU ? fluid_nu(in.w, k.dt) : FluidNU<T>{};
    fluid_position<T, D, GRAV, HSE, LIM, LaneShift, true, NU>(in.u, in.bc, in.phi, in.gh, in.u3, k, nu, hi, ho, un);
    const bool out = in.valid && in.co >= 0 && in.co < nx;
    if (out) {
#pragma unroll
      for (int i = 0; i < 5; ++i) st(a.uo[i], in.o3, un[i]);
    }
    if (CFL) {
      // the cell-centred field of the output cell c-3 is the one position
      // c-3 loaded, three lanes down (the same row for every output lane)
      T b3[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) b3[j] = lane_shr(lane_shr(lane_shr(in.bc.v[j])));
      int cell_bad = 0;
      T sp[3];
      cell_cfl_speeds<T>(un, b3, a.gamma, g, sp, cell_bad);
      if (out) {
        if (NU) {
          cnu = fmax(cnu, cfl_of_cell(sp, (double)in.w[1], (double)in.wy, (double)in.wz, g));
        } else {
#pragma unroll
          for (int dd = 0; dd < 3; ++dd) smax[dd] = fmax(smax[dd], sp[dd]);
        }
        bad |= cell_bad;
      }
    }
  };
  In cur = load(0);
  for (int it = 0; it < nit; it += 2) {
    const In nxt = load(it + 1);
    compute(cur, hA, hB);
    cur = load(it + 2);
    compute(nxt, hB, hA);
  }
  if (CFL) publish_cfl(NU ? cnu : cfl_of(smax, g), bad, const_cast<Scalars*>(a.sc));
}

// ------------------------------------------------------------ B_d (fused)
// One kernel per field sweep: the transverse advection of b_t1 and b_t2 and
// the constraint update of b_d from the same edge fluxes (Eq. 64), without
// an edge-flux array in HBM.  A thread owns the face rows (t1-face c1, t2-cell
// c2) of b_t1, (t1-cell c1, t2-face c2) of b_t2 and (c1, c2) of b_d; the edge
// fluxes of the neighbouring rows c1+1 and c2+1 that the constraint needs are
// recomputed from the same inputs (bitwise the values their owners compute).
template <typename T>
struct FieldArgs {
  const T* rho;
  const T* md;             // momentum along d (the fluid state is held fixed)
  const T* bt[2];          // b_t1, b_t2 (input)
  const T* bd;             // b_d (input)
  T* bto[2];               // outputs
  T* bdo;
  const T* wid[3];         // irregular mesh: cell widths per axis, else null
  Geo g;
  int seg, nseg;           // strided policy
  int rows_per_wave;       // lanes policy
  const Scalars* sc;
  double ih[3];            // 1 / h_d
};

template <typename T>
struct FieldLaunch {
  const T* rho;
  const T* md;
  const T* bt[2];
  const T* bd;
  T* bto[2];
  T* bdo;
  const T* wid[3];  // irregular meshes: every table box's cell widths per axis (at BoxDesc::woff), else null
  WorkList wl;
  Scalars* sc;
};

template <typename T, int KIND>
__device__ __forceinline__ FieldArgs<T> field_view(const FieldLaunch<T>& L, const BoxDesc& d) {
  FieldArgs<T> a;
  const long long off = d.off;
  a.rho = L.rho + off;
  a.md = L.md + off;
  a.bt[0] = L.bt[0] + off;
  a.bt[1] = L.bt[1] + off;
  a.bd = L.bd + off;
  a.bto[0] = L.bto[0] + off;
  a.bto[1] = L.bto[1] + off;
  a.bdo = L.bdo + off;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.wid[i] = L.wid[i] ? L.wid[i] + d.woff[i] : nullptr;
  a.g = d.g;
  const int D = KIND - K_FIELD_X;
  a.seg = d.par[KIND];
  a.nseg = d.nseg[KIND];
  a.rows_per_wave = d.par[KIND];
  a.sc = L.sc + d.slot;
#pragma unroll
  for (int i = 0; i < 3; ++i) a.ih[i] = d.ih[i];
  (void)D;
  return a;
}

template <typename T>
struct RowHist {
  T w1, w2, b1, b2, b3, b4, f2, p1, vb1, vb2, vb3, fp3, fp4, fp5, P2;
  __device__ void zero() { w1 = w2 = b1 = b2 = b3 = b4 = f2 = p1 = vb1 = vb2 = vb3 = fp3 = fp4 = fp5 = P2 = T(0); }
};

// One position of one face row of b_t along d: Eq. (65) face velocity w0 at
// cell c, Eq. (66) smoothing, Eq. (68) interface velocity, Eq. (67)
// first-order upwind predictor flux, second-order limited upwind corrector
// flux (end of Sect. 2.4), Eq. (63).  Gives the edge flux at d-face c-3 (the
// interface between c-4 and c-3) and, for NEED_BN, the new b_t of cell c-4.
// Irregular mesh (Sect. 2.5): the weights that put the limited slopes of cells
// c-4 (upwind side "up") and c-3 ("dn") on the interface between them, as in
// the fluid corrector; k_half and k_full are then those of cells c-2 and c-4.
template <typename T>
struct FieldW {
  T wl4, wr4, wl3, wr3;
};

template <typename T, int LIM, typename H, bool NEED_BN, bool RELOAD_B4, bool NU = false>
__device__ __forceinline__ T row_position(T w0, T bb, T b4_loaded, T k_half, T k_full, const FieldW<T>& fw,
                                          const RowHist<T>& hi, RowHist<T>& ho, T& bn) {
  const T w1 = H::prev(w0, hi.w1, ho.w1);
  const T w2 = H::prev(w1, hi.w2, ho.w2);
  // outer neighbours first: an odd face velocity gives exact negatives here
  // and V = 0 exactly, which the <= 0 branch of Eq. (67) decides
  const T vbc = T(0.25) * ((w2 + w0) + T(2) * w1);   // v-bar of c-1
  const T b1 = H::prev(bb, hi.b1, ho.b1);                   // b of c-1
  const T fc = vbc * b1;                            // f of c-1
  const T vb1 = H::prev(vbc, hi.vb1, ho.vb1);                // v-bar of c-2
  const T V = T(0.5) * (vb1 + vbc);                 // interface c-3/2
  const T f2 = H::prev(fc, hi.f2, ho.f2);                   // f of c-2
  const T P1 = V > T(0) ? f2 : fc;                  // Phi1 at c-3/2
  const T p1 = H::prev(P1, hi.p1, ho.p1);                   // Phi1 at c-5/2
  const T b2 = H::prev(b1, hi.b2, ho.b2);                   // b of c-2
  const T bp = b2 - k_half * (P1 - p1);             // b' of c-2
  const T fp2 = vb1 * bp;                           // f' of c-2
  const T vb2 = H::prev(vb1, hi.vb2, ho.vb2);                // v-bar of c-3
  const T vb3 = H::prev(vb2, hi.vb3, ho.vb3);                // v-bar of c-4
  const T V7 = T(0.5) * (vb3 + vb2);                // interface c-7/2
  const T fp3 = H::prev(fp2, hi.fp3, ho.fp3);
  const T fp4 = H::prev(fp3, hi.fp4, ho.fp4);
  const T fp5 = H::prev(fp4, hi.fp5, ho.fp5);
  T up, dn;
  if (!NU) {
    up = fp4 + T(0.5) * limit<T, LIM>(fp4 - fp5, fp3 - fp4);
    dn = fp3 - T(0.5) * limit<T, LIM>(fp3 - fp4, fp2 - fp3);
  } else {
    up = fp4 + limit<T, LIM>(fw.wl4 * (fp4 - fp5), fw.wr4 * (fp3 - fp4));
    dn = fp3 - limit<T, LIM>(fw.wl3 * (fp3 - fp4), fw.wr3 * (fp2 - fp3));
  }
  const T P2c = V7 > T(0) ? up : dn;                // Phi2 at c-7/2
  if (NEED_BN) {
    const T P2 = H::prev(P2c, hi.P2, ho.P2);                // Phi2 at c-9/2
    T b4;
    if (RELOAD_B4) {
      b4 = b4_loaded;
    } else {
      const T b3 = H::prev(b2, hi.b3, ho.b3);
      b4 = H::prev(b3, hi.b4, ho.b4);
    }
    bn = b4 - k_full * (P2c - P2);
  }
  return P2c;
}

template <typename T>
struct FieldConsts {
  T k_half, k_full, dt, ih1, ih2;
};

// The step factors of a field sweep along D (see fluid_consts).
template <typename T, int D>
__device__ __forceinline__ FieldConsts<T> field_consts(const FieldArgs<T>& a) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  FieldConsts<T> k;
  k.k_half = (T)a.sc->kh[D];
  k.k_full = (T)a.sc->kf[D];
  k.dt = (T)a.sc->dt;
  k.ih1 = (T)a.ih[T1];
  k.ih2 = (T)a.ih[T2];
  return k;
}

// Offsets a position needs besides the d offset.  Cells are relative to the
// thread's own cell (c1, c2) mapped into the box (on the outflow face rows
// c = n_t the mapped cell is n_t - 1, exactly the ghost the boundary copies);
// faces are relative to the face-row base (c1, c2).
struct FieldOffsets {
  long long c1m, c1p, c2m, c2p;   // cells (c1-1, c2), (c1+1, c2), (c1, c2-1), (c1, c2+1)
  long long f1p, f2p;             // t1-face c1+1, t2-face c2+1
};

template <int D>
__device__ __forceinline__ FieldOffsets field_offsets(const Geo& g, int c1, int c2) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  FieldOffsets o;
  const int m1 = map_cell(c1, g.n[T1], g.bc[T1]);
  const int m2 = map_cell(c2, g.n[T2], g.bc[T2]);
  o.c1m = (long long)(map_cell(c1 - 1, g.n[T1], g.bc[T1]) - m1) * g.st[T1];
  o.c1p = (long long)(map_cell(c1 + 1, g.n[T1], g.bc[T1]) - m1) * g.st[T1];
  o.c2m = (long long)(map_cell(c2 - 1, g.n[T2], g.bc[T2]) - m2) * g.st[T2];
  o.c2p = (long long)(map_cell(c2 + 1, g.n[T2], g.bc[T2]) - m2) * g.st[T2];
  o.f1p = (long long)(map_face(c1 + 1, g.n[T1], g.bc[T1]) - c1) * g.st[T1];
  o.f2p = (long long)(map_face(c2 + 1, g.n[T2], g.bc[T2]) - c2) * g.st[T2];
  return o;
}

// The same offsets for the x sweep's rows (t1 = y, t2 = z), in bytes, with
// the cheap maps (the neighbours are within one period); base is the face
// row's element offset y st1 + z st2, which the lanes cursor keeps.
// All in unsigned arithmetic: a difference that is negative wraps, and adding
// it to an offset wraps back (every offset is below 2^32 bytes).
struct RowOffsets {
  unsigned base, ownc;             // face row (c1, c2) and its mapped own cell
  unsigned c1m, c1p, c2m, c2p, f1p, f2p;
};

template <typename T>
__device__ __forceinline__ void row_offsets(const Geo& g, int c1, int c2, unsigned base, RowOffsets& r) {
  constexpr unsigned z = sizeof(T);
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];
  const int n1 = g.n[1], n2 = g.n[2], b1 = g.bc[1], b2 = g.bc[2];
  const int m1 = map_cell_near(c1, n1, b1), m2 = map_cell_near(c2, n2, b2);
  r.base = base * z;
  r.ownc = (base + (unsigned)(m1 - c1) * st1 + (unsigned)(m2 - c2) * st2) * z;
  r.c1m = (unsigned)(map_cell_near(c1 - 1, n1, b1) - m1) * st1 * z;
  r.c1p = (unsigned)(map_cell_near(c1 + 1, n1, b1) - m1) * st1 * z;
  r.c2m = (unsigned)(map_cell_near(c2 - 1, n2, b2) - m2) * st2 * z;
  r.c2p = (unsigned)(map_cell_near(c2 + 1, n2, b2) - m2) * st2 * z;
  r.f1p = (unsigned)(map_face_near(c1 + 1, n1, b1) - c1) * st1 * z;
  r.f2p = (unsigned)(map_face_near(c2 + 1, n2, b2) - c2) * st2 * z;
}

// Byte offsets of everything one position reads, relative to the arrays'
// base pointers (which carry the d offset when it is wave-uniform).
struct FieldLane {
  unsigned cc, c1m, c1p, c2m, c2p;  // cells (c1, c2) and its four transverse neighbours
  unsigned fA, fB, fC, fD;          // b_t1 at t1-faces c1, c1+1; b_t2 at t2-faces c2, c2+1
};

template <typename T>
__device__ __forceinline__ FieldLane field_lane(long long base, long long ownc, const FieldOffsets& o, long long off) {
  constexpr long long z = sizeof(T);
  FieldLane l;
  l.cc = (unsigned)((ownc + off) * z);
  l.c1m = (unsigned)((ownc + off + o.c1m) * z);
  l.c1p = (unsigned)((ownc + off + o.c1p) * z);
  l.c2m = (unsigned)((ownc + off + o.c2m) * z);
  l.c2p = (unsigned)((ownc + off + o.c2p) * z);
  l.fA = (unsigned)((base + off) * z);
  l.fB = (unsigned)((base + off + o.f1p) * z);
  l.fC = l.fA;
  l.fD = (unsigned)((base + off + o.f2p) * z);
  return l;
}

// Inputs of one position of the four face rows (loads only, so that they can
// be issued a position ahead of their use).
template <typename T>
struct FieldIn {
  T md[5], rho[5];  // cells (c1, c2), (c1-1, c2), (c1+1, c2), (c1, c2-1), (c1, c2+1)
  T b[4];           // b_t1 at t1-faces c1, c1+1; b_t2 at t2-faces c2, c2+1
  T b4a, b4c;       // b_t1, b_t2 of cell c-4 (lanes policy)
  T bd3;            // b_d at d-face c-3, which the constraint update of this position rewrites
};

template <typename T>
__device__ __forceinline__ FieldIn<T> field_load(const T* md, const T* rho, const T* bt0, const T* bt1,
                                                  const FieldLane& l) {
  FieldIn<T> in;
  const unsigned c[5] = {l.cc, l.c1m, l.c1p, l.c2m, l.c2p};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    in.md[i] = ld(md, c[i]);
    in.rho[i] = ld(rho, c[i]);
  }
  in.b[0] = ld(bt0, l.fA);
  in.b[1] = ld(bt0, l.fB);
  in.b[2] = ld(bt1, l.fC);
  in.b[3] = ld(bt1, l.fD);
  in.b4a = in.b4c = in.bd3 = T(0);
  return in;
}

// Irregular mesh: the factors of one face row set (fixed along the pencil):
// per t-face the weights of its low and high cell in the interpolation of
// Eq. (65) (each the other cell's width over their sum), and 1/width of the
// thread's cell across t1 and t2 for Eq. (64).
template <typename T>
struct FieldRowNU {
  T a[4][2];  // faces A (t1-face c1), B (c1+1), C (t2-face c2), D (c2+1): low, high
  T ih1, ih2;
};
template <typename T>
__device__ __forceinline__ FieldRowNU<T> field_row_nu(T w1m, T w10, T w1p, T w2m, T w20, T w2p) {
  FieldRowNU<T> r;
  const T sA = rcp(w1m + w10), sB = rcp(w10 + w1p), sC = rcp(w2m + w20), sD = rcp(w20 + w2p);
  r.a[0][0] = w10 * sA;
  r.a[0][1] = w1m * sA;
  r.a[1][0] = w1p * sB;
  r.a[1][1] = w10 * sB;
  r.a[2][0] = w20 * sC;
  r.a[2][1] = w2m * sC;
  r.a[3][0] = w2p * sD;
  r.a[3][1] = w20 * sD;
  r.ih1 = rcp(w10);
  r.ih2 = rcp(w20);
  return r;
}
// Irregular mesh: the per-position factors from the widths of cells c-5 .. c-2.
template <typename T>
struct FieldPosNU {
  T kh, kf;
  FieldW<T> w;
};
template <typename T>
__device__ __forceinline__ FieldPosNU<T> field_pos_nu(const T* w, T dt) {
  FieldPosNU<T> f;
  f.kh = T(0.5) * dt * rcp(w[3]);
  f.kf = dt * rcp(w[1]);
  f.w.wl4 = w[1] * rcp(w[0] + w[1]);
  f.w.wr4 = w[1] * rcp(w[1] + w[2]);
  f.w.wl3 = w[2] * rcp(w[1] + w[2]);
  f.w.wr3 = w[2] * rcp(w[2] + w[3]);
  return f;
}
// Eq. (65) on an irregular mesh: linear interpolation between the two cell
// centres, two separate products (never fused, so the value is exactly odd
// when the velocities and widths are mirrored).
template <typename T>
__device__ __forceinline__ T face_interp(T alo, T vlo, T ahi, T vhi) {
  const T p = alo * vlo;
  const T q = ahi * vhi;
  return p + q;
}

// All four face rows at one position.
template <typename T, int LIM, typename H, bool RELOAD_B4, bool NU = false>
__device__ __forceinline__ void field_compute(const FieldIn<T>& in, const FieldConsts<T>& k, const FieldRowNU<T>& rn,
                                              const FieldPosNU<T>& pn, const RowHist<T>* hi, RowHist<T>* ho, T& bn1,
                                              T& bn2, T& dbd) {
  // v_d of the five cells around the thread's pencil (Sect. 2.4: the fluid
  // state current at B_d)
  T v[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = in.md[i] * rcp(in.rho[i]);
  // Eq. (65) on the four t-faces
  T wA, wB, wC, wD;
  if (!NU) {
    wA = T(0.5) * (v[1] + v[0]);
    wB = T(0.5) * (v[0] + v[2]);
    wC = T(0.5) * (v[3] + v[0]);
    wD = T(0.5) * (v[0] + v[4]);
  } else {
    wA = face_interp(rn.a[0][0], v[1], rn.a[0][1], v[0]);
    wB = face_interp(rn.a[1][0], v[0], rn.a[1][1], v[2]);
    wC = face_interp(rn.a[2][0], v[3], rn.a[2][1], v[0]);
    wD = face_interp(rn.a[3][0], v[0], rn.a[3][1], v[4]);
  }
  const T kh = NU ? pn.kh : k.k_half, kf = NU ? pn.kf : k.k_full;
  T dummy;
  const T eA = row_position<T, LIM, H, true, RELOAD_B4, NU>(wA, in.b[0], in.b4a, kh, kf, pn.w, hi[0], ho[0], bn1);
  const T eB = row_position<T, LIM, H, false, false, NU>(wB, in.b[1], T(0), kh, kf, pn.w, hi[1], ho[1], dummy);
  const T eC = row_position<T, LIM, H, true, RELOAD_B4, NU>(wC, in.b[2], in.b4c, kh, kf, pn.w, hi[2], ho[2], bn2);
  const T eD = row_position<T, LIM, H, false, false, NU>(wD, in.b[3], T(0), kh, kf, pn.w, hi[3], ho[3], dummy);
  // Eq. (64), physical signs: d/dt b_d = d_t1 Phi^t1 + d_t2 Phi^t2
  dbd = k.dt * ((eB - eA) * (NU ? rn.ih1 : k.ih1) + (eD - eC) * (NU ? rn.ih2 : k.ih2));
}

// Strided policy (d = y or z).
template <typename T, int D, int LIM, bool NU>
__global__ __launch_bounds__(256) void field_strided_kernel(FieldLaunch<T> FL) {
  static_assert(D != 0, "x sweeps use the lanes policy");
  constexpr int A = 0;
  constexpr int O = 3 - D;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const BoxDesc* d;
  int lw;
  if (!work_item<K_FIELD_X + D>(FL.wl, d, lw)) return;
  const FieldArgs<T> a = field_view<T, K_FIELD_X + D>(FL, *d);
  const Geo& g = a.g;
  const int nD = g.n[D];
  const int rA = g.n[A] + g.bc[A];  // outflow adds the face row n
  const int rO = g.n[O] + g.bc[O];
  int sg, p;
  bool active;
  if (!strided_map(lw, rA, rO, a.nseg, FL.wl.row_groups, sg, p, active)) return;
  const int s0 = sg * a.seg;
  const int s1 = min(nD, s0 + a.seg);
  const bool last = (s1 == nD);
  const bool outD = g.bc[D] == 1;
  int c[3];
  c[A] = p % rA;
  c[O] = p / rA;
  c[D] = 0;
  const int c1 = c[T1], c2 = c[T2];
  const bool own1 = active && c2 < g.n[T2];   // b_t1 row is real
  const bool own2 = active && c1 < g.n[T1];   // b_t2 row is real
  const bool ownd = own1 && own2;             // b_d row is real
  const long long stD = g.st[D];
  const long long base = (long long)c1 * g.st[T1] + (long long)c2 * g.st[T2];
  const long long ownc = (long long)map_cell(c1, g.n[T1], g.bc[T1]) * g.st[T1] +
                         (long long)map_cell(c2, g.n[T2], g.bc[T2]) * g.st[T2];
  const FieldOffsets oc = field_offsets<D>(g, c1, c2);
  const FieldConsts<T> k = field_consts<T, D>(a);
  RowHist<T> hA[4], hB[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hA[q].zero();
    hB[q].zero();
  }
  const FieldLane l = field_lane<T>(base, ownc, oc, 0);  // lane byte offsets, fixed along the pencil
  FieldRowNU<T> rn{};
  if (NU) {
    const T* w1 = a.wid[T1];
    const T* w2 = a.wid[T2];
    const int n1 = g.n[T1], n2 = g.n[T2], b1 = g.bc[T1], b2 = g.bc[T2];
    rn = field_row_nu(width_at(w1, c1 - 1, n1, b1), width_at(w1, c1, n1, b1), width_at(w1, c1 + 1, n1, b1),
                      width_at(w2, c2 - 1, n2, b2), width_at(w2, c2, n2, b2), width_at(w2, c2 + 1, n2, b2));
  }
  auto load = [&](int it) {
    const int s = s0 - 4 + it;  // uniform
    const long long off = (long long)map_cell(s, nD, g.bc[D]) * stD;
    FieldIn<T> in = field_load<T>(in_sgpr(a.md + off), in_sgpr(a.rho + off), in_sgpr(a.bt[0] + off),
                                  in_sgpr(a.bt[1] + off), l);
    // b_d at d-face s-3, issued with the other loads (the constraint update
    // of this position rewrites it); the mapped face is in range everywhere
    in.bd3 = ld(in_sgpr(a.bd + (long long)map_face(s - 3, nD, g.bc[D]) * stD), l.fA);
    return in;
  };
  auto compute = [&](int it, const FieldIn<T>& in, const RowHist<T>* hi, RowHist<T>* ho) {
    const int s = s0 - 4 + it;
    T bn1, bn2, dbd;
    FieldPosNU<T> pn{};
    if (NU) {
      T w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] = width_at(a.wid[D], s - 5 + j, nD, g.bc[D]);
      pn = field_pos_nu(w, k.dt);
    }
    field_compute<T, LIM, StridedHist, false, NU>(in, k, rn, pn, hi, ho, bn1, bn2, dbd);
    if (it >= 8 && s - 4 < s1) {
      const long long ob = (long long)(s - 4) * stD;
      if (own1) st(in_sgpr(a.bto[0] + ob), l.fA, bn1);
      if (own2) st(in_sgpr(a.bto[1] + ob), l.fA, bn2);
    }
    const int fd = s - 3;
    if (ownd && it >= 7 && (fd < s1 || (last && outD && fd == nD))) {
      const long long of = (long long)fd * stD;
      st(in_sgpr(a.bdo + of), l.fA, in.bd3 + dbd);
    }
  };
  // positions s0-4 .. s1+3, padded to an even count (the pad writes nothing;
  // the lookahead reads at most two positions past the end, mapped in range).
  // The lookahead costs one wave per SIMD in FP32 (5 -> 4) and hides more
  // than that (measured).
  const int npos = (s1 - s0) + 8;
  FieldIn<T> cur = load(0);
  for (int it = 0; it < npos; it += 2) {
    const FieldIn<T> nxt = load(it + 1);
    compute(it, cur, hA, hB);
    cur = load(it + 2);
    compute(it + 1, nxt, hB, hA);
  }
}

// The x field sweep with one face row (y, z) per wave, on a uniform mesh.
// The row, its base and its neighbour offsets are wave-uniform, so every
// load and store takes a scalar base and the lane's x offset only, and an
// iteration that lies inside the row (every cell it reaches in [0, n_x))
// takes the x index unmapped.  Iteration it covers positions
// it STEP .. it STEP + STEP - 1 of the row (the last one partly), its first
// HALO lanes recomputing the positions before them as in the general path.
template <typename T, int LIM>
__device__ __forceinline__ void field_lanes_row(const FieldArgs<T>& a, const FieldConsts<T>& k, int y, int zc) {
  const Geo& g = a.g;
  const int nx = g.n[0];
  const bool outx = g.bc[0] == 1;
  const int L = nx + 8;
  constexpr int HALO = 8, STEP = 64 - HALO;
  const int lane = threadIdx.x & 63;
  constexpr unsigned z = sizeof(T);
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];
  RowOffsets ro;
  row_offsets<T>(g, y, zc, (unsigned)y * st1 + (unsigned)zc * st2, ro);
  const bool own1 = zc < g.n[2], own2 = y < g.n[1];
  auto at = [](const T* p, unsigned b) {
    return in_sgpr((const T*)((const char*)p + (unsigned)__builtin_amdgcn_readfirstlane((int)b)));
  };
  auto at_out = [](T* p, unsigned b) {
    return in_sgpr((T*)((char*)p + (unsigned)__builtin_amdgcn_readfirstlane((int)b)));
  };
  const unsigned cn[5] = {ro.ownc, ro.ownc + ro.c1m, ro.ownc + ro.c1p, ro.ownc + ro.c2m, ro.ownc + ro.c2p};
  const T* md[5];
  const T* rh[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    md[i] = at(a.md, cn[i]);
    rh[i] = at(a.rho, cn[i]);
  }
  const T* bA = at(a.bt[0], ro.base);
  const T* bB = at(a.bt[0], ro.base + ro.f1p);
  const T* bC = at(a.bt[1], ro.base);
  const T* bD = at(a.bt[1], ro.base + ro.f2p);
  const T* bd = at(a.bd, ro.base);
  T* o1 = at_out(a.bto[0], ro.base);
  T* o2 = at_out(a.bto[1], ro.base);
  T* od = at_out(a.bdo, ro.base);
  RowHist<T> hA[4], hB[4];  // unused by the carry-free policy
  struct In {
    FieldIn<T> f;
    unsigned oc, o4, of;  // x byte offsets of cells c and c-4 and of d-face c-3
    int cpos;
    bool valid;
  };
  auto load = [&](int it) {
    In in;
    const int p0 = it * STEP - HALO;  // position of lane 0 (uniform)
    const int p = p0 + lane;
    in.valid = lane >= HALO && p < L;
    const int c0 = p0 - 4;            // cell index of lane 0
    if (c0 >= 4 && c0 + 63 < nx) {    // uniform: the whole iteration inside the row
      in.cpos = p - 4;
      in.oc = (unsigned)in.cpos * z;
      in.o4 = in.oc - 4 * z;
      in.of = in.oc - 3 * z;
    } else {
      // clamped as in the general path: every index stays in the box
      in.cpos = min(max(p, 0), L - 1) - 4;
      in.oc = (unsigned)map_cell_near(in.cpos, nx, g.bc[0]) * z;
      in.o4 = (unsigned)map_cell_near(in.cpos - 4, nx, g.bc[0]) * z;
      in.of = (unsigned)map_face_near(in.cpos - 3, nx, g.bc[0]) * z;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      in.f.md[i] = ld(md[i], in.oc);
      in.f.rho[i] = ld(rh[i], in.oc);
    }
    in.f.b[0] = ld(bA, in.oc);
    in.f.b[1] = ld(bB, in.oc);
    in.f.b[2] = ld(bC, in.oc);
    in.f.b[3] = ld(bD, in.oc);
    in.f.b4a = ld(bA, in.o4);
    in.f.b4c = ld(bC, in.o4);
    in.f.bd3 = ld(bd, in.of);
    return in;
  };
  auto compute = [&](const In& in, const RowHist<T>* hi, RowHist<T>* ho) {
    T bn1, bn2, dbd;
    field_compute<T, LIM, LaneShift, true, false>(in.f, k, FieldRowNU<T>{}, FieldPosNU<T>{}, hi, ho, bn1, bn2, dbd);
    const int cb = in.cpos - 4;
    if (in.valid && cb >= 0 && cb < nx) {
      if (own1) st(o1, in.o4, bn1);
      if (own2) st(o2, in.o4, bn2);
    }
    const int fd = in.cpos - 3;
    if (in.valid && own1 && own2 && fd >= 0 && (fd < nx || (outx && fd == nx))) st(od, in.of, in.f.bd3 + dbd);
  };
  const int nit = (L + STEP - 1) / STEP;
  In cur = load(0);
  for (int it = 0; it < nit; it += 2) {
    const In nxt = load(it + 1);
    compute(cur, hA, hB);
    cur = load(it + 2);
    compute(nxt, hB, hA);
  }
}

// Lanes policy (d = x): waves stream whole rows (y, z) of faces, each padded
// by 4 positions before and 4 after.
template <typename T, int LIM, bool NU>
__global__ __launch_bounds__(256) void field_lanes_kernel(FieldLaunch<T> FL) {
  constexpr int D = 0;
  const BoxDesc* d;
  int lw;
  if (!work_item<K_FIELD_X>(FL.wl, d, lw)) return;
  const FieldArgs<T> a = field_view<T, K_FIELD_X>(FL, *d);
  const Geo& g = a.g;
  const int nx = g.n[0];
  const bool outx = g.bc[0] == 1;
  const int L = nx + 8;
  const int ry = g.n[1] + g.bc[1];
  const int rz = g.n[2] + g.bc[2];
  const long long nrows = (long long)ry * rz;
  const long long wave = lw;
  const int lane = threadIdx.x & 63;
  const long long r0 = wave * a.rows_per_wave;
  if (r0 >= nrows) return;  // whole wave exits together
  if (!NU && a.rows_per_wave == 1) {
    const int r = __builtin_amdgcn_readfirstlane((int)r0);
    const int zr = r / ry;
    field_lanes_row<T, LIM>(a, field_consts<T, D>(a), r - zr * ry, zr);
    return;
  }
  const int rows = (int)min((long long)a.rows_per_wave, nrows - r0);
  const int npos = rows * L;
  // lanes 0..HALO-1 recompute the last positions of the previous iteration:
  // the new transverse face of lane i depends on lanes i-8 .. i (the
  // corrector flux and its neighbour, the limited slopes over three
  // predictor fluxes, the predictor's upwind fluxes and the smoothed face
  // velocity each reach back), the edge flux of the normal update on lanes
  // i-7 .. i, so lanes 8..63 are exact
  constexpr int HALO = 8, STEP = 64 - HALO;
  const int nit = (npos + STEP - 1) / STEP;
  const FieldConsts<T> k = field_consts<T, D>(a);
  RowHist<T> hA[4], hB[4];  // unused by the carry-free policy
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];  // arrays < 2^32 bytes
  const unsigned up = st2 - (unsigned)(ry - 1) * st1;
  RowCursor rc;
  rc.init(lane - HALO, L, (int)r0, rows, ry, st1, st2, up);  // the halo lanes start before the stream (clamped to its start)
  RowOffsets ro;
  bool own1 = false, own2 = false;
  FieldRowNU<T> rnr{};  // irregular mesh: the factors of the current row
  struct In {
    FieldIn<T> f;
    FieldRowNU<T> rn;
    T w[4];              // irregular mesh: widths of cells c-5 .. c-2 along x
    unsigned b4off, fo;  // byte offsets of cell c-4 and d-face c-3 in the row
    int cpos;
    bool valid, own1, own2;
  };
  constexpr unsigned z = sizeof(T);
  auto load = [&](int it) {
    if (rc.moved) {
      row_offsets<T>(g, rc.y, rc.z, rc.base, ro);  // y, z face rows
      own1 = rc.z < g.n[2];
      own2 = rc.y < g.n[1];
      if (NU) {
        const int n1 = g.n[1], n2 = g.n[2], b1 = g.bc[1], b2 = g.bc[2], y = rc.y, zc = rc.z;
        rnr = field_row_nu(width_at(a.wid[1], y - 1, n1, b1), width_at(a.wid[1], y, n1, b1),
                           width_at(a.wid[1], y + 1, n1, b1), width_at(a.wid[2], zc - 1, n2, b2),
                           width_at(a.wid[2], zc, n2, b2), width_at(a.wid[2], zc + 1, n2, b2));
      }
    }
    In in;
    in.valid = lane >= HALO && it * STEP + lane - HALO < npos;
    in.cpos = min(max(rc.cp, 0), L - 1) - 4;  // cell index along x (-4 .. nx+3), clamped as in the fluid sweep
    in.own1 = own1;
    in.own2 = own2;
    const unsigned xb = (unsigned)map_cell_near(in.cpos, nx, g.bc[0]) * z;
    FieldLane l;
    l.cc = ro.ownc + xb;
    l.c1m = l.cc + ro.c1m;
    l.c1p = l.cc + ro.c1p;
    l.c2m = l.cc + ro.c2m;
    l.c2p = l.cc + ro.c2p;
    l.fA = ro.base + xb;
    l.fB = l.fA + ro.f1p;
    l.fC = l.fA;
    l.fD = l.fA + ro.f2p;
    in.f = field_load<T>(a.md, a.rho, a.bt[0], a.bt[1], l);
    in.b4off = ro.base + (unsigned)map_cell_near(in.cpos - 4, nx, g.bc[0]) * z;
    in.f.b4a = ld(a.bt[0], in.b4off);
    in.f.b4c = ld(a.bt[1], in.b4off);
    // d-face c-3 (mapped, in range for every lane); b_d there is rewritten by
    // this position's constraint update, so it is loaded with the inputs
    in.fo = ro.base + (unsigned)map_face_near(in.cpos - 3, nx, g.bc[0]) * z;
    in.f.bd3 = ld(a.bd, in.fo);
    if (NU) {
      in.rn = rnr;
#pragma unroll
      for (int j = 0; j < 4; ++j) in.w[j] = width_at(a.wid[0], in.cpos - 5 + j, nx, g.bc[0]);
    }
    rc.advance(L, rows, ry, st1, up, STEP);
    return in;
  };
  auto compute = [&](const In& in, const RowHist<T>* hi, RowHist<T>* ho) {
    T bn1, bn2, dbd;
    const FieldPosNU<T> pn = NU ? field_pos_nu(in.w, k.dt) : FieldPosNU<T>{};
    field_compute<T, LIM, LaneShift, true, NU>(in.f, k, in.rn, pn, hi, ho, bn1, bn2, dbd);
    const int cb = in.cpos - 4;
    if (in.valid && cb >= 0 && cb < nx) {
      if (in.own1) st(a.bto[0], in.b4off, bn1);
      if (in.own2) st(a.bto[1], in.b4off, bn2);
    }
    const int fd = in.cpos - 3;
    if (in.valid && in.own1 && in.own2 && fd >= 0 && (fd < nx || (outx && fd == nx)))
      st(a.bdo, in.fo, in.f.bd3 + dbd);
  };
  In cur = load(0);
  for (int it = 0; it < nit; it += 2) {
    const In nxt = load(it + 1);
    compute(cur, hA, hB);
    cur = load(it + 2);
    compute(nxt, hB, hA);
  }
}

// ------------------------------------------------------------ B_x, two positions per lane
// The x field sweep with lane l holding stream positions 2l and 2l+1 of a
// 128-position window.  The pipeline runs stage by stage over both: the
// value one position back is the lane's own register for 2l+1 and the
// neighbour lane's (one DPP shift) for 2l, so each history value costs one
// shift per two cells.  As in the one-position kernel, the first lanes of a
// window recompute the positions the previous one ended on (8 positions, 4
// lanes), so nothing crosses windows.
template <typename T>
__device__ __forceinline__ void prev2(const T (&x)[2], T (&p)[2]) {
  p[1] = x[0];
  p[0] = lane_shr(x[1]);
}

// row_position for both positions of the lane.
template <typename T, int LIM, bool NEED_BN>
__device__ __forceinline__ void row_position2(const T (&w0)[2], const T (&bb)[2], const T (&b4)[2], T k_half,
                                              T k_full, T (&bn)[2], T (&P2c)[2]) {
  T w1[2], w2[2], vbc[2], b1[2], fc[2], vb1[2], V[2], f2[2], P1[2], p1[2], b2[2], bp[2], fp2[2];
  T vb2[2], vb3[2], fp3[2], fp4[2], fp5[2];
  prev2(w0, w1);
  prev2(w1, w2);
#pragma unroll
  for (int j = 0; j < 2; ++j) vbc[j] = T(0.25) * ((w2[j] + w0[j]) + T(2) * w1[j]);  // v-bar of c-1 (as above)
  prev2(bb, b1);
#pragma unroll
  for (int j = 0; j < 2; ++j) fc[j] = vbc[j] * b1[j];
  prev2(vbc, vb1);
#pragma unroll
  for (int j = 0; j < 2; ++j) V[j] = T(0.5) * (vb1[j] + vbc[j]);
  prev2(fc, f2);
#pragma unroll
  for (int j = 0; j < 2; ++j) P1[j] = V[j] > T(0) ? f2[j] : fc[j];
  prev2(P1, p1);
  prev2(b1, b2);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    bp[j] = b2[j] - k_half * (P1[j] - p1[j]);
    fp2[j] = vb1[j] * bp[j];
  }
  prev2(vb1, vb2);
  prev2(vb2, vb3);
  prev2(fp2, fp3);
  prev2(fp3, fp4);
  prev2(fp4, fp5);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const T V7 = T(0.5) * (vb3[j] + vb2[j]);
    const T up = fp4[j] + T(0.5) * limit<T, LIM>(fp4[j] - fp5[j], fp3[j] - fp4[j]);
    const T dn = fp3[j] - T(0.5) * limit<T, LIM>(fp3[j] - fp4[j], fp2[j] - fp3[j]);
    P2c[j] = V7 > T(0) ? up : dn;
  }
  if (NEED_BN) {
    T P2[2];
    prev2(P2c, P2);
#pragma unroll
    for (int j = 0; j < 2; ++j) bn[j] = b4[j] - k_full * (P2c[j] - P2[j]);
  }
}

template <typename T, int LIM>
__global__ __launch_bounds__(256) void field_lanes2_kernel(FieldLaunch<T> FL) {
  constexpr int D = 0;
  const BoxDesc* d;
  int lw;
  if (!work_item<K_FIELD_X>(FL.wl, d, lw)) return;
  const FieldArgs<T> a = field_view<T, K_FIELD_X>(FL, *d);
  const Geo& g = a.g;
  const int nx = g.n[0];
  const bool outx = g.bc[0] == 1;
  const int L = nx + 8;
  const int ry = g.n[1] + g.bc[1];
  const int rz = g.n[2] + g.bc[2];
  const long long nrows = (long long)ry * rz;
  const int lane = threadIdx.x & 63;
  const long long r0 = (long long)lw * a.rows_per_wave;
  if (r0 >= nrows) return;  // whole wave exits together
  const int rows = (int)min((long long)a.rows_per_wave, nrows - r0);
  const int npos = rows * L;
  constexpr int HALO = 8, STEP = 128 - HALO;  // positions
  const int nit = (npos + STEP - 1) / STEP;
  const FieldConsts<T> k = field_consts<T, D>(a);
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];  // arrays < 2^32 bytes
  const unsigned up = st2 - (unsigned)(ry - 1) * st1;
  RowCursor rc[2];
  RowOffsets ro[2];
  bool own1[2] = {false, false}, own2[2] = {false, false};
#pragma unroll
  for (int j = 0; j < 2; ++j) rc[j].init(2 * lane + j - HALO, L, (int)r0, rows, ry, st1, st2, up);
  constexpr unsigned z = sizeof(T);
  struct In {
    FieldIn<T> f;
    unsigned b4off, fo;
    int cpos;
    bool valid, own1, own2;
  };
  auto load1 = [&](int it, int j) {
    if (rc[j].moved) {
      row_offsets<T>(g, rc[j].y, rc[j].z, rc[j].base, ro[j]);
      own1[j] = rc[j].z < g.n[2];
      own2[j] = rc[j].y < g.n[1];
    }
    In in;
    in.valid = 2 * lane + j >= HALO && it * STEP + 2 * lane + j - HALO < npos;
    in.cpos = min(max(rc[j].cp, 0), L - 1) - 4;  // clamped as in the fluid sweep
    in.own1 = own1[j];
    in.own2 = own2[j];
    const unsigned xb = (unsigned)map_cell_near(in.cpos, nx, g.bc[0]) * z;
    FieldLane l;
    l.cc = ro[j].ownc + xb;
    l.c1m = l.cc + ro[j].c1m;
    l.c1p = l.cc + ro[j].c1p;
    l.c2m = l.cc + ro[j].c2m;
    l.c2p = l.cc + ro[j].c2p;
    l.fA = ro[j].base + xb;
    l.fB = l.fA + ro[j].f1p;
    l.fC = l.fA;
    l.fD = l.fA + ro[j].f2p;
    in.f = field_load<T>(a.md, a.rho, a.bt[0], a.bt[1], l);
    in.b4off = ro[j].base + (unsigned)map_cell_near(in.cpos - 4, nx, g.bc[0]) * z;
    in.f.b4a = ld(a.bt[0], in.b4off);
    in.f.b4c = ld(a.bt[1], in.b4off);
    in.fo = ro[j].base + (unsigned)map_face_near(in.cpos - 3, nx, g.bc[0]) * z;
    in.f.bd3 = ld(a.bd, in.fo);
    rc[j].advance(L, rows, ry, st1, up, STEP);
    return in;
  };
  auto compute = [&](const In (&in)[2]) {
    T wA[2], wB[2], wC[2], wD[2], bA[2], bB[2], bC[2], bD[2], b4a[2], b4c[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      T v[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) v[i] = in[j].f.md[i] * rcp(in[j].f.rho[i]);
      wA[j] = T(0.5) * (v[1] + v[0]);
      wB[j] = T(0.5) * (v[0] + v[2]);
      wC[j] = T(0.5) * (v[3] + v[0]);
      wD[j] = T(0.5) * (v[0] + v[4]);
      bA[j] = in[j].f.b[0];
      bB[j] = in[j].f.b[1];
      bC[j] = in[j].f.b[2];
      bD[j] = in[j].f.b[3];
      b4a[j] = in[j].f.b4a;
      b4c[j] = in[j].f.b4c;
    }
    T bn1[2], bn2[2], eA[2], eB[2], eC[2], eD[2], dummy[2];
    row_position2<T, LIM, true>(wA, bA, b4a, k.k_half, k.k_full, bn1, eA);
    row_position2<T, LIM, false>(wB, bB, b4a, k.k_half, k.k_full, dummy, eB);
    row_position2<T, LIM, true>(wC, bC, b4c, k.k_half, k.k_full, bn2, eC);
    row_position2<T, LIM, false>(wD, bD, b4c, k.k_half, k.k_full, dummy, eD);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      // Eq. (64), physical signs
      const T dbd = k.dt * ((eB[j] - eA[j]) * k.ih1 + (eD[j] - eC[j]) * k.ih2);
      const int cb = in[j].cpos - 4;
      if (in[j].valid && cb >= 0 && cb < nx) {
        if (in[j].own1) st(a.bto[0], in[j].b4off, bn1[j]);
        if (in[j].own2) st(a.bto[1], in[j].b4off, bn2[j]);
      }
      const int fd = in[j].cpos - 3;
      if (in[j].valid && in[j].own1 && in[j].own2 && fd >= 0 && (fd < nx || (outx && fd == nx)))
        st(a.bdo, in[j].fo, in[j].f.bd3 + dbd);
    }
  };
  for (int it = 0; it < nit; ++it) {
    In in[2];
    in[0] = load1(it, 0);
    in[1] = load1(it, 1);
    compute(in);
  }
}

// ------------------------------------------------------------ CFL + state check
template <typename T>
struct CheckLaunch {
  const T* u[5];
  const T* b[3];
  const T* wid[3];  // irregular meshes: every table box's cell widths per axis (at BoxDesc::woff), else null
  double gamma;
  WorkList wl;
  Scalars* sc;
};

// Eq. (14)-(15) on the stored state: the CFL speed of every cell (the same
// function, hence bitwise the same value, as the reduction fused into the
// last sweep of a step) and the state check (rho > 0, p > 0, every value
// finite).  A wave covers 64 * par consecutive cells of its box (x fastest);
// each lane steps its cell index by 64, never dividing inside the loop.
template <typename T>
__global__ __launch_bounds__(256) void check_cfl_kernel(CheckLaunch<T> L) {
  const BoxDesc* d;
  int lw;
  if (!work_item<K_CHECK>(L.wl, d, lw)) return;
  const Geo g = d->g;
  const long long off = d->off;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const long long ncell = (long long)n0 * n1 * n2;
  const long long c0 = (long long)lw * 64 * d->par[K_CHECK];
  const long long c1 = min(ncell, c0 + 64ll * d->par[K_CHECK]);
  const T* u[5];
  const T* b[3];
#pragma unroll
  for (int f = 0; f < 5; ++f) u[f] = L.u[f] + off;
#pragma unroll
  for (int f = 0; f < 3; ++f) b[f] = L.b[f] + off;
  const unsigned st1 = (unsigned)g.st[1], st2 = (unsigned)g.st[2];
  constexpr unsigned z4 = sizeof(T);
  long long c = c0 + (threadIdx.x & 63);
  int x = (int)(c % n0);
  const long long r = c / n0;
  int y = (int)(r % n1);
  int zz = (int)(r / n1);
  T smax[3] = {T(0), T(0), T(0)};
  double cnu = 0.0;                      // irregular mesh: per-cell speeds over widths
  const bool nu = L.wid[0] != nullptr;   // uniform across the launch
  const T* wx = nu ? L.wid[0] + d->woff[0] : nullptr;
  const T* wy = nu ? L.wid[1] + d->woff[1] : nullptr;
  const T* wz = nu ? L.wid[2] + d->woff[2] : nullptr;
  int bad = 0;
  for (; c < c1; c += 64) {
    const unsigned s = (unsigned)x + (unsigned)y * st1 + (unsigned)zz * st2;
    const unsigned o = s * z4;
    T uc[5], bc[3];
#pragma unroll
    for (int f = 0; f < 5; ++f) uc[f] = ld(u[f], o);
    const unsigned sx = (unsigned)(map_face_near(x + 1, n0, g.bc[0]) - x);
    const unsigned sy = (unsigned)(map_face_near(y + 1, n1, g.bc[1]) - y) * st1;
    const unsigned sz = (unsigned)(map_face_near(zz + 1, n2, g.bc[2]) - zz) * st2;
    bc[0] = T(0.5) * (ld(b[0], o) + ld(b[0], (s + sx) * z4));
    bc[1] = T(0.5) * (ld(b[1], o) + ld(b[1], (s + sy) * z4));
    bc[2] = T(0.5) * (ld(b[2], o) + ld(b[2], (s + sz) * z4));
    T sp[3];
    cell_cfl_speeds<T>(uc, bc, L.gamma, g, sp, bad);
    if (nu) {
      cnu = fmax(cnu, cfl_of_cell(sp, (double)wx[x], (double)wy[y], (double)wz[zz], g));
    } else {
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) smax[dd] = fmax(smax[dd], sp[dd]);
    }
    x += 64;
    while (x >= n0) {
      x -= n0;
      if (++y == n1) {
        y = 0;
        ++zz;
      }
    }
  }
  publish_cfl(nu ? cnu : cfl_of(smax, g), bad, L.sc + d->slot);
}

}  // namespace fish
