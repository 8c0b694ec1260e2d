// step_kernels.h -- the small kernels of the engine: per-box step scalars
// (CFL step, time, status), the fixed-order FP64 diagnostics and the
// self-tests of the lane shift and of the FP64 reciprocal and square root.
// Included by engine.hip only.
#pragma once

#include "sweeps.h"

namespace fish {

// The step size of every sub-operator and the factors the sweeps take from
// it, dt / (2 h_d) and dt / h_d per axis (evaluated once per step, not in
// every wave of every sweep).
__device__ __forceinline__ void set_step(Scalars* s, const Geo& g, double dt) {
  s->dt = dt;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    s->kh[d] = dt / (2.0 * g.h[d]);
    s->kf[d] = dt / g.h[d];
  }
}

// Per-box step scalars; one thread per box of the table.
__global__ void reset_cmax_kernel(const BoxDesc* boxes, int nb, Scalars* sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) sc[boxes[i].slot].cmax_bits = 0ull;
}

// dt = k / cmax (Eq. 14); a bad reduction marks the state and stops the box.
__global__ void finalize_dt_kernel(const BoxDesc* boxes, int nb, Scalars* sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  Scalars* s = sc + boxes[i].slot;
  const double cmax = __longlong_as_double((long long)s->cmax_bits);
  if (!(cmax > 0.0) || !isfinite(cmax) || s->status) {
    s->status |= 1;
    set_step(s, boxes[i].g, 0.0);
    return;
  }
  double dt = boxes[i].cfl / cmax;
  if (s->has_end) {
    // the double step advances 2 dt: no further than t_end (a step of
    // (t_end - t)/2 lands on t_end exactly), none once it is reached
    const double rest = s->t_end - s->t;
    dt = rest > 0.0 ? fmin(dt, 0.5 * rest) : 0.0;
  }
  set_step(s, boxes[i].g, dt);
}

// The start of a double step, one thread per box: the step size of every
// sub-operator (dt > 0 as given, else k / C from the CFL speed of the current
// state, Eq. 14, clamped to an end time, as finalize_dt_kernel), the time the
// step reaches (t + 2 dt, Eqs. 12-13) and the count of steps taken with
// dt > 0, and the CFL maximum cleared for the reduction fused into the step's
// last sweep (no other sweep of the step touches it).
__global__ void begin_step_kernel(const BoxDesc* boxes, int nb, Scalars* sc, double dt_given) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  Scalars* s = sc + boxes[i].slot;
  if (dt_given > 0.0) {
    set_step(s, boxes[i].g, dt_given);
  } else {
    const double cmax = __longlong_as_double((long long)s->cmax_bits);
    double dt = 0.0;
    if (!(cmax > 0.0) || !isfinite(cmax) || s->status) {
      s->status |= 1;
    } else {
      dt = boxes[i].cfl / cmax;
      if (s->has_end) {
        const double rest = s->t_end - s->t;
        dt = rest > 0.0 ? fmin(dt, 0.5 * rest) : 0.0;
      }
    }
    set_step(s, boxes[i].g, dt);
  }
  if (s->dt > 0.0) {
    s->t += 2.0 * s->dt;
    s->taken += 1;
  }
  s->cmax_bits = 0ull;
}

// A given step size for every box of the table.
__global__ void set_dt_kernel(const BoxDesc* boxes, int nb, Scalars* sc, double dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) set_step(sc + boxes[i].slot, boxes[i].g, dt);
}
__global__ void set_end_kernel(Scalars* sc, double t_end, int on) {
  sc->t_end = t_end;
  sc->has_end = on;
}
__global__ void set_scalars_kernel(Scalars* sc, double t, int status) {
  sc->t = t;
  sc->status = status;
  sc->cmax_bits = 0ull;
  sc->dt = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) sc->kh[d] = sc->kf[d] = 0.0;
  sc->t_end = 0.0;
  sc->has_end = 0;
  sc->taken = 0;
}

// ------------------------------------------------------------ diagnostics
template <typename T>
struct DiagArgs {
  const T* u[5];
  const T* b[3];
  const T* wid[3];   // irregular mesh: cell widths per axis (all three set), else null
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
    // cell widths; on a uniform mesh the volume and face areas are applied
    // once at the end, on an irregular one each cell and face carries its own
    // (Sect. 2.5), and the final factors are 1
    const bool nu = a.wid[0] != nullptr;
    const double hx = nu ? (double)a.wid[0][i] : g.h[0];
    const double hy = nu ? (double)a.wid[1][j] : g.h[1];
    const double hz = nu ? (double)a.wid[2][k] : g.h[2];
    const double cw = nu ? hx * hy * hz : 1.0;
    const double ax = nu ? hy * hz : 1.0, ay = nu ? hx * hz : 1.0, az = nu ? hx * hy : 1.0;
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[f] += (double)a.u[f][s] * cw;
    const long long sx = s + (long long)(map_face(i + 1, g.n[0], g.bc[0]) - i) * g.st[0];
    const long long sy = s + (long long)(map_face(j + 1, g.n[1], g.bc[1]) - j) * g.st[1];
    const long long sz = s + (long long)(map_face(k + 1, g.n[2], g.bc[2]) - k) * g.st[2];
    // Eq. (62), each difference over its cell's width
    const double div = ((double)a.b[0][sx] - (double)a.b[0][s]) / hx +
                       ((double)a.b[1][sy] - (double)a.b[1][s]) / hy +
                       ((double)a.b[2][sz] - (double)a.b[2][s]) / hz;
    acc[8] = fmax(acc[8], fabs(div));
    // face sums over real faces: the low face of every cell, plus face n on
    // outflow axes (owned by the last cell)
    const double bx = (double)a.b[0][s], by = (double)a.b[1][s], bz = (double)a.b[2][s];
    acc[5] += bx * ax;
    acc[6] += by * ay;
    acc[7] += bz * az;
    acc[9] = fmax(acc[9], fmax(fabs(bx), fmax(fabs(by), fabs(bz))));
    if (g.bc[0] == 1 && i == g.n[0] - 1) {
      const double v = (double)a.b[0][sx];
      acc[5] += v * ax;
      acc[9] = fmax(acc[9], fabs(v));
    }
    if (g.bc[1] == 1 && j == g.n[1] - 1) {
      const double v = (double)a.b[1][sy];
      acc[6] += v * ay;
      acc[9] = fmax(acc[9], fabs(v));
    }
    if (g.bc[2] == 1 && k == g.n[2] - 1) {
      const double v = (double)a.b[2][sz];
      acc[7] += v * az;
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

// Self-test of the lane-shift primitive: out[64*it + lane] = the value of
// lane - 1 of (100*it + lane), 0 in lane 0, over two iterations (128 entries).
__global__ void lane_shift_selftest_kernel(float* out) {
  const int lane = threadIdx.x & 63;
  for (int it = 0; it < 2; ++it) {
    const float cur = (float)(100 * it + lane);
    out[64 * it + lane] = lane_shr(cur);
  }
}

// Self-test of the FP64 reciprocal and square root the sweeps use:
// r[i] = rcp(x[i]), s[i] = fsqrt(x[i]) for i < n.
__global__ void math_selftest_kernel(const double* x, double* r, double* s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    r[i] = rcp(x[i]);
    s[i] = fsqrt(x[i]);
  }
}

}  // namespace fish
