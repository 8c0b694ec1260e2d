// launch_defs.h -- definitions of the sweep launches (launch_api.h) and of
// the engine's sub-operators that build their arguments.  Included only by
// the launch_*.hip translation units, each of which instantiates one
// precision and one sweep kind, so that the kernels compile in parallel.
#pragma once

#include "launch.h"
#include "launch_api.h"
#include "sweeps.h"

namespace fish {

// ------------------------------------------------------------ fluid sweeps
template <typename T, int D, int GRAV, bool HSE, int LIM, bool NU>
void fluid_kernel(const FluidLaunch<T>& L, bool cfl, bool x_strided, hipStream_t stream) {
  if (L.wl.nwaves == 0) return;
  const dim3 grid(grid_for((long long)L.wl.nwaves * 64));
  if constexpr (D == 0) {
    if (x_strided && !cfl)
      hipLaunchKernelGGL((fluid_strided_kernel<T, 0, GRAV, HSE, LIM, NU>), grid, dim3(kBlock), 0, stream, L);
    else if (cfl)
      hipLaunchKernelGGL((fluid_lanes_kernel<T, GRAV, HSE, LIM, true, NU>), grid, dim3(kBlock), 0, stream, L);
    else
      hipLaunchKernelGGL((fluid_lanes_kernel<T, GRAV, HSE, LIM, false, NU>), grid, dim3(kBlock), 0, stream, L);
  } else {
    hipLaunchKernelGGL((fluid_strided_kernel<T, D, GRAV, HSE, LIM, NU>), grid, dim3(kBlock), 0, stream, L);
  }
}

template <typename T, int D, int GRAV, bool HSE, int LIM>
void fluid_mesh(const SweepSel& s, const FluidLaunch<T>& L, bool cfl) {
  if (s.nonuniform)
    fluid_kernel<T, D, GRAV, HSE, LIM, true>(L, cfl, s.x_strided, s.stream);
  else
    fluid_kernel<T, D, GRAV, HSE, LIM, false>(L, cfl, s.x_strided, s.stream);
}

template <typename T, int D, int LIM>
void fluid_gravity(const SweepSel& s, const FluidLaunch<T>& L, bool cfl) {
  if (!s.gravity)
    fluid_mesh<T, D, 0, false, LIM>(s, L, cfl);
  else if (s.gravity == 1)
    s.hse ? fluid_mesh<T, D, 1, true, LIM>(s, L, cfl) : fluid_mesh<T, D, 1, false, LIM>(s, L, cfl);
  else
    s.hse ? fluid_mesh<T, D, 2, true, LIM>(s, L, cfl) : fluid_mesh<T, D, 2, false, LIM>(s, L, cfl);
}

template <typename T, int D>
void launch_fluid_sweep(const SweepSel& s, const FluidLaunch<T>& L, bool cfl) {
  if (s.limiter == 0)
    fluid_gravity<T, D, 0>(s, L, cfl);
  else if (s.limiter == 1)
    fluid_gravity<T, D, 1>(s, L, cfl);
  else
    fluid_gravity<T, D, 2>(s, L, cfl);
}

// ------------------------------------------------------------ field sweeps
template <typename T, int D, int LIM, bool NU>
void field_kernel(const SweepSel& s, const FieldLaunch<T>& L) {
  if (L.wl.nwaves == 0) return;
  const dim3 grid(grid_for((long long)L.wl.nwaves * 64));
  if constexpr (D == 0) {
    if (s.lanes2 && !NU)  // two positions per lane: uniform meshes only
      hipLaunchKernelGGL((field_lanes2_kernel<T, LIM>), grid, dim3(kBlock), 0, s.stream, L);
    else
      hipLaunchKernelGGL((field_lanes_kernel<T, LIM, NU>), grid, dim3(kBlock), 0, s.stream, L);
  } else {
    hipLaunchKernelGGL((field_strided_kernel<T, D, LIM, NU>), grid, dim3(kBlock), 0, s.stream, L);
  }
}

template <typename T, int D>
void launch_field_sweep(const SweepSel& s, const FieldLaunch<T>& L) {
  // the limiter switch (limiter 2) is a fluid choice: the field advection keeps van Leer
  if (s.limiter == 0)
    s.nonuniform ? field_kernel<T, D, 0, true>(s, L) : field_kernel<T, D, 0, false>(s, L);
  else
    s.nonuniform ? field_kernel<T, D, 1, true>(s, L) : field_kernel<T, D, 1, false>(s, L);
}

// ------------------------------------------------------------ the engine's sub-operators
inline SweepSel Engine::sweep_sel() const {
  SweepSel s;
  s.limiter = cfg.limiter;
  s.gravity = cfg.gravity;
  s.hse = cfg.hse;
  s.nonuniform = nonuniform;
  s.lanes2 = tuning.groups[K_FIELD_X] != 0;
  s.x_strided = tuning.groups[K_FLUID_X] != 0;
  s.stream = cfg.stream;
  return s;
}

template <typename T, int D>
int Engine::fluid_dispatch() {
  // y or z with one cell in every box: the identity, left out (x never is:
  // its last sweep of a step reduces the CFL speed)
  if (D != 0 && flat[D]) return 0;
  FluidLaunch<T> L;
  for (int k = 0; k < 5; ++k) {
    L.u[k] = (const T*)pool[cur[k]][k].ptr;
    L.uo[k] = (T*)pool[1 - cur[k]][k].ptr;
  }
  for (int k = 0; k < 3; ++k) L.b[k] = (const T*)pool[cur[5 + k]][5 + k].ptr;
  L.phi = (const T*)phi.ptr;
  for (int k = 0; k < 3; ++k) L.wid[k] = nonuniform ? (const T*)wid[k].ptr : nullptr;
  L.gamma = cfg.gamma;
  L.alpha = cfg.alpha;
  L.wl = make_wl(this, K_FLUID_X + D);
  L.sc = (Scalars*)scal.ptr;
  {
    TimedLaunch tl(this, 1);
    launch_fluid_sweep<T, D>(sweep_sel(), L, D == 0 && last_fluid_cfl);
  }
  for (int k = 0; k < 5; ++k) cur[k] = 1 - cur[k];
  return launch_check();
}

template <typename T, int D>
int Engine::field_sweep() {
  const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  FieldLaunch<T> L;
  L.rho = (const T*)pool[cur[0]][0].ptr;
  L.md = (const T*)pool[cur[1 + D]][1 + D].ptr;
  L.bt[0] = (const T*)pool[cur[5 + t1]][5 + t1].ptr;
  L.bt[1] = (const T*)pool[cur[5 + t2]][5 + t2].ptr;
  L.bd = (const T*)pool[cur[5 + D]][5 + D].ptr;
  L.bto[0] = (T*)pool[1 - cur[5 + t1]][5 + t1].ptr;
  L.bto[1] = (T*)pool[1 - cur[5 + t2]][5 + t2].ptr;
  L.bdo = (T*)pool[1 - cur[5 + D]][5 + D].ptr;
  for (int k = 0; k < 3; ++k) L.wid[k] = nonuniform ? (const T*)wid[k].ptr : nullptr;
  L.wl = make_wl(this, K_FIELD_X + D);
  L.sc = (Scalars*)scal.ptr;
  if (L.wl.nwaves > 0) {
    TimedLaunch tl(this, 2);
    launch_field_sweep<T, D>(sweep_sel(), L);
  }
  for (int f = 5; f < 8; ++f) cur[f] = 1 - cur[f];
  return launch_check();
}

}  // namespace fish
