// launch_defs.h -- the sweep launches of the engine (kernel selection by
// precision, direction, gravity form, HSE, limiter and mesh).  Included only
// by the launch_*.hip translation units, each of which instantiates one
// precision and one sweep kind, so that the kernels compile in parallel.
#pragma once

#include "launch.h"
#include "sweeps.h"

namespace fish {

// ------------------------------------------------------------ sub-operators
template <typename T, int D, int GRAV, bool HSE, int LIM>
void Engine::launch_fluid_mesh() {
  if (nonuniform)
    launch_fluid<T, D, GRAV, HSE, LIM, true>();
  else
    launch_fluid<T, D, GRAV, HSE, LIM, false>();
}

template <typename T, int D, int GRAV, bool HSE, int LIM, bool NU>
void Engine::launch_fluid() {
  FluidLaunch<T> L;
  for (int k = 0; k < 5; ++k) {
    L.u[k] = (const T*)pool[cur[k]][k].ptr;
    L.uo[k] = (T*)pool[1 - cur[k]][k].ptr;
  }
  for (int k = 0; k < 3; ++k) L.b[k] = (const T*)pool[cur[5 + k]][5 + k].ptr;
  L.phi = (const T*)phi.ptr;
  for (int k = 0; k < 3; ++k) L.wid[k] = NU ? (const T*)wid[k].ptr : nullptr;
  L.gamma = cfg.gamma;
  L.alpha = cfg.alpha;
  L.wl = make_wl(this, K_FLUID_X + D);
  L.sc = (Scalars*)scal.ptr;
  if (L.wl.nwaves == 0) return;
  const dim3 grid(grid_for((long long)L.wl.nwaves * 64));
  TimedLaunch tl(this, 1);
  if constexpr (D == 0) {
    if (last_fluid_cfl)
      hipLaunchKernelGGL((fluid_lanes_kernel<T, GRAV, HSE, LIM, true, NU>), grid, dim3(kBlock), 0, cfg.stream, L);
    else
      hipLaunchKernelGGL((fluid_lanes_kernel<T, GRAV, HSE, LIM, false, NU>), grid, dim3(kBlock), 0, cfg.stream, L);
  } else {
    constexpr int DD = D;
    hipLaunchKernelGGL((fluid_strided_kernel<T, DD, GRAV, HSE, LIM, NU>), grid, dim3(kBlock), 0, cfg.stream, L);
  }
}

template <typename T, int D, int LIM>
void Engine::fluid_dispatch_lim() {
  if (!cfg.gravity)
    launch_fluid_mesh<T, D, 0, false, LIM>();
  else if (cfg.gravity == 1)
    cfg.hse ? launch_fluid_mesh<T, D, 1, true, LIM>() : launch_fluid_mesh<T, D, 1, false, LIM>();
  else
    cfg.hse ? launch_fluid_mesh<T, D, 2, true, LIM>() : launch_fluid_mesh<T, D, 2, false, LIM>();
}

template <typename T, int D>
int Engine::fluid_dispatch() {
  if (cfg.limiter == 0)
    fluid_dispatch_lim<T, D, 0>();
  else if (cfg.limiter == 1)
    fluid_dispatch_lim<T, D, 1>();
  else
    fluid_dispatch_lim<T, D, 2>();
  for (int k = 0; k < 5; ++k) cur[k] = 1 - cur[k];
  return launch_check();
}

template <typename T, int D, int LIM>
int Engine::field_sweep_lim() {
  if (nonuniform)
    launch_field<T, D, LIM, true>();
  else
    launch_field<T, D, LIM, false>();
  for (int f = 5; f < 8; ++f) cur[f] = 1 - cur[f];
  return launch_check();
}

template <typename T, int D, int LIM, bool NU>
void Engine::launch_field() {
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
  for (int k = 0; k < 3; ++k) L.wid[k] = NU ? (const T*)wid[k].ptr : nullptr;
  L.wl = make_wl(this, K_FIELD_X + D);
  L.sc = (Scalars*)scal.ptr;
  if (L.wl.nwaves > 0) {
    const dim3 grid(grid_for((long long)L.wl.nwaves * 64));
    TimedLaunch tl(this, 2);
    if constexpr (D == 0) {
      if (tuning.groups[K_FIELD_X] && !NU)  // two positions per lane: uniform meshes only
        hipLaunchKernelGGL((field_lanes2_kernel<T, LIM>), grid, dim3(kBlock), 0, cfg.stream, L);
      else
        hipLaunchKernelGGL((field_lanes_kernel<T, LIM, NU>), grid, dim3(kBlock), 0, cfg.stream, L);
    } else {
      constexpr int DD = D;
      hipLaunchKernelGGL((field_strided_kernel<T, DD, LIM, NU>), grid, dim3(kBlock), 0, cfg.stream, L);
    }
  }
}

template <typename T, int D>
int Engine::field_sweep() {
  // the limiter switch (limiter 2) is a fluid choice: the field advection keeps van Leer
  return cfg.limiter == 0 ? field_sweep_lim<T, D, 0>() : field_sweep_lim<T, D, 1>();
}

}  // namespace fish
