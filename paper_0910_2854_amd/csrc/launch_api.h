// launch_api.h -- the launches of the sweep kernels as free functions: the
// kernel is chosen from the scheme settings (precision and direction by
// template, gravity form, HSE, limiter and mesh at run time) and launched on
// the given stream.  The engine and the allocation-free step both launch
// through these; their definitions are instantiated in the launch_*.hip
// translation units, one precision and sweep kind each.
#pragma once

#include <hip/hip_runtime.h>

#include "sweeps.h"

namespace fish {

struct SweepSel {
  int limiter = 1;         // 0 minmod, 1 van Leer, 2 the Mach switch (fluid only)
  int gravity = 0;         // 0 none, 1 unsplit, 2 split
  int hse = 0;
  bool nonuniform = false; // per-cell widths (the launch carries them)
  bool lanes2 = false;     // x field sweep: two stream positions per lane (uniform meshes)
  bool x_strided = false;  // x fluid sweep without the CFL reduction: the strided policy, lanes along y
  hipStream_t stream = nullptr;
};

// L_D over the list in L.wl; cfl: the x sweep also reduces the CFL speed of
// the state it writes (the last sub-operator of a double step).
template <typename T, int D>
void launch_fluid_sweep(const SweepSel& s, const FluidLaunch<T>& L, bool cfl);

// B_D over the list in L.wl.
template <typename T, int D>
void launch_field_sweep(const SweepSel& s, const FieldLaunch<T>& L);

// The CFL reduction and state check over the list in L.wl (engine.hip).
template <typename T>
void launch_check(const CheckLaunch<T>& L, hipStream_t stream);

// The start of a double step over the first nb boxes of a table
// (engine.hip): the step size (dt > 0 as given, else the CFL step of Eq. 14
// from the boxes' CFL maxima) with its factors, t += 2 dt, and the CFL
// maximum cleared for the step's last sweep.
void launch_begin_step(const BoxDesc* boxes, int nb, Scalars* sc, double dt, hipStream_t stream);

// The work shape of a box alone in its table at the default tuning (as the
// engine plans it): per kind the parameter of BoxDesc::par, the segments per
// pencil of BoxDesc::nseg and the waves of its work list.
void plan_single_box(const int n[3], const int bc[3], int par[K_NUM], int nseg[K_NUM], long long waves[K_NUM]);

}  // namespace fish
