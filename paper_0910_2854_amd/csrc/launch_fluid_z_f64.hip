// launch_fluid_z_f64.hip -- the FP64 fluid sweep L_z and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<double, 2>();
template void launch_fluid_sweep<double, 2>(const SweepSel&, const FluidLaunch<double>&, bool);
}  // namespace fish
