// launch_fluid_x_f64.hip -- the FP64 fluid sweep L_x and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<double, 0>();
template void launch_fluid_sweep<double, 0>(const SweepSel&, const FluidLaunch<double>&, bool);
}  // namespace fish
