// launch_fluid_y_f64.hip -- the FP64 fluid sweep L_y and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<double, 1>();
template void launch_fluid_sweep<double, 1>(const SweepSel&, const FluidLaunch<double>&, bool);
}  // namespace fish
