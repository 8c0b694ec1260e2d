// launch_fluid_x_f32.hip -- the FP32 fluid sweep L_x and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<float, 0>();
template void launch_fluid_sweep<float, 0>(const SweepSel&, const FluidLaunch<float>&, bool);
}  // namespace fish
