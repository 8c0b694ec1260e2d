// launch_fluid_y_f32.hip -- the FP32 fluid sweep L_y and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<float, 1>();
template void launch_fluid_sweep<float, 1>(const SweepSel&, const FluidLaunch<float>&, bool);
}  // namespace fish
