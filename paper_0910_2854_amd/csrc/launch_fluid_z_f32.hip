// launch_fluid_z_f32.hip -- the FP32 fluid sweep L_z and its kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::fluid_dispatch<float, 2>();
template void launch_fluid_sweep<float, 2>(const SweepSel&, const FluidLaunch<float>&, bool);
}  // namespace fish
