// launch_field_f32.hip -- the FP32 field sweeps B_x, B_y, B_z and their kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::field_sweep<float, 0>();
template void launch_field_sweep<float, 0>(const SweepSel&, const FieldLaunch<float>&);
template int Engine::field_sweep<float, 1>();
template void launch_field_sweep<float, 1>(const SweepSel&, const FieldLaunch<float>&);
template int Engine::field_sweep<float, 2>();
template void launch_field_sweep<float, 2>(const SweepSel&, const FieldLaunch<float>&);
}  // namespace fish
