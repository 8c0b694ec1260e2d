// launch_field_f64.hip -- the FP64 field sweeps B_x, B_y, B_z and their kernel variants (launch_defs.h).
#include "launch_defs.h"

namespace fish {
template int Engine::field_sweep<double, 0>();
template void launch_field_sweep<double, 0>(const SweepSel&, const FieldLaunch<double>&);
template int Engine::field_sweep<double, 1>();
template void launch_field_sweep<double, 1>(const SweepSel&, const FieldLaunch<double>&);
template int Engine::field_sweep<double, 2>();
template void launch_field_sweep<double, 2>(const SweepSel&, const FieldLaunch<double>&);
}  // namespace fish
