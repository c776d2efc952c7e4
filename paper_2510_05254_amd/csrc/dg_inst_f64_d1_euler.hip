// Stage-kernel and 1-D multi-step instantiations: double, 1-D, isothermal Euler, N = 1..8.
#include "dg_multistep.hpp"
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f64_d1_euler(int N) { return pick_stage_n<double, 1, 1>(N); }
StageXFn stage_x_fn_f64_d1_euler(int N) { return pick_stage_x_n<double, 1, 1>(N); }
BatchFn batch_fn_f64_d1_euler(int N) { return pick_batch_n<double, 1, 1>(N); }
BatchXFn batch_x_fn_f64_d1_euler(int N) { return pick_batch_x_n<double, 1, 1>(N); }
MsFn ms_fn_f64_euler(int N) { return ms::pick_ms1<double, 1>(N); }
int ms_cap_f64_euler(int N) { return ms::cap1<double, 1>(N); }
}  // namespace dg
