// Stage-kernel and 1-D multi-step instantiations: double, 1-D, advection, N = 1..8.
#include "dg_multistep.hpp"
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f64_d1_adv(int N) { return pick_stage_n<double, 1, 0>(N); }
StageXFn stage_x_fn_f64_d1_adv(int N) { return pick_stage_x_n<double, 1, 0>(N); }
BatchFn batch_fn_f64_d1_adv(int N) { return pick_batch_n<double, 1, 0>(N); }
BatchXFn batch_x_fn_f64_d1_adv(int N) { return pick_batch_x_n<double, 1, 0>(N); }
MsFn ms_fn_f64_adv(int N) { return ms::pick_ms1<double, 0>(N); }
int ms_cap_f64_adv(int N) { return ms::cap1<double, 0>(N); }
}  // namespace dg
