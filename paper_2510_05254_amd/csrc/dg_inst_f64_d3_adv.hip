// Stage-kernel instantiations: double, 3-D, advection, N = 1..8.
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f64_d3_adv(int N) { return pick_stage_n<double, 3, 0>(N); }
StageXFn stage_x_fn_f64_d3_adv(int N) { return pick_stage_x_n<double, 3, 0>(N); }
BatchFn batch_fn_f64_d3_adv(int N) { return pick_batch_n<double, 3, 0>(N); }
BatchXFn batch_x_fn_f64_d3_adv(int N) { return pick_batch_x_n<double, 3, 0>(N); }
}  // namespace dg
