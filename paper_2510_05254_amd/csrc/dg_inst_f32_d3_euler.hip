// Stage-kernel instantiations: float, 3-D, isothermal Euler, N = 1..8.
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f32_d3_euler(int N) { return pick_stage_n<float, 3, 1>(N); }
StageXFn stage_x_fn_f32_d3_euler(int N) { return pick_stage_x_n<float, 3, 1>(N); }
BatchFn batch_fn_f32_d3_euler(int N) { return pick_batch_n<float, 3, 1>(N); }
BatchXFn batch_x_fn_f32_d3_euler(int N) { return pick_batch_x_n<float, 3, 1>(N); }
}  // namespace dg
