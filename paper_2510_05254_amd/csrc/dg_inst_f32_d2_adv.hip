// Stage-kernel instantiations: float, 2-D, advection, N = 1..8.
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f32_d2_adv(int N) { return pick_stage_n<float, 2, 0>(N); }
StageXFn stage_x_fn_f32_d2_adv(int N) { return pick_stage_x_n<float, 2, 0>(N); }
BatchFn batch_fn_f32_d2_adv(int N) { return pick_batch_n<float, 2, 0>(N); }
BatchXFn batch_x_fn_f32_d2_adv(int N) { return pick_batch_x_n<float, 2, 0>(N); }
}  // namespace dg
