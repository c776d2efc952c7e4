// Stage-kernel instantiations: double, 1-D, advection, N = 1..8.
#include "dg_stage.hpp"

namespace dg {
StageFn stage_fn_f64_d1_adv(int N) { return pick_stage_n<double, 1, 0>(N); }
BatchFn batch_fn_f64_d1_adv(int N) { return pick_batch_n<double, 1, 0>(N); }
}  // namespace dg
