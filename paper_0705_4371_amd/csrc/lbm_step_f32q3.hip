// lbm_step_f32q3.hip -- instantiation of the time-step kernels (step, ranking,
// selection, reset) for float populations on D1Q3.
#include "lbm_step.hpp"

namespace lbm {

hipError_t launch_step_f32q3(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return step_q<float, 3>(a, pull, s, ev0, ev1);
}

}  // namespace lbm
