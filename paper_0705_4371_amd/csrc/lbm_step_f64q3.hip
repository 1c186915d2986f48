// lbm_step_f64q3.hip -- instantiation of the time-step kernels (step, ranking,
// selection, reset) for double populations on D1Q3.
#include "lbm_step.hpp"

namespace lbm {

hipError_t launch_step_f64q3(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return step_q<double, 3>(a, pull, s, ev0, ev1);
}

}  // namespace lbm
