// lbm_step_f64q9.hip -- instantiation of the time-step kernels (step, ranking,
// selection, reset) for double populations on D2Q9.
#include "lbm_step.hpp"

namespace lbm {

hipError_t launch_step_f64q9(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  return step_q<double, 9>(a, pull, s, ev0, ev1);
}

}  // namespace lbm
