// lbm_fstep_f32.hip -- instantiation of the f*_M time-step kernels (pull,
// moments, Newton solve, screen, collision; fallback) for float populations.
#include "lbm_step.hpp"

namespace lbm {

hipError_t launch_fstep_f32(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
  return pull ? fstep_p<float, true>(a, fa, start, s, ev0, ev1) : fstep_p<float, false>(a, fa, start, s, ev0, ev1);
}

int fstep_resident_f32(int start, bool pull, bool elbm) { return fstep_resident_p<float>(start, pull, elbm); }

}  // namespace lbm
