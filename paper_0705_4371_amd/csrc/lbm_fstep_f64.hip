// lbm_fstep_f64.hip -- instantiation of the f*_M time-step kernels (pull,
// moments, Newton solve, screen, collision; fallback) for double populations.
#include "lbm_step.hpp"

namespace lbm {

hipError_t launch_fstep_f64(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
  return pull ? fstep_p<double, true>(a, fa, start, s, ev0, ev1) : fstep_p<double, false>(a, fa, start, s, ev0, ev1);
}

int fstep_resident_f64(int start, bool pull, bool elbm) { return fstep_resident_p<double>(start, pull, elbm); }

}  // namespace lbm
