// Step kernels instantiated for the SRT collision (one translation
// unit per operator, so that they compile in parallel).
#include "lbm_step.h"

namespace lbm {
hipError_t launch_step_srt(const StepLaunch &L, hipStream_t s) { return launch_step_coll<0>(L, s); }
}  // namespace lbm
