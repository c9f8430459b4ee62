// Instantiations of the sampling interpreter: double amplitudes, trace mode (forced outcomes and faults, probabilities, final vectors).
// (One translation unit per precision and mode, so that the build compiles
// them in parallel.)
#include "shot.h"

namespace clifft {

hipError_t launch_trace_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  return launch_g<double, true>(P, A, L, st);
}

}  // namespace clifft
