// Instantiations of the sampling interpreter: float amplitudes.
// (One translation unit per precision and mode, so that the build compiles
// them in parallel.)
#include "shot.h"

namespace clifft {

hipError_t launch_sample_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  return launch_g<float, false>(P, A, L, st);
}

}  // namespace clifft
