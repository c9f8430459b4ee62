// Instantiations of the sampling interpreter with post-selection and
// stratified fault sampling compiled in: float amplitudes.
#include "shot.h"

namespace clifft {

hipError_t launch_sample_ext_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  return launch_g<float, false, true>(P, A, L, st);
}

}  // namespace clifft
