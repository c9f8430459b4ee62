// Vector-only stream of the split form, FP32 amplitudes (the interpreter of
// shot.h without Pauli frames: the frame bits it needs come precomputed).
#include "shot.h"

namespace clifft {

hipError_t launch_vsample_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  return launch_vonly<float>(P, A, L, st);
}

}  // namespace clifft
