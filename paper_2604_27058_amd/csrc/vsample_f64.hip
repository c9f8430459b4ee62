// Vector-only stream of the split form, FP64 amplitudes (the interpreter of
// shot.h without Pauli frames: the frame bits it needs come precomputed).
#include "shot.h"

namespace clifft {

hipError_t launch_vsample_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  return launch_vonly<double>(P, A, L, st);
}

}  // namespace clifft
