// Batched launch of many programs: the plain instantiation of the queue
// kernels (batch_kernel.h).
#include "batch_kernel.h"

namespace clifft {

hipError_t launch_batch(const BatchArgs& groups, int grid_groups, const BatchArgs& waves, int grid_waves,
                        const BatchArgs& lanes, int grid_lanes, size_t lds_bytes, bool fp64, hipStream_t st) {
  return launch_batch_impl<false>(groups, grid_groups, waves, grid_waves, lanes, grid_lanes, lds_bytes, fp64, st);
}

}  // namespace clifft
