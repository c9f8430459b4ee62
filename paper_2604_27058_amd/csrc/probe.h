// Rate probes (measurement support, not part of sampling).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace clifft {

// kind 0 copies n bytes (a multiple of 16) from src to dst; kind 1 runs n
// iterations of 16 VALU instructions per thread and writes one word per
// thread to dst; kind 2 reads n bytes of src and writes one 16-byte XOR per
// thread to dst.  Workgroups of 256 threads.
hipError_t launch_probe(int kind, void* dst, const void* src, uint64_t n, int grid, hipStream_t stream);

}  // namespace clifft
