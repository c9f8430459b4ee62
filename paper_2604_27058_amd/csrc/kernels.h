// Launch interface of the sampling kernels (device side of the runtime).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "program.h"

namespace clifft {

struct KArgs {
  uint64_t shots, seed, offset;
  uint64_t* meas;  // [nrec][ceil(shots/64)] or null
  uint64_t* det;   // [ndet][ceil(shots/64)] or null
  uint64_t* obs;   // [nobs][ceil(shots/64)] or null
  void* workspace; // global active vectors (HBM tier) or null
  // forced / trace mode only
  const uint32_t* forced_m;      // [shots][nevents] or null
  const int32_t* forced_faults;  // [shots][nsites] outcome or -1, or null
  double* probs;                 // [shots][nevents] P(m = 1) or null
  double* phi_out;               // [shots][2^kmax][2] or null
  int* error;                    // device flag word (trace mode)
};

struct LaunchShape {
  int G;            // threads per shot: 1, 64 or 256
  int grid;         // workgroups of 256 threads
  size_t lds_bytes; // dynamic LDS per workgroup
  bool global_vec;  // active vectors in the global workspace
};

hipError_t launch_sample(const DevProgram& P, const KArgs& A, const LaunchShape& L, bool fp64, bool trace,
                         hipStream_t stream);
size_t lds_bytes_for(const DevProgram& P, int G, bool global_vec, bool fp64);

}  // namespace clifft
