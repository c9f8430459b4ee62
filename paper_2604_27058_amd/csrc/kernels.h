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
  double* gamma_out;             // [shots][2] global scalar (re, im) or null
  double* expval;                // [nprobes][shots] expectation-value probes or null
  int* error;                    // device flag word (trace mode)
  // split form: needed-bit rows [nbits][ceil(shots/64)], written by the frame
  // stream and read by the vector stream
  uint64_t* nbits;
  uint32_t list_cap = 0xFFFFFFFFu;  // bit-sliced fault-list capacity (tests may lower it)
  int32_t strat_r = -1;             // stratified: exactly this many faults per shot (P.strat), or -1
};

struct LaunchShape {
  int G;            // threads per shot: 1, 64 or 256
  int grid;         // workgroups of 256 threads
  size_t lds_bytes; // dynamic LDS per workgroup
  bool global_vec;  // active vectors in the global workspace
  bool spec;        // bit-sliced: the program-specialized kernel
  // split form: the frame-only stream on the bit-sliced kernel (fgrid
  // workgroups of 64 threads), then the vector-only stream with the shape
  // above, then the record fix-up
  bool split;
  int fgrid;
  bool flane;       // split: frames too wide for LDS rows, so the frame pass
                    // runs shot per lane (fgrid workgroups of 256 threads)
};

// Batched launch: many programs, one persistent kernel.
struct BatchProgram {
  DevProgram P;
  uint64_t shots, seed, offset;
  uint64_t meas_off, det_off, obs_off;  // row-block offsets (uint64 words) in the batch outputs
  int32_t G;                            // 1 (64-shot tiles per wave) or 256 (one shot per workgroup)
  int32_t pad;
};
struct BatchItem {
  uint32_t prog;   // index into the program table
  uint32_t kind;   // 1: four 64-shot tiles (one per wave); 256: one shot
  uint64_t first;  // first tile (kind 1), first of four shots (kind 64) or the shot (kind 256)
};
// One queue of a batched launch (all items of one kind), its items grouped
// by the frame width W of their program: items [wstart[W-1], wstart[W]).
struct BatchArgs {
  const BatchProgram* progs;
  const BatchItem* items;
  uint64_t nitems;
  uint64_t wstart[5];
  uint32_t* counter;      // claim counters (one 64-bit slot per width), zeroed before the launch
  uint64_t *meas, *det, *obs;
  void* workspace;
  uint64_t slot_bytes;    // workspace bytes per workgroup
  uint32_t rec_words;     // max records + detectors + observables over programs
};
// The shot-per-workgroup queue, the shot-per-wave queue, then the
// shot-per-lane queue, each as one persistent kernel per frame width present
// (instantiated for that width), in turn on the stream (they share the
// workspace).  The queues' counter blocks are the 32-bit words at
// groups.counter + 8 q + 2 (W - 1), q = 0, 1, 2: twelve 64-bit slots.
hipError_t launch_batch(const BatchArgs& groups, int grid_groups, const BatchArgs& waves, int grid_waves,
                        const BatchArgs& lanes, int grid_lanes, size_t lds_bytes, bool fp64, hipStream_t stream);
// The same with post-selection compiled in (batches holding post-selected programs).
hipError_t launch_batch_ext(const BatchArgs& groups, int grid_groups, const BatchArgs& waves, int grid_waves,
                            const BatchArgs& lanes, int grid_lanes, size_t lds_bytes, bool fp64, hipStream_t stream);

hipError_t launch_zero(uint64_t* p, size_t n, hipStream_t stream);
// The allocation-free entry point's fixed device workspace: kScratchBytes at
// the address *ptr on the current device (looked up on the first call per
// device).  Calls that overlap on one device share it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_region(void** ptr);
// Bit-sliced Pauli-frame kernel (k_max = 0): 32 shots per lane, one 64-thread
// workgroup per 2048-shot tile.
hipError_t launch_frames(const DevProgram& P, const KArgs& A, int grid, hipStream_t stream);
size_t frames_lds_rows(const DevProgram& P, int strat_r = -1);
hipError_t launch_sample(const DevProgram& P, const KArgs& A, const LaunchShape& L, bool fp64, bool trace,
                         hipStream_t stream);
size_t lds_bytes_for(const DevProgram& P, int G, bool global_vec, bool fp64);
// Interpreter instantiations, one translation unit each (sample_*.hip, trace_*.hip).
hipError_t launch_sample_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
hipError_t launch_sample_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
hipError_t launch_trace_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
// With post-selection and stratified sampling compiled in (sample_ext_*.hip).
hipError_t launch_sample_ext_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
hipError_t launch_sample_ext_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
hipError_t launch_trace_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
// Split form: the vector-only stream (vsample_*.hip) and the record fix-up:
// rows[i] (an output row: meas, then det, then obs) ^= XOR of the outcome
// rows mrows[xdep[xdep_off[rows[i]] ..]] over every word.
hipError_t launch_vsample_f32(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
hipError_t launch_vsample_f64(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t stream);
struct FixupArgs {
  uint64_t *meas, *det, *obs;
  int32_t nrec, ndet, nobs;
  const uint32_t* rows;      // output rows with a nonempty dependency
  uint32_t nrows;
  const uint32_t* xdep_off;  // per output row
  const uint32_t* xdep;
  const uint64_t* mrows;     // [nactive][words] active outcomes
  uint64_t words;
};
hipError_t launch_fixup(const FixupArgs& F, hipStream_t stream);
// The split form's vector pass (record rows zero-filled first where the
// shot-granular tiers OR their bits into them).
hipError_t launch_vector_pass(const DevProgram& P, const KArgs& A, const LaunchShape& L, bool fp64,
                              hipStream_t stream);

}  // namespace clifft
