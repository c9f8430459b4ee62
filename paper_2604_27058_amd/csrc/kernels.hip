// Launch dispatch of the sampling kernels and the record zero-fill kernel.
// The interpreter itself is in shot.h; its instantiations are spread over
// sample_f32.hip, sample_f64.hip, trace_f32.hip and trace_f64.hip, the
// bit-sliced kernel is in frames.hip and the batched launch in batch.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace clifft {

// Fixed device scratch of the allocation-free sampling entry point: it holds
// the active-vector workspace of the HBM tiers.  Each device that loads the
// library keeps its own copy until the process ends.  In host code the
// array's name is not a device address; scratch_region() returns the address
// of the current device's copy (looked up once per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_region(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// Zero-fill of record rows (a plain kernel rather than a memset node, so the
// whole call can be captured in a graph).
__global__ void k_zero(uint64_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_zero(uint64_t* p, size_t n, hipStream_t st) {
  if (!p || n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

static void zero_records(const DevProgram& P, const KArgs& A, hipStream_t st) {
  const size_t words = (A.shots + 63) / 64;
  uint64_t* rows[3] = {A.meas, A.det, A.obs};
  const size_t counts[3] = {(size_t)P.nrec, (size_t)P.ndet, (size_t)P.nobs};
  for (int i = 0; i < 3; i++) {
    size_t n = counts[i] * words;
    if (!rows[i] || n == 0) continue;
    int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, rows[i], n);
  }
}

hipError_t launch_vector_pass(const DevProgram& P, const KArgs& A, const LaunchShape& L, bool fp64,
                              hipStream_t st) {
  if (L.G == 256 || L.G == 64) zero_records(P, A, st);
  return fp64 ? launch_vsample_f64(P, A, L, st) : launch_vsample_f32(P, A, L, st);
}

hipError_t launch_sample(const DevProgram& P, const KArgs& A, const LaunchShape& L, bool fp64, bool debug,
                         hipStream_t st) {
  if (L.G == 256 || L.G == 64 || (L.G < 0 && P.has_post)) {
    // shot-granular tiers OR their record bits into zero-filled rows; the
    // bit-sliced kernel skips the rows left once post-selection has
    // rejected every shot of a wave
    const size_t words = (A.shots + 63) / 64;
    uint64_t* rows[3] = {A.meas, A.det, A.obs};
    const size_t counts[3] = {(size_t)P.nrec, (size_t)P.ndet, (size_t)P.nobs};
    for (int i = 0; i < 3; i++) {
      size_t n = counts[i] * words;
      if (!rows[i] || n == 0) continue;
      int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
      hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, rows[i], n);
    }
  }
  if (P.has_post && A.expval && P.nprobes > 0) {
    // probes a rejected shot does not reach read 0
    const size_t n = (size_t)P.nprobes * A.shots;
    hipLaunchKernelGGL(k_zero, dim3((int)std::min<size_t>(1024, (n + 255) / 256)), dim3(256), 0, st,
                       (uint64_t*)A.expval, n);
  }
  if (L.G < 0) return launch_frames(P, A, L.grid, st);
  // post-selected programs and stratified calls take the kernels that have
  // those paths compiled in (the trace kernels always do)
  const bool ext = P.has_post || A.strat_r >= 0;
  if (fp64) return debug ? launch_trace_f64(P, A, L, st) : ext ? launch_sample_ext_f64(P, A, L, st)
                                                              : launch_sample_f64(P, A, L, st);
  return debug ? launch_trace_f32(P, A, L, st) : ext ? launch_sample_ext_f32(P, A, L, st) : launch_sample_f32(P, A, L, st);
}

// Record fix-up of the split form: one thread per word of a dependent row.
__global__ void k_fixup(FixupArgs F) {
  const uint64_t n = (uint64_t)F.nrows * F.words;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = F.rows[i / F.words];
    const uint64_t w = i % F.words;
    uint64_t acc = 0;
    for (uint32_t e = F.xdep_off[r]; e < F.xdep_off[r + 1]; e++) acc ^= F.mrows[(size_t)F.xdep[e] * F.words + w];
    uint64_t* dst;
    if (r < (uint32_t)F.nrec) dst = F.meas ? F.meas + (size_t)r * F.words : nullptr;
    else if (r < (uint32_t)(F.nrec + F.ndet)) dst = F.det ? F.det + (size_t)(r - F.nrec) * F.words : nullptr;
    else dst = F.obs ? F.obs + (size_t)(r - F.nrec - F.ndet) * F.words : nullptr;
    if (dst) dst[w] ^= acc;
  }
}

hipError_t launch_fixup(const FixupArgs& F, hipStream_t st) {
  const uint64_t n = (uint64_t)F.nrows * F.words;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<uint64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_fixup, dim3(blocks), dim3(256), 0, st, F);
  return hipGetLastError();
}

size_t lds_bytes_for(const DevProgram& P, int G, bool global_vec, bool fp64) {
  const int units = G == 256 ? 1 : 4;
  const size_t nwords_rec = (size_t)(P.nrec + P.ndet + P.nobs);
  const size_t rec_stride = (nwords_rec + 1) & ~(size_t)1;
  size_t bytes = units * rec_stride * 8 + 64;
  if (!global_vec && P.kmax > 0) {
    size_t el = (size_t)1 << P.kmax;
    size_t amp = fp64 ? 16 : 8;
    bytes += units * el * amp * (G == 1 ? 64 : 1);
  }
  return bytes;
}

}  // namespace clifft
