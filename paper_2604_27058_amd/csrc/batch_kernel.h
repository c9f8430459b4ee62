// Batched launch of many programs (persistent queue kernels): the kernel
// templates, instantiated without (batch.hip) and with (batch_ext.hip) the
// post-selection and stratified-sampling paths.
#pragma once
#include <algorithm>

#include "shot.h"

namespace clifft {

// ------------------------------------------------------------------ batched launch
// One persistent launch over many programs of different width and active
// dimension.  Workgroups claim items in the order the host sorted them
// (longest first) from an atomic counter; an item is either four 64-shot
// tiles of a shot-per-lane program (one tile per wave) or one shot of a
// shot-per-workgroup program.  Every active vector lives in the workgroup's
// slice of the global workspace.
template <int W, typename R, int KIND, bool EXT>
__device__ __forceinline__ void batch_item(const BatchArgs& B, const BatchProgram& bp, const BatchItem& it, uint64_t* rec,
                           double* red, unsigned char* slot) {
  const DevProgram& P = bp.P;
  KArgs A{};
  A.shots = bp.shots;
  A.seed = bp.seed;
  A.offset = bp.offset;
  A.meas = B.meas ? B.meas + bp.meas_off : nullptr;
  A.det = B.det ? B.det + bp.det_off : nullptr;
  A.obs = B.obs ? B.obs + bp.obs_off : nullptr;
  const uint32_t nwords_rec = (uint32_t)(P.nrec + P.ndet + P.nobs);
  const uint64_t words = (bp.shots + 63) / 64;
  const int lane = threadIdx.x & 63;
  if constexpr (KIND == 1) {
    const int wv = (int)rfl(threadIdx.x >> 6);
    const uint64_t tile = it.first + (uint64_t)wv;
    uint64_t* wrec = rec + (size_t)wv * B.rec_words;
    if (tile < words) {
      for (uint32_t r = (uint32_t)lane; r < nwords_rec; r += 64) wrec[r] = 0;
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const size_t per = 64 * ((size_t)1 << P.kmax);  // each wave: two buffers
      cpx<R>* base = (cpx<R>*)slot + (size_t)wv * 2 * per;
      if (P.kmax == 0) {
        Shot<W, 1, R, false, false, kUnroll, false, false, EXT> sh{P, A, Group<1>{lane}, Vec<1, R>{base, lane}, wrec, red, lane,
                                       A.offset + tile * 64 + lane, tile * 64 + lane};
        sh.run();
      } else {
        Shot<W, 1, R, false, true, kUnroll, true, false, EXT> sh{P, A, Group<1>{lane}, Vec<1, R>{base, lane}, wrec, red, lane,
                                                      A.offset + tile * 64 + lane, tile * 64 + lane, base + per};
        sh.run();
      }
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const uint64_t nvalid = min((uint64_t)64, A.shots - tile * 64);
      const uint64_t vmask = nvalid == 64 ? ~0ull : ((1ull << nvalid) - 1ull);
      for (uint32_t r = (uint32_t)lane; r < nwords_rec; r += 64) {
        uint64_t v = wrec[r] & vmask;
        if (r < (uint32_t)P.nrec) {
          if (A.meas) A.meas[(size_t)r * words + tile] = v;
        } else if (r < (uint32_t)(P.nrec + P.ndet)) {
          if (A.det) A.det[(size_t)(r - P.nrec) * words + tile] = v;
        } else {
          if (A.obs) A.obs[(size_t)(r - P.nrec - P.ndet) * words + tile] = v;
        }
      }
    }
  } else if constexpr (KIND == 64) {
    // up to four shots, one per wave, each with its own two buffers
    const int wv = (int)rfl(threadIdx.x >> 6);
    const uint64_t sh_i = it.first + (uint64_t)wv;
    uint64_t* wrec = rec + (size_t)wv * B.rec_words;
    if (sh_i < bp.shots) {
      for (uint32_t r = (uint32_t)lane; r < nwords_rec; r += 64) wrec[r] = 0;
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const uint64_t g = rfl((uint32_t)sh_i) | (sh_i & 0xFFFFFFFF00000000ull);
      const size_t per = (size_t)1 << P.kmax;
      cpx<R>* base = (cpx<R>*)slot + (size_t)wv * 2 * per;
      Shot<W, 64, R, false, true, unroll_for<R, true>(), true, false, EXT, true, false> sh{P, A, Group<64>{lane}, Vec<64, R>{base, lane}, wrec,
                                                               red, 0, A.offset + g, g, base + per};
      sh.run();
      __builtin_amdgcn_wave_barrier();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const uint64_t bit = 1ull << (g & 63);
      const size_t word = (size_t)(g >> 6);
      for (uint32_t r = (uint32_t)lane; r < nwords_rec; r += 64) {
        if (!(wrec[r] & 1ull)) continue;
        uint64_t* dst;
        if (r < (uint32_t)P.nrec) dst = A.meas ? A.meas + (size_t)r * words + word : nullptr;
        else if (r < (uint32_t)(P.nrec + P.ndet)) dst = A.det ? A.det + (size_t)(r - P.nrec) * words + word : nullptr;
        else dst = A.obs ? A.obs + (size_t)(r - P.nrec - P.ndet) * words + word : nullptr;
        if (dst) atomicOr((unsigned long long*)dst, (unsigned long long)bit);
      }
    }
  } else {
    const uint64_t g = rfl((uint32_t)it.first) | (it.first & 0xFFFFFFFF00000000ull);
    for (uint32_t r = threadIdx.x; r < nwords_rec; r += 256) rec[r] = 0;
    __syncthreads();
    Shot<W, 256, R, false, true, unroll_for<R, true>(), true, false, EXT, true, false> sh{P, A, Group<256>{(int)threadIdx.x},
                                                              Vec<256, R>{(cpx<R>*)slot, lane}, rec, red, 0, A.offset + g,
                                                              g, (cpx<R>*)slot + ((size_t)1 << P.kmax)};
    sh.run();
    __syncthreads();
    const uint64_t bit = 1ull << (g & 63);
    const size_t word = (size_t)(g >> 6);
    for (uint32_t r = threadIdx.x; r < nwords_rec; r += 256) {
      if (!(rec[r] & 1ull)) continue;
      uint64_t* dst;
      if (r < (uint32_t)P.nrec) dst = A.meas ? A.meas + (size_t)r * words + word : nullptr;
      else if (r < (uint32_t)(P.nrec + P.ndet)) dst = A.det ? A.det + (size_t)(r - P.nrec) * words + word : nullptr;
      else dst = A.obs ? A.obs + (size_t)(r - P.nrec - P.ndet) * words + word : nullptr;
      if (dst) atomicOr((unsigned long long*)dst, (unsigned long long)bit);
    }
  }
  __syncthreads();
}

// KIND 256: the shot-per-workgroup queue; KIND 64: four shots per
// workgroup, one per wave; KIND 1: the shot-per-lane tiles.  Separate
// kernels, so that each path gets the registers it needs.  The cooperative
// kinds inline the interpreter for every frame width and would need about
// 200 VGPRs (two waves per SIMD); they are held to four waves per SIMD,
// which spills a few values to scratch and runs the batched set 1.2x faster.
template <typename R, int KIND, bool EXT, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == 1 ? 1 : 4))) void k_batch(BatchArgs B) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* rec = (uint64_t*)smem;  // 4 * rec_words
  double* red = (double*)(smem + (size_t)4 * B.rec_words * 8);
  uint32_t* claim = (uint32_t*)(smem + (size_t)4 * B.rec_words * 8 + 64);
  unsigned char* slot = (unsigned char*)B.workspace + (size_t)blockIdx.x * B.slot_bytes;
  for (;;) {
    if (threadIdx.x == 0) *claim = atomicAdd(B.counter, 1u);
    __syncthreads();
    const uint32_t item = rfl(*claim);
    __syncthreads();
    if ((uint64_t)item >= B.nitems) break;
    const BatchItem it = B.items[item];
    const BatchProgram& bp = B.progs[it.prog];
    batch_item<W, R, KIND, EXT>(B, bp, it, rec, red, slot);
  }
}

template <typename R, int KIND, bool EXT, int W>
static hipError_t launch_batch_w(const BatchArgs& B, int grid, size_t lds_bytes, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_batch<R, KIND, EXT, W>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_batch<R, KIND, EXT, W>), dim3(grid), dim3(256), lds_bytes, st, B);
  return hipGetLastError();
}

// One queue: a kernel per frame width present, on that width's items (a
// kernel instantiated for one width needs far fewer registers than one
// that inlines the interpreter for all four).
template <typename R, int KIND, bool EXT>
static hipError_t launch_batch_t(const BatchArgs& B, int grid, size_t lds_bytes, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int w = 1; w <= 4 && e == hipSuccess; w++) {
    const uint64_t n = B.wstart[w] - B.wstart[w - 1];
    if (!n) continue;
    BatchArgs S = B;
    S.items = B.items + B.wstart[w - 1];
    S.nitems = n;
    S.counter = B.counter + 2 * (w - 1);
    const int g = (int)std::min<uint64_t>((uint64_t)grid, n);
    if (w == 1) e = launch_batch_w<R, KIND, EXT, 1>(S, g, lds_bytes, st);
    else if (w == 2) e = launch_batch_w<R, KIND, EXT, 2>(S, g, lds_bytes, st);
    else if (w == 3) e = launch_batch_w<R, KIND, EXT, 3>(S, g, lds_bytes, st);
    else e = launch_batch_w<R, KIND, EXT, 4>(S, g, lds_bytes, st);
  }
  return e;
}

template <bool EXT>
hipError_t launch_batch_impl(const BatchArgs& groups, int grid_groups, const BatchArgs& waves, int grid_waves,
                             const BatchArgs& lanes, int grid_lanes, size_t lds_bytes, bool fp64, hipStream_t st) {
  // the claim counters: three blocks of four 64-bit slots (one per width)
  hipError_t e = launch_zero((uint64_t*)groups.counter, 12, st);
  if (e == hipSuccess && groups.nitems)
    e = fp64 ? launch_batch_t<double, 256, EXT>(groups, grid_groups, lds_bytes, st)
             : launch_batch_t<float, 256, EXT>(groups, grid_groups, lds_bytes, st);
  if (e == hipSuccess && waves.nitems)
    e = fp64 ? launch_batch_t<double, 64, EXT>(waves, grid_waves, lds_bytes, st)
             : launch_batch_t<float, 64, EXT>(waves, grid_waves, lds_bytes, st);
  if (e == hipSuccess && lanes.nitems)
    e = fp64 ? launch_batch_t<double, 1, EXT>(lanes, grid_lanes, lds_bytes, st)
             : launch_batch_t<float, 1, EXT>(lanes, grid_lanes, lds_bytes, st);
  return e;
}

}  // namespace clifft
