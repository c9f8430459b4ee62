// Rate probes: kernels whose work is known exactly, timed by the caller to
// state achievable rates beside the published peaks.
#include "probe.h"

namespace clifft {

// A plain device copy.
__global__ __launch_bounds__(256) void k_probe_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// A read-only sweep: every thread XORs the 16-byte elements it reads and
// writes one element, so the reads cannot be dropped.
__global__ __launch_bounds__(256) void k_probe_read(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
  uint4 acc = make_uint4(0, 0, 0, 0);
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = g; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint4 v = src[i];
    acc.x ^= v.x;
    acc.y ^= v.y;
    acc.z ^= v.z;
    acc.w ^= v.w;
  }
  dst[g] = acc;
}

// Eight independent chains a = (a ^ c) + c: each iteration issues exactly
// 16 VALU instructions per lane (written out so that none is fused away).
__global__ __launch_bounds__(256) void k_probe_int(uint32_t* dst, uint32_t iters) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = 0x9E3779B9u;
  uint32_t a0 = g * 8, a1 = g * 8 + 1, a2 = g * 8 + 2, a3 = g * 8 + 3;
  uint32_t a4 = g * 8 + 4, a5 = g * 8 + 5, a6 = g * 8 + 6, a7 = g * 8 + 7;
#define CLIFFT_PROBE_STEP(a) asm volatile("v_xor_b32 %0, %1, %0\n\tv_add_u32 %0, %1, %0" : "+v"(a) : "v"(c))
#pragma unroll 4
  for (uint32_t i = 0; i < iters; i++) {
    CLIFFT_PROBE_STEP(a0);
    CLIFFT_PROBE_STEP(a1);
    CLIFFT_PROBE_STEP(a2);
    CLIFFT_PROBE_STEP(a3);
    CLIFFT_PROBE_STEP(a4);
    CLIFFT_PROBE_STEP(a5);
    CLIFFT_PROBE_STEP(a6);
    CLIFFT_PROBE_STEP(a7);
  }
#undef CLIFFT_PROBE_STEP
  dst[g] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

hipError_t launch_probe(int kind, void* dst, const void* src, uint64_t n, int grid, hipStream_t st) {
  if (kind == 0) hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, (size_t)(n / 16));
  else if (kind == 1) hipLaunchKernelGGL(k_probe_int, dim3(grid), dim3(256), 0, st, (uint32_t*)dst, (uint32_t)n);
  else hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, (size_t)(n / 16));
  return hipGetLastError();
}

}  // namespace clifft
