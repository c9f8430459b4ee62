// Counter-based random numbers of the stochastic contract, device side.
// Self-contained (no includes, plain integer types) so that the same text
// serves the kernels built ahead of time and the program-specialized kernels
// compiled at run time.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each multiplier's full
// 64-bit product is one v_mad_u64_u32 (both halves at once).
#pragma once

namespace clifft_rng {

struct U4 {
  unsigned int w0, w1, w2, w3;
};

__device__ __forceinline__ U4 philox(unsigned int c0, unsigned int c1, unsigned int c2, unsigned int c3,
                                     unsigned int k0, unsigned int k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
    const unsigned int n0 = (unsigned int)(p1 >> 32) ^ c1 ^ k0, n2 = (unsigned int)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (unsigned int)p1;
    c2 = n2;
    c3 = (unsigned int)p0;
  }
  return U4{c0, c1, c2, c3};
}

// counter = (index, purpose, shot_lo, shot_hi), key = (seed_lo, seed_hi)
__device__ __forceinline__ U4 draw(unsigned int index, unsigned int purpose, unsigned long long shot,
                                   unsigned long long seed) {
  return philox(index, purpose, (unsigned int)shot, (unsigned int)(shot >> 32), (unsigned int)seed,
                (unsigned int)(seed >> 32));
}

// u = ((w1 << 32 | w0) >> 11) * 2^-53, in [0, 1)
__device__ __forceinline__ double uniform53(const U4& w) {
  const unsigned long long v = ((unsigned long long)w.w1 << 32) | w.w0;
  return (double)(v >> 11) * 0x1.0p-53;
}

}  // namespace clifft_rng
