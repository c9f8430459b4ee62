// Device helpers of the program-specialized bit-sliced kernels.  The runtime
// compiles this text (after philox.h and spec_args.h) together with a kernel
// body generated from one compiled program, so it uses plain types and no
// headers.  The arithmetic is that of the stochastic contract: the gap
// sampler over survival products (Section 3.2, jump to the next realized
// fault) with Philox draws keyed by the global shot index.
#pragma once

namespace clifft_spec {

using clifft_rng::draw;
using clifft_rng::U4;
using clifft_rng::uniform53;

constexpr unsigned int kChunk = 4096;
constexpr unsigned int kPurposeNoise = 0x4E000000u;
constexpr unsigned int kPurposeRbit = 0x52000000u;
constexpr unsigned int kShotsPerLane = 32;
constexpr unsigned int kListCap = 24;

// outcomes of a site: DEPOLARIZE1 3, DEPOLARIZE2 15, fixed Pauli errors 1
__device__ __forceinline__ unsigned int outcomes(unsigned int type) { return type == 0 ? 3u : type == 1 ? 15u : 1u; }

// First fault at or after local index cur of `chunk` for one shot (S = the
// chunk's survival products); returns the absolute site (chunk end when
// none), advances *ord and sets *outcome for a fault.
// s_end: S[len] of the chunk when the caller knows it (single-chunk
// programs pass it as a literal), negative to read it from S.
__device__ __forceinline__ unsigned int next_fault(const SpecArgs& A, const double* S, double s_end,
                                                   unsigned int nsites, unsigned int chunk, unsigned int cur,
                                                   unsigned int* ord, unsigned long long shot, unsigned int* outcome) {
  const U4 w = draw((*ord)++, kPurposeNoise | chunk, shot, A.seed);
  const unsigned int rest = nsites - chunk * kChunk;
  const unsigned int len = rest < kChunk ? rest : kChunk;
  const double tau = cur ? uniform53(w) * S[cur] : uniform53(w);  // S[0] = 1
  unsigned int lo = cur, hi = len;
  if ((s_end >= 0.0 ? s_end : S[len]) > tau) lo = len;  // no fault in the rest of the chunk
  while (lo < hi) {
    const unsigned int mid = (lo + hi) >> 1;
    if (S[mid + 1] <= tau) hi = mid;
    else lo = mid + 1;
  }
  const unsigned int nf = chunk * kChunk + lo;
  if (lo < len) {
    const unsigned long long w64 = ((unsigned long long)w.w3 << 32) | w.w2;
    *outcome = (unsigned int)__umul64hi(w64, (unsigned long long)outcomes(A.site_type[nf]));
  }
  return nf;
}

// Survival products of chunk c: the LDS copy (one chunk) or global memory.
__device__ __forceinline__ const double* chunk_surv(const SpecArgs& A, const double* lds, unsigned int c) {
  return lds ? lds : A.surv + (unsigned long long)c * (kChunk + 1);
}

// Inserts key into the lane's ascending list of n (< cap) or cap keys in
// the rows L (row i at L[i * 64 + lane]); when the list is full the largest
// key is dropped.
__device__ __forceinline__ void list_insert(unsigned int* L, int lane, unsigned int n, unsigned int cap,
                                            unsigned int key) {
  if (n >= cap && L[(cap - 1) * 64 + lane] <= key) return;  // above every kept key
  unsigned int k = n < cap ? n : cap - 1;
  while (k > 0 && L[(k - 1) * 64 + lane] > key) {
    L[k * 64 + lane] = L[(k - 1) * 64 + lane];
    k--;
  }
  L[k * 64 + lane] = key;
}

// The lane's faults (32 shots from s0) as keys (site << 9 | shot << 4 |
// outcome): the cap smallest keys >= lo_key go to the list, ascending (so in
// site order); returns how many keys >= lo_key exist.  A lane with more
// faults than the list holds calls again with lo_key above its last applied
// key (the draws are stateless, so the faults are the same).  cap >= 1.
__device__ __forceinline__ unsigned int build_list(const SpecArgs& A, const double* lds, double s_end,
                                                   unsigned int nsites, unsigned int nchunks, unsigned long long s0,
                                                   unsigned int* L, int lane, unsigned int cap, unsigned int lo_key) {
  // One draw per iteration over (shot, chunk, draw) in that order, so that
  // lanes advance independently: the wave pays 32 x chunks draws plus the
  // largest fault count among its lanes, not a second draw for every shot
  // in which any lane saw a fault.
  unsigned int cnt = 0, j = 0, c = 0, ord = 0, cur = 0;
  while (j < kShotsPerLane) {
    const unsigned int end = (c + 1) * kChunk < nsites ? (c + 1) * kChunk : nsites;
    unsigned int o = 0;
    const unsigned int nf = next_fault(A, chunk_surv(A, lds, c), s_end, nsites, c, cur, &ord, A.offset + s0 + j, &o);
    if (nf < end) {
      const unsigned int key = (nf << 9) | (j << 4) | o;
      if (key >= lo_key) {
        list_insert(L, lane, cnt < cap ? cnt : cap, cap, key);
        cnt++;
      }
      cur = nf - c * kChunk + 1;
    } else {  // no more faults in this chunk for shot j
      ord = 0;
      cur = 0;
      if (++c == nchunks) {
        c = 0;
        j++;
      }
    }
  }
  return cnt;
}

}  // namespace clifft_spec
