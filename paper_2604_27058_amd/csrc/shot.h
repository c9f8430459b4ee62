// HIP kernels for gfx950: persistent shot-parallel interpreter of the
// compiled instruction stream (the paper's sample-time virtual machine,
// Section 3.2), re-designed for CDNA4.
//
// Execution shapes (template G = threads per shot):
//   G = 1    shot per lane: 64 shots per wave; Pauli frames live in VGPRs as
//            W 64-bit words per lane; the active vector of each lane lives in
//            LDS, interleaved so that amplitude i of the 64 lanes is one
//            contiguous 512-byte row (conflict-free).
//   G = 64   shot per wave: the frames are wave-uniform (SGPR/SALU); the 2^k
//            amplitudes are spread over the lanes (LDS).
//   G = 256  shot per workgroup: as G = 64 with workgroup barriers between
//            array passes; the active vector is in LDS or in a global
//            workspace slice (HBM) for large k.
// Records are bit-packed 64 shots per word (record-major) and staged in LDS
// per 64-shot tile.
// Pauli-frame-only programs (k_max = 0) also have a bit-sliced kernel
// (k_frames: 32 shots per lane, one LDS row per frame bit), and many programs
// can share one persistent launch (k_batch).
//
// Paper passages: Definition 2 (frame-factored state), Appendix B.1
// (rotations: phase / expansion / active), Appendix B.2 (measurements:
// dormant deterministic, dormant random, active mask / interfere),
// Appendix B.3 (conditional Paulis: noise and feed-forward), Section 3.2
// (sparse noise sampling by jumping to the next fault).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"
#include "philox.h"
#include "program.h"

namespace clifft {

#define DEV static __device__ __forceinline__
#define MDEV __device__ __forceinline__
#define DEV_HOST_INLINE static __host__ __device__ __forceinline__

// ------------------------------------------------------------------ RNG
using clifft_rng::draw;
using clifft_rng::U4;
using clifft_rng::uniform53;

// ------------------------------------------------------------------ helpers
// Complex amplitude.  Copies are member-wise: a struct copy of two doubles
// otherwise lowers to memcpy and keeps pass buffers in scratch memory.
template <typename R>
struct cpx {
  R re, im;
  cpx() = default;
  __host__ __device__ constexpr cpx(R r, R i) : re(r), im(i) {}
  __host__ __device__ constexpr cpx(const cpx& o) : re(o.re), im(o.im) {}
  __host__ __device__ cpx& operator=(const cpx& o) {
    re = o.re;
    im = o.im;
    return *this;
  }
};

DEV uint32_t ins0(uint32_t p, int s) { return ((p >> s) << (s + 1)) | (p & ((1u << s) - 1u)); }

// Frame words as a small vector value: a word chosen by a run-time qubit
// index then lowers to register selects, where a plain array would be
// turned into a variable offset into private (scratch) memory.
template <int W>
using Words = uint64_t __attribute__((ext_vector_type(W)));

template <int W>
struct Frame {
  Words<W> x, z;
};

template <int W>
DEV uint32_t getbit(const Words<W>& a, int q) {
  uint64_t v = a[0];
#pragma unroll
  for (int w = 1; w < W; w++)
    if ((q >> 6) == w) v = a[w];
  return (uint32_t)(v >> (q & 63)) & 1u;
}

template <int W>
DEV void xorbit(Words<W>& a, int q, uint32_t b) {
#pragma unroll
  for (int w = 0; w < W; w++)
    if ((q >> 6) == w) a[w] ^= (uint64_t)b << (q & 63);
}

template <int W>
DEV uint32_t parity_and(const Words<W>& a, const uint64_t* m) {
  uint64_t acc = 0;
#pragma unroll
  for (int w = 0; w < W; w++) acc ^= a[w] & m[w];
  return (uint32_t)__popcll(acc) & 1u;
}

// Fan of CNOT v->q (q in mask): x ^= x_v * mask, z_v ^= parity(z & mask).
template <int W>
DEV void fan_cx(Frame<W>& f, int v, const uint64_t* m) {
  uint64_t sel = 0ull - (uint64_t)getbit<W>(f.x, v);
  uint32_t pz = parity_and<W>(f.z, m);
#pragma unroll
  for (int w = 0; w < W; w++) f.x[w] ^= sel & m[w];
  xorbit<W>(f.z, v, pz);
}
// Fan of CZ v,q: z ^= x_v * mask, z_v ^= parity(x & mask).
template <int W>
DEV void fan_cz(Frame<W>& f, int v, const uint64_t* m) {
  uint64_t sel = 0ull - (uint64_t)getbit<W>(f.x, v);
  uint32_t px = parity_and<W>(f.x, m);
#pragma unroll
  for (int w = 0; w < W; w++) f.z[w] ^= sel & m[w];
  xorbit<W>(f.z, v, px);
}
// Fan of CNOT q->v: x_v ^= parity(x & mask), z ^= z_v * mask.
template <int W>
DEV void fan_2(Frame<W>& f, int v, const uint64_t* m) {
  uint64_t sel = 0ull - (uint64_t)getbit<W>(f.z, v);
  uint32_t px = parity_and<W>(f.x, m);
#pragma unroll
  for (int w = 0; w < W; w++) f.z[w] ^= sel & m[w];
  xorbit<W>(f.x, v, px);
}
template <int W>
DEV void frame_s(Frame<W>& f, int v) { xorbit<W>(f.z, v, getbit<W>(f.x, v)); }
template <int W>
DEV void frame_h(Frame<W>& f, int v) {
  uint32_t d = getbit<W>(f.x, v) ^ getbit<W>(f.z, v);
  xorbit<W>(f.x, v, d);
  xorbit<W>(f.z, v, d);
}
template <int W>
DEV void frame_xor(Frame<W>& f, const uint64_t* px, const uint64_t* pz) {
#pragma unroll
  for (int w = 0; w < W; w++) { f.x[w] ^= px[w]; f.z[w] ^= pz[w]; }
}

// Scalar (SMEM) view of program data: uniform addresses read through the
// constant address space so that the compiler issues s_load.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
DEV cptr<T> as_const(const T* p) { return (cptr<T>)(p); }

DEV uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// One 16-byte instruction through the scalar cache.
DEV GInstr load_instr(const GInstr* code, int pc) {
  cptr<uint32_t> w = (cptr<uint32_t>)(as_const(code) + pc);
  uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
  GInstr in;
  in.op = (uint8_t)(w0 & 0xFF);
  in.flags = (uint8_t)((w0 >> 8) & 0xFF);
  in.v = (uint16_t)(w0 >> 16);
  in.s = (uint16_t)(w1 & 0xFFFF);
  in.u = (uint16_t)(w1 >> 16);
  in.a = w2;
  in.b = w3;
  return in;
}
DEV double rfl(double v) {
  uint64_t b = __double_as_longlong(v);
  uint32_t lo = rfl((uint32_t)b), hi = rfl((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ------------------------------------------------------------------ group context
template <int G>
struct Group {
  int tid;  // thread index inside the shot group
  __device__ void sync() const {
    if constexpr (G == 256) __syncthreads();
    else if constexpr (G == 64) { __builtin_amdgcn_wave_barrier(); __atomic_signal_fence(__ATOMIC_SEQ_CST); }
  }
  __device__ double sum(double v, double* red) const {
    if constexpr (G == 1) {
      return v;
    } else {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if constexpr (G == 64) {
        return rfl(v);
      } else {
        int wv = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[wv] = v;
        __syncthreads();
        double t = red[0] + red[1] + red[2] + red[3];
        return rfl(t);
      }
    }
  }
};

// Amplitude storage: G == 1 lane-interleaved (element i of lane l at i*64+l),
// otherwise element i of the group's vector at i.
template <int G, typename R>
struct Vec {
  cpx<R>* base;
  int lane;
  __device__ cpx<R>& operator[](uint32_t i) const {
    if constexpr (G == 1) return base[(size_t)i * 64 + lane];
    else return base[i];
  }
};

template <int N>
struct IntC {
  static constexpr int value = N;
};

// Iterate p over [0, n) split among the threads of a group.
#define FOR_GROUP(p, n) for (uint32_t p = (G == 1 ? 0u : (uint32_t)grp.tid); p < (n); p += (G == 1 ? 1u : (uint32_t)G))

// Unrolled passes over the active vector.  Iteration p touches an element
// set disjoint from every other iteration's, so a batch of U iterations
// issues all its loads before its stores (U independent loads in flight per
// lane) without any hazard.
constexpr int kUnroll = 4;        // iterations in flight per lane, vectors on chip
constexpr int kUnrollGlobal = 8;  // FP32 vectors in HBM: more bytes in flight per wave
template <typename R, bool GLOBAL>
constexpr int unroll_for() { return GLOBAL && sizeof(R) == 4 ? kUnrollGlobal : kUnroll; }
// log2 of the amplitudes in one 128-byte line
template <typename R>
constexpr int kLineBits() { return sizeof(R) == 4 ? 4 : 3; }

// Read-modify-write of one element per iteration: i = idx(p).
template <int G, typename R, int U, typename IdxF, typename BodyF>
DEV void pass1(const Group<G>& grp, const Vec<G, R>& vec, uint32_t n, IdxF idx, BodyF body) {
  const uint32_t st = G == 1 ? 1u : (uint32_t)G;
  for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += U * st) {
    uint32_t ii[U];
    cpx<R> a[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      uint32_t p = base + u * st;
      ii[u] = idx(p < n ? p : base);
      if (p < n) a[u] = vec[ii[u]];
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (base + u * st < n) vec[ii[u]] = body(a[u]);
  }
}

// Read-modify-write of a pair per iteration: (i0, i1) = idx(p).
template <int G, typename R, int U, typename IdxF, typename BodyF>
DEV void pass2(const Group<G>& grp, const Vec<G, R>& vec, uint32_t n, IdxF idx, BodyF body) {
  const uint32_t st = G == 1 ? 1u : (uint32_t)G;
  for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += U * st) {
    uint32_t i0[U], i1[U];
    cpx<R> a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      uint32_t p = base + u * st;
      idx(p < n ? p : base, i0[u], i1[u]);
      if (p < n) { a[u] = vec[i0[u]]; b[u] = vec[i1[u]]; }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (base + u * st < n) {
        body(a[u], b[u]);
        vec[i0[u]] = a[u];
        vec[i1[u]] = b[u];
      }
  }
}

// Two reads, one write per iteration: out[wi(p)] = body(in[r0(p)], in[r1(p)])
// (r1 may equal r0).  Used where a pass writes fewer elements than it reads.
template <int G, typename R, int U, typename IdxF, typename BodyF>
DEV void pass21(const Group<G>& grp, const Vec<G, R>& vec, uint32_t n, IdxF idx, BodyF body) {
  const uint32_t st = G == 1 ? 1u : (uint32_t)G;
  for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += U * st) {
    uint32_t r0[U], r1[U], wi[U];
    cpx<R> a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      uint32_t p = base + u * st;
      idx(p < n ? p : base, r0[u], r1[u], wi[u]);
      if (p < n) { a[u] = vec[r0[u]]; b[u] = vec[r1[u]]; }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (base + u * st < n) vec[wi[u]] = body(a[u], b[u]);
  }
}

// Work-item order of the cooperative HBM passes (one shot per wave or
// workgroup).  Such a pass reads each element pair at affine images of its
// item index q; when a pair's partner mask crosses 128-byte lines while the
// measured axis lies inside a line, the natural order touches every line
// for half its elements and fetches it again from HBM for the other half.
// Here the items of one aligned group of 2^nv lanes share q >> nv and span
// v[0..nv), chosen so that the group's reads fill whole lines: q maps to
// dep(q >> nv) ^ sum_i q_i v_i, dep inserting zeros at the pivots of v
// (the highest bit of each, distinct after elimination) and at the pass's
// fixed-zero bit.
struct LineEnum {
  uint32_t v[4];
  int nv;
  int pos[5];  // ascending zero-insertion positions (unused entries last)
  int npos;
  uint32_t xo;  // sum of v over the low bits of the lane's items (bind)
  // The passes step q by multiples of 64 from the lane's own index, so the
  // low nv (<= 4) bits of q are the lane's: their part of the sum is fixed.
  MDEV void bind(uint32_t lane_q) {
    xo = 0;
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (i < nv && ((lane_q >> i) & 1u)) xo ^= v[i];
  }
  MDEV uint32_t operator()(uint32_t q) const {
    uint32_t j = q >> nv;
#pragma unroll
    for (int i = 0; i < 5; i++)
      if (i < npos) j = ins0(j, pos[i]);
    return j ^ xo;
  }
};

// cand: candidate spanning vectors (0 = none; zero at the fixed bit `zero`,
// or zero < 0 for none), in order of preference; at most four are kept
// after elimination.  Constant indices only, so that everything stays in
// registers.
template <int NC>
DEV LineEnum line_enum(const uint32_t (&cand)[NC], int zero) {
  LineEnum E;
  E.nv = 0;
  int piv[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; i++) E.v[i] = 0;
#pragma unroll
  for (int c = 0; c < NC; c++) {
    uint32_t x = cand[c];
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (i < E.nv && ((x >> piv[i]) & 1u)) x ^= E.v[i];
    if (x && E.nv < 4) {
      const int pb = 31 - __clz(x);
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (i < E.nv && ((E.v[i] >> pb) & 1u)) E.v[i] ^= x;
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (i == E.nv) {
          E.v[i] = x;
          piv[i] = pb;
        }
      E.nv++;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; i++) E.pos[i] = i < E.nv ? piv[i] : 64;
  E.pos[4] = zero >= 0 ? zero : 64;
  E.npos = E.nv + (zero >= 0 ? 1 : 0);
#pragma unroll
  for (int i = 0; i < 4; i++)  // sorting network, ascending
#pragma unroll
    for (int j = 0; j < 4 - i; j++)
      if (E.pos[j] > E.pos[j + 1]) {
        const int t = E.pos[j];
        E.pos[j] = E.pos[j + 1];
        E.pos[j + 1] = t;
      }
  return E;
}

// Read-only pairs accumulated into two FP64 sums (the body also gets the
// iteration index).
template <int G, typename R, int U, typename IdxF, typename BodyF>
DEV void reduce2(const Group<G>& grp, const Vec<G, R>& vec, uint32_t n, IdxF idx, BodyF body, double& s0,
                 double& s1) {
  const uint32_t st = G == 1 ? 1u : (uint32_t)G;
  for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += U * st) {
    cpx<R> a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      uint32_t p = base + u * st;
      uint32_t i0, i1;
      idx(p < n ? p : base, i0, i1);
      if (p < n) { a[u] = vec[i0]; b[u] = vec[i1]; }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (base + u * st < n) body(a[u], b[u], base + u * st, s0, s1);
  }
}

// Gather pass into another buffer: dst[o] = gen(o) for o = ord(p), p in
// [0, n) (ord a permutation of [0, n); gen reads the source); all U values
// of a batch are formed before the stores.
template <int G, typename R, int U, typename OrdF, typename GenF>
DEV void pass1_to(const Group<G>& grp, const Vec<G, R>& dst, uint32_t n, OrdF ord, GenF gen) {
  const uint32_t st = G == 1 ? 1u : (uint32_t)G;
  for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += U * st) {
    cpx<R> v[U];
    uint32_t o[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t p = base + u * st;
      o[u] = ord(p < n ? p : base);
      if (p < n) v[u] = gen(o[u]);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t p = base + u * st;
      if (p < n) dst[o[u]] = v[u];
    }
  }
}

template <typename R>
DEV cpx<R> cmul(cpx<R> a, R cr, R ci) { return cpx<R>{a.re * cr - a.im * ci, a.re * ci + a.im * cr}; }
template <typename R>
DEV double norm2(cpx<R> a) { return (double)a.re * (double)a.re + (double)a.im * (double)a.im; }

// ------------------------------------------------------------------ noise state
struct Noise {
  uint32_t chunk, ord, nf, nf_out;
};

DEV uint32_t nout_of(uint32_t t) { return t == S_DEP1 ? 3u : t == S_DEP2 ? 15u : 1u; }

// Next fault at or after local index cur of the current chunk (Section 3.2,
// jump to the next realized fault).  tau = u * S[cur]; the fault is the
// smallest j with S[j+1] <= tau, j == len meaning none left in the chunk.
DEV void next_fault(const DevProgram& P, Noise& ns, uint32_t cur, uint64_t shot, uint64_t seed) {
  U4 w = draw(ns.ord++, kPurposeNoise | ns.chunk, shot, seed);
  const double* S = P.surv + (size_t)ns.chunk * (kChunk + 1);
  uint32_t len = min((uint32_t)kChunk, (uint32_t)P.nsites - ns.chunk * (uint32_t)kChunk);
  double tau = uniform53(w) * S[cur];
  uint32_t lo = cur, hi = len;
  if (S[len] > tau) lo = len;  // no fault in the rest of the chunk (same answer as the search)
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (S[mid + 1] <= tau) hi = mid;
    else lo = mid + 1;
  }
  ns.nf = ns.chunk * (uint32_t)kChunk + lo;
  if (lo < len) {
    uint64_t w64 = ((uint64_t)w.w3 << 32) | w.w2;
    ns.nf_out = (uint32_t)__umul64hi(w64, (uint64_t)nout_of(P.site_type[ns.nf]));
  }
}

DEV uint32_t fault_outcome(const DevProgram& P, uint32_t site, const U4& w) {
  const uint64_t w64 = ((uint64_t)w.w3 << 32) | w.w2;
  return (uint32_t)__umul64hi(w64, (uint64_t)nout_of(P.site_type[site]));
}

// Stratified sampling (Section 3.2, rare-event sampling): with s >= 1 faults
// left from site cur on, the next one is at the smallest t >= cur with
// e_s(t + 1) <= u e_s(cur) (tab: the rows of DevProgram::strat, in HBM or
// staged in LDS); t <= nsites - s since e_s vanishes once fewer than s
// sites remain.
DEV uint32_t strat_site(const double* tab, uint32_t nsites, uint32_t s, uint32_t cur, const U4& w) {
  const double* E = tab + (size_t)(s - 1) * (nsites + 1);
  const double tau = uniform53(w) * E[cur];
  uint32_t lo = cur, hi = nsites - s;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (E[mid + 1] <= tau) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Noise state of a stratified shot: chunk counts the faults still to place
// and ord the faults placed (fault i comes from draw i of kPurposeStrat).
DEV void next_fault_strat(const DevProgram& P, Noise& ns, uint32_t cur, uint64_t shot, uint64_t seed) {
  if (ns.chunk == 0) {
    ns.nf = 0xFFFFFFFFu;
    return;
  }
  const U4 w = draw(ns.ord++, kPurposeStrat, shot, seed);
  ns.nf = strat_site(P.strat, (uint32_t)P.nsites, ns.chunk, cur, w);
  ns.nf_out = fault_outcome(P, ns.nf, w);
  ns.chunk--;
}

template <int W>
DEV void apply_fault(const DevProgram& P, Frame<W>& T, Frame<W>& N, uint32_t site, uint32_t o) {
  uint32_t t = P.site_type[site];
  const uint64_t* img = P.masks + P.site_img[site];
  uint32_t la, lb = 0;
  if (t == S_DEP1) la = o + 1;
  else if (t == S_DEP2) { la = (o + 1) >> 2; lb = (o + 1) & 3; }
  else la = t - 1;  // X_ERROR 1, Y_ERROR 2, Z_ERROR 3
  uint64_t ex[W], ez[W];
#pragma unroll
  for (int w = 0; w < W; w++) { ex[w] = 0; ez[w] = 0; }
  // image layout per qubit: X~ (x words, z words) then Z~ (x words, z words)
  const uint32_t L[2] = {la, lb};
#pragma unroll
  for (int qi = 0; qi < 2; qi++) {
    uint32_t l = L[qi];
    const uint64_t* ix = img + (size_t)qi * 4 * W;
    const uint64_t* iz = ix + 2 * W;
    uint64_t ux = (l == 1 || l == 2) ? ~0ull : 0ull;
    uint64_t uz = (l == 2 || l == 3) ? ~0ull : 0ull;
    if (qi == 1 && t != S_DEP2) break;
#pragma unroll
    for (int w = 0; w < W; w++) {
      ex[w] ^= (ix[w] & ux) ^ (iz[w] & uz);
      ez[w] ^= (ix[W + w] & ux) ^ (iz[W + w] & uz);
    }
  }
  frame_xor<W>(T, ex, ez);
  frame_xor<W>(N, ex, ez);
}

// Power of i that a fired fault contributes to the global scalar (trace
// mode; Appendix B.3): the fired Pauli is the product of its qubits'
// letters' signed images (Y = i X Z), written E = i^e X^ex Z^ez, and
// E X^x Z^z = i^(e + 2|ez & x|) X^(ex ^ x) Z^(ez ^ z) for the frame X^x Z^z.
template <int W>
DEV int fault_phase(const DevProgram& P, const Words<W>& fx, uint32_t site, uint32_t o) {
  const uint32_t t = P.site_type[site];
  const uint64_t* img = P.masks + P.site_img[site];
  const uint32_t sg = P.site_sign[site];
  uint32_t la, lb = 0;
  if (t == S_DEP1) la = o + 1;
  else if (t == S_DEP2) { la = (o + 1) >> 2; lb = (o + 1) & 3; }
  else la = t - 1;
  int e = 0;
  uint64_t px[W], pz[W];
#pragma unroll
  for (int w = 0; w < W; w++) { px[w] = 0; pz[w] = 0; }
  const uint32_t L[2] = {la, lb};
  for (int qi = 0; qi < 2; qi++) {
    if (qi == 1 && t != S_DEP2) break;
    const uint32_t l = L[qi];
    if (l == 0) continue;
    const uint64_t* ax = img + (size_t)qi * 4 * W;  // X image: x words, z words
    const uint64_t* bx = ax + 2 * W;                // Z image: x words, z words
    const int rx = (sg >> (2 * qi)) & 1, rz = (sg >> (2 * qi + 1)) & 1;
    uint64_t qx[W], qz[W];
    int eq = 0;
#pragma unroll
    for (int w = 0; w < W; w++) {
      if (l == 1) { qx[w] = ax[w]; qz[w] = ax[W + w]; eq += __popcll(ax[w] & ax[W + w]); }
      else if (l == 3) { qx[w] = bx[w]; qz[w] = bx[W + w]; eq += __popcll(bx[w] & bx[W + w]); }
      else {
        qx[w] = ax[w] ^ bx[w];
        qz[w] = ax[W + w] ^ bx[W + w];
        eq += __popcll(ax[w] & ax[W + w]) + __popcll(bx[w] & bx[W + w]) + 2 * __popcll(ax[W + w] & bx[w]);
      }
    }
    eq += l == 1 ? 2 * rx : l == 3 ? 2 * rz : 1 + 2 * rx + 2 * rz;
#pragma unroll
    for (int w = 0; w < W; w++) {
      eq += 2 * __popcll(pz[w] & qx[w]);
      px[w] ^= qx[w];
      pz[w] ^= qz[w];
    }
    e += eq;
  }
#pragma unroll
  for (int w = 0; w < W; w++) e += 2 * __popcll(pz[w] & fx[w]);
  return e & 3;
}

// ------------------------------------------------------------------ one shot
// OOP: active vectors in HBM with a second buffer of the same size; active
// measurements collapse out of place (alternating buffers) and read through
// their folded localization passes.  EXT: post-selection (OP_POSTSELECT) and
// stratified fault sampling are compiled in (always in trace mode); the
// plain kernels leave them out so that their code and registers stay those
// of plain sampling.  PAIR: paired measurement collapses on the cooperative
// HBM tiers (left out of the batched kernels, whose vectors mostly stay in
// the caches and whose registers are tighter).
template <int W, int G, typename R, bool DBG, bool VEC, int U = kUnroll, bool OOP = false, bool VONLY = false,
          bool EXT = false, bool LINE = true, bool PAIR = false>
struct Shot {
  static constexpr bool kExt = EXT || DBG;
  // line-complete item orders in the cooperative HBM passes (LineEnum)
  static constexpr bool kLine = G > 1 && OOP && LINE;
  static constexpr bool kPairLine = kLine && sizeof(R) == 8;
  // Without that order (FP32) a pair's passes read whole lines only when
  // every slot they move (the measured slots of the pair and of the pair
  // whose joint sums they take, and a single collapse's own) lies above the
  // line bits; lower ones cost 2-8 lines per line of data, more than the
  // pair saves, so FP32 pairs only such measurements, and only on vectors
  // of 2^17 amplitudes or more (measured: below that the pairs' passes cost
  // FP32 more than the bytes they save).
  static constexpr int kPairMinSlot = kPairLine ? 0 : kLineBits<R>();
  static constexpr int kPairMinK = kPairLine ? 3 : 17;
  const DevProgram& P;
  const KArgs& A;
  Group<G> grp;
  Vec<G, R> vec;
  uint64_t* rec;  // LDS record words of the tile (R + D + O)
  double* red;    // LDS reduction scratch (G == 256)
  int slane;      // shot index inside the 64-shot tile
  uint64_t shot;  // global shot index (G == 1: per lane)
  uint64_t local; // shot index relative to the call (debug buffers)
  cpx<R>* alt = nullptr;  // OOP: the other buffer
  // G == 1: the lane's shot was rejected by post-selection.  The lane keeps
  // executing the stream (its wave-uniform state must stay uniform) but
  // writes nothing more; G > 1 units end the shot at once instead.
  bool post_dead = false;

  // The next active measurement after instruction pc (whose collapse fuses
  // it): its slot and type and the localization passes folded into it.
  MDEV void peek_next_measurement(int pc, uint32_t& s2, bool& x2, uint32_t& tm2, uint32_t& sm2, bool& as2) const {
    tm2 = sm2 = 0;
    as2 = false;
    for (int q = pc + 1;; q++) {
      const GInstr g = load_instr(P.code, q);
      if (g.op == OP_APERM) tm2 = g.a;
      else if (g.op == OP_ASIGN) sm2 = g.a;
      else if (g.op == OP_AS) as2 = true;
      else if (g.op == OP_MACTZ || g.op == OP_MACTX || g.op == OP_END) {
        s2 = g.s;
        x2 = g.op == OP_MACTX;
        return;
      }
    }
  }

  // An active measurement ahead of pc and the localization passes folded
  // into it (pc = -1 at the end of the stream).
  struct MeasAhead {
    int pc;
    uint32_t s, tm, sm;
    bool as, x;
    uint8_t flags;
  };
  MDEV MeasAhead peek_meas(int pc) const {
    MeasAhead m{-1, 0u, 0u, 0u, false, false, 0};
    for (int q = pc + 1;; q++) {
      const GInstr g = load_instr(P.code, q);
      if (g.op == OP_APERM) m.tm = g.a;
      else if (g.op == OP_ASIGN) m.sm = g.a;
      else if (g.op == OP_AS) m.as = true;
      else if (g.op == OP_MACTZ || g.op == OP_MACTX || g.op == OP_END) {
        m.pc = g.op == OP_END ? -1 : q;
        m.s = g.s;
        m.x = g.op == OP_MACTX;
        m.flags = g.flags;
        return m;
      }
    }
  }
  // Paired collapses: a partner read through folded localization passes
  // (the sign from its index, then the factor i), and the unnormalised kept
  // branch b of a pair (a, c): a or c, or a +- c for an X-type measurement.
  static MDEV cpx<R> pair_phase(cpx<R> x, uint32_t i1, uint32_t sm, bool as) {
    const cpx<R> y = (__popc(i1 & sm) & 1) ? cpx<R>{-x.re, -x.im} : x;
    return as ? cpx<R>{-y.im, y.re} : y;
  }
  static MDEV cpx<R> pair_comb(cpx<R> a, cpx<R> c, bool x, uint32_t b) {
    if (x) return b ? cpx<R>{a.re - c.re, a.im - c.im} : cpx<R>{a.re + c.re, a.im + c.im};
    return b ? c : a;
  }
  // Quad q of a vector of kq slots under measurement a and then b (on a's
  // result, whose slot a.s holds the former top slot kq-1): o[0], o[1] are
  // a's pair that gives b's first member u1 (top slot kq-2 moved into b.s),
  // o[2], o[3] the pair that gives b's partner, read at u2i ^ b.tm.
  static MDEV void pair_quad(uint32_t q, int kq, const MeasAhead& a, const MeasAhead& b, uint32_t (&o)[4],
                             uint32_t& u2i) {
    const int ta = kq - 1, tb = kq - 2;
    const uint32_t ba = 1u << a.s, bb = 1u << b.s;
    const uint32_t u1 = (int)b.s == tb ? q : ((q & ~bb) | (((q >> b.s) & 1u) << tb));
    u2i = u1 | bb;
    const uint32_t u2 = u2i ^ b.tm;
    o[0] = (int)a.s == ta ? u1 : ((u1 & ~ba) | (((u1 >> a.s) & 1u) << ta));
    o[1] = (o[0] | ba) ^ a.tm;
    o[2] = (int)a.s == ta ? u2 : ((u2 & ~ba) | (((u2 >> a.s) & 1u) << ta));
    o[3] = (o[2] | ba) ^ a.tm;
  }
  // the quad's part of the joint branch sums t[2 ba + bb] (raw: a factor
  // 1/2 per X-type measurement left out)
  static MDEV void pair_sums(const cpx<R> (&y)[4], const uint32_t (&o)[4], uint32_t u2i, const MeasAhead& a,
                             const MeasAhead& b, double (&t)[4]) {
    const uint32_t ba = 1u << a.s;
    const cpx<R> c1 = pair_phase(y[1], o[0] | ba, a.sm, a.as), c2 = pair_phase(y[3], o[2] | ba, a.sm, a.as);
#pragma unroll
    for (uint32_t e = 0; e < 2; e++) {
      const cpx<R> y1 = pair_comb(y[0], c1, a.x, e);
      const cpx<R> y2 = pair_phase(pair_comb(y[2], c2, a.x, e), u2i, b.sm, b.as);
      if (b.x) {
        t[2 * e] += norm2(cpx<R>{y1.re + y2.re, y1.im + y2.im});
        t[2 * e + 1] += norm2(cpx<R>{y1.re - y2.re, y1.im - y2.im});
      } else {
        t[2 * e] += norm2(y1);
        t[2 * e + 1] += norm2(y2);
      }
    }
  }

  // The lane's items of this measurement's paired pass in the line-complete
  // order precomputed with the program (identity when it has none of this
  // kind, and in FP32, where the order's registers cost the workgroup tier
  // a wave per SIMD and its time more than the order saves).  The order inserts zero bits at its pivots and adds the lane's
  // combination xo; the items of a lane step by G, so the inserted value
  // steps by a constant carried across the pivot bits.
  struct PairWalk {
    uint32_t j, holes, inc, xo;
    MDEV uint32_t cur() const { return j ^ xo; }
    MDEV void next() { j = ((j | holes) + inc) & ~holes; }
  };
  MDEV PairWalk pair_walk(const GInstr& in, int kind) const {
    uint32_t v[4] = {0u, 0u, 0u, 0u}, holes = 0;
    int nv = 0;
    if (kPairLine && in.u != 0) {
      const PairLine& L = P.pline[2u * in.u + (sizeof(R) == 8 ? 1u : 0u)];
      if (L.kind == kind) {
#pragma unroll
        for (int i = 0; i < 4; i++) v[i] = L.v[i];
        nv = L.nv;
#pragma unroll
        for (int i = 0; i < 5; i++)
          if (i < L.npos) holes |= 1u << L.pos[i];
      }
    }
    auto deposit = [&](uint32_t a) {
      uint32_t h = holes;
      while (h) {
        a = ins0(a, __builtin_ctz(h));
        h &= h - 1u;
      }
      return a;
    };
    const uint32_t tid = (uint32_t)grp.tid;
    PairWalk w;
    w.holes = holes;
    w.j = deposit(tid >> nv);
    w.inc = deposit((uint32_t)G >> nv);
    w.xo = 0;
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (i < nv && ((tid >> i) & 1u)) w.xo ^= v[i];
    return w;
  }

  MDEV bool writer() const { return (G == 1 || grp.tid == 0) && local < A.shots && !(kExt && post_dead); }

  MDEV void put(uint32_t r, uint32_t m) {
    if constexpr (G == 1) {
      uint64_t word = __ballot(m && !(kExt && post_dead));
      if ((threadIdx.x & 63) == 0) rec[r] = word;
    } else {
      if (grp.tid == 0) rec[r] |= (uint64_t)m << slane;
    }
  }
  MDEV uint32_t xor_refs(uint32_t a, uint32_t u) {
    // G == 1: whole 64-shot words; otherwise this shot's bit
    uint64_t acc = 0;
    cptr<uint32_t> refs = as_const(P.refs);
    for (uint32_t i = 0; i < u; i++) acc ^= rec[refs[a + i]];
    if constexpr (G == 1) {
      uint32_t lane = threadIdx.x & 63;
      return (uint32_t)(acc >> lane) & 1u;
    } else {
      return (uint32_t)(acc >> slane) & 1u;
    }
  }

  // Vector-only stream of the split form: needed bit `row` of this shot
  // (written by the frame stream with every active outcome 0), corrected by
  // the parity of its dependency mask with the active outcomes so far.
  // Shot-granular tiers fetch the first kNbitPre rows of the shot once, one
  // row per lane, into wave-uniform masks.
  static constexpr int kNbitPre = 256;
  uint64_t nbm[kNbitPre / 64];
  MDEV void fetch_nbits() {
    if constexpr (G > 1 && VONLY) {
      const uint64_t words = (A.shots + 63) / 64;
      const uint32_t lane = threadIdx.x & 63;
#pragma unroll
      for (int q = 0; q < kNbitPre / 64; q++) {
        const uint32_t row = (uint32_t)q * 64 + lane;
        uint32_t b = 0;
        if (q * 64 < P.nbits && row < (uint32_t)P.nbits && local < A.shots)
          b = (uint32_t)(A.nbits[(size_t)row * words + (local >> 6)] >> (local & 63)) & 1u;
        nbm[q] = __ballot(b);
      }
    }
  }
  MDEV uint32_t raw_nbit(uint32_t row) const {
    if constexpr (G > 1) {
      if (row < (uint32_t)kNbitPre) {
        uint64_t w = nbm[0];
#pragma unroll
        for (int q = 1; q < kNbitPre / 64; q++)
          if ((row >> 6) == (uint32_t)q) w = nbm[q];
        return (uint32_t)(w >> (row & 63)) & 1u;
      }
    }
    const uint64_t words = (A.shots + 63) / 64;
    return (uint32_t)(A.nbits[(size_t)row * words + (local >> 6)] >> (local & 63)) & 1u;
  }
  MDEV uint32_t nbit(uint32_t row, const uint64_t (&mb)[kSplitWords]) const {
    uint32_t b = raw_nbit(row);
    cptr<uint64_t> dep = as_const(P.vdep) + (size_t)row * P.dep_words;
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kSplitWords; q++)
      if (q < P.dep_words) acc ^= dep[q] & mb[q];
    return b ^ ((uint32_t)__popcll(acc) & 1u);
  }

  __device__ __forceinline__ void run() {
    Frame<W> T, N;
    uint64_t mb[kSplitWords];  // vector-only stream: active outcomes so far (bit = active index)
#pragma unroll
    for (int q = 0; q < kSplitWords; q++) mb[q] = 0;
    if constexpr (VONLY) fetch_nbits();
#pragma unroll
    for (int w = 0; w < W; w++) { T.x[w] = T.z[w] = N.x[w] = N.z[w] = 0; }
    const uint64_t seed = A.seed;
    int k = 0;
    uint32_t last_m = 0, last_pn = 0;
    uint32_t rb_blk = 0xFFFFFFFFu;
    U4 rb{0, 0, 0, 0};
    double carry0 = 0, carry1 = 0;  // branch sums of the next active measurement (fused)
    bool carry_valid = false;
    // Paired collapses (the cooperative HBM tiers, Appendix B.2 for two
    // measurements A and B with only frame work between them): from the
    // joint branch sums S[bA][bB], A is sampled from the marginals and its
    // collapse waits; B, sampled from S[bA][.], collapses the vector along
    // both axes in one pass (reads 2^k, writes 2^(k-2)) instead of two
    // (2^k + 2^(k-1) read, 2^(k-1) + 2^(k-2) written).  The joint sums are
    // taken by the collapse before A as it writes its outputs (by quads of
    // A and B), or with nothing carried by one pass over the vector.  B's
    // frame bits are read at B as usual.
    constexpr bool kPair = G > 1 && OOP && PAIR;
    bool pj_valid = false;                 // joint sums carried
    double pj00 = 0, pj01 = 0, pj10 = 0, pj11 = 0;
    bool pair_pend = false;                // A sampled, collapse pending
    uint32_t pa_s = 0, pa_tm = 0, pa_sm = 0, pa_b = 0;
    bool pa_as = false, pa_x = false;
    double pb0 = 0, pb1 = 0;               // B's raw sums given A's branch
    uint32_t pend_tm = 0, pend_sm = 0;  // folded localization passes of the next measurement
    bool pend_as = false;
    // Out of place: the last dfr expansions are not applied yet; element x
    // is vec[x mod 2^(k-dfr)] times beta[t] for every set bit t of
    // x >> (k-dfr) (an expansion multiplies its new upper half by a phase).
    constexpr int ND = OOP ? kDeferMax : 1;
    // passes through the factors run one iteration at a time: their reads
    // mostly hit the cache (each stored element serves up to 2^dfr outputs)
    // and a deeper unroll would cost the whole kernel occupancy
    constexpr int UD = 1;
    int dfr = 0;
    cpx<R> beta[ND];
#pragma unroll
    for (int t = 0; t < ND; t++) beta[t] = cpx<R>{(R)1, (R)0};
    auto fac = [&](uint32_t c) {
      cpx<R> f = (c & 1u) ? beta[0] : cpx<R>{(R)1, (R)0};
#pragma unroll
      for (int t = 1; t < ND; t++) {
        const cpx<R> b = ((c >> t) & 1u) ? beta[t] : cpx<R>{(R)1, (R)0};
        f = cpx<R>{f.re * b.re - f.im * b.im, f.re * b.im + f.im * b.re};
      }
      return f;
    };
    // writes the deferred part: x = lo | c << (k-dfr) for c != 0, with c the
    // fastest index so that each stored element is read once per group of c
    auto materialize = [&]() {
      if constexpr (OOP) {
        if (dfr == 0) return;
        const int m = k - dfr;
        const uint32_t n = 1u << k, cm = (1u << dfr) - 1u;
        const uint32_t st = G == 1 ? 1u : (uint32_t)G;
        for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += UD * st) {
          cpx<R> y[UD];
#pragma unroll
          for (int u = 0; u < UD; u++) {
            const uint32_t qq = base + u * st;
            if (qq < n && (qq & cm)) {
              const cpx<R> a = vec[qq >> dfr], f = fac(qq & cm);
              y[u] = cpx<R>{a.re * f.re - a.im * f.im, a.re * f.im + a.im * f.re};
            }
          }
#pragma unroll
          for (int u = 0; u < UD; u++) {
            const uint32_t qq = base + u * st;
            if (qq < n && (qq & cm)) vec[(qq >> dfr) | ((qq & cm) << m)] = y[u];
          }
        }
        grp.sync();
        dfr = 0;
      }
    };
    // Trace mode tracks the global scalar of the frame-factored state
    // (Definition 2): an exact power of i from frame conjugations and
    // products (Appendix B.3), rotation phases (the factor e^{-i theta} that
    // the kernels leave out of the vector, and dormant-Z phases), and
    // 2^{-1/2} per expansion since the last collapse (the vector is left
    // unnormalised by expansions and renormalised by a collapse).
    int g_ipow = 0, g_nexp = 0;
    double g_re = 1.0, g_im = 0.0;
    auto g_rot = [&](uint32_t ci, bool flip) {  // gamma *= e^{-i theta}, theta sign-flipped by the frame
      if constexpr (DBG) {
        const double c = P.consts[4 * ci + 2], sn = flip ? -P.consts[4 * ci + 3] : P.consts[4 * ci + 3];
        const double re = g_re * c + g_im * sn;
        g_im = g_im * c - g_re * sn;
        g_re = re;
      }
    };
    auto g_h = [&](int q) {  // frame conjugation by H_q: (-1)^(x_q z_q)
      if constexpr (DBG) g_ipow += 2 * (int)(getbit<W>(T.x, q) & getbit<W>(T.z, q));
    };
    Noise ns{0, 0, 0xFFFFFFFFu, 0};
    if (P.nsites > 0) {
      if (DBG && A.forced_faults) ns.nf = 0xFFFFFFFFu;
      else if (kExt && A.strat_r >= 0) {
        ns.chunk = (uint32_t)A.strat_r;
        next_fault_strat(P, ns, 0, shot, seed);
      } else
        next_fault(P, ns, 0, shot, seed);
    }
    if (VEC && P.kmax > 0) {
      FOR_GROUP(p, 1u) vec[p] = cpx<R>{(R)1, (R)0};
      grp.sync();
    }
    cptr<uint64_t> masks = as_const(P.masks);
    for (int pc = 0;; pc++) {
      const GInstr in = load_instr(P.code, pc);
      const int v = in.v;
      const int s = in.s;
      if constexpr (G == 1 && kExt) {
        // every lane of the wave rejected by post-selection: leave together
        // (a wave-uniform exit, so that the instruction fetch stays scalar)
        if (P.has_post && !__ballot(!post_dead)) goto done;
      }
      switch (in.op) {
        case OP_END:
          goto done;
        case OP_FANCX: {
          uint64_t m[W];
#pragma unroll
          for (int w = 0; w < W; w++) m[w] = masks[in.a + w];
          fan_cx<W>(T, v, m);
          fan_cx<W>(N, v, m);
          break;
        }
        case OP_FANCZ: {
          uint64_t m[W];
#pragma unroll
          for (int w = 0; w < W; w++) m[w] = masks[in.a + w];
          if constexpr (DBG) g_ipow += 2 * (int)(getbit<W>(T.x, v) & parity_and<W>(T.x, m));
          fan_cz<W>(T, v, m);
          fan_cz<W>(N, v, m);
          break;
        }
        case OP_FAN2: {
          uint64_t m[W];
#pragma unroll
          for (int w = 0; w < W; w++) m[w] = masks[in.a + w];
          fan_2<W>(T, v, m);
          fan_2<W>(N, v, m);
          break;
        }
        case OP_FS:
          if constexpr (DBG) g_ipow += (int)getbit<W>(T.x, v);  // S X S^dag = Y = i X Z
          frame_s<W>(T, v);
          frame_s<W>(N, v);
          break;
        case OP_FH:
          g_h(v);
          frame_h<W>(T, v);
          frame_h<W>(N, v);
          break;
        case OP_PHASE: {
          if constexpr (DBG) {
            uint64_t m[W];
#pragma unroll
            for (int w = 0; w < W; w++) m[w] = masks[in.a + w];
            g_rot(in.b, parity_and<W>(T.x, m) != 0);
          }
          break;
        }
        case OP_APERM: {
          if constexpr (!VEC) break;
          else {
          if (OOP && (in.flags & F_FOLD_NEXT)) {  // read through by the next measurement
            pend_tm = in.a;
            break;
          }
          carry_valid = false;
          pj_valid = false;
          materialize();
          // control slot s, targets tm: i -> i ^ tm for i with bit s set; each
          // pair is visited once from the member with target bit t0 clear
          const uint32_t tm = in.a, bs = 1u << s;
          const int t0 = __ffs(tm) - 1;
          const int lo = min(s, t0), hi = max(s, t0);
          pass2<G, R, U>(grp, vec, 1u << (k - 2),
                      [&](uint32_t p, uint32_t& i0, uint32_t& i1) { i0 = ins0(ins0(p, lo), hi) | bs; i1 = i0 ^ tm; },
                      [](cpx<R>& a, cpx<R>& b) { cpx<R> t = a; a = b; b = t; });
          grp.sync();
          }
          break;
        }
        case OP_ASIGN: {
          if constexpr (!VEC) break;
          else {
          if (OOP && (in.flags & F_FOLD_NEXT)) {
            pend_sm = in.a;
            break;
          }
          carry_valid = false;
          pj_valid = false;
          materialize();
          // -1 on i with bit s set and odd parity of i & sm: enumerate i with
          // bits s and c (lowest of sm) free, then fix bit c to make it odd
          const uint32_t sm = in.a, bs = 1u << s;
          const int c = __ffs(sm) - 1;
          const int lo = min(s, c), hi = max(s, c);
          pass1<G, R, U>(grp, vec, 1u << (k - 2),
                      [&](uint32_t p) {
                        uint32_t i = ins0(ins0(p, lo), hi) | bs;
                        return i | ((uint32_t)((__popc(i & sm) & 1) ^ 1) << c);
                      },
                      [](cpx<R> a) { return cpx<R>{-a.re, -a.im}; });
          grp.sync();
          }
          break;
        }
        case OP_APERM2: {
          if constexpr (!VEC) break;
          else {
          carry_valid = false;
          pj_valid = false;
          materialize();
          // flip bit s where parity(i & sm) is odd: pairs along s with odd parity
          const uint32_t sm = in.a, bs = 1u << s;
          const int c = __ffs(sm) - 1;
          const int lo = min(s, c), hi = max(s, c);
          pass2<G, R, U>(grp, vec, 1u << (k - 2),
                      [&](uint32_t p, uint32_t& i0, uint32_t& i1) {
                        uint32_t i = ins0(ins0(p, lo), hi);
                        i0 = i | ((uint32_t)((__popc(i & sm) & 1) ^ 1) << c);
                        i1 = i0 | bs;
                      },
                      [](cpx<R>& a, cpx<R>& b) { cpx<R> t = a; a = b; b = t; });
          grp.sync();
          }
          break;
        }
        case OP_AS: {
          if constexpr (!VEC) break;
          else {
          if (OOP && (in.flags & F_FOLD_NEXT)) {
            pend_as = true;
            break;
          }
          carry_valid = false;
          pj_valid = false;
          materialize();
          const uint32_t bs = 1u << s;
          pass1<G, R, U>(grp, vec, 1u << (k - 1), [&](uint32_t p) { return ins0(p, s) | bs; },
                      [](cpx<R> a) { return cpx<R>{-a.im, a.re}; });
          grp.sync();
          }
          break;
        }
        case OP_AH: {
          if constexpr (!VEC) break;
          else {
          carry_valid = false;
          pj_valid = false;
          if constexpr (!OOP) materialize();
          const R h = (R)0.70710678118654752440;
          const uint32_t bs = 1u << s;
          if constexpr (OOP) {
            // out of place: a rotation on this slot that directly follows is
            // applied to the written upper halves, and folded localization
            // passes are read through (the element of i1 is that of i1 ^ tm,
            // signed by parity(i1 & sm), times i for S), as are deferred
            // expansions (element x is stored[x mod 2^dm] times its factor)
            const int dm = k - dfr;
            const uint32_t lmask = (1u << dm) - 1u;
            auto rdx = [&](uint32_t x) {
              const cpx<R> e = vec[x & lmask], f = fac(x >> dm);
              return cpx<R>{e.re * f.re - e.im * f.im, e.re * f.im + e.im * f.re};
            };
            const GInstr nx = load_instr(P.code, pc + 1);
            const bool rot = nx.op == OP_AROT && nx.s == s;
            R rr = (R)1, ri = (R)0;
            if (rot) {
              double c2 = P.consts[4 * nx.a], s2 = P.consts[4 * nx.a + 1];
              const bool flip = VONLY ? nbit(nx.v, mb) != 0 : getbit<W>(T.x, nx.v) != 0;
              if (flip) s2 = -s2;
              rr = (R)c2;
              ri = (R)s2;
              g_rot(nx.a, flip);
            }
            const uint32_t tm = pend_tm, sm = pend_sm;
            const bool fas = pend_as;
            const Vec<G, R> dst{alt, vec.lane};
            const uint32_t n = 1u << (k - 1), st = G == 1 ? 1u : (uint32_t)G;
            constexpr int UH = G == 1 ? 1 : (U >= 4 ? U / 4 : 1);
            for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n; base += UH * st) {
              uint32_t ii[UH];
              cpx<R> a[UH], c[UH];
#pragma unroll
              for (int u = 0; u < UH; u++) {
                const uint32_t q = base + u * st;
                ii[u] = ins0(q < n ? q : base, s);
                if (q < n) {
                  a[u] = rdx(ii[u]);
                  c[u] = rdx((ii[u] | bs) ^ tm);
                }
              }
#pragma unroll
              for (int u = 0; u < UH; u++) {
                if (base + u * st >= n) continue;
                const uint32_t i1 = ii[u] | bs;
                cpx<R> y = (__popc(i1 & sm) & 1) ? cpx<R>{-c[u].re, -c[u].im} : c[u];
                if (fas) y = cpx<R>{-y.im, y.re};
                dst[ii[u]] = cpx<R>{h * (a[u].re + y.re), h * (a[u].im + y.im)};
                dst[i1] = cmul(cpx<R>{h * (a[u].re - y.re), h * (a[u].im - y.im)}, rr, ri);
              }
            }
            cpx<R>* t = vec.base;
            vec.base = alt;
            alt = t;
            pend_tm = pend_sm = 0;
            pend_as = false;
            dfr = 0;
            if (rot) pc++;
          } else {
            pass2<G, R, U>(grp, vec, 1u << (k - 1),
                        [&](uint32_t p, uint32_t& i0, uint32_t& i1) { i0 = ins0(p, s); i1 = i0 | bs; },
                        [h](cpx<R>& a, cpx<R>& b) {
                          cpx<R> x{h * (a.re + b.re), h * (a.im + b.im)};
                          b = cpx<R>{h * (a.re - b.re), h * (a.im - b.im)};
                          a = x;
                        });
          }
          grp.sync();
          }
          break;
        }
        case OP_EXPAND: {
          if constexpr (!VEC) break;
          else {
          carry_valid = false;
          pj_valid = false;
          // Appendix B.1 case 2: H_v takes |0>_v to |+>_v (frames conjugated);
          // then exp(-i theta' Z_v) on the new axis, theta' sign-flipped by
          // x_v of the frame.  The common phase e^{-i theta'} is global, so
          // the new half is the old one times e^{2 i theta'}.
          bool flip;
          if constexpr (VONLY) {
            flip = nbit(v, mb) != 0;
          } else {
            g_h(v);
            frame_h<W>(T, v);
            frame_h<W>(N, v);
            flip = getbit<W>(T.x, v) != 0;
          }
          double c2 = P.consts[4 * in.a], s2 = P.consts[4 * in.a + 1];
          if (flip) s2 = -s2;
          g_rot(in.a, flip);
          g_nexp++;
          const R cr = (R)c2, ci = (R)s2;
          if constexpr (OOP) {
            // deferred: the new top slot's factor; when all are taken, the
            // oldest (slot k - dfr) is applied first, as an expansion would
            if (dfr == ND) {
              const uint32_t n = 1u << (k - dfr);
              const cpx<R> b0 = beta[0];
              pass21<G, R, U>(grp, vec, n, [&](uint32_t p, uint32_t& r0, uint32_t& r1, uint32_t& w) { r0 = r1 = p; w = p | n; },
                              [b0](cpx<R> a, cpx<R>) { return cmul(a, b0.re, b0.im); });
              grp.sync();
#pragma unroll
              for (int t = 0; t + 1 < ND; t++) beta[t] = beta[t + 1];
              dfr--;
            }
#pragma unroll
            for (int t = 0; t < ND; t++)
              if (t == dfr) beta[t] = cpx<R>{cr, ci};
            dfr++;
            k++;
            break;
          }
          const uint32_t n = 1u << k;
          pass21<G, R, U>(grp, vec, n, [&](uint32_t p, uint32_t& r0, uint32_t& r1, uint32_t& w) { r0 = r1 = p; w = p | n; },
                       [cr, ci](cpx<R> a, cpx<R>) { return cmul(a, cr, ci); });
          k++;
          grp.sync();
          }
          break;
        }
        case OP_AROT: {
          if constexpr (!VEC) break;
          else {
          carry_valid = false;
          pj_valid = false;
          materialize();
          double c2 = P.consts[4 * in.a], s2 = P.consts[4 * in.a + 1];
          const bool flip = VONLY ? nbit(v, mb) != 0 : getbit<W>(T.x, v) != 0;
          if (flip) s2 = -s2;
          g_rot(in.a, flip);
          const R cr = (R)c2, ci = (R)s2;
          const uint32_t bs = 1u << s;
          pass1<G, R, U>(grp, vec, 1u << (k - 1), [&](uint32_t p) { return ins0(p, s) | bs; },
                      [cr, ci](cpx<R> a) { return cmul(a, cr, ci); });
          grp.sync();
          }
          break;
        }
        case OP_MSTATIC: {
          uint64_t m[W];
#pragma unroll
          for (int w = 0; w < W; w++) m[w] = masks[in.a + w];
          uint32_t mm = parity_and<W>(T.x, m) ^ (uint32_t)(in.flags & F_SIGN);
          last_pn = parity_and<W>(N.x, m);
          if constexpr (DBG) {
            if (A.probs && writer()) A.probs[local * P.nevents + in.b] = (double)mm;
            if (A.forced_m && writer() && A.forced_m[local * P.nevents + in.b] != mm) atomicOr(A.error, 2);
          }
          last_m = mm;
          int r = as_const(P.ev_rec)[in.b];
          if (r >= 0) put((uint32_t)r, mm);
          break;
        }
        case OP_MRANDOM: {
          uint32_t j = in.b;
          uint32_t p = getbit<W>(T.z, v), pn = getbit<W>(N.z, v);
          uint32_t mm;
          if constexpr (DBG) {
            if (A.probs && writer()) A.probs[local * P.nevents + j] = 0.5;
          }
          if (DBG && A.forced_m) {
            mm = local < A.shots ? A.forced_m[local * P.nevents + j] : 0u;
            if constexpr (G > 1) mm = rfl(mm);
          } else {
            if ((j >> 7) != rb_blk) {
              rb_blk = j >> 7;
              rb = draw(rb_blk, kPurposeRbit, shot, seed);
            }
            uint32_t bi = j & 127, word = bi >> 5;
            uint32_t wv = word == 0 ? rb.w0 : word == 1 ? rb.w1 : word == 2 ? rb.w2 : rb.w3;
            mm = ((wv >> (bi & 31)) & 1u) ^ pn;
          }
          uint32_t b = mm ^ (uint32_t)(in.flags & F_SIGN) ^ p;
          g_h(v);  // H_v absorbed into the frames
          frame_h<W>(T, v);
          frame_h<W>(N, v);
          if constexpr (DBG) g_ipow += 2 * (int)(b & getbit<W>(T.z, v));  // X^x Z^z X_v = (-1)^{z_v} X^(x^v) Z^z
          xorbit<W>(T.x, v, b);
          last_m = mm;
          last_pn = pn;
          int r = as_const(P.ev_rec)[j];
          if (r >= 0) put((uint32_t)r, mm);
          break;
        }
        case OP_MACTZ:
        case OP_MACTX: {
          if constexpr (!VEC) break;
          else {
          const bool isx = in.op == OP_MACTX;
          uint32_t j = in.b;
          uint32_t sign = in.flags & F_SIGN;
          uint32_t p, pn;
          if constexpr (VONLY) {
            p = nbit(v, mb);
            pn = raw_nbit(v + 1);
          } else {
            p = isx ? getbit<W>(T.z, v) : getbit<W>(T.x, v);
            pn = isx ? getbit<W>(N.z, v) : getbit<W>(N.x, v);
          }
          const uint32_t bs = 1u << s;
          const uint32_t half = 1u << (k - 1);
          // paired collapses (see kPair): A of a pair (its collapse waits)
          // or B (the collapse along both axes)
          int pmode = 0;
          MeasAhead pmB{};
          if constexpr (kPair) {
            if (pair_pend) {
              pmode = 2;
            } else if ((in.flags & F_FUSE_NEXT) && k >= kPairMinK && dfr == 0 && (pj_valid || !carry_valid) &&
                       s >= kPairMinSlot) {
              pmB = peek_meas(pc);
              if ((int)pmB.s >= kPairMinSlot) pmode = 1;
            }
          }
          // branch sums (Appendix B.2): |a|^2 per half along the axis, or
          // |a +- b|^2 of the fold for an X-type measurement
          auto branch_sums = [](bool x, cpx<R> a, cpx<R> b, double& x0, double& x1) {
            if (x) {
              x0 += norm2(cpx<R>{a.re + b.re, a.im + b.im});
              x1 += norm2(cpx<R>{a.re - b.re, a.im - b.im});
            } else {
              x0 += norm2(a);
              x1 += norm2(b);
            }
          };
          // the partner (measured bit set) of a pair, read through the folded
          // localization passes: element (i1 ^ tm) times the phase at i1
          const uint32_t tm = pend_tm, sm = pend_sm;
          const bool fas = pend_as;
          auto partner = [&](cpx<R> x, uint32_t i1) {
            cpx<R> y = (__popc(i1 & sm) & 1) ? cpx<R>{-x.re, -x.im} : x;
            return fas ? cpx<R>{-y.im, y.re} : y;
          };
          double s0 = 0, s1 = 0;
          // Deferred expansions (out of place): element lo | c << dm is
          // stored[lo] times F(c), the product of beta over the set bits of c
          // (|F| = 1), and its measured partner is (lo ^ dlo, c ^ dc).  Over
          // the combinations c of one stored pair, the Z branch sums are nc
          // times the stored ones, and the X cross term Re(conj(a) p) sums to
          // Re(conj(va) pv Gam), Gam = sum over c of sigma_c F(c ^ dc) conj F(c)
          // (sigma_c: the sign of the measured-slot phase from the bits of c).
          const bool dfd = OOP && dfr > 0;
          const int dm = k - dfr;
          const uint32_t lmask = (1u << dm) - 1u, cmask = (1u << dfr) - 1u;
          const uint32_t bsc = dfd && s >= dm ? (1u << (s - dm)) : 0u;
          const uint32_t dlo = (bs ^ tm) & lmask, dc = dfd ? ((bs ^ tm) >> dm) & cmask : 0u;
          const uint32_t bsl = bs & lmask, sml = sm & lmask, smc = dfd ? (sm >> dm) & cmask : 0u;
          const uint32_t npairs = s < dm ? (1u << (dm - 1)) : (1u << dm);
          // phase of a stored partner from the stored bits of its index
          auto partner_lo = [&](cpx<R> x, uint32_t lo) {
            cpx<R> y = (__popc((lo | bsl) & sml) & 1) ? cpx<R>{-x.re, -x.im} : x;
            return fas ? cpx<R>{-y.im, y.re} : y;
          };
          if (kPair && pmode == 2) {
            // B: its sums given A's branch
            s0 = pb0;
            s1 = pb1;
          } else if (kPair && pmode == 1) {
            // A: the marginals of the joint sums of A and B (carried, or
            // from one pass over the vector)
            if (!pj_valid) {
              const MeasAhead me{pc, (uint32_t)s, tm, sm, fas, isx, in.flags};
              PairWalk E = pair_walk(in, PP_JOINT_READ);
              double t[4] = {0, 0, 0, 0};
              for (uint32_t q = (uint32_t)grp.tid; q < (1u << (k - 2)); q += (uint32_t)G, E.next()) {
                uint32_t o[4], u2i;
                pair_quad(E.cur(), k, me, pmB, o, u2i);
                cpx<R> y[4];
#pragma unroll
                for (int e = 0; e < 4; e++) y[e] = vec[o[e]];
                pair_sums(y, o, u2i, me, pmB, t);
              }
              pj00 = grp.sum(t[0], red);
              pj01 = grp.sum(t[1], red);
              pj10 = grp.sum(t[2], red);
              pj11 = grp.sum(t[3], red);
            }
            const double f = pmB.x ? 0.5 : 1.0;
            s0 = f * (pj00 + pj01);
            s1 = f * (pj10 + pj11);
          } else if (carry_valid) {
            // accumulated by the previous measurement's collapse pass
            s0 = carry0;
            s1 = carry1;
          } else if (dfd) {
            const double nc = (double)(s < dm ? (1u << dfr) : (1u << (dfr - 1)));
            double gre = 0, gim = 0;
            if (isx) {
              for (uint32_t c = 0; c <= cmask; c++) {
                if (c & bsc) continue;
                const cpx<R> f = fac(c), g = fac(c ^ dc);
                double re = (double)g.re * f.re + (double)g.im * f.im;
                double im = (double)g.im * f.re - (double)g.re * f.im;
                if (__popc((c | bsc) & smc) & 1) { re = -re; im = -im; }
                gre += re;
                gim += im;
              }
            }
            reduce2<G, R, (U > 4 ? 4 : U)>(grp, vec, npairs,
                             [&](uint32_t q, uint32_t& i0, uint32_t& i1) {
                               i0 = s < dm ? ins0(q, s) : q;
                               i1 = i0 ^ dlo;
                             },
                             [&](cpx<R> va, cpx<R> vc, uint32_t q, double& x0, double& x1) {
                               const cpx<R> pv = partner_lo(vc, s < dm ? ins0(q, s) : q);
                               if (isx) {
                                 const double t = nc * (norm2(va) + norm2(pv));
                                 const double wre = (double)va.re * pv.re + (double)va.im * pv.im;
                                 const double wim = (double)va.re * pv.im - (double)va.im * pv.re;
                                 const double cr = 2.0 * (wre * gre - wim * gim);
                                 x0 += t + cr;
                                 x1 += t - cr;
                               } else {
                                 x0 += nc * norm2(va);
                                 x1 += nc * norm2(pv);
                               }
                             },
                             s0, s1);
            s0 = grp.sum(s0, red);
            s1 = grp.sum(s1, red);
          } else {
            // the pairs' first members (bit s clear); on the cooperative HBM
            // tiers in line-complete order: the line bits other than s, and
            // the partner mask's bits outside them when s is a line bit
            LineEnum E{};
            if constexpr (kLine) {
              constexpr int LB = kLineBits<R>();
              uint32_t cand[LB + 1];
              uint32_t inc = 0;
#pragma unroll
              for (int b = 0; b < LB; b++) {
                cand[b] = (b != (int)s && b < k) ? 1u << b : 0u;
                inc |= cand[b];
              }
              cand[LB] = (int)s < LB ? tm & ~inc : 0u;
              E = line_enum(cand, s);
              E.bind((uint32_t)grp.tid);
            }
            auto first = [&](uint32_t q) -> uint32_t {
              if constexpr (kLine) return E(q);
              else return ins0(q, s);
            };
            reduce2<G, R, U>(grp, vec, half,
                             [&](uint32_t q, uint32_t& i0, uint32_t& i1) { i0 = first(q); i1 = (i0 | bs) ^ tm; },
                             [&](cpx<R> a, cpx<R> c, uint32_t q, double& x0, double& x1) {
                               branch_sums(isx, a, partner(c, first(q) | bs), x0, x1);
                             },
                             s0, s1);
            s0 = grp.sum(s0, red);
            s1 = grp.sum(s1, red);
          }
          if (isx) { s0 *= 0.5; s1 *= 0.5; }
          double tot = s0 + s1;
          uint32_t bm1 = 1u ^ sign ^ p;  // virtual branch of m = 1
          double sb1 = bm1 ? s1 : s0;
          uint32_t mm;
          if constexpr (DBG) {
            if (A.probs && writer()) A.probs[local * P.nevents + j] = sb1 / tot;
          }
          if (DBG && A.forced_m) {
            mm = local < A.shots ? A.forced_m[local * P.nevents + j] : 0u;
            if constexpr (G > 1) mm = rfl(mm);
          } else {
            U4 w = draw(j, kPurposeAmeas, shot, seed);
            double pref1 = ((bm1 ^ pn) ? s1 : s0) / tot;  // P(m_ref = 1)
            mm = (uniform53(w) < pref1 ? 1u : 0u) ^ pn;
          }
          uint32_t b = mm ^ sign ^ p;
          double sb = b ? s1 : s0;
          if (!(sb > 1e-300 * tot)) {
            if constexpr (DBG) {
              if (writer()) atomicOr(A.error, 2);
            }
            sb = tot > 0 ? tot : 1.0;
          }
          const R scale = (R)(1.0 / sqrt(sb));
          const R fs = isx ? (R)0.70710678118654752440 : (R)1;
          const R sgn = b ? (R)-1 : (R)1;
          const int top = k - 1;
          const uint32_t tb = 1u << top;
          auto out1 = [&](cpx<R> a, cpx<R> c) -> cpx<R> {
            if (isx) return cpx<R>{fs * scale * (a.re + sgn * c.re), fs * scale * (a.im + sgn * c.im)};
            return b ? cpx<R>{scale * c.re, scale * c.im} : cpx<R>{scale * a.re, scale * a.im};
          };
          // the next measurement (after this demotion), when fused: its slot,
          // type and folded localization passes
          const bool fuse = (in.flags & F_FUSE_NEXT) && k >= 2;
          uint32_t s2 = 0, tm2 = 0, sm2 = 0;
          bool nx = false, as2 = false;
          if (fuse) peek_next_measurement(pc, s2, nx, tm2, sm2, as2);
          const uint32_t b2 = 1u << s2;
          auto partner2 = [&](cpx<R> x, uint32_t i1) {
            cpx<R> y = (__popc(i1 & sm2) & 1) ? cpx<R>{-x.re, -x.im} : x;
            return as2 ? cpx<R>{-y.im, y.re} : y;
          };
          // a pair follows: the joint sums of the next two measurements
          // instead (cooperative HBM tiers)
          MeasAhead pm2{}, pm3{};
          bool joint2 = false;
          if constexpr (kPair) {
            if (fuse && !dfd && k - 1 >= kPairMinK && (pmode == 2 || s >= kPairMinSlot)) {
              pm2 = peek_meas(pc);
              if ((pm2.flags & F_FUSE_NEXT) && (int)pm2.s >= kPairMinSlot) {
                pm3 = peek_meas(pm2.pc);
                joint2 = (int)pm3.s >= kPairMinSlot;
              }
            }
          }
          const uint32_t st = G == 1 ? 1u : (uint32_t)G;
          double n0 = 0, n1 = 0;
          bool fused_sums = false, pj_new = false;
          if constexpr (OOP) {
            // out of place into the other buffer: output o (new slot s holds
            // the former top bit) reads its pair through the folded passes
            const Vec<G, R> dst{alt, vec.lane};
            auto one = [&](uint32_t o) {
              const uint32_t base = s == top ? o : ((o & ~bs) | (((o >> s) & 1u) << top));
              const uint32_t i1 = base | bs;
              return out1(vec[base], partner(vec[i1 ^ tm], i1));
            };
            if (kPair && pmode == 1) {
              // A: sampled and recorded; its collapse waits for B
              pa_s = (uint32_t)s;
              pa_tm = tm;
              pa_sm = sm;
              pa_as = fas;
              pa_x = isx;
              pa_b = b;
              pb0 = b ? pj10 : pj00;
              pb1 = b ? pj11 : pj01;
              pair_pend = true;
            } else if (kPair && pmode == 2) {
              // B: the vector (k + 1 slots, A not collapsed yet) collapses
              // along both axes; element u of A's result (unnormalised) and
              // element w of the result
              const int topA = k, topB = k - 1;
              const uint32_t bsA = 1u << pa_s;
              auto ua = [&](uint32_t u) {
                const uint32_t v0 = (int)pa_s == topA ? u : ((u & ~bsA) | (((u >> pa_s) & 1u) << topA));
                return pair_comb(vec[v0], pair_phase(vec[(v0 | bsA) ^ pa_tm], v0 | bsA, pa_sm, pa_as), pa_x, pa_b);
              };
              const R f = isx ? fs * scale : scale;
              auto wv = [&](uint32_t w) {
                const uint32_t u1 = s == topB ? w : ((w & ~bs) | (((w >> s) & 1u) << topB));
                const uint32_t u2i = u1 | bs;
                const cpx<R> r = pair_comb(ua(u1), partner(ua(u2i ^ tm), u2i), isx, b);
                return cpx<R>{f * r.re, f * r.im};
              };
              const uint32_t nw = half;  // k - 1 slots
              if (joint2) {
                PairWalk E = pair_walk(in, PP_PAIR_JOINT);
                double jt[4] = {0, 0, 0, 0};
                for (uint32_t q = (uint32_t)grp.tid; q < (nw >> 2); q += st, E.next()) {
                  uint32_t o[4], u2i;
                  pair_quad(E.cur(), k - 1, pm2, pm3, o, u2i);
                  cpx<R> y[4];
#pragma unroll
                  for (int e = 0; e < 4; e++) y[e] = wv(o[e]);
#pragma unroll
                  for (int e = 0; e < 4; e++) dst[o[e]] = y[e];
                  pair_sums(y, o, u2i, pm2, pm3, jt);
                }
                pj00 = grp.sum(jt[0], red);
                pj01 = grp.sum(jt[1], red);
                pj10 = grp.sum(jt[2], red);
                pj11 = grp.sum(jt[3], red);
                pj_new = true;
              } else if (fuse) {
                PairWalk E = pair_walk(in, PP_PAIR_NEXT);
                for (uint32_t q = (uint32_t)grp.tid; q < (nw >> 1); q += st, E.next()) {
                  const uint32_t j0 = ins0(E.cur(), (int)s2), j1 = (j0 | b2) ^ tm2;
                  const cpx<R> y0 = wv(j0), y1 = wv(j1);
                  dst[j0] = y0;
                  dst[j1] = y1;
                  branch_sums(nx, y0, partner2(y1, j0 | b2), n0, n1);
                }
                fused_sums = true;
              } else {
                PairWalk E = pair_walk(in, PP_PAIR);
                for (uint32_t q = (uint32_t)grp.tid; q < nw; q += st, E.next()) {
                  const uint32_t w = E.cur();
                  dst[w] = wv(w);
                }
              }
              pair_pend = false;
            } else if (dfd) {
              // each stored pair is read once; the outputs of its deferred
              // combinations follow a Gray-code walk over c (one factor per
              // step on each side)
              const cpx<R> g0 = fac(dc);
              const R sg0 = (__popc(bsc & smc) & 1) ? (R)-1 : (R)1;
              // output of input lo | c << dm (the top bit moves to slot s)
              auto oidx = [&](uint32_t lo, uint32_t c) {
                const uint32_t i0 = lo | (c << dm);
                return s == top ? i0 : ((i0 & ~tb) | (((i0 >> top) & 1u) << s));
              };
              // one Gray-code step (bit t, to value nb) of a walk whose c is
              // offset by off: its element factor and its partner factor
              auto step = [&](cpx<R>& x, cpx<R>& y, int t, bool nb, uint32_t off) {
                const cpx<R> bt = beta[t];
                const bool xb = nb ^ ((off >> t) & 1u);
                x = cmul(x, bt.re, xb ? bt.im : -bt.im);
                const bool yb = xb ^ ((dc >> t) & 1u);  // bit t of (c ^ off) ^ dc
                const R sg = ((smc >> t) & 1u) ? (R)-1 : (R)1;
                y = cmul(y, sg * bt.re, yb ? sg * bt.im : -sg * bt.im);
              };
              // The next measurement (fused) pairs output o with o ^ d2 (the
              // member with bit s2 clear first).  In stored and deferred bits
              // d2 is (d2lo, d2c): the pair of the output of (lo, c) is the
              // output of (lo ^ d2lo, c ^ d2c), from the same stored pair when
              // d2lo = 0; piv is the bit that orders the two members.
              const uint32_t cm1 = (1u << (dfr - 1)) - 1u;
              auto to_c = [&](uint32_t M) {
                return ((M >> dm) & cm1 & ~bsc) | (s != top ? ((M >> s) & 1u) << (dfr - 1) : 0u);
              };
              const uint32_t d2 = fuse ? b2 ^ tm2 : 0u;
              const uint32_t d2lo = d2 & lmask & ~bsl, d2c = fuse ? to_c(d2) : 0u;
              const bool same_row = d2lo == 0;
              const uint32_t piv = same_row ? (d2c & (0u - d2c)) : (d2lo & (0u - d2lo));
              const int pb = __ffs(piv) - 1;
              const uint32_t nq = !fuse ? npairs : same_row ? npairs : npairs >> 1;
              // stored index of row A of iteration q (pivot bit clear when the
              // two rows differ)
              auto row_a = [&](uint32_t q) {
                if (!fuse || same_row) return s < dm ? ins0(q, s) : q;
                if (s < dm) return ins0(ins0(q, min((int)s, pb)), max((int)s, pb));
                return ins0(q, pb);
              };
              auto sigma = [&](uint32_t c) { return (__popc((c | bsc) & smc) & 1) ? (R)-1 : (R)1; };
              if (G == 1 && fuse) {
                // one lane walks c and c ^ d2c in step over the stored pairs
                // at lo and lo ^ d2lo, writing both outputs and summing them
                // (the cooperative tiers leave the sums to the next
                // measurement's own streaming reduction, which they run faster)
                const cpx<R> f2 = fac(d2c), g2 = fac(d2c ^ dc);
                const R sg2 = sigma(d2c);
                // a plain loop over the steps (unrolled, the two walks would
                // cost the kernel its occupancy); beta[t] by selection
                auto beta_at = [&](int t) {
                  // constant indices only: a loop here would leave beta in memory
                  static_assert(ND == 4, "four deferred factors");
                  const cpx<R> b01 = t == 1 ? beta[1] : beta[0];
                  const cpx<R> b23 = t == 3 ? beta[3] : beta[2];
                  return t >= 2 ? b23 : b01;
                };
                auto step_d = [&](cpx<R>& x, cpx<R>& y, int t, bool nb, uint32_t off) {
                  const cpx<R> bt = beta_at(t);
                  const bool xb = nb ^ ((off >> t) & 1u);
                  x = cmul(x, bt.re, xb ? bt.im : -bt.im);
                  const bool yb = xb ^ ((dc >> t) & 1u);
                  const R sg = ((smc >> t) & 1u) ? (R)-1 : (R)1;
                  y = cmul(y, sg * bt.re, yb ? sg * bt.im : -sg * bt.im);
                };
                const uint32_t nc = 1u << dfr;
                for (uint32_t q = G == 1 ? 0u : (uint32_t)grp.tid; q < nq; q += st) {
                  const uint32_t la = row_a(q);
                  const uint32_t lb = la ^ d2lo;
                  cpx<R> xa = vec[la];
                  cpx<R> ya = partner_lo(vec[la ^ dlo], la);
                  cpx<R> xb = vec[lb];
                  cpx<R> yb = partner_lo(vec[lb ^ dlo], lb);
                  ya = cmul(ya, sg0 * g0.re, sg0 * g0.im);
                  xb = cmul(xb, f2.re, f2.im);
                  yb = cmul(yb, sg2 * g2.re, sg2 * g2.im);
                  for (uint32_t j = 0; j < nc; j++) {
                    const uint32_t c = j ^ (j >> 1);
                    if (j) {
                      const int t = __builtin_ctz(j);
                      const bool nb = (c >> t) & 1u;
                      step_d(xa, ya, t, nb, 0u);
                      step_d(xb, yb, t, nb, d2c);
                    }
                    if ((c & bsc) || (same_row && (c & piv))) continue;  // a partner, or emitted from its pair
                    const uint32_t oa = oidx(la, c), ob = oidx(lb, c ^ d2c);
                    const cpx<R> va = out1(xa, ya), vb = out1(xb, yb);
                    dst[oa] = va;
                    dst[ob] = vb;
                    const bool a0 = !(oa & b2);
                    branch_sums(nx, a0 ? va : vb, partner2(a0 ? vb : va, (a0 ? oa : ob) | b2), n0, n1);
                  }
                }
                fused_sums = true;
              } else {
                auto walk = [&](auto DT) {
                  constexpr int D = decltype(DT)::value;
                  for (uint32_t q = G == 1 ? 0u : (uint32_t)grp.tid; q < npairs; q += st) {
                    const uint32_t lo = s < dm ? ins0(q, s) : q;
                    cpx<R> av = vec[lo];
                    cpx<R> pv = partner_lo(vec[lo ^ dlo], lo);
                    pv = cmul(pv, sg0 * g0.re, sg0 * g0.im);
                    auto put_out = [&](uint32_t c) {
                      if (c & bsc) return;
                      dst[oidx(lo, c)] = out1(av, pv);
                    };
                    put_out(0);
#pragma unroll
                    for (int j = 1; j < (1 << D); j++) {
                      const int t = __builtin_ctz(j);
                      const uint32_t c = (uint32_t)(j ^ (j >> 1));
                      step(av, pv, t, (c >> t) & 1u, 0u);
                      put_out(c);
                    }
                  }
                };
                if (dfr == 1) walk(IntC<1>{});
                else if (dfr == 2) walk(IntC<2 <= ND ? 2 : 1>{});
                else if (dfr == 3) walk(IntC<3 <= ND ? 3 : 1>{});
                else walk(IntC<4 <= ND ? 4 : 1>{});
              }
              dfr = 0;
            } else if (kPair && joint2) {
              // outputs by quads of the next two measurements, summed as
              // they are written
              PairWalk E = pair_walk(in, PP_SINGLE_JOINT);
              double jt[4] = {0, 0, 0, 0};
              for (uint32_t q = (uint32_t)grp.tid; q < (half >> 2); q += st, E.next()) {
                uint32_t o[4], u2i;
                pair_quad(E.cur(), k - 1, pm2, pm3, o, u2i);
                cpx<R> y[4];
#pragma unroll
                for (int e = 0; e < 4; e++) y[e] = one(o[e]);
#pragma unroll
                for (int e = 0; e < 4; e++) dst[o[e]] = y[e];
                pair_sums(y, o, u2i, pm2, pm3, jt);
              }
              pj00 = grp.sum(jt[0], red);
              pj01 = grp.sum(jt[1], red);
              pj10 = grp.sum(jt[2], red);
              pj11 = grp.sum(jt[3], red);
              pj_new = true;
            } else if (fuse) {
              // outputs (j0, j1): the next measurement's pair through its own
              // folded passes, summed as it is written
              constexpr int UP = U >= 2 ? U / 2 : 1;
              const uint32_t n2 = half >> 1;
              // j0 (bit s2 clear) in line-complete order on the cooperative
              // tiers: each group of lanes reads whole lines through both
              // partner masks (m of this measurement, m2 of the next)
              LineEnum E{};
              if constexpr (kLine) {
                const uint32_t m2 = b2 ^ tm2;
                auto sig_inv = [&](uint32_t x) { return s == top ? x : ((x & ~tb) | (((x >> top) & 1u) << s)); };
                constexpr int LB = kLineBits<R>();
                uint32_t cand[LB + 2];
                uint32_t inc = 0;
#pragma unroll
                for (int b = 0; b < LB; b++) {
                  cand[b] = (b != (int)s && b != (int)s2 && b < top) ? 1u << b : 0u;
                  inc |= cand[b];
                }
                cand[LB] = 0u;
                if ((int)s < LB && (tm & ~inc)) {
                  uint32_t x = sig_inv(tm & ~inc);
                  if ((x >> s2) & 1u) x ^= m2;
                  cand[LB] = x;
                }
                cand[LB + 1] = 0u;
                if (s2 != s && (int)s2 < LB) {
                  const uint32_t sm2 = s == top ? m2 : ((m2 & ~bs) | (((m2 >> s) & 1u) << top));
                  cand[LB + 1] = sig_inv((sm2 ^ b2) & ~inc);
                }
                E = line_enum(cand, s2);
                E.bind((uint32_t)grp.tid);
              }
              for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n2; base += UP * st) {
                uint32_t j0[UP];
                cpx<R> y0[UP], y1[UP];
#pragma unroll
                for (int u = 0; u < UP; u++) {
                  const uint32_t q = base + u * st;
                  if constexpr (kLine) j0[u] = E(q < n2 ? q : base);
                  else j0[u] = ins0(q < n2 ? q : base, s2);
                  if (q < n2) {
                    y0[u] = one(j0[u]);
                    y1[u] = one((j0[u] | b2) ^ tm2);
                  }
                }
#pragma unroll
                for (int u = 0; u < UP; u++)
                  if (base + u * st < n2) {
                    dst[j0[u]] = y0[u];
                    dst[(j0[u] | b2) ^ tm2] = y1[u];
                    branch_sums(nx, y0[u], partner2(y1[u], j0[u] | b2), n0, n1);
                  }
              }
              fused_sums = true;
            } else {
              // outputs in line-complete order on the cooperative tiers
              LineEnum E{};
              if constexpr (kLine) {
                auto sig_inv = [&](uint32_t x) { return s == top ? x : ((x & ~tb) | (((x >> top) & 1u) << s)); };
                constexpr int LB = kLineBits<R>();
                uint32_t cand[LB + 1];
                uint32_t inc = 0;
#pragma unroll
                for (int b = 0; b < LB; b++) {
                  cand[b] = (b != (int)s && b < top) ? 1u << b : 0u;
                  inc |= cand[b];
                }
                cand[LB] = (int)s < LB ? sig_inv(tm & ~inc) : 0u;
                E = line_enum(cand, -1);
                E.bind((uint32_t)grp.tid);
              }
              pass1_to<G, R, U>(grp, dst, half,
                                [&](uint32_t p) -> uint32_t {
                                  if constexpr (kLine) return E(p);
                                  else return p;
                                },
                                one);
            }
            if (!(kPair && pmode == 1)) {
              cpx<R>* t = vec.base;
              vec.base = alt;
              alt = t;
            }
          } else {
            // in place (on-chip vectors; folded passes are never skipped here,
            // so only a directly following measurement is fused): the kept
            // half (or fold) is written in place; the top slot k-1 takes the
            // place of slot s (no hazard: every thread owns its outputs and
            // reads only them and the elements above them)
            const bool fuse_here = fuse && tm2 == 0 && sm2 == 0 && !as2;
            if (fuse_here && s == top) {
              constexpr int UP = U >= 4 ? U / 4 : 1;
              const uint32_t n2 = half >> 1;
              for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n2; base += UP * st) {
                uint32_t oo[UP];
                cpx<R> x0[UP], x1[UP], y0[UP], y1[UP];
#pragma unroll
                for (int u = 0; u < UP; u++) {
                  const uint32_t q = base + u * st;
                  oo[u] = ins0(q < n2 ? q : base, s2);
                  if (q < n2) {
                    x0[u] = vec[oo[u]];
                    x1[u] = vec[oo[u] | tb];
                    y0[u] = vec[oo[u] | b2];
                    y1[u] = vec[oo[u] | b2 | tb];
                  }
                }
#pragma unroll
                for (int u = 0; u < UP; u++)
                  if (base + u * st < n2) {
                    const cpx<R> lo = out1(x0[u], x1[u]), hi = out1(y0[u], y1[u]);
                    vec[oo[u]] = lo;
                    vec[oo[u] | b2] = hi;
                    branch_sums(nx, lo, hi, n0, n1);
                  }
              }
              fused_sums = true;
            } else if (fuse_here && s2 != s) {
              // four outputs {o, o|bs, o|b2, o|bs|b2} from eight inputs (new
              // bit s of an output is the former top bit of its inputs); the
              // next axis pairs (o, o|b2) and (o|bs, o|bs|b2)
              const uint32_t n4 = half >> 2;
              const int lo_b = min((int)s, (int)s2), hi_b = max((int)s, (int)s2);
              for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n4; base += st) {
                const uint32_t o = ins0(ins0(base, lo_b), hi_b);
                const cpx<R> i0 = vec[o], i1 = vec[o | bs], i2 = vec[o | tb], i3 = vec[o | tb | bs];
                const cpx<R> i4 = vec[o | b2], i5 = vec[o | b2 | bs], i6 = vec[o | b2 | tb], i7 = vec[o | b2 | tb | bs];
                const cpx<R> r0 = out1(i0, i1), r1 = out1(i2, i3), r2 = out1(i4, i5), r3 = out1(i6, i7);
                vec[o] = r0;
                vec[o | bs] = r1;
                vec[o | b2] = r2;
                vec[o | bs | b2] = r3;
                branch_sums(nx, r0, r2, n0, n1);
                branch_sums(nx, r1, r3, n0, n1);
              }
              fused_sums = true;
            } else if (s == top) {
              pass21<G, R, U>(grp, vec, half,
                              [&](uint32_t q, uint32_t& r0, uint32_t& r1, uint32_t& w) { r0 = w = q; r1 = q | bs; },
                              [&](cpx<R> a, cpx<R> c) { return out1(a, c); });
            } else {
              // pair (j0, j1 = j0 | bs) of outputs reads its own two elements
              // and the two above them in the top slot
              const uint32_t n4 = half >> 1;
              for (uint32_t base = G == 1 ? 0u : (uint32_t)grp.tid; base < n4; base += U * st) {
                uint32_t jj[U];
                cpx<R> a0[U], a1[U], c0[U], c1[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                  uint32_t q = base + u * st;
                  jj[u] = ins0(q < n4 ? q : base, s);
                  if (q < n4) {
                    a0[u] = vec[jj[u]];
                    a1[u] = vec[jj[u] | bs];
                    c0[u] = vec[jj[u] | tb];
                    c1[u] = vec[jj[u] | bs | tb];
                  }
                }
#pragma unroll
                for (int u = 0; u < U; u++)
                  if (base + u * st < n4) {
                    const cpx<R> lo = out1(a0[u], a1[u]), hi = out1(c0[u], c1[u]);
                    vec[jj[u]] = lo;
                    vec[jj[u] | bs] = hi;
                    // next axis == s: the two outputs are its pair
                    if (fuse_here) branch_sums(nx, lo, hi, n0, n1);
                  }
              }
              fused_sums = fuse_here;
            }
          }
          pend_tm = pend_sm = 0;
          pend_as = false;
          carry_valid = fused_sums;
          pj_valid = pj_new;
          if (fused_sums) {
            carry0 = grp.sum(n0, red);
            carry1 = grp.sum(n1, red);
          }
          k--;
          grp.sync();
          g_nexp = 0;  // the kept branch is normalised
          if constexpr (VONLY) {
            mb[in.a >> 6] |= (uint64_t)mm << (in.a & 63);
          } else {
            if (isx) { g_h(v); frame_h<W>(T, v); frame_h<W>(N, v); }
            if constexpr (DBG) g_ipow += 2 * (int)(b & getbit<W>(T.z, v));
            xorbit<W>(T.x, v, b);
          }
          last_m = mm;
          last_pn = pn;
          int r = as_const(P.ev_rec)[j];
          if (r >= 0) put((uint32_t)r, mm);
          }
          break;
        }
        case OP_CPAULI: {
          uint64_t px[W], pz[W], zero[W];
#pragma unroll
          for (int w = 0; w < W; w++) {
            px[w] = masks[in.a + w];
            pz[w] = masks[in.a + W + w];
            zero[w] = 0;
          }
          uint64_t mm = 0ull - (uint64_t)last_m, mp = 0ull - (uint64_t)last_pn;
          uint64_t ax[W], az[W], bx[W], bz[W];
#pragma unroll
          for (int w = 0; w < W; w++) {
            ax[w] = px[w] & mm; az[w] = pz[w] & mm;
            bx[w] = px[w] & mp; bz[w] = pz[w] & mp;
          }
          (void)zero;
          if constexpr (DBG) {
            // X^m of the reset: the signed image E = (-1)^r i^|ex & ez| X^ex Z^ez
            if (last_m) {
              int e = 2 * (int)(in.flags & F_SIGN);
#pragma unroll
              for (int w = 0; w < W; w++) e += __popcll(px[w] & pz[w]) + 2 * __popcll(pz[w] & T.x[w]);
              g_ipow += e;
            }
          }
          frame_xor<W>(T, ax, az);
          frame_xor<W>(N, bx, bz);
          break;
        }
        case OP_EXPVAL: {
          // <psi|P|psi> (expectation-value probe): with the virtual observable
          // g = U_C^dagger P U_C, the Pauli frame contributes (-1)^c (its
          // commutation with g), and g acts on the active vector through its
          // letters on active slots (Z on a dormant |0> is 1; X there gives 0):
          // <phi|g_A|phi> / <phi|phi>, summed in FP64
          uint64_t gx[W], gz[W];
#pragma unroll
          for (int w = 0; w < W; w++) {
            gx[w] = masks[in.a + w];
            gz[w] = masks[in.a + W + w];
          }
          const uint32_t c = parity_and<W>(T.x, gz) ^ parity_and<W>(T.z, gx) ^ (uint32_t)(in.flags & F_SIGN);
          double e = 0;
          if (!(in.flags & F_ZERO)) {
            if constexpr (VEC) {
              materialize();
              const uint32_t xm = (uint32_t)masks[in.a + 2 * W], zm = (uint32_t)masks[in.a + 2 * W + 1];
              double sre = 0, sim = 0, nrm = 0;
              FOR_GROUP(i, (1u << k)) {
                const cpx<R> a = vec[i], b = vec[i ^ xm];
                // conj(a) * (-1)^{|(i ^ xm) & zm|} * b
                const double sg = (__popc((i ^ xm) & zm) & 1) ? -1.0 : 1.0;
                sre += sg * ((double)a.re * b.re + (double)a.im * b.im);
                sim += sg * ((double)a.re * b.im - (double)a.im * b.re);
                nrm += norm2(a);
              }
              sre = grp.sum(sre, red);
              sim = grp.sum(sim, red);
              nrm = grp.sum(nrm, red);
              // times i^{|xm & zm|} (one i per Y letter), real part
              const int ny = __popc(xm & zm) & 3;
              const double re = ny == 0 ? sre : ny == 1 ? -sim : ny == 2 ? -sre : sim;
              e = re / nrm;
            } else {
              e = 1.0;  // k_max = 0: the active vector is [1] and g has no X support
            }
          }
          if (A.expval && writer()) A.expval[(size_t)in.b * A.shots + local] = c ? -e : e;
          break;
        }
        case OP_CFEED: {
          // feed-forward Pauli (Appendix B.3) on the full frame when record b
          // of this shot is 1; the noise frame only follows physical faults
          uint32_t m;
          if constexpr (G == 1) {
            m = (uint32_t)(rec[in.b] >> (threadIdx.x & 63)) & 1u;
          } else {
            grp.sync();  // the record bit is staged by the group's first thread
            m = (uint32_t)(rec[in.b] >> slane) & 1u;
          }
          if (m) {
            uint64_t px[W], pz[W];
#pragma unroll
            for (int w = 0; w < W; w++) {
              px[w] = masks[in.a + w];
              pz[w] = masks[in.a + W + w];
            }
            if constexpr (DBG) {
              int e = 2 * (int)(in.flags & F_SIGN);
#pragma unroll
              for (int w = 0; w < W; w++) e += __popcll(px[w] & pz[w]) + 2 * __popcll(pz[w] & T.x[w]);
              g_ipow += e;
            }
            frame_xor<W>(T, px, pz);
          }
          break;
        }
        case OP_NOISE: {
          if constexpr (DBG) {
            if (A.forced_faults) {
              for (uint32_t st = in.a; st < in.b; st++) {
                int o = local < A.shots ? A.forced_faults[local * P.nsites + st] : -1;
                if (o >= 0) {
                  g_ipow += fault_phase<W>(P, T.x, st, (uint32_t)o);
                  apply_fault<W>(P, T, N, st, (uint32_t)o);
                }
              }
              break;
            }
          }
          const uint32_t hi = in.b;
          if constexpr (kExt) {
            if (A.strat_r >= 0) {
              // stratified: the faults come in site order, no chunks
              while (ns.nf < hi) {
                if constexpr (DBG) g_ipow += fault_phase<W>(P, T.x, ns.nf, ns.nf_out);
                apply_fault<W>(P, T, N, ns.nf, ns.nf_out);
                next_fault_strat(P, ns, ns.nf + 1, shot, seed);
              }
              break;
            }
          }
          while (ns.nf < hi) {
            uint32_t cend = min((ns.chunk + 1) * (uint32_t)kChunk, (uint32_t)P.nsites);
            if (ns.nf >= cend) {
              ns.chunk++;
              ns.ord = 0;
              next_fault(P, ns, 0, shot, seed);
              continue;
            }
            if constexpr (DBG) g_ipow += fault_phase<W>(P, T.x, ns.nf, ns.nf_out);
            apply_fault<W>(P, T, N, ns.nf, ns.nf_out);
            next_fault(P, ns, ns.nf - ns.chunk * (uint32_t)kChunk + 1, shot, seed);
          }
          break;
        }
        case OP_DET: {
          uint32_t d = xor_refs(in.a, in.u);
          put((uint32_t)P.nrec + in.b, d);
          break;
        }
        case OP_EMIT:
        case OP_MACTF: {
          // frame-only stream of the split form on the shot-per-lane tier
          // (frames too wide for the bit-sliced kernel's LDS rows)
          if constexpr (G == 1 && !VEC) {
            const uint64_t words = (A.shots + 63) / 64;
            const uint32_t lane = threadIdx.x & 63;
            uint64_t* row = A.nbits + (size_t)in.u * words + (local >> 6);
            if (in.op == OP_EMIT) {
              const uint64_t wb = __ballot(getbit<W>(T.x, v));
              if (lane == 0) row[0] = wb;
              break;
            }
            const bool isx = (in.flags & F_XMEAS) != 0;
            const uint32_t p = isx ? getbit<W>(T.z, v) : getbit<W>(T.x, v);
            const uint32_t pn = isx ? getbit<W>(N.z, v) : getbit<W>(N.x, v);
            const uint64_t wp = __ballot(p), wn = __ballot(pn);
            if (lane == 0) {
              row[0] = wp;
              row[words] = wn;
            }
            if (isx) {
              frame_h<W>(T, v);
              frame_h<W>(N, v);
            }
            xorbit<W>(T.x, v, getbit<W>(T.x, v) ^ (uint32_t)(in.flags & F_SIGN));  // x_v = sign
            last_m = 0;
            last_pn = pn;
            const int r = as_const(P.ev_rec)[in.b];
            if (r >= 0) put((uint32_t)r, 0u);
          }
          break;
        }
        case OP_OBS: {
          uint32_t d = xor_refs(in.a, in.u);
          uint32_t r = (uint32_t)P.nrec + (uint32_t)P.ndet + in.b;
          if constexpr (G == 1) {
            uint64_t word = __ballot(d && !(kExt && post_dead));
            if ((threadIdx.x & 63) == 0) rec[r] ^= word;
          } else {
            if (grp.tid == 0) rec[r] ^= (uint64_t)d << slane;
          }
          break;
        }
        default:
          // post-selection (Section 3.2): the detector is recorded, then a
          // shot reading 1 ends here with its observables cleared (records
          // not yet written stay 0).  Only the EXT kernels have this path;
          // programs holding OP_POSTSELECT run on them alone.
          if constexpr (kExt) {
            if (in.op == OP_POSTSELECT) {
              if constexpr (G > 1) grp.sync();  // record bits are staged by the group's first thread
              const uint32_t d = xor_refs(in.a, in.u);
              put((uint32_t)P.nrec + in.b, d);
              const uint32_t r0 = (uint32_t)(P.nrec + P.ndet);
              if constexpr (G == 1) {
                const uint64_t rej = __ballot(d && !post_dead);
                if (rej && (threadIdx.x & 63) == 0)
                  for (uint32_t o = 0; o < (uint32_t)P.nobs; o++) rec[r0 + o] &= ~rej;
                post_dead = post_dead || d;
              } else {
                if (rfl(d)) {  // one shot per group: the same value in every wave
                  if (grp.tid == 0)
                    for (uint32_t o = 0; o < (uint32_t)P.nobs; o++) rec[r0 + o] &= ~(1ull << slane);
                  goto done;
                }
              }
            }
          }
          break;
      }
    }
  done:
    if constexpr (DBG) {
      if (A.gamma_out && writer()) {
        const double sc = exp2(-0.5 * (double)g_nexp);
        const int e = g_ipow & 3;
        // i^e (g_re + i g_im) 2^{-n/2}
        const double re = e == 0 ? g_re : e == 1 ? -g_im : e == 2 ? -g_re : g_im;
        const double im = e == 0 ? g_im : e == 1 ? g_re : e == 2 ? -g_im : -g_re;
        A.gamma_out[local * 2] = re * sc;
        A.gamma_out[local * 2 + 1] = im * sc;
      }
      if (A.phi_out && local < A.shots && P.kmax == 0) {
        // no active vector exists: the state is the trivial [1]
        if (writer()) {
          A.phi_out[local * 2] = 1.0;
          A.phi_out[local * 2 + 1] = 0.0;
        }
      } else if (VEC && A.phi_out && local < A.shots && !(kExt && post_dead)) {
        if constexpr (OOP) materialize();
        // final active vector (its length 2^k is program-determined)
        FOR_GROUP(p, (1u << k)) {
          cpx<R> a = vec[p];
          A.phi_out[(local << P.kmax) * 2 + 2 * p] = (double)a.re;
          A.phi_out[(local << P.kmax) * 2 + 2 * p + 1] = (double)a.im;
        }
      }
    }
    grp.sync();
  }
};

// ------------------------------------------------------------------ kernel
// One persistent launch: units (lanes-of-a-wave for G = 1, waves for G = 64,
// workgroups for G = 256) take 64-shot tiles round-robin.
template <int W, int G, typename R, bool GLOBAL, bool DBG, bool VEC, bool VONLY = false, bool EXT = false,
          bool PAIR = false>
__global__ __launch_bounds__(256) void k_sample(DevProgram P, KArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int units_per_block = G == 256 ? 1 : 4;
  const int unit_in_block = G == 256 ? 0 : (int)rfl(threadIdx.x >> 6);
  const uint64_t unit = (uint64_t)blockIdx.x * units_per_block + unit_in_block;
  const uint64_t nunits = (uint64_t)gridDim.x * units_per_block;
  const uint32_t nwords_rec = (uint32_t)(P.nrec + P.ndet + P.nobs);
  const uint32_t rec_stride = (nwords_rec + 1) & ~1u;  // keep 16-byte alignment
  uint64_t* rec = (uint64_t*)smem + (size_t)unit_in_block * rec_stride;
  unsigned char* after_rec = smem + (size_t)units_per_block * rec_stride * 8;
  double* red = (double*)after_rec;
  cpx<R>* arr_lds = (cpx<R>*)(after_rec + 64);
  const size_t vec_elems = (size_t)1 << P.kmax;
  cpx<R>* base;
  cpx<R>* alt = nullptr;
  if constexpr (GLOBAL) {
    // two buffers per unit (active measurements collapse from one into the other)
    const size_t per = vec_elems * (G == 1 ? 64 : 1);
    base = (cpx<R>*)A.workspace + unit * per * 2;
    alt = base + per;
  } else {
    base = arr_lds + (size_t)unit_in_block * vec_elems * (G == 1 ? 64 : 1);
  }
  const int lane = threadIdx.x & 63;
  const int tid = G == 256 ? (int)threadIdx.x : lane;
  const uint64_t ntiles = (A.shots + 63) / 64;
  const uint64_t words = ntiles;
  if constexpr (G > 1) {
    // One shot per workgroup (G = 256) or per wave (G = 64): shots (not
    // tiles) are spread over the units so that small shot counts still fill
    // the device; record bits are staged per shot (bit 0) and ORed into the
    // zero-filled outputs.
    auto unit_sync = [] {
      if constexpr (G == 256) __syncthreads();
      else { __builtin_amdgcn_wave_barrier(); __atomic_signal_fence(__ATOMIC_SEQ_CST); }
    };
    for (uint64_t sh_i = unit; sh_i < A.shots; sh_i += nunits) {
      for (uint32_t r = (uint32_t)tid; r < nwords_rec; r += G) rec[r] = 0;
      unit_sync();
      uint64_t g = rfl((uint32_t)sh_i) | (sh_i & 0xFFFFFFFF00000000ull);
      Shot<W, G, R, DBG, VEC, unroll_for<R, GLOBAL>(), GLOBAL, VONLY, EXT, true, PAIR> sh{P, A, Group<G>{tid}, Vec<G, R>{base, lane}, rec, red, 0,
                                                                  A.offset + g, g, alt};
      sh.run();
      unit_sync();
      const uint64_t bit = 1ull << (g & 63);
      const size_t word = (size_t)(g >> 6);
      for (uint32_t r = (uint32_t)tid; r < nwords_rec; r += G) {
        if (!(rec[r] & 1ull)) continue;
        uint64_t* dst;
        if (r < (uint32_t)P.nrec) dst = A.meas ? A.meas + (size_t)r * words + word : nullptr;
        else if (r < (uint32_t)(P.nrec + P.ndet)) dst = A.det ? A.det + (size_t)(r - P.nrec) * words + word : nullptr;
        else dst = A.obs ? A.obs + (size_t)(r - P.nrec - P.ndet) * words + word : nullptr;
        if (dst) atomicOr((unsigned long long*)dst, (unsigned long long)bit);
      }
      unit_sync();
    }
    return;
  }
  for (uint64_t tile = unit; tile < ntiles; tile += nunits) {
    for (uint32_t r = (uint32_t)tid; r < nwords_rec; r += 64) rec[r] = 0;
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if constexpr (G == 1) {
      Shot<W, G, R, DBG, VEC, unroll_for<R, GLOBAL>(), GLOBAL, VONLY, EXT, true, PAIR> sh{P, A, Group<G>{tid}, Vec<G, R>{base, lane}, rec, red, lane,
                                                                  A.offset + tile * 64 + lane, tile * 64 + lane, alt};
      sh.run();
    } else {
      uint32_t nsh = (uint32_t)min((uint64_t)64, A.shots - tile * 64);
      for (uint32_t sl = 0; sl < nsh; sl++) {
        uint64_t g = rfl((uint32_t)(tile * 64 + sl)) | ((tile * 64 + sl) & 0xFFFFFFFF00000000ull);
        Shot<W, G, R, DBG, VEC, unroll_for<R, GLOBAL>(), GLOBAL, VONLY, EXT, true, PAIR> sh{P, A, Group<G>{tid}, Vec<G, R>{base, lane}, rec, red,
                                                                    (int)sl, A.offset + g, g, alt};
        sh.run();
      }
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // flush the tile's record words (bits of shots beyond the end cleared)
    const uint64_t nvalid = min((uint64_t)64, A.shots - tile * 64);
    const uint64_t vmask = nvalid == 64 ? ~0ull : ((1ull << nvalid) - 1ull);
    for (uint32_t r = (uint32_t)tid; r < nwords_rec; r += 64) {
      uint64_t v = rec[r] & vmask;
      if (r < (uint32_t)P.nrec) {
        if (A.meas) A.meas[(size_t)r * words + tile] = v;
      } else if (r < (uint32_t)(P.nrec + P.ndet)) {
        if (A.det) A.det[(size_t)(r - P.nrec) * words + tile] = v;
      } else {
        if (A.obs) A.obs[(size_t)(r - P.nrec - P.ndet) * words + tile] = v;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
}

// ------------------------------------------------------------------ dispatch table
template <int W, int G, typename R, bool GLOBAL, bool DBG, bool VEC, bool VONLY = false, bool EXT = false,
          bool PAIR = false>
inline hipError_t launch_one(const DevProgram& P, const KArgs& A, int grid, size_t lds, hipStream_t st) {
  static bool attr = false;  // allow the whole 160 KB of LDS for dynamic use
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sample<W, G, R, GLOBAL, DBG, VEC, VONLY, EXT, PAIR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_sample<W, G, R, GLOBAL, DBG, VEC, VONLY, EXT, PAIR>), dim3(grid), dim3(256), lds, st, P, A);
  return hipGetLastError();
}

// The vector-only stream of the split form (no frames: W = 1).
template <typename R>
inline hipError_t launch_vonly(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  if (L.G == 1) {
    if (L.global_vec) return launch_one<1, 1, R, true, false, true, true>(P, A, L.grid, L.lds_bytes, st);
    return launch_one<1, 1, R, false, false, true, true>(P, A, L.grid, L.lds_bytes, st);
  }
  if (L.G == 64) {
    if (L.global_vec) return launch_one<1, 64, R, true, false, true, true>(P, A, L.grid, L.lds_bytes, st);
    return launch_one<1, 64, R, false, false, true, true>(P, A, L.grid, L.lds_bytes, st);
  }
  if (L.global_vec) return launch_one<1, 256, R, true, false, true, true>(P, A, L.grid, L.lds_bytes, st);
  return launch_one<1, 256, R, false, false, true, true>(P, A, L.grid, L.lds_bytes, st);
}

template <int G, typename R, bool GLOBAL, bool DBG, bool VEC = true, bool EXT = false, bool PAIR = false>
inline hipError_t launch_w(const DevProgram& P, const KArgs& A, int grid, size_t lds, hipStream_t st) {
  switch (P.W) {
    case 1: return launch_one<1, G, R, GLOBAL, DBG, VEC, false, EXT, PAIR>(P, A, grid, lds, st);
    case 2: return launch_one<2, G, R, GLOBAL, DBG, VEC, false, EXT, PAIR>(P, A, grid, lds, st);
    case 3: return launch_one<3, G, R, GLOBAL, DBG, VEC, false, EXT, PAIR>(P, A, grid, lds, st);
    case 4: return launch_one<4, G, R, GLOBAL, DBG, VEC, false, EXT, PAIR>(P, A, grid, lds, st);
  }
  return hipErrorInvalidValue;
}

// EXT: the instantiations with post-selection and stratified sampling
// (sample_ext_*.hip), for programs and calls that use them.  The
// cooperative HBM tiers of plain sampling take the instantiation with paired
// collapses only for programs that pair some measurements at this precision
// (DevProgram::has_pairs): compiled in, the pair code alone costs the
// interpreter up to 15% on programs that never use it.  The trace kernels
// always have it.
template <typename R, bool DBG, bool EXT = false>
inline hipError_t launch_g(const DevProgram& P, const KArgs& A, const LaunchShape& L, hipStream_t st) {
  if (L.G == 1) {
    // Pauli-frame-only programs get an instantiation without any active-vector code
    if (P.kmax == 0) return launch_w<1, R, false, DBG, false, EXT>(P, A, L.grid, L.lds_bytes, st);
    if (L.global_vec) return launch_w<1, R, true, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
    return launch_w<1, R, false, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
  }
  constexpr bool kPairs = !EXT;
  const bool pairs = DBG || P.has_pairs[sizeof(R) == 8 ? 1 : 0] != 0;
  if (L.G == 64) {
    if (L.global_vec) {
      if (kPairs && pairs) return launch_w<64, R, true, DBG, true, EXT, kPairs>(P, A, L.grid, L.lds_bytes, st);
      if constexpr (!DBG) return launch_w<64, R, true, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
    }
    return launch_w<64, R, false, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
  }
  if (L.global_vec) {
    if (kPairs && pairs) return launch_w<256, R, true, DBG, true, EXT, kPairs>(P, A, L.grid, L.lds_bytes, st);
    if constexpr (!DBG) return launch_w<256, R, true, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
  }
  return launch_w<256, R, false, DBG, true, EXT>(P, A, L.grid, L.lds_bytes, st);
}

}  // namespace clifft
