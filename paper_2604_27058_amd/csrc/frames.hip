// Bit-sliced Pauli-frame kernel for programs without an active vector
// (k_max = 0): 32 shots per lane, one LDS row per frame bit.
#include "shot.h"

namespace clifft {

// ------------------------------------------------------------------ bit-sliced frames
// Pauli-frame-only programs (k_max = 0): every lane carries 32 shots, one bit
// per shot, so a frame bit of one virtual qubit for the 64 x 32 shots of a
// wave is one 256-byte LDS row (lane l owns word l: conflict free).  Frame
// instructions become a few word operations per touched qubit for 2048
// shots; dispatch is paid once per 2048 shots.  The stochastic contract is
// the per-shot one of the other kernels (each shot keeps its own gap-sampler
// cursor), so records are identical.
constexpr int kShotsPerLane = 32;

struct FrameRows {
  uint32_t* base;  // LDS rows of 64 words
  int lane;
  __device__ uint32_t& operator()(uint32_t row) const { return base[row * 64u + (uint32_t)lane]; }
};

// first fault at or after local index cur of `chunk` for one shot; returns
// the absolute site (chunk end when none) and advances *ord
template <bool LDS_SURV>
DEV uint32_t bs_next_fault(const DevProgram& P, const double* surv_lds, uint32_t chunk, uint32_t cur, uint32_t* ord,
                           uint64_t shot, uint64_t seed, uint32_t* outcome = nullptr) {
  U4 w = draw((*ord)++, kPurposeNoise | chunk, shot, seed);
  const double* S = LDS_SURV ? surv_lds : P.surv + (size_t)chunk * (kChunk + 1);
  uint32_t len = min((uint32_t)kChunk, (uint32_t)P.nsites - chunk * (uint32_t)kChunk);
  double tau = uniform53(w) * S[cur];
  uint32_t lo = cur, hi = len;
  if (S[len] > tau) lo = len;  // no fault in the rest of the chunk (same answer as the search)
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (S[mid + 1] <= tau) hi = mid;
    else lo = mid + 1;
  }
  const uint32_t nf = chunk * (uint32_t)kChunk + lo;
  if (outcome && lo < len) {
    const uint64_t w64 = ((uint64_t)w.w3 << 32) | w.w2;
    *outcome = (uint32_t)__umul64hi(w64, (uint64_t)nout_of(P.site_type[nf]));
  }
  return nf;
}

template <int W>
DEV void bs_apply_fault(const DevProgram& P, const FrameRows& F, uint32_t N, uint32_t site, uint32_t o, uint32_t bit) {
  uint32_t t = P.site_type[site];
  const uint64_t* img = P.masks + P.site_img[site];
  uint32_t la, lb = 0;
  if (t == S_DEP1) la = o + 1;
  else if (t == S_DEP2) { la = (o + 1) >> 2; lb = (o + 1) & 3; }
  else la = t - 1;
  for (int qi = 0; qi < (t == S_DEP2 ? 2 : 1); qi++) {
    const uint32_t l = qi ? lb : la;
    const uint64_t ux = (l == 1 || l == 2) ? ~0ull : 0ull, uz = (l == 2 || l == 3) ? ~0ull : 0ull;
    const uint64_t* ix = img + (size_t)qi * 4 * W;
    const uint64_t* iz = ix + 2 * W;
    for (int w = 0; w < W; w++) {
      uint64_t ex = (ix[w] & ux) ^ (iz[w] & uz);
      uint64_t ez = (ix[W + w] & ux) ^ (iz[W + w] & uz);
      while (ex) {
        uint32_t q = (uint32_t)(w * 64 + __ffsll((unsigned long long)ex) - 1);
        ex &= ex - 1;
        F(q) ^= bit;          // full x
        F(2 * N + q) ^= bit;  // noise x
      }
      while (ez) {
        uint32_t q = (uint32_t)(w * 64 + __ffsll((unsigned long long)ez) - 1);
        ez &= ez - 1;
        F(N + q) ^= bit;      // full z
        F(3 * N + q) ^= bit;  // noise z
      }
    }
  }
}

// LDS rows: [0,4N) frames (full x, full z, noise x, noise z), then one row
// per detector and observable accumulator, then the dormant-random bit rows
// of the current 128-event block, then the lane's fault list (or per-shot
// noise cursors: site; draw ordinal | chunk << 16), then a row that stays
// zero and a row that absorbs stores of unused slots (so batched accesses
// need no branches), then the survival products when they fit.
constexpr int kSurvLdsMax = 2048;  // survival products staged in LDS (single chunk, up to this many sites)
constexpr int kListCap = 24;       // faults per lane kept in the precomputed list
constexpr size_t kStratLdsMax = 16384;  // stratified tables staged in LDS up to this many bytes
DEV_HOST_INLINE bool frames_surv_in_lds(const DevProgram& P) { return P.nchunks == 1 && P.nsites < kSurvLdsMax; }
// Low-noise programs precompute each lane's faults into a site-sorted list
// (expected faults per lane at most a quarter of the list; stratified: all
// 32 shots' faults fit the list); others keep one sampler cursor per shot.
DEV_HOST_INLINE bool frames_fault_list(const DevProgram& P, int strat_r) {
  if (strat_r >= 0) return P.nsites < (1 << 23) && strat_r * kShotsPerLane <= kListCap;
  return P.nsites < (1 << 23) && (double)P.exp_faults * kShotsPerLane <= kListCap / 4;
}
// Stratified tables e_1 .. e_r (nsites + 1 doubles each) staged in LDS.
DEV_HOST_INLINE bool frames_strat_in_lds(const DevProgram& P, int strat_r) {
  return strat_r > 0 && (size_t)strat_r * (size_t)(P.nsites + 1) * 8 <= kStratLdsMax;
}
DEV_HOST_INLINE size_t frames_surv_rows(const DevProgram& P) {
  return frames_surv_in_lds(P) ? ((size_t)(P.nsites + 1) * 8 + 255) / 256 : 0;  // doubles, in 256-byte rows
}
size_t frames_lds_rows(const DevProgram& P, int strat_r) {
  size_t rows = (size_t)4 * P.nq + P.ndet_rows + P.nobs + (P.rblk_max > 0 ? P.rblk_max : 1);
  rows += frames_fault_list(P, strat_r) ? kListCap : 2 * kShotsPerLane;
  rows += 2;  // zero row, dump row
  rows += frames_surv_rows(P);
  if (frames_strat_in_lds(P, strat_r)) rows += ((size_t)strat_r * (P.nsites + 1) * 8 + 255) / 256;
  return rows;
}

// Up to four set bits of a wave-uniform mask word (qubit wbase + bit),
// removed from m; returns how many.
MDEV int take4(uint64_t& m, uint32_t wbase, uint32_t (&q)[4]) {
  int n = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    q[i] = m ? wbase + (uint32_t)__ffsll((unsigned long long)m) - 1 : 0u;
    n += m ? 1 : 0;
    m &= m - 1;
  }
  return n;
}

// EXT: post-selection and stratified sampling compiled in.
template <int W, bool LDS_SURV, bool LIST, bool EXT>
__global__ __launch_bounds__(64) void k_frames(DevProgram P, KArgs A) {
  extern __shared__ __align__(16) uint32_t sm[];
  const int lane = threadIdx.x;
  const uint32_t N = (uint32_t)P.nq;
  const FrameRows F{sm, lane};
  const uint32_t ACC = 4 * N, RB = ACC + (uint32_t)(P.ndet_rows + P.nobs);
  // LIST: rows [NF, NF + kListCap) hold the fault list; otherwise per-shot
  // cursors: next fault site at NF + s, draw ordinal | chunk << 16 at OC + s
  const uint32_t NF = RB + (uint32_t)(P.rblk_max > 0 ? P.rblk_max : 1), OC = NF + kShotsPerLane;
  const uint32_t ZR = NF + (LIST ? kListCap : 2 * kShotsPerLane), DR = ZR + 1;
  double* surv = (double*)(sm + (size_t)(DR + 1) * 64);
  // stratified tables: staged after the survival products when small
  const bool strat = EXT && A.strat_r >= 0;
  const bool strat_lds = EXT && frames_strat_in_lds(P, A.strat_r);
  double* strat_tab_lds = (double*)(sm + (size_t)(DR + 1 + frames_surv_rows(P)) * 64);
  const double* stab = strat_lds ? strat_tab_lds : P.strat;
  const uint32_t NS = (uint32_t)P.nsites;
  F(ZR) = 0;
  if (LDS_SURV)
    for (int i = lane; i <= P.nsites; i += 64) surv[i] = P.surv[i];
  if (strat_lds)
    for (int i = lane; i < A.strat_r * (P.nsites + 1); i += 64) strat_tab_lds[i] = P.strat[i];
  __syncthreads();
  const uint64_t seed = A.seed;
  const uint64_t words64 = (A.shots + 63) / 64;
  const uint64_t tiles = (A.shots + 64 * kShotsPerLane - 1) / (64 * kShotsPerLane);
  uint32_t* meas32 = (uint32_t*)A.meas;
  uint32_t* det32 = (uint32_t*)A.det;
  uint32_t* obs32 = (uint32_t*)A.obs;
  uint32_t* bits32 = (uint32_t*)A.nbits;  // split form: needed-bit rows
  cptr<uint64_t> masks = as_const(P.masks);
  cptr<uint32_t> rec_tgt_off = as_const(P.rec_tgt_off), rec_tgt = as_const(P.rec_tgt);
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t s0 = tile * (64 * kShotsPerLane) + (uint64_t)lane * kShotsPerLane;  // first shot of the lane
    const uint32_t valid = s0 >= A.shots ? 0u : (A.shots - s0 >= 32 ? ~0u : ((1u << (A.shots - s0)) - 1u));
    const size_t col = (size_t)(s0 >> 5);  // 32-bit column of this lane in the record rows
    const bool store = col < 2 * words64;  // inside the buffer (bits past the last shot are written as 0)
    for (uint32_t r = 0; r < RB; r++) F(r) = 0;
    uint32_t min_nf = 0xFFFFFFFFu;
    uint32_t lcnt = 0, lhead = 0;
    const uint32_t lcap = min((uint32_t)kListCap, A.list_cap);
    bool lovf = false;
    if (LIST && P.nsites > 0) {
      // every fault of the lane's 32 shots, as (site << 9 | shot << 4 | outcome)
      for (int j = 0; j < kShotsPerLane; j++) {
        const uint64_t shot = A.offset + s0 + j;
        if (strat) {
          // stratified: exactly strat_r faults, in site order
          uint32_t cur = 0;
          for (uint32_t i = 0; i < (uint32_t)A.strat_r; i++) {
            const U4 w = draw(i, kPurposeStrat, shot, seed);
            const uint32_t nf = strat_site(stab, NS, (uint32_t)A.strat_r - i, cur, w);
            if (lcnt < lcap) F(NF + lcnt) = (nf << 9) | ((uint32_t)j << 4) | fault_outcome(P, nf, w);
            else lovf = true;
            lcnt++;
            cur = nf + 1;
          }
          continue;
        }
        for (uint32_t c = 0; c < (uint32_t)P.nchunks; c++) {
          const uint32_t cend = min((c + 1) * (uint32_t)kChunk, (uint32_t)P.nsites);
          uint32_t ord = 0, cur = 0;
          for (;;) {
            uint32_t o = 0;
            const uint32_t nf = bs_next_fault<LDS_SURV>(P, surv, c, cur, &ord, shot, seed, &o);
            if (nf >= cend) break;
            if (lcnt < lcap) F(NF + lcnt) = (nf << 9) | ((uint32_t)j << 4) | o;
            else lovf = true;
            lcnt++;
            cur = nf - c * (uint32_t)kChunk + 1;
          }
        }
      }
      const uint32_t n = min(lcnt, lcap);
      for (uint32_t i = 1; i < n; i++) {  // insertion sort by site
        const uint32_t e = F(NF + i);
        uint32_t kk = i;
        while (kk > 0 && F(NF + kk - 1) > e) {
          F(NF + kk) = F(NF + kk - 1);
          kk--;
        }
        F(NF + kk) = e;
      }
    }
    // per-shot noise cursors (stratified: the next fault and the faults
    // placed so far)
    if (!LIST && P.nsites > 0) {
      for (int j = 0; j < kShotsPerLane; j++) {
        uint32_t ord = 0, nf = 0xFFFFFFFFu;
        if (!strat) nf = bs_next_fault<LDS_SURV>(P, surv, 0, 0, &ord, A.offset + s0 + j, seed);
        else if (A.strat_r > 0) nf = strat_site(stab, NS, (uint32_t)A.strat_r, 0, draw(ord++, kPurposeStrat, A.offset + s0 + j, seed));
        F(NF + j) = nf;
        F(OC + j) = ord;
        min_nf = min(min_nf, nf);
      }
    }
    uint32_t alive = valid;  // shots not rejected by post-selection
    uint32_t last_m = 0, last_pn = 0;
    uint32_t rblk = 0xFFFFFFFFu;
    for (int pc = 0;; pc++) {
      const GInstr in = load_instr(P.code, pc);
      const uint32_t v = in.v;
      // leave when every shot of the wave is rejected by post-selection
      // (a wave-uniform exit; a lane with no live shot writes only zeros)
      if (in.op == OP_END || (EXT && P.has_post && !__ballot(alive != 0))) break;
      switch (in.op) {
        case OP_FANCX:
        case OP_FANCZ:
        case OP_FAN2: {
          // target rows T ^= the pivot word, parity of rows Q into the pivot;
          // four targets (both frames) per round trip
          const uint32_t xv = F(v), zv = F(N + v), nxv = F(2 * N + v), nzv = F(3 * N + v);
          const bool cx = in.op == OP_FANCX;
          const uint32_t tf = cx ? 0u : N, qf = cx ? N : 0u;  // row offsets of T and Q in the full frame
          const uint32_t sf = in.op == OP_FAN2 ? zv : xv, sn = in.op == OP_FAN2 ? nzv : nxv;
          uint32_t par = 0, npar = 0;
          for (int w = 0; w < W; w++) {
            uint64_t m = masks[in.a + w];
            while (m) {
              uint32_t q[4];
              const int n = take4(m, (uint32_t)w * 64, q);
              uint32_t rt[4], rq[4], a[4], b[4], c[4], d[4];
#pragma unroll
              for (int i = 0; i < 4; i++) {
                rt[i] = i < n ? tf + q[i] : DR;
                rq[i] = i < n ? qf + q[i] : ZR;
              }
#pragma unroll
              for (int i = 0; i < 4; i++) {
                a[i] = F(rt[i]);
                b[i] = F(rt[i] == DR ? DR : rt[i] + 2 * N);
                c[i] = F(rq[i]);
                d[i] = F(rq[i] == ZR ? ZR : rq[i] + 2 * N);
              }
#pragma unroll
              for (int i = 0; i < 4; i++) {
                F(rt[i]) = a[i] ^ sf;
                F(rt[i] == DR ? DR : rt[i] + 2 * N) = b[i] ^ sn;
                par ^= c[i];
                npar ^= d[i];
              }
            }
          }
          if (in.op == OP_FAN2) {
            F(v) = xv ^ par;
            F(2 * N + v) = nxv ^ npar;
          } else {
            F(N + v) = zv ^ par;
            F(3 * N + v) = nzv ^ npar;
          }
          break;
        }
        case OP_FS: {
          const uint32_t x = F(v), z = F(N + v), nx = F(2 * N + v), nz = F(3 * N + v);
          F(N + v) = z ^ x;
          F(3 * N + v) = nz ^ nx;
          break;
        }
        case OP_FH: {
          const uint32_t x = F(v), z = F(N + v), nx = F(2 * N + v), nz = F(3 * N + v);
          F(v) = z;
          F(N + v) = x;
          F(2 * N + v) = nz;
          F(3 * N + v) = nx;
          break;
        }
        case OP_MSTATIC:
        case OP_MRANDOM: {
          uint32_t mm, pn;
          if (in.op == OP_MSTATIC) {
            // parity of the x rows over the measured Z-string, both frames
            mm = (in.flags & F_SIGN) ? ~0u : 0u;
            pn = 0;
            for (int w = 0; w < W; w++) {
              uint64_t m = masks[in.a + w];
              while (m) {
                uint32_t q[4];
                const int n = take4(m, (uint32_t)w * 64, q);
                uint32_t a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                  a[i] = F(i < n ? q[i] : ZR);
                  b[i] = F(i < n ? 2 * N + q[i] : ZR);
                }
                mm ^= a[0] ^ a[1] ^ a[2] ^ a[3];
                pn ^= b[0] ^ b[1] ^ b[2] ^ b[3];
              }
            }
          } else {
            const uint32_t j = in.b, blk = j >> 7;
            if (blk != rblk) {
              // bits of this block's dormant random events for the lane's 32
              // shots, eight events per pass, gathered in registers
              const uint32_t o0 = P.rblk_off[blk], o1 = P.rblk_off[blk + 1];
              for (uint32_t g = o0; g < o1; g += 8) {
                uint32_t e[8], bits[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                  e[i] = g + i < o1 ? (uint32_t)P.rblk_ev[g + i] : 0u;
                  bits[i] = 0;
                }
                for (int s = 0; s < kShotsPerLane; s++) {
                  const U4 w = draw(blk, kPurposeRbit, A.offset + s0 + s, seed);
#pragma unroll
                  for (int i = 0; i < 8; i++) {
                    const uint32_t h = e[i] >> 5;
                    const uint32_t wv = h == 0 ? w.w0 : h == 1 ? w.w1 : h == 2 ? w.w2 : w.w3;
                    bits[i] |= ((wv >> (e[i] & 31)) & 1u) << s;
                  }
                }
#pragma unroll
                for (int i = 0; i < 8; i++)
                  if (g + i < o1) F(RB + (g - o0) + i) = bits[i];
              }
              rblk = blk;
            }
            const uint32_t x = F(v), z = F(N + v), nx = F(2 * N + v), nz = F(3 * N + v), rb = F(RB + in.u);
            pn = nz;
            mm = rb ^ pn;
            const uint32_t b = mm ^ z ^ ((in.flags & F_SIGN) ? ~0u : 0u);
            // H absorbed after the outcome, then the correction X^b
            F(v) = z ^ b;
            F(N + v) = x;
            F(2 * N + v) = nz;
            F(3 * N + v) = nx;
          }
          last_m = mm;
          last_pn = pn;
          const int r = as_const(P.ev_rec)[in.b];
          if (r >= 0) {
            if (meas32 && store) meas32[(size_t)r * 2 * words64 + col] = mm & alive;
            // accumulators fed by this record, four per round trip
            const uint32_t t1 = rec_tgt_off[r + 1];
            for (uint32_t t = rec_tgt_off[r]; t < t1; t += 4) {
              uint32_t rr[4], a[4];
#pragma unroll
              for (int i = 0; i < 4; i++) rr[i] = t + i < t1 ? ACC + rec_tgt[t + i] : DR;
#pragma unroll
              for (int i = 0; i < 4; i++) a[i] = F(rr[i]);
#pragma unroll
              for (int i = 0; i < 4; i++) F(rr[i]) = a[i] ^ mm;
            }
          }
          break;
        }
        case OP_CPAULI: {
          // X^m on the x rows (full frame), X^pn (noise frame); same for Z
          for (int zpart = 0; zpart < 2; zpart++) {
            const uint32_t off = zpart ? N : 0u;
            for (int w = 0; w < W; w++) {
              uint64_t m = masks[in.a + zpart * W + w];
              while (m) {
                uint32_t q[4], rf[4], rn[4], a[4], b[4];
                const int n = take4(m, (uint32_t)w * 64, q);
#pragma unroll
                for (int i = 0; i < 4; i++) {
                  rf[i] = i < n ? off + q[i] : DR;
                  rn[i] = i < n ? 2 * N + off + q[i] : DR;
                }
#pragma unroll
                for (int i = 0; i < 4; i++) {
                  a[i] = F(rf[i]);
                  b[i] = F(rn[i]);
                }
#pragma unroll
                for (int i = 0; i < 4; i++) {
                  F(rf[i]) = a[i] ^ last_m;
                  F(rn[i]) = b[i] ^ last_pn;
                }
              }
            }
          }
          break;
        }
        case OP_NOISE: {
          const uint32_t hi = in.b;
          if (LIST) {
            if (!lovf) {
              while (lhead < lcnt) {
                const uint32_t e = F(NF + lhead);
                if ((e >> 9) >= hi) break;
                bs_apply_fault<W>(P, F, N, e >> 9, e & 15u, 1u << ((e >> 4) & 31u));
                lhead++;
              }
            } else {
              // list overflow (rare): re-draw this block's faults per shot from
              // the start of each chunk it touches (stateless, same faults)
              const uint32_t lo = in.a;
              for (int j = 0; j < kShotsPerLane; j++) {
                const uint64_t shot = A.offset + s0 + j;
                if (strat) {
                  uint32_t cur = 0;
                  for (uint32_t i = 0; i < (uint32_t)A.strat_r && cur < hi; i++) {
                    const U4 w = draw(i, kPurposeStrat, shot, seed);
                    const uint32_t nf = strat_site(stab, NS, (uint32_t)A.strat_r - i, cur, w);
                    if (nf >= lo && nf < hi) bs_apply_fault<W>(P, F, N, nf, fault_outcome(P, nf, w), 1u << j);
                    cur = nf + 1;
                  }
                  continue;
                }
                for (uint32_t c = lo / (uint32_t)kChunk; c * (uint32_t)kChunk < hi; c++) {
                  const uint32_t cend = min(min((c + 1) * (uint32_t)kChunk, (uint32_t)P.nsites), hi);
                  uint32_t ord = 0, cur = 0;
                  for (;;) {
                    uint32_t o = 0;
                    const uint32_t nf = bs_next_fault<LDS_SURV>(P, surv, c, cur, &ord, shot, seed, &o);
                    if (nf >= cend) break;
                    if (nf >= lo) bs_apply_fault<W>(P, F, N, nf, o, 1u << j);
                    cur = nf - c * (uint32_t)kChunk + 1;
                  }
                }
              }
            }
            break;
          }
          if (min_nf < hi) {
            // which of the lane's shots have a fault before hi: 32 independent
            // LDS loads, then a mask
            uint32_t due = 0;
#pragma unroll
            for (int s = 0; s < kShotsPerLane; s++) due |= (uint32_t)(F(NF + s) < hi) << s;
            while (due) {
              const int s = __ffs(due) - 1;
              due &= due - 1;
              uint32_t nf = F(NF + s);
              if (strat) {
                uint32_t ord = F(OC + s);
                const uint64_t shot = A.offset + s0 + s;
                while (nf < hi) {
                  // the outcome comes from the draw that placed this fault
                  bs_apply_fault<W>(P, F, N, nf, fault_outcome(P, nf, draw(ord - 1, kPurposeStrat, shot, seed)), 1u << s);
                  if (ord == (uint32_t)A.strat_r) nf = 0xFFFFFFFFu;
                  else {
                    nf = strat_site(stab, NS, (uint32_t)A.strat_r - ord, nf + 1, draw(ord, kPurposeStrat, shot, seed));
                    ord++;
                  }
                }
                F(NF + s) = nf;
                F(OC + s) = ord;
              } else {
                uint32_t oc = F(OC + s);
                uint32_t chunk = oc >> 16, ord = oc & 0xFFFFu;
                const uint64_t shot = A.offset + s0 + s;
                while (nf < hi) {
                  const uint32_t cend = min((chunk + 1) * (uint32_t)kChunk, (uint32_t)P.nsites);
                  if (nf >= cend) {
                    chunk++;
                    ord = 0;
                    nf = bs_next_fault<LDS_SURV>(P, surv, chunk, 0, &ord, shot, seed);
                    continue;
                  }
                  // the outcome comes from the draw that placed this fault
                  U4 w = draw(ord - 1, kPurposeNoise | chunk, shot, seed);
                  const uint64_t w64 = ((uint64_t)w.w3 << 32) | w.w2;
                  const uint32_t o = (uint32_t)__umul64hi(w64, (uint64_t)nout_of(P.site_type[nf]));
                  bs_apply_fault<W>(P, F, N, nf, o, 1u << s);
                  nf = bs_next_fault<LDS_SURV>(P, surv, chunk, nf - chunk * (uint32_t)kChunk + 1, &ord, shot, seed);
                }
                F(NF + s) = nf;
                F(OC + s) = ord | (chunk << 16);
              }
            }
            uint32_t nmin = 0xFFFFFFFFu;
#pragma unroll
            for (int s = 0; s < kShotsPerLane; s++) nmin = min(nmin, F(NF + s));
            min_nf = nmin;
          }
          break;
        }
        case OP_DET:
          if (det32 && store) det32[(size_t)in.b * 2 * words64 + col] = F(ACC + in.s) & alive;
          F(ACC + in.s) = 0;  // the row is reused by a later detector
          break;
        case OP_POSTSELECT: {
          // post-selection (Section 3.2): shots whose detector reads 1 are
          // rejected; later record words carry only the live shots' bits
          if constexpr (EXT) {
            const uint32_t d = F(ACC + in.s);
            if (det32 && store) det32[(size_t)in.b * 2 * words64 + col] = d & alive;
            F(ACC + in.s) = 0;
            alive &= ~d;
          }
          break;
        }
        case OP_EMIT:
          // frame-only stream of the split form: a rotation's sign bit
          if (bits32 && store) bits32[(size_t)in.u * 2 * words64 + col] = F(v) & valid;
          break;
        case OP_MACTF: {
          // frame side of an active measurement taken with outcome 0: its
          // frame and noise parities for the vector stream, H_v (X-type),
          // x_v = sign; the record row stays 0 until the fix-up
          const bool isx = (in.flags & F_XMEAS) != 0;
          const uint32_t x = F(v), z = F(N + v), nx = F(2 * N + v), nz = F(3 * N + v);
          const uint32_t pn = isx ? nz : nx;
          if (bits32 && store) {
            bits32[(size_t)in.u * 2 * words64 + col] = (isx ? z : x) & valid;
            bits32[(size_t)(in.u + 1) * 2 * words64 + col] = pn & valid;
          }
          if (isx) {
            F(N + v) = x;
            F(2 * N + v) = nz;
            F(3 * N + v) = nx;
          }
          F(v) = (in.flags & F_SIGN) ? ~0u : 0u;
          last_m = 0;
          last_pn = pn;
          const int r = as_const(P.ev_rec)[in.b];
          if (r >= 0 && meas32 && store) meas32[(size_t)r * 2 * words64 + col] = 0;
          break;
        }
        default:  // OP_OBS: accumulated from its records; no active-vector ops exist here
          break;
      }
    }
    if (obs32 && store)
      for (int o = 0; o < P.nobs; o++) obs32[(size_t)o * 2 * words64 + col] = F(ACC + P.ndet_rows + o) & alive;
  }
}

template <bool LS, bool LI, bool EXT>
static hipError_t launch_frames_t(const DevProgram& P, const KArgs& A, int grid, size_t lds, hipStream_t st) {
  static bool attr[5] = {false, false, false, false, false};
  const void* fn = P.W == 1   ? (const void*)k_frames<1, LS, LI, EXT>
                   : P.W == 2 ? (const void*)k_frames<2, LS, LI, EXT>
                   : P.W == 3 ? (const void*)k_frames<3, LS, LI, EXT>
                              : (const void*)k_frames<4, LS, LI, EXT>;
  if (!attr[P.W]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr[P.W] = true;
  }
  switch (P.W) {
    case 1: hipLaunchKernelGGL((k_frames<1, LS, LI, EXT>), dim3(grid), dim3(64), lds, st, P, A); break;
    case 2: hipLaunchKernelGGL((k_frames<2, LS, LI, EXT>), dim3(grid), dim3(64), lds, st, P, A); break;
    case 3: hipLaunchKernelGGL((k_frames<3, LS, LI, EXT>), dim3(grid), dim3(64), lds, st, P, A); break;
    default: hipLaunchKernelGGL((k_frames<4, LS, LI, EXT>), dim3(grid), dim3(64), lds, st, P, A); break;
  }
  return hipGetLastError();
}

template <bool EXT>
static hipError_t launch_frames_e(const DevProgram& P, const KArgs& A, int grid, size_t lds, hipStream_t st) {
  const bool ls = frames_surv_in_lds(P), li = frames_fault_list(P, A.strat_r);
  if (ls && li) return launch_frames_t<true, true, EXT>(P, A, grid, lds, st);
  if (ls) return launch_frames_t<true, false, EXT>(P, A, grid, lds, st);
  if (li) return launch_frames_t<false, true, EXT>(P, A, grid, lds, st);
  return launch_frames_t<false, false, EXT>(P, A, grid, lds, st);
}

hipError_t launch_frames(const DevProgram& P, const KArgs& A, int grid, hipStream_t st) {
  const size_t lds = frames_lds_rows(P, A.strat_r) * 64 * 4;
  // post-selected programs and stratified calls take the EXT kernels
  if (P.has_post || A.strat_r >= 0) return launch_frames_e<true>(P, A, grid, lds, st);
  return launch_frames_e<false>(P, A, grid, lds, st);
}

}  // namespace clifft
