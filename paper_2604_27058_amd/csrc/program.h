// Compiled program layout shared by the host compiler, the runtime and the
// HIP kernels.  Everything here is plain data: a flat 16-byte instruction
// stream plus side tables, uploaded once per program and read through the
// scalar cache by every wave (the stream is wave-uniform by Theorem 1: the
// Clifford frame, the active set and k(t) do not depend on any sample).
#pragma once
#include <stdint.h>

namespace clifft {

constexpr int kChunk = 4096;      // noise sites per survival table (gap sampler)
constexpr int kMaxWords = 4;      // frames up to 256 qubits
constexpr int kMaxK = 30;         // active dimension limit of the format

// Opcodes.  F* act on the Pauli frames only (both the full frame and the
// noise-only frame); A* act on the active vector only; the measurement and
// expansion opcodes do both.
enum Op : uint8_t {
  OP_END = 0,
  OP_FANCX,    // CNOT v->q for q in mask (v is the control)      v, a=mask
  OP_FANCZ,    // CZ v,q for q in mask                              v, a=mask
  OP_FAN2,     // CNOT q->v for q in mask (v is the target)         v, a=mask
  OP_FS,       // S on v                                            v
  OP_FH,       // H on v                                            v
  OP_APERM,    // array part of a CNOT fan: control slot s, targets slots a
  OP_ASIGN,    // array part of a CZ fan: slot s with slots a
  OP_APERM2,   // array part of a target fan: target slot s, controls slots a
  OP_AS,       // array S on slot s
  OP_AH,       // array H on slot s
  OP_EXPAND,   // H on dormant v, new slot s = k, then rotation      v, s, a=const
  OP_AROT,     // diagonal rotation on active v at slot s            v, s, a=const
  OP_MSTATIC,  // deterministic Z-string measurement                 a=mask(z, W words), b=event
  OP_MRANDOM,  // dormant X_v measurement, then H_v absorbed         v, b=event, u=index among the
               //   dormant random events of the event's 128-block
  OP_MACTZ,    // active Z_v measurement (mask), demote slot s       v, s, b=event (u, flags: fusion)
  OP_MACTX,    // active X_v measurement (interfere), demote slot s  v, s, b=event (u, flags: fusion)
  OP_CPAULI,   // reset correction X^m (noise part X^pn)             a=mask(x,z), b=event
  OP_NOISE,    // noise sites [a, b)
  OP_DET,      // detector b = XOR of records refs[a .. a+u); s = its accumulator row
  OP_OBS,      // observable b ^= XOR of records refs[a .. a+u)
  OP_PHASE,    // rotation whose generator is a Z string on dormant qubits   a=mask(z), b=const
               //   (Appendix B.1 case 1): only the global scalar changes
  // Frame-only stream of the split form (below): the frame side of the
  // vector instructions, for the bit-sliced frame kernel.
  OP_EMIT,     // write bit x_v of the full frame to needed-bit row u
  OP_MACTF,    // frame side of an active measurement with outcome 0: write p
               //   (x_v, or z_v for F_XMEAS) to row u and the noise frame's to
               //   row u + 1; H_v for F_XMEAS; then x_v = sign; record 0  v, u, b=event
  OP_CFEED,    // feed-forward Pauli (Appendix B.3): if record b is 1,     a=mask(x,z), b=record
               //   the full frame takes the image (sign in F_SIGN)
  OP_EXPVAL,   // expectation value of a virtual observable (probe b):    a=mask(x,z) then the
               //   slot masks of its active X and Z letters (2 words); F_SIGN, F_ZERO
  OP_POSTSELECT,  // post-selected detector (Section 3.2): as OP_DET; a shot whose detector
               //   reads 1 ends there, its observables read 0 and its later records stay 0
  OP_COUNT
};

// flags
constexpr uint8_t F_SIGN = 1;        // sign bit of the localized observable (of the image, for OP_CPAULI)
// Localization passes of an active measurement or H (Appendix A with an
// active pivot): an OP_APERM, then an OP_ASIGN, then an OP_AS, each
// optional, on the measured (or H) slot and directly before that
// instruction among the vector instructions.  They permute and rephase only
// the elements whose bit on that slot is set, so kernels that work out of
// place skip them (F_FOLD_NEXT) and read the next pass through them.
constexpr uint8_t F_FOLD_NEXT = 8;
// Active measurement whose next vector instruction, after folded passes, is
// again an active measurement: this measurement's collapse pass accumulates
// that one's branch sums (F_FUSE_NEXT), and it skips its own reduction.
constexpr uint8_t F_FUSE_NEXT = 2;
constexpr uint8_t F_XMEAS = 4;  // OP_MACTF: the measurement is X-type (interfere)
constexpr uint8_t F_ZERO = 16;  // OP_EXPVAL: X support on a dormant qubit, the value is 0
// Kernels that collapse out of place keep up to this many trailing
// expansions unapplied: the vector is then the stored 2^(k-d) amplitudes
// times one phase factor per deferred top slot (an expansion only multiplies
// its new upper half by a phase), and the next active measurement reads it
// through them; any other vector instruction writes the deferred part first.
constexpr int kDeferMax = 4;

struct GInstr {
  uint8_t op;
  uint8_t flags;
  uint16_t v;   // virtual qubit
  uint16_t s;   // slot (array axis)
  uint16_t u;   // small count
  uint32_t a;   // mask offset / slot mask / const index / site lo / refs offset
  uint32_t b;   // event / site hi / detector or observable index
};
static_assert(sizeof(GInstr) == 16, "instruction must be 16 bytes");

// Noise site types
enum SiteType : uint8_t { S_DEP1 = 0, S_DEP2 = 1, S_XERR = 2, S_YERR = 3, S_ZERR = 4 };

// Philox counter purposes of the stochastic contract
constexpr uint32_t kPurposeNoise = 0x4E000000u;  // | chunk
constexpr uint32_t kPurposeRbit = 0x52000000u;
constexpr uint32_t kPurposeAmeas = 0x41000000u;
constexpr uint32_t kPurposeStrat = 0x53000000u;  // stratified sampling: fault i of the shot

// Split form.  Every frame bit and every record of a shot is an affine
// function over GF(2) of the shot's faults, dormant random bits and active
// measurement outcomes, and the active vector reads the frames only through a
// few bits (a rotation's sign, an active measurement's frame and noise
// parities).  So a program can run as
//   1. the frame-only stream (bit-sliced, 32 shots per lane) with every active
//      outcome taken as 0, writing records and the needed bits;
//   2. the vector-only stream, one shot per lane, wave or workgroup, each
//      needed bit corrected by the parity of its dependency mask with the
//      shot's active outcomes so far, writing the active outcomes;
//   3. a fix-up XORing into each record row the outcome rows its dependency
//      lists.
// At most kSplitMaxActive active measurements (dependency masks of
// kSplitWords 64-bit words).
constexpr int kSplitMaxActive = 256;
constexpr int kSplitWords = kSplitMaxActive / 64;

// Paired measurement collapses on the cooperative HBM tiers: the pass an
// active measurement runs for a pair (the joint-sum read pass of its first
// measurement A; the collapse of a single measurement that takes the joint
// sums of the next two; the collapse of B, carrying the next two's joint
// sums, the next one's sums, or none) and its line-complete item order,
// precomputed per element size.  GInstr.u of an active measurement indexes
// the table (entry 2u for FP32, 2u + 1 for FP64; u = 0: none); the kernel
// uses an entry only when its kind is the pass it runs.
enum PairPass : int8_t { PP_NONE = 0, PP_JOINT_READ = 1, PP_SINGLE_JOINT = 2, PP_PAIR_JOINT = 3, PP_PAIR_NEXT = 4, PP_PAIR = 5 };
struct PairLine {
  uint32_t v[4];  // spanning directions of a lane group's items
  int8_t pos[5];  // zero-insertion positions, ascending
  int8_t nv, npos, kind;
};
static_assert(sizeof(PairLine) == 24, "pair order entry must be 24 bytes");

// Device-side view of one program (all pointers are device addresses).
struct DevProgram {
  const GInstr* code;
  const uint64_t* masks;     // W-word Pauli masks
  const double* consts;      // (cos 2theta, sin 2theta, cos theta, sin theta) per rotation angle
  const uint32_t* refs;      // record references of detectors / observables
  const int32_t* ev_rec;     // event -> record index or -1
  const uint8_t* site_type;  // per noise site
  const uint32_t* site_img;  // per site: offset of its images in masks (2 or 4 images x 2W words)
  const uint8_t* site_sign;  // per site: sign bits of those images (bit 2i: X image of its qubit i, 2i+1: Z)
  const double* surv;        // per chunk: kChunk + 1 survival products
  const uint32_t* rec_tgt_off;  // per record: first entry in rec_tgt (nrec + 1 entries)
  const uint32_t* rec_tgt;      // accumulators (detector d, or ndet + observable o) a record feeds
  const uint32_t* rblk_off;     // per 128-event block: first entry in rblk_ev (nblocks + 1 entries)
  const uint8_t* rblk_ev;       // event ordinal mod 128 of each dormant random event of the block
  int32_t nq, W, kmax, ncode;
  int32_t nevents, nrec, ndet, nobs;
  int32_t nprobes;
  int32_t nsites, nchunks;
  int32_t rblk_max;             // most dormant random events in one 128-event block
  int32_t ndet_rows;            // detector accumulator rows (observables follow them)
  float exp_faults;             // expected realized faults per shot (sum of site probabilities)
  // split form, vector-only view: needed bits of the shot ([rows][words],
  // bit-packed like records) and each row's dependency mask over the active
  // outcomes (kSplitWords words per row); null elsewhere
  const uint64_t* vdep;
  int32_t nbits;                // needed-bit rows
  int32_t dep_words;            // words per dependency mask actually used (<= kSplitWords)
  int32_t has_post;             // the stream holds OP_POSTSELECT (shots may end early)
  // Stratified sampling (Section 3.2, rare-event sampling): row s - 1 holds
  // e_s(t), t = 0 .. nsites, the elementary symmetric polynomial of degree s
  // of the odds p / (1 - p) of the sites t .. nsites - 1; given s faults
  // left from site j on, the next one lies at or after t with probability
  // e_s(t) / e_s(j).  Null until a stratified call uploads it.
  const double* strat;
  int32_t strat_rows;
  const PairLine* pline;  // paired-pass item orders (see PairLine)
  int32_t has_pairs[2];   // some measurements collapse in pairs (FP32, FP64)
};

}  // namespace clifft
