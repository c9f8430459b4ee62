/*
 * clifft.h -- C-ABI of the MI355X (gfx950) sample-many engine for
 * near-Clifford circuits (frame-factored simulation, Chase & Labib, "Clifft").
 *
 * The library compiles a circuit once on the host (Section 3.1 of the paper:
 * Clifford frame absorption by Heisenberg mapping, Definition 1 / Eq. 1;
 * Pauli localization, Lemma 1 and Appendix A) and then samples it many times
 * on the GPU (Section 3.2: per-shot Pauli-frame updates, sparse noise
 * sampling, active-vector expansion / rotation / measurement, Appendix B).
 *
 * Conventions used by every entry point:
 *   - Circuit text: a Stim-style subset, extended with non-Clifford
 *     rotations (Section 3.1, front end).  Gates H S S_DAG X Y Z CX (CNOT)
 *     CZ SWAP; rotations T = exp(-i pi/8 Z), T_DAG = exp(+i pi/8 Z),
 *     R_Z(phi) = exp(-i phi Z / 2), R_X(phi), R_Y(phi) likewise about X and
 *     Y, R_PAULI(phi) P... = exp(-i phi P / 2) for Pauli products P written
 *     X0*Y3*Z5, U3(theta, phi, lambda) (the matrix [[c, -e^{i l} s],
 *     [e^{i p} s, e^{i (p + l)} c]], c = cos(theta/2), s = sin(theta/2));
 *     M MX MR R, MPP P... (one record per product, eigenvalue (-1)^m);
 *     record-controlled Paulis CX / CY / CZ rec[-k] q (a Pauli on q when the
 *     record is 1; Appendix B.3); EXP_VAL P... (expectation-value probes,
 *     see clifft_sample_expval); noise DEPOLARIZE1(p) DEPOLARIZE2(p)
 *     X_ERROR(p) Y_ERROR(p) Z_ERROR(p); DETECTOR rec[-k]...;
 *     OBSERVABLE_INCLUDE(i) rec[-k]...; REPEAT n { ... }; TICK and
 *     coordinates are ignored.  At most 256 qubits, k_max <= 30.
 *   - Records are bit-packed and record-major: for a call with `shots`
 *     shots, words = ceil(shots / 64); bit (s % 64) of word
 *     out[r * words + s / 64] is record r of shot s.  Bits of shots beyond
 *     `shots` in the last word are written as zero.
 *   - Determinism: records are a pure function of (program, seed, global
 *     shot index = shot_offset + s); they do not depend on the launch shape,
 *     on the split of a run into calls, or on the precision for circuits
 *     whose active dimension stays 0.
 *   - Errors: every function returns a clifft_status; nothing is thrown
 *     across the ABI.  clifft_last_error() returns a message for the last
 *     failing call of the calling thread.
 *   - Device work is queued on `stream` (a hipStream_t, NULL for the null
 *     stream) of the current HIP device; sampling calls return after the
 *     launch is queued, except the trace call which synchronizes.
 */
#ifndef CLIFFT_H
#define CLIFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clifft_program clifft_program; /* opaque, owned by the library */

typedef enum clifft_status {
  CLIFFT_OK = 0,
  CLIFFT_E_PARSE = 1,              /* malformed circuit text */
  CLIFFT_E_UNSUPPORTED = 2,        /* instruction outside the supported subset */
  CLIFFT_E_CAPACITY = 3,           /* too many qubits, k_max too large, buffer too small */
  CLIFFT_E_INVALID_ARG = 4,        /* null pointer where one is required, bad option */
  CLIFFT_E_DEVICE = 5,             /* HIP error (launch, allocation, copy) */
  CLIFFT_E_IMPOSSIBLE_OUTCOME = 6  /* trace mode: forced outcome of probability 0 */
} clifft_status;

typedef enum clifft_precision { CLIFFT_FP32 = 0, CLIFFT_FP64 = 1 } clifft_precision;

typedef struct clifft_info {
  int32_t num_qubits;        /* N */
  int32_t frame_words;       /* W = ceil(N / 64) */
  int32_t k_max;             /* peak active dimension (Section 2.2) */
  int32_t num_events;        /* measurement events incl. resets */
  int32_t num_measurements;  /* recorded measurements */
  int32_t num_detectors;
  int32_t num_observables;
  int32_t num_noise_sites;
  int32_t num_instructions;  /* length of the compiled stream */
  int32_t num_random_events; /* dormant random measurements (Appendix B.2) */
  int32_t num_active_events; /* measurements on the active vector */
  int32_t num_probes;        /* expectation-value probes (EXP_VAL) */
  int32_t num_postselected;  /* post-selected detectors (clifft_compile_opts) */
} clifft_info;

/* Launch configuration; zero-initialize for automatic choices. */
typedef struct clifft_launch {
  int32_t precision;        /* clifft_precision of the active-vector amplitudes;
                               probability reductions and renormalization
                               factors are FP64 in both */
  int32_t threads_per_shot; /* 0 automatic, else 1 (shot per lane), 64 (shot per
                               wave), 256 (shot per workgroup) or -32 (32 shots
                               per lane, bit-sliced Pauli frames; k_max = 0 only,
                               not in trace mode) */
  int32_t grid;             /* workgroups (256 threads); 0 = fill the device */
  int32_t vector_in_hbm;    /* 0 automatic (HBM only when LDS is too small),
                               1 force the global workspace, -1 force LDS */
  int32_t specialize;       /* 1 a bit-sliced kernel generated for this
                               program and compiled at run time (see
                               clifft_specialize; an error on any other tier),
                               -1 never, 0 automatic (the interpreter unless
                               the autotuner chose the specialized kernel) */
  int32_t split;            /* 1, 2, 3 the split form (programs with an active
                               vector and at most 256 active measurements):
                               the Pauli frames of every shot run bit-sliced
                               with the active outcomes taken as 0 (records
                               and the frame bits the vector reads are affine
                               over GF(2) in those outcomes), then the vector
                               instructions alone at threads_per_shot /
                               vector_in_hbm / grid, then a fix-up XORs the
                               outcomes into the records they feed; same
                               records as the whole-program interpreter.
                               The frame pass runs bit-sliced (2), shot per
                               lane with frames in VGPRs (3), or (1) bit-sliced
                               when its rows fit in LDS and there are at least
                               two 2048-shot tiles per CU.
                               -1 never, 0 automatic (the autotuner's choice) */
} clifft_launch;

/* Compile options; zero-initialize (or pass NULL) for the defaults. */
typedef struct clifft_compile_opts {
  int32_t hir_passes;  /* optimisation passes on the Heisenberg representation
                          before localization (Section 3.1, middle end), a bit
                          mask: 1 peephole (fuse adjacent rotations about one
                          generator, cancel inverse pairs, absorb a resulting
                          Clifford rotation into the frame), 2 commuting
                          reorder (measurements earlier, non-Clifford
                          rotations later, across operations they commute
                          with).  0: none, so that k(t) is that of the
                          operations as written.  4: lower through the
                          Heisenberg representation without optimizing it
                          (the same program as 0; for testing) */
  int32_t k_limit;     /* E_CAPACITY if the peak active dimension exceeds this
                          (0: the format limit, 30) */
  int32_t drop_phases; /* 1: leave out the instructions whose only effect is a
                          phase of the global scalar (rotations about dormant
                          Z strings, Appendix B.1 case 1); the trace call's
                          global scalar then misses those phases.  0: keep */
  const uint64_t* postselect; /* post-selected detectors (Section 3.2,
                          post-selection overhead), host memory read during
                          the call: bit d % 64 of word d / 64 set for
                          detector d, in the order DETECTOR instructions
                          appear; NULL for none.  Each becomes an
                          OP_POSTSELECT instruction: a shot whose detector
                          reads 1 is rejected and ends there.  Its records up
                          to that detector (which reads 1) are written as
                          usual; every later measurement and detector record,
                          every observable record and every probe not yet
                          reached read 0.  So a shot was kept iff all its
                          post-selected detectors read 0.  Records of kept
                          shots equal those of the same program without
                          post-selection.  Such programs do not use the split
                          form or the specialized kernel.  E_INVALID_ARG if a
                          set bit names no detector. */
  int32_t postselect_words; /* words in postselect (0 with NULL), or -1 to
                          post-select every detector (postselect ignored) */
} clifft_compile_opts;

/* Compile circuit text (len bytes, need not be NUL-terminated) into a
 * program (Section 3.1: Heisenberg mapping of the physical operations into
 * the virtual basis, Definition 1 / Eq. 1; Pauli localization, Lemma 1 and
 * Appendix A; lowering to a flat instruction stream).  opts may be NULL.
 * Host only; no device work.  *out receives a handle that the caller
 * releases with clifft_program_free.  Errors: E_PARSE, E_UNSUPPORTED,
 * E_CAPACITY, E_INVALID_ARG (null text or out, bad option). */
clifft_status clifft_compile(const char* text, size_t len, const clifft_compile_opts* opts, clifft_program** out);

/* Static properties of a compiled program (Theorem 1: fixed before sampling). */
clifft_status clifft_program_info(const clifft_program* p, clifft_info* out);

/* Active dimension after each compiled instruction (k(t), Theorem 1), and
 * the class of each measurement event (0 deterministic, 1 dormant random,
 * 2 active).  Host arrays of capacity `cap`; *n receives the full length. */
clifft_status clifft_k_profile(const clifft_program* p, int32_t* out, size_t cap, size_t* n);
clifft_status clifft_event_classes(const clifft_program* p, int32_t* out, size_t cap, size_t* n);

/* Virtual qubit held by each active-vector slot at the end of the program
 * (host array of k_max entries); *k receives the final active dimension. */
clifft_status clifft_final_slots(const clifft_program* p, int32_t* slots, int32_t* k);

/* Algorithmic work of one shot, summed over the compiled stream with the
 * active dimension in force at each instruction (the per-shot cost of
 * Section 2.6, asymptotic complexity, made concrete).  Integer work
 * counts 32-bit lane operations (a 64-bit word operation is two); noise work
 * uses the expected number of realized faults; vector traffic is the bytes
 * an unfused pass per instruction reads and writes at `precision`. */
typedef struct clifft_cost {
  double int_ops;         /* 32-bit integer lane-operations (frames, noise, records) */
  double flops;           /* floating-point operations on the active vector */
  double vector_bytes;    /* active-vector bytes read + written */
  double record_bytes;    /* bit-packed record bytes written */
  double expected_faults; /* mean number of realized faults */
  double instructions;    /* compiled instructions executed */
  double int_ops_bitsliced; /* integer lane-operations per shot of the bit-sliced form (32 shots per
                               frame word; per-shot random draws and outcome bits counted in full) */
  double vector_bytes_fused; /* active-vector bytes of the fused passes of the shot-per-lane tier
                               with vectors in HBM (folded localization passes and deferred
                               expansions move nothing, a collapse reads the vector and writes
                               half, carried branch sums skip the reduction) */
  double vector_bytes_fused_group; /* the same for a shot per wave or per workgroup (a collapse
                               through deferred expansions carries no branch sums there; two
                               consecutive measurements with only frame work between them
                               collapse together, Appendix B.2 applied to both) */
  double vector_bytes_fused_batch; /* the group tiers of the batched launch, which collapse one
                               measurement at a time */
  double paired_measurements; /* measurements that start a paired collapse on the group tiers at
                               this precision (0: the launch takes the instantiation without
                               the pair code) */
} clifft_cost;
clifft_status clifft_cost_model(const clifft_program* p, int32_t precision, clifft_cost* out);

/* The item orders the compiler stored for the paired measurement passes of
 * the cooperative HBM tiers (Appendix B.2 applied to two consecutive active
 * measurements; the orders only make the passes read whole cache lines).
 * out (capacity cap int32 values; may be NULL) receives 25 values per
 * measurement that runs such a pass: its instruction index, the pass kind
 * (1 the read pass of a pair's first measurement, 2 a single collapse taking
 * the next two's joint sums, 3/4/5 a pair's collapse carrying the next two's
 * joint sums / the next one's sums / nothing), n (the pass's items are
 * q < 2^n), then for FP32 and for FP64: nv, npos, pos[5], v[4] (item q maps
 * to the zero insertion of q >> nv at pos[0..npos) XOR the v[i] of q's low
 * bits).  *n_out receives the total count.  Host only. */
clifft_status clifft_pair_orders(const clifft_program* p, int32_t* out, size_t cap, size_t* n_out);

/* The launch configuration a sample call of `shots` shots would use with
 * `cfg` (NULL = automatic): *out receives precision, threads_per_shot,
 * grid and vector_in_hbm (1 HBM workspace, -1 LDS) after the automatic
 * choices are made.  Host only. */
clifft_status clifft_resolve_launch(const clifft_program* p, const clifft_launch* cfg, uint64_t shots,
                                    clifft_launch* out);

/* Launch-shape autotuner: times the candidate tiers (threads per shot 1,
 * 64, 256; vectors in LDS or HBM; for k_max = 0 also the bit-sliced
 * interpreter and, when the program qualifies, its specialized kernel) and
 * grid sizes (1 to 32 workgroups per CU) on a trial of up to `shots` shots
 * (at most 2^24 for k_max = 0, 2^18 below k_max = 13, 8 per CU above) at
 * `precision`, on `stream` of the current device, and stores the fastest in
 * the program.  Later calls whose cfg leaves threads_per_shot, grid,
 * vector_in_hbm and specialize at 0 use it (also for
 * clifft_workspace_size).  Allocates and frees temporary device buffers;
 * synchronizes.  *out (optional) receives the chosen configuration. */
clifft_status clifft_autotune(clifft_program* p, uint64_t shots, int32_t precision, void* stream, clifft_launch* out);

/* Program-specialized bit-sliced kernel (Pauli-frame-only programs,
 * k_max = 0): generates a HIP kernel in which the compiled stream is
 * unrolled and every frame row is a register, and compiles it for gfx950
 * (hiprtc).  Host only: the code object is kept in the program and loaded on
 * a device at its first launch.  Records are identical to the interpreter's
 * (same stochastic contract).  Idempotent.  Errors: E_UNSUPPORTED (the
 * program does not qualify: k_max > 0, more than 200 frame and accumulator
 * rows, more than 600 instructions, or noise too dense for the per-lane
 * fault list), E_DEVICE (run-time compilation failed).  `log` (optional, cap
 * bytes, NUL-terminated) receives the reason or the compiler log. */
clifft_status clifft_specialize(clifft_program* p, char* log, size_t cap);

/* Bytes of caller-provided device workspace a sample call of `shots` shots
 * needs with this configuration (0 when the active vectors fit in LDS and
 * the split form is not used).  Vectors in HBM take two buffers of
 * 2^k_max amplitudes per shot in flight: active measurements collapse from
 * one into the other.  The split form adds its needed-bit and outcome rows
 * (bit-packed, one row per needed bit and per active measurement). */
clifft_status clifft_workspace_size(const clifft_program* p, const clifft_launch* cfg, uint64_t shots, size_t* bytes);

/* Sample `shots` shots with global indices shot_offset .. shot_offset+shots-1
 * and Philox seed `seed` (Section 3.2: every shot resets the frames and the
 * active vector, runs the compiled stream -- Pauli-frame updates, sparse
 * noise sampling by jumping to the next realized fault, expansion, rotation
 * and measurement of the active vector, Appendix B -- and writes its
 * measurement, detector and observable records).  meas / det / obs are device buffers of
 * num_measurements / num_detectors / num_observables rows of
 * ceil(shots / 64) uint64 words (any may be NULL to skip it).  workspace is
 * a device buffer of at least clifft_workspace_size bytes (may be NULL when
 * that size is 0).  cfg may be NULL (automatic).  The program is uploaded to
 * the current device on first use and kept in the handle.  The call only
 * queues work on `stream`; launch errors are returned as E_DEVICE. */
clifft_status clifft_sample(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                            const clifft_launch* cfg, void* workspace, size_t workspace_bytes, uint64_t* meas,
                            uint64_t* det, uint64_t* obs, void* stream);

/* Sampling with expectation-value probes (Section 3.2, post-selection
 * overhead: probes read the frame-factored runtime state inline; Appendix C
 * uses one for a logical <Y>).  Each EXP_VAL P instruction of the circuit
 * is probe i (in program order) and gives, per shot, <psi|P|psi> of the
 * shot's state at that point: with g = U_C^dagger P U_C, (-1)^c <phi|g_A|phi>
 * / <phi|phi> where c is the commutation of the Pauli frame with g and g_A
 * its letters on active axes, or 0 when g has X support on a dormant qubit.
 * Same arguments as clifft_sample, plus expval: device [num_probes][shots]
 * double (probe-major; NULL to skip).  The reduction is FP64 in both
 * precisions.  Programs with probes do not run on the bit-sliced tier or in
 * the split form, and the batched launch does not return probe values. */
clifft_status clifft_sample_expval(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                   const clifft_launch* cfg, void* workspace, size_t workspace_bytes, uint64_t* meas,
                                   uint64_t* det, uint64_t* obs, double* expval, void* stream);

/* Stratified sampling (Section 3.2, rare-event sampling: batches conditioned
 * on a fixed number of realized faults, weighted by the probability of that
 * number).  Like clifft_sample, except that every shot has exactly `faults`
 * noise sites firing, the set drawn from the distribution of independent
 * sites conditioned on that count: fault i of shot s (in site order) is the
 * inverse-transform draw i of the Philox stream of purpose 0x53000000 from
 * one past the previous fault, with P(next fault at or after site t | f
 * faults left from site j on) = e_f(t) / e_f(j), e_f(t) the elementary
 * symmetric polynomial of degree f of the odds p / (1 - p) of the sites
 * t .. N-1; the fired Pauli comes from the same draw as in plain sampling.
 * Weight the stratum by clifft_fault_count_pmf.  The first call for a fault
 * count uploads tables of (faults x num_noise_sites) doubles to the device
 * (kept with the program; at most 1 GiB, else E_CAPACITY).  Runs on the
 * interpreter tiers and the bit-sliced tier; E_INVALID_ARG if cfg asks for
 * the split form or the specialized kernel, if faults < 0 or exceeds the
 * number of sites, or if no configuration has that many faults;
 * E_UNSUPPORTED if a site has probability 1. */
clifft_status clifft_sample_stratified(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                       int32_t faults, const clifft_launch* cfg, void* workspace,
                                       size_t workspace_bytes, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                       void* stream);

/* Weights of the strata (Section 3.2, rare-event sampling): pmf[r] = the
 * probability that exactly r noise sites fire, r = 0 .. rmax (Poisson-
 * binomial over the sites' probabilities), into host memory of rmax + 1
 * doubles.  Host only.  E_UNSUPPORTED if a site has probability 1,
 * E_CAPACITY if the weights overflow. */
clifft_status clifft_fault_count_pmf(const clifft_program* p, int32_t rmax, double* pmf);

/* Allocation-free sampling, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, records and launch choices as clifft_sample,
 * without the workspace: the active-vector workspace of the HBM tiers is a
 * fixed device array of 64 MiB inside the library (each device that loads
 * the library holds one until the process ends).  When the chosen launch
 * needs more than that, the call uses fewer persistent workgroups (records
 * do not depend on the grid); it returns E_CAPACITY when one workgroup's
 * vectors alone exceed 64 MiB or when cfg fixes a grid whose workspace does
 * not fit.  The call allocates nothing: the program must already be
 * resident on the current device (E_INVALID_ARG otherwise; any clifft_sample
 * call on the device uploads it), and a program-specialized kernel not yet
 * loaded on the device is replaced by the bit-sliced interpreter, which
 * writes the same records (E_INVALID_ARG if cfg demands it).  Nothing in
 * the array needs to start at zero (every shot initializes its vectors).
 * Calls that overlap in time on one device share the array and race: the
 * caller orders them (one stream, or events).  Queues work on `stream` and
 * returns. */
clifft_status clifft_sample_noalloc(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                    const clifft_launch* cfg, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                    void* stream);

/* Trace mode (testing; the forced-outcome call of the frame-factored state,
 * Definition 2 / Eq. 2: psi = gamma U_C P~ (phi_A (x) |0>_D)): like
 * clifft_sample, and in addition
 *   forced_m       device [shots][num_events] uint32 outcomes to force, or NULL
 *   forced_faults  device [shots][num_noise_sites] int32 fault outcome index
 *                  (-1 none) replacing the noise sampler, or NULL
 *   probs          device [shots][num_events] double, P(m = 1) of each event
 *                  (Appendix B.2), or NULL
 *   phi            device [shots][2^k_max][2] double, final active vector in
 *                  the program's final slot order (clifft_final_slots), or NULL
 *   gamma          device [shots][2] double, the final global scalar, or NULL:
 *                  phases of frame conjugations and products (Appendix B.3),
 *                  of rotations (Appendix B.1) and the normalisation of phi,
 *                  so that gamma * phi is the physical amplitude vector
 *                  relative to U_C P~ with no further phase or scale
 * Not available on the bit-sliced tier.  Synchronizes `stream`; returns
 * E_IMPOSSIBLE_OUTCOME if a forced outcome had zero probability. */
clifft_status clifft_sample_trace(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                  const clifft_launch* cfg, const uint32_t* forced_m, const int32_t* forced_faults,
                                  double* probs, double* phi, double* gamma, void* workspace,
                                  size_t workspace_bytes, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                  void* stream);

/* ---- Batched launch (Section 3.2: shots, and here whole programs, are
 * independent, so many compiled programs share one launch): many programs
 * of different width and active dimension sampled by one persistent launch
 * per tier (work items: single
 * shots of shot-per-workgroup programs, groups of four shots of
 * shot-per-wave programs and 64-shot tiles of shot-per-lane programs,
 * ordered longest first by the cost model, claimed dynamically). */
typedef struct clifft_batch clifft_batch; /* opaque, owned by the library */

/* Prepare a batch of n programs (which must stay alive while the batch
 * exists), shots[i] shots of program i with Philox seed seeds[i] (host
 * arrays).  cfg: precision, optional threads_per_shot (0 automatic per
 * program, 1, 64 or 256 for all) and grid.  Uploads the item table to the
 * current device (allocates device memory, owned by the batch). */
clifft_status clifft_batch_create(const clifft_program* const* progs, int32_t n, const uint64_t* shots,
                                  const uint64_t* seeds, const clifft_launch* cfg, clifft_batch** out);

/* Sizes of the three output buffers in uint64 words, the workspace in bytes
 * and (if not NULL, n entries) the threads per shot chosen per program. */
clifft_status clifft_batch_sizes(const clifft_batch* b, uint64_t* meas_words, uint64_t* det_words,
                                 uint64_t* obs_words, size_t* workspace_bytes, int32_t* threads_per_shot);

/* Offsets (uint64 words) of program i's rows inside the three output
 * buffers; program i's records are then laid out as in clifft_sample. */
clifft_status clifft_batch_layout(const clifft_batch* b, int32_t i, uint64_t* meas_off, uint64_t* det_off,
                                  uint64_t* obs_off);

/* Sample every program of the batch in one launch on `stream` (plus small
 * zero-fill kernels for the outputs).  meas / det / obs: device buffers of
 * the sizes above (any may be NULL); workspace: device buffer of at least
 * the size above.  Records equal those of clifft_sample on each program. */
clifft_status clifft_batch_sample(const clifft_batch* b, void* workspace, size_t workspace_bytes, uint64_t* meas,
                                  uint64_t* det, uint64_t* obs, void* stream);

void clifft_batch_free(clifft_batch* b);

/* Release a program and its device copies. */
void clifft_program_free(clifft_program* p);

/* ---- Rate probes (measurement support, not part of sampling): kernels
 * whose work is known exactly, for the caller to time on `stream` and so
 * state achievable rates beside the published peaks.
 *   kind 0: copy n bytes (a multiple of 16) from src to dst, both device
 *           buffers of the caller (grid-stride, 16-byte elements);
 *   kind 1: n iterations (< 2^32) of 16 full-rate 32-bit VALU instructions
 *           per thread (eight independent xor/add chains); dst is a device
 *           buffer of grid * 256 uint32 that receives one word per thread,
 *           the XOR of the chains a <- (a ^ 0x9E3779B9) + 0x9E3779B9 started
 *           at 8 * thread + j;
 *   kind 2: read n bytes (a multiple of 16) of src; dst is a device buffer
 *           of grid * 256 16-byte elements that receives, per thread, the
 *           XOR of the elements it read (grid-stride). 
 * grid: workgroups of 256 threads.  Asynchronous; errors as status codes. */
clifft_status clifft_probe(int32_t kind, void* dst, const void* src, uint64_t n, int32_t grid, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* clifft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLIFFT_H */
