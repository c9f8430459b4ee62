// Host compiler interface (circuit text -> CompiledProgram).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "program.h"

namespace clifft {

struct CompiledProgram {
  int nq = 0, W = 1, kmax = 0;
  int nevents = 0, nrec = 0, ndet = 0, nobs = 0, nchunks = 0;
  std::vector<GInstr> code;
  std::vector<int> k_after;        // active dimension after each instruction
  std::vector<uint64_t> masks;     // W-word masks and 2W-word Pauli images
  std::vector<double> consts;      // (cos 2theta, sin 2theta, cos theta, sin theta) per angle
  std::vector<uint32_t> refs;      // detector / observable record references
  std::vector<int32_t> ev_rec;     // event -> record index or -1
  std::vector<int> ev_class;       // event -> 0 deterministic, 1 dormant random, 2 active
  std::vector<uint8_t> site_type;  // per noise site
  std::vector<double> site_p;      // per noise site probability
  std::vector<uint32_t> site_img;  // per site offset of its images in masks
  std::vector<uint8_t> site_sign;  // per site sign bits of its images (bit 2i X, 2i+1 Z of qubit i)
  std::vector<double> surv;        // nchunks x (kChunk + 1) survival products
  std::vector<int> final_slots;    // virtual qubit held by each slot at the end
  std::vector<uint32_t> rec_tgt_off, rec_tgt;  // record -> detector/observable accumulator rows
  int ndet_rows = 0;                           // detector accumulator rows (reused over time)
  std::vector<uint32_t> rblk_off;              // 128-event block -> its dormant random events
  std::vector<uint8_t> rblk_ev;
  int rblk_max = 0;
  bool has_cfeed = false;          // feed-forward Paulis (need record bits: not on the bit-sliced kernels)
  int nprobes = 0;                 // expectation-value probes (not on the bit-sliced kernels or the split form)
  int npost = 0;                   // post-selected detectors (OP_POSTSELECT; not in the split form)
  std::vector<PairLine> pline;     // paired-pass item orders (program.h), two per entry, entry 0 unused
  std::vector<int> pline_items;    // per entry: the pass's items are q < 2^pline_items
  // split form (program.h): valid when split_ok
  bool split_ok = false;
  int nactive = 0;                 // active measurement events
  int nbits = 0;                   // needed-bit rows (a rotation: one; an active measurement: two)
  int dep_words = 1;               // 64-bit words per dependency mask
  std::vector<GInstr> fcode;       // frame-only stream (k_max 0 for the bit-sliced kernel)
  std::vector<GInstr> vcode;       // vector-only stream (v: needed-bit row; MACT: a = active index)
  std::vector<int> vk_after;       // active dimension after each vector instruction
  std::vector<uint64_t> vdep;      // [nbits][dep_words] dependency masks of the needed bits
  std::vector<int32_t> vev_rec;    // event -> active index or -1 (the vector stream's records)
  std::vector<uint32_t> xdep_off;  // per output row (meas, det, obs): first entry in xdep
  std::vector<uint32_t> xdep;      // active outcome rows XORed into each output row
};

// Algorithmic work of one shot (see cost_model in compiler.cpp).
struct CostModel {
  double int_ops = 0;          // 32-bit integer lane-operations
  double flops = 0;            // floating-point operations on the active vector
  double vector_bytes = 0;     // active-vector bytes read + written (unfused)
  double record_bytes = 0;     // bit-packed record bytes written
  double expected_faults = 0;  // mean realized faults
  double instructions = 0;     // compiled instructions executed
  double int_ops_bitsliced = 0;  // integer lane-operations per shot when 32 shots share each frame word
  double vector_bytes_fused = 0;        // active-vector bytes of the fused passes, shot per lane in HBM
  double vector_bytes_fused_group = 0;  // the same for a shot per wave or per workgroup
  double vector_bytes_fused_batch = 0;  // the group tiers of the batched launch (no paired collapses)
  int pair_starts = 0;                  // measurements that start a pair on the group tiers
};
CostModel cost_model(const CompiledProgram& P, bool fp64);

// Compile options (see clifft_compile_opts in include/clifft.h).
struct CompileOptions {
  int hir_passes = 0;     // bit 1 peephole, bit 2 commuting reorder
  int k_limit = 0;        // reject k_max above this (0: kMaxK)
  bool drop_phases = false;  // omit OP_PHASE instructions
  std::vector<uint64_t> postselect;  // bit d: detector d is post-selected
  bool postselect_all = false;       // every detector is post-selected
};

// Returns 0 on success, 1 parse error, 2 unsupported instruction, 3 capacity,
// 4 invalid option (a post-selected detector the circuit does not have).
int compile_text(const char* text, size_t len, const CompileOptions& opts, CompiledProgram& out, std::string& err);

}  // namespace clifft
