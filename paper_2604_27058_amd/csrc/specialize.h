// Program-specialized bit-sliced kernels: for a Pauli-frame-only program
// (k_max = 0) the host writes a HIP kernel in which the compiled stream is
// unrolled into straight-line code, every frame, accumulator and random-bit
// row is a register at a constant index, and each noise block applies the
// lane's precomputed faults through a switch over its own sites.  The
// kernel is compiled at run time (hiprtc) for gfx950 and keeps the
// stochastic contract of every other kernel, so its records are identical.
#pragma once
#include <string>
#include <vector>

#include "compiler.h"

namespace clifft {

// Whether the program can be specialized; *why receives the reason if not.
bool spec_supported(const CompiledProgram& P, std::string* why);

// Kernel source (prelude + generated body), entry point "clifft_frames_spec".
std::string spec_source(const CompiledProgram& P);

// Compiles source for gfx950; returns true and the code object, or false
// and the compiler log.
bool spec_compile(const std::string& src, std::vector<char>* code, std::string* log);

constexpr const char* kSpecEntry = "clifft_frames_spec";

}  // namespace clifft
