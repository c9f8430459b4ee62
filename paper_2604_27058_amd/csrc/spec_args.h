// Kernel argument block of the program-specialized bit-sliced kernels, shared
// by the host runtime and the device code compiled at run time (plain types,
// identical layout on both sides).
#pragma once

namespace clifft_spec {

struct SpecArgs {
  unsigned long long shots, seed, offset;
  unsigned long long words64;      // ceil(shots / 64): words per record row
  unsigned int* meas32;            // record rows viewed as 32-bit words, or null
  unsigned int* det32;
  unsigned int* obs32;
  const double* surv;              // nchunks x (4096 + 1) survival products
  const unsigned char* site_type;  // per noise site (DEPOLARIZE1, DEPOLARIZE2, X, Y, Z error)
  unsigned int list_cap;           // fault-list capacity (tests may lower it)
  unsigned int pad;
};

}  // namespace clifft_spec
