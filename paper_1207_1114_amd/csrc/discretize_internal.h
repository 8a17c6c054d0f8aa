// Device greedy discretisation: the per-pair descriptor shared by the host
// API and the kernels.  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace fpfp {

struct GreedyPair {
  const float* X;       // n x np, row pitch ldx (device)
  long long ldx;
  int n, np;
  int32_t* match;       // n entries (device): column of row i, or -1
  uint64_t* suitor;     // np keys (device scratch): best proposal so far
  unsigned* flags;      // [0] non-finite entry seen, [1] proposal cap hit
  long long row_begin;  // first row / column of this pair in the batch's
  long long col_begin;  // global numbering (ascending over pairs)
};

}  // namespace fpfp
