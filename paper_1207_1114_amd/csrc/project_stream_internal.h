// Streaming projection: device state shared by the host API and the
// kernels.  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace fpfp {

struct StreamState {
  float* Y;             // N x N, row pitch N (the caller's matrix, in place)
  long long N;
  double* a;            // N: (1 - r_i) / N of the current iterate
  float* b;             // N: (1 - c_j) / N
  float* rowpart;       // [TC][N] row partials of each tile column
  float* colpart;       // [TR][N] column partials of each tile row
  float* tmax;          // [TR * TC] tile max|dY|
  double* spart;        // [nrb] partials of s, one per reduce block
  float* mpart;         // [nrb] max|dY| of each tile row, one per reduce block
  double* scal;         // [0] s = 1^T Y 1, [1] last max|dY|
  unsigned* counters;   // [0] passes run
  unsigned* ctl;        // 0 running, 1 converged, 2 non-finite
};

}  // namespace fpfp
