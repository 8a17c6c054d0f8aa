// Greedy discretisation on the device (Lu, Huang & Liu, arXiv 1207.1114,
// Sec. 4.5): repeatedly take the largest remaining entry of X, match its row
// and column, and remove both; ties go to the smaller row-major index.
//
// The rule fixes a strict total order on the entries (value, then index),
// and the greedy matching is then the unique stable matching of the two
// sides when both rank partners by that order.  Row-proposing deferred
// acceptance reaches the stable matching from any interleaving of its steps,
// so it is computed here in parallel: every unmatched row proposes to its
// best column among those whose current suitor ranks below the proposal;
// a column keeps the better of the two by a 64-bit atomic max on the packed
// key; a displaced row is taken over by the wave that displaced it and
// proposes again.  The result equals the sequential rule entry for entry.
//
// Keys: high 32 bits = the value mapped to an unsigned integer that orders
// like the float (negative zero taken as zero), low 32 bits = the complement
// of the row-major index, so a larger key is a larger value or, on equal
// values, a smaller index.  Key 0 marks a free column (every finite value
// maps above it).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "discretize_internal.h"

namespace fpfp {

__device__ __forceinline__ unsigned ordered_bits(float x) {
  const unsigned b = __float_as_uint(x == 0.0f ? 0.0f : x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t entry_key(float x, unsigned idx) {
  return ((uint64_t)ordered_bits(x) << 32) | (uint64_t)(0xFFFFFFFFu - idx);
}

__device__ __forceinline__ unsigned key_index(uint64_t k) {
  return 0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFu);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Index of the pair whose [begin, begin + count) range holds g (begins are
// ascending).
template <class F>
__device__ __forceinline__ int find_pair(int batch, long long g, F begin) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin(mid) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Thread g: row g of the batch -> match -1; column g -> free; flags cleared.
__global__ void greedy_init(const GreedyPair* P, int batch,
                            long long total_rows, long long total_cols) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < total_rows) {
    const int b = find_pair(batch, g, [&](int k) { return P[k].row_begin; });
    P[b].match[g - P[b].row_begin] = -1;
  }
  if (g < total_cols) {
    const int b = find_pair(batch, g, [&](int k) { return P[k].col_begin; });
    P[b].suitor[g - P[b].col_begin] = 0ull;
    if (g == P[b].col_begin) {
      P[b].flags[0] = 0u;
      P[b].flags[1] = 0u;
    }
  }
}

// One wave per row of the batch: the row's proposal chain.
__global__ void __launch_bounds__(256)
greedy_propose(const GreedyPair* P, int batch, long long total_rows) {
  const int lane = threadIdx.x & 63;
  const long long g = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= total_rows) return;
  const int b = find_pair(batch, g, [&](int k) { return P[k].row_begin; });
  const GreedyPair p = P[b];
  const int np = p.np;
  int i = (int)(g - p.row_begin);
  // Every accepted proposal raises one column's key, each column's key takes
  // at most n values, and a rejection follows another wave's acceptance, so
  // a chain is shorter than 2 n n' + 2 steps; the cap only guards the exit.
  const long long cap = 2LL * p.n * np + 2;
  bool bad = false;
  long long step = 0;
  for (;; ++step) {
    if (step >= cap) {
      if (lane == 0)
        __hip_atomic_store(p.flags + 1, 1u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    const float* row = p.X + (long long)i * p.ldx;
    const unsigned base = (unsigned)i * (unsigned)np;
    uint64_t best = 0ull;
    for (int j = lane; j < np; j += 64) {
      const float x = row[j];
      bad |= !isfinite(x);
      const uint64_t k = entry_key(x, base + (unsigned)j);
      const uint64_t s = __hip_atomic_load(p.suitor + j, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      if (k > s && k > best) best = k;
    }
    best = wave_max_u64(best);
    if (best == 0ull) break;  // no column takes row i: it stays unmatched
    const int j = (int)(key_index(best) - base);
    uint64_t old = 0ull;
    if (lane == 0)
      old = __hip_atomic_fetch_max(p.suitor + j, best, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, 64);
    if (old < best) {          // accepted
      if (old == 0ull) break;  // the column was free: the chain ends
      i = (int)(key_index(old) / (unsigned)np);  // the displaced row
    }
    // rejected: a better proposal arrived first; row i looks again
  }
  if (__any(bad) && lane == 0)
    __hip_atomic_store(p.flags, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread g: column g of the batch writes its row's match.
__global__ void greedy_emit(const GreedyPair* P, int batch,
                            long long total_cols) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_cols) return;
  const int b = find_pair(batch, g, [&](int k) { return P[k].col_begin; });
  const GreedyPair& p = P[b];
  if (p.flags[0] != 0u || p.flags[1] != 0u) return;
  const int j = (int)(g - p.col_begin);
  const uint64_t s = p.suitor[j];
  if (s != 0ull) p.match[key_index(s) / (unsigned)p.np] = j;
}

}  // namespace fpfp

extern "C" hipError_t fpfp_greedy_launch(const fpfp::GreedyPair* P_dev,
                                         int batch, long long total_rows,
                                         long long total_cols,
                                         hipStream_t stream) {
  const long long span = total_rows > total_cols ? total_rows : total_cols;
  fpfp::greedy_init<<<dim3((unsigned)((span + 255) / 256)), dim3(256), 0,
                      stream>>>(P_dev, batch, total_rows, total_cols);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fpfp::greedy_propose<<<dim3((unsigned)((total_rows + 3) / 4)), dim3(256), 0,
                         stream>>>(P_dev, batch, total_rows);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  fpfp::greedy_emit<<<dim3((unsigned)((total_cols + 255) / 256)), dim3(256),
                      0, stream>>>(P_dev, batch, total_cols);
  return hipGetLastError();
}
