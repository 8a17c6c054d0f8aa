// Host discretisation of a soft assignment X into a partial permutation
// (Lu, Huang & Liu, arXiv 1207.1114, Sec. 4.5).
//
// * Greedy (the paper's rule, taken from spectral matching): repeatedly pick
//   the largest remaining entry, match its row and column, and remove both.
//   Implemented as one sort of all entries by (value desc, row-major index
//   asc) followed by a scan that accepts an entry when its row and column are
//   still free, which selects exactly the same entries in the same order.
// * Hungarian: the injective map of the smaller side that maximises
//   sum_i X[i, m(i)], by the shortest-augmenting-path method with dual
//   potentials (Kuhn-Munkres in its O(n^2 m) form), in float64.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <vector>

#include "fastpfp.h"

namespace {

// Minimum-cost assignment of every row of an r x c cost matrix (r <= c).
// Returns col_of_row.
std::vector<int> min_cost_rows(const std::vector<double>& cost, int r, int c) {
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<double> u(r + 1, 0.0), v(c + 1, 0.0);
  std::vector<int> row_of(c + 1, 0), prev(c + 1, 0);
  std::vector<double> dist(c + 1);
  std::vector<char> done(c + 1);
  for (int i = 1; i <= r; ++i) {
    // Grow a shortest-path tree from row i over the reduced costs until it
    // reaches a free column, then flip the path.
    row_of[0] = i;
    int j0 = 0;
    std::fill(dist.begin(), dist.end(), INF);
    std::fill(done.begin(), done.end(), 0);
    do {
      done[j0] = 1;
      const int i0 = row_of[j0];
      double best = INF;
      int j1 = 0;
      const double* crow = &cost[(size_t)(i0 - 1) * c];
      for (int j = 1; j <= c; ++j) {
        if (done[j]) continue;
        const double red = crow[j - 1] - u[i0] - v[j];
        if (red < dist[j]) {
          dist[j] = red;
          prev[j] = j0;
        }
        if (dist[j] < best) {
          best = dist[j];
          j1 = j;
        }
      }
      for (int j = 0; j <= c; ++j) {
        if (done[j]) {
          u[row_of[j]] += best;
          v[j] -= best;
        } else {
          dist[j] -= best;
        }
      }
      j0 = j1;
    } while (row_of[j0] != 0);
    do {
      const int j1 = prev[j0];
      row_of[j0] = row_of[j1];
      j0 = j1;
    } while (j0 != 0);
  }
  std::vector<int> col_of(r, -1);
  for (int j = 1; j <= c; ++j)
    if (row_of[j] > 0) col_of[row_of[j] - 1] = j - 1;
  return col_of;
}

}  // namespace

extern "C" fastpfp_status fastpfp_discretize(int n, int np, const float* X,
                                             int ldx, int method,
                                             int32_t* match, double* score) {
  if (n < 1 || np < 1 || !X || !match || ldx < np)
    return FASTPFP_ERR_INVALID_ARG;
  if (method != FASTPFP_HUNGARIAN && method != FASTPFP_GREEDY)
    return FASTPFP_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < np; ++j)
      if (!std::isfinite(X[(size_t)i * ldx + j])) return FASTPFP_ERR_NUMERIC;
  std::fill(match, match + n, -1);
  if (method == FASTPFP_GREEDY) {
    std::vector<int64_t> order((size_t)n * np);
    std::iota(order.begin(), order.end(), 0);
    auto val = [&](int64_t k) { return X[(size_t)(k / np) * ldx + k % np]; };
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      const float va = val(a), vb = val(b);
      return va > vb || (va == vb && a < b);
    });
    std::vector<char> col_used(np, 0);
    int left = std::min(n, np);
    for (int64_t k : order) {
      const int i = (int)(k / np), j = (int)(k % np);
      if (match[i] < 0 && !col_used[j]) {
        match[i] = j;
        col_used[j] = 1;
        if (--left == 0) break;
      }
    }
  } else if (n <= np) {
    std::vector<double> cost((size_t)n * np);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < np; ++j)
        cost[(size_t)i * np + j] = -(double)X[(size_t)i * ldx + j];
    std::vector<int> c = min_cost_rows(cost, n, np);
    for (int i = 0; i < n; ++i) match[i] = c[i];
  } else {
    std::vector<double> cost((size_t)np * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < np; ++j)
        cost[(size_t)j * n + i] = -(double)X[(size_t)i * ldx + j];
    std::vector<int> r = min_cost_rows(cost, np, n);
    for (int j = 0; j < np; ++j) match[r[j]] = j;
  }
  if (score) {
    double s = 0.0;
    for (int i = 0; i < n; ++i)
      if (match[i] >= 0) s += (double)X[(size_t)i * ldx + match[i]];
    *score = s;
  }
  return FASTPFP_OK;
}
