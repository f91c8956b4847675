// Flat pair lists for the per-pair sweep kernels (large padded bond
// dimensions): the pairs of every task of one launch, numbered task by task.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qk_internal.h"

struct QkPairTable {
  QkTask t[QK_MAX_TASKS];
  int64_t pair_begin[QK_MAX_TASKS + 1];
  int n_tasks;
};

// Fills the table; every task must have bond dimension T. Returns the total
// number of pairs, or -1 for an invalid task list.
inline int64_t qk_pair_table_fill(const QkTask* tasks, int n_tasks, int T, QkPairTable& tab) {
  if (n_tasks < 1 || n_tasks > QK_MAX_TASKS) return -1;
  int64_t acc = 0;
  for (int k = 0; k < n_tasks; ++k) {
    if (tasks[k].T != T) return -1;
    tab.t[k] = tasks[k];
    tab.pair_begin[k] = acc;
    acc += tasks[k].symmetric ? tasks[k].na * (tasks[k].na + 1) / 2 : tasks[k].na * tasks[k].nb;
  }
  tab.pair_begin[n_tasks] = acc;
  tab.n_tasks = n_tasks;
  return acc;
}

// (i, j) of local pair l: row-major over na x nb, or the upper triangle
// (j >= i) of n x n row by row
__device__ inline void qk_pair_of(const QkTask& t, int64_t l, int64_t& i, int64_t& j) {
  if (!t.symmetric) {
    i = l / t.nb;
    j = l - i * t.nb;
    return;
  }
  const int64_t n = t.na;
  // rows before row i: i n - i (i - 1) / 2
  const double b2 = 2.0 * (double)n + 1.0;
  int64_t r = (int64_t)((b2 - sqrt(b2 * b2 - 8.0 * (double)l)) * 0.5);
  if (r < 0) r = 0;
  if (r > n - 1) r = n - 1;
  auto before = [&](int64_t q) { return q * n - q * (q - 1) / 2; };
  while (r > 0 && before(r) > l) --r;
  while (r + 1 < n && before(r + 1) <= l) ++r;
  i = r;
  j = r + (l - before(r));
}

// Global pair p -> task index and (i, j).
__device__ inline const QkTask& qk_pair_lookup(const QkPairTable& tab, int64_t p, int64_t& i,
                                               int64_t& j) {
  int k = 0;
  while (k + 1 < tab.n_tasks && tab.pair_begin[k + 1] <= p) ++k;
  qk_pair_of(tab.t[k], p - tab.pair_begin[k], i, j);
  return tab.t[k];
}

// Writes entry (i, j) of an output matrix, and (j, i) for symmetric tasks.
__device__ inline void qk_pair_put(const QkTask& t, double* ptr, int64_t ld, int64_t i, int64_t j,
                                   double v) {
  if (!ptr) return;
  ptr[i * ld + j] = v;
  if (t.symmetric && j != i) ptr[j * ld + i] = v;
}
