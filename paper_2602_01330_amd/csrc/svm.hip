// SVM training and one-against-one prediction on precomputed kernel
// matrices (Eqs. (1), (2), (4), (5); multiclass by one-against-one voting,
// Section II-B).
//
// Training solves the dual of Eqs. (1)-(2) by sequential minimal
// optimisation with the second-order pair selection of Fan, Chen and Lin
// (JMLR 6, 2005). One workgroup owns one binary problem (one pair of
// classes); all problems of a class set run in one launch. Thread k owns the
// problem's samples t = k, k + 256, ...: their multiplier a_t, gradient G_t
// and diagonal K_tt live in a global scratch slice that only that thread
// writes, so one step needs four barriers: one per block reduction (i, the
// stopping gap, j) and one for the broadcast of the step.
//
// Per step, in the problem's sample order, with v_t = -y_t G_t:
//   i = argmax v over I_up, m = v_i; M = min v over I_low; stop if m - M < eps;
//   j = argmin over t in I_low, v_t < m, of -(m - v_t)^2 / a_it,
//       a_it = K_ii + K_tt - 2 K_it (tau when not positive);
//   s = min((m - v_j) / a_ij, room of a_i, room of a_j); a_i += y_i s,
//   a_j -= y_j s (a coordinate reaching a bound is set to it);
//   G_t += y_t ((K_it - K_jt) s).
// Ties go to the smallest index. FP contraction is off in this file, so each
// product and sum is rounded on its own, in the order written, and the pair
// choices match a plain FP64 evaluation of the same formulas.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "qk_internal.h"

#pragma clang fp contract(off)

namespace {

constexpr int kSvmThreads = 256;
constexpr int kSvmWaves = kSvmThreads / 64;
constexpr double kSvmTau = 1e-12;

struct ArgBest {
  double v;
  int i;
};

// larger value wins; equal values: smaller index
__device__ inline ArgBest better_max(ArgBest a, ArgBest b) {
  return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}
// smaller value wins; equal values: smaller index
__device__ inline ArgBest better_min(ArgBest a, ArgBest b) {
  return (b.v < a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}

template <bool kMax>
__device__ ArgBest block_arg(ArgBest x, ArgBest* red) {
  for (int off = 32; off > 0; off >>= 1) {
    ArgBest o{__shfl_xor(x.v, off, 64), __shfl_xor(x.i, off, 64)};
    x = kMax ? better_max(x, o) : better_min(x, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  ArgBest r = red[0];
  for (int w = 1; w < kSvmWaves; ++w) r = kMax ? better_max(r, red[w]) : better_min(r, red[w]);
  return r;  // every thread holds the same result
}

__global__ __launch_bounds__(kSvmThreads) void svm_smo_kernel(
    const double* __restrict__ K, int64_t ld_k, const int32_t* __restrict__ idx,
    const double* __restrict__ yv, const int64_t* __restrict__ off, double C, double eps,
    int64_t max_iter, double* __restrict__ alpha, double* __restrict__ grad,
    double* __restrict__ diag, double* __restrict__ coef, int64_t ld_coef, int64_t n_all,
    double* __restrict__ b_out, int64_t* __restrict__ iters_out) {
  __shared__ ArgBest red_up[kSvmWaves], red_low[kSvmWaves], red_j[kSvmWaves];
  __shared__ double bc[3];  // step s, new a_i, new a_j
  const int p = blockIdx.x;
  const int64_t base = off[p];
  const int np = (int)(off[p + 1] - base);
  const int32_t* ix = idx + base;
  const double* y = yv + base;
  double* a = alpha + base;
  double* G = grad + base;
  double* dg = diag + base;
  const int tid = threadIdx.x;

  for (int t = tid; t < np; t += kSvmThreads) {
    a[t] = 0.0;
    G[t] = -1.0;
    dg[t] = K[(int64_t)ix[t] * ld_k + ix[t]];
  }
  __syncthreads();

  int64_t it = 0;
  while (it < max_iter) {
    // pair selection, first half: i and the stopping gap
    ArgBest up{-DBL_MAX, INT_MAX}, low{DBL_MAX, INT_MAX};
    bool any_up = false, any_low = false;
    for (int t = tid; t < np; t += kSvmThreads) {
      const double v = y[t] > 0.0 ? -G[t] : G[t];
      const double at = a[t];
      if ((y[t] > 0.0 && at < C) || (y[t] < 0.0 && at > 0.0)) {
        any_up = true;
        up = better_max(up, ArgBest{v, t});
      }
      if ((y[t] > 0.0 && at > 0.0) || (y[t] < 0.0 && at < C)) {
        any_low = true;
        low = better_min(low, ArgBest{v, t});
      }
    }
    if (!any_up) up.i = INT_MAX;
    if (!any_low) low.i = INT_MAX;
    up = block_arg<true>(up, red_up);
    low = block_arg<false>(low, red_low);
    if (up.i >= np || low.i >= np) break;  // one of the sets is empty
    const double m = up.v;
    if (!(m - low.v >= eps)) break;         // converged (or a non-finite gap)
    const int i = up.i;
    const double* Ki = K + (int64_t)ix[i] * ld_k;
    const double Kii = dg[i];
    // second half: j by the second-order gain
    ArgBest jb{DBL_MAX, INT_MAX};
    for (int t = tid; t < np; t += kSvmThreads) {
      const double v = y[t] > 0.0 ? -G[t] : G[t];
      const double at = a[t];
      const bool in_low = (y[t] > 0.0 && at > 0.0) || (y[t] < 0.0 && at < C);
      if (in_low && v < m) {
        const double bt = m - v;
        double q = (Kii + dg[t]) - 2.0 * Ki[ix[t]];
        q = q > 0.0 ? q : kSvmTau;
        jb = better_min(jb, ArgBest{-(bt * bt) / q, t});
      }
    }
    jb = block_arg<false>(jb, red_j);
    if (jb.i >= np) break;  // no admissible partner (non-finite values)
    const int j = jb.i;
    const double* Kj = K + (int64_t)ix[j] * ld_k;
    if (tid == 0) {
      double q = (Kii + dg[j]) - 2.0 * Ki[ix[j]];
      if (!(q > 0.0)) q = kSvmTau;
      const double vj = y[j] > 0.0 ? -G[j] : G[j];
      const double s_star = (m - vj) / q;
      const double room_i = y[i] > 0.0 ? C - a[i] : a[i];
      const double room_j = y[j] > 0.0 ? a[j] : C - a[j];
      const double s = fmin(s_star, fmin(room_i, room_j));
      bc[0] = s;
      bc[1] = s == room_i ? (y[i] > 0.0 ? C : 0.0) : a[i] + y[i] * s;
      bc[2] = s == room_j ? (y[j] > 0.0 ? 0.0 : C) : a[j] - y[j] * s;
    }
    __syncthreads();
    const double s = bc[0];
    for (int t = tid; t < np; t += kSvmThreads) {
      const int64_t c = ix[t];
      G[t] = G[t] + y[t] * ((Ki[c] - Kj[c]) * s);
      if (t == i) a[t] = bc[1];
      if (t == j) a[t] = bc[2];
    }
    ++it;
  }
  __syncthreads();

  // bias from the KKT conditions, summed in sample order by one thread
  if (tid == 0) {
    double acc = 0.0, lo = -DBL_MAX, hi = DBL_MAX;
    int64_t nfree = 0;
    bool has_lo = false, has_hi = false;
    for (int t = 0; t < np; ++t) {
      const double v = y[t] > 0.0 ? -G[t] : G[t];
      if (a[t] > 0.0 && a[t] < C) {
        acc = acc + v;
        ++nfree;
      } else if ((a[t] == 0.0 && y[t] > 0.0) || (a[t] == C && y[t] < 0.0)) {
        lo = has_lo ? fmax(lo, v) : v;
        has_lo = true;
      } else {
        hi = has_hi ? fmin(hi, v) : v;
        has_hi = true;
      }
    }
    double b = 0.0;
    if (nfree > 0) b = acc / (double)nfree;
    else if (has_lo && has_hi) b = (lo + hi) / 2.0;
    else if (has_lo) b = lo;
    else if (has_hi) b = hi;
    b_out[p] = b;
    iters_out[p] = it;
  }
  // dense coefficient row: a_t y_t at the problem's samples, zero elsewhere
  double* crow = coef + (int64_t)p * ld_coef;
  for (int64_t c = tid; c < n_all; c += kSvmThreads) crow[c] = 0.0;
  __syncthreads();
  for (int t = tid; t < np; t += kSvmThreads) crow[ix[t]] = a[t] * y[t];
}

// One workgroup per kernel row: the decision value of every problem
// (Eq. (5)), then the one-against-one vote.
__global__ __launch_bounds__(kSvmThreads) void svm_predict_kernel(
    const double* __restrict__ K, int64_t ld_k, int64_t n, const double* __restrict__ coef,
    int64_t ld_coef, const double* __restrict__ b, int n_classes, double* __restrict__ f,
    int64_t ld_f, int32_t* __restrict__ labels) {
  __shared__ double red[kSvmWaves];
  __shared__ int votes[64];
  const int64_t r = blockIdx.x;
  const double* row = K + r * ld_k;
  const int tid = threadIdx.x;
  if (tid < 64) votes[tid] = 0;
  int p = 0;
  for (int ca = 0; ca < n_classes; ++ca) {
    for (int cb = ca + 1; cb < n_classes; ++cb, ++p) {
      const double* cr = coef + (int64_t)p * ld_coef;
      double acc = 0.0;
      for (int64_t c = tid; c < n; c += kSvmThreads) acc = acc + cr[c] * row[c];
      for (int o = 32; o > 0; o >>= 1) acc = acc + __shfl_xor(acc, o, 64);
      if ((tid & 63) == 0) red[tid >> 6] = acc;
      __syncthreads();
      if (tid == 0) {
        const double fv = ((red[0] + red[1]) + (red[2] + red[3])) + b[p];
        if (f) f[r * ld_f + p] = fv;
        ++votes[fv > 0.0 ? ca : cb];
      }
      __syncthreads();  // red is rewritten by the next problem
    }
  }
  if (tid == 0 && labels) {
    int best = 0;
    for (int c = 1; c < n_classes; ++c)
      if (votes[c] > votes[best]) best = c;
    labels[r] = best;
  }
}

}  // namespace

hipError_t qk_launch_svm_smo(const double* k, int64_t ld_k, const int32_t* idx, const double* y,
                             const int64_t* off, int n_problems, double C, double eps,
                             int64_t max_iter, double* alpha, double* grad, double* diag,
                             double* coef, int64_t ld_coef, int64_t n_all, double* b,
                             int64_t* iters, hipStream_t s) {
  if (n_problems == 0) return hipSuccess;
  hipLaunchKernelGGL(svm_smo_kernel, dim3((unsigned)n_problems), dim3(kSvmThreads), 0, s, k,
                     ld_k, idx, y, off, C, eps, max_iter, alpha, grad, diag, coef, ld_coef,
                     n_all, b, iters);
  return hipGetLastError();
}

hipError_t qk_launch_svm_predict(const double* k, int64_t m, int64_t n, int64_t ld_k,
                                 const double* coef, int64_t ld_coef, const double* b,
                                 int n_classes, double* f, int64_t ld_f, int32_t* labels,
                                 hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(svm_predict_kernel, dim3((unsigned)m), dim3(kSvmThreads), 0, s, k, ld_k, n,
                     coef, ld_coef, b, n_classes, f, ld_f, labels);
  return hipGetLastError();
}
