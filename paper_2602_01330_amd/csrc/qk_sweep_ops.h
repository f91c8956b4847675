// The two accumulation steps of a transfer-matrix site, as explicit FMA
// sequences shared by every VALU sweep kernel (tile kernel, pair-level
// refinement, large-bond kernel), so that all of them take the same
// operations in the same order for an entry:
//   G[a][b'] += E[a][b] B^s[b][b']            (complex)
//   E'[a'][b'] += conj(A^s[a][a']) G[a][b']   (complex)
#pragma once

#include <hip/hip_runtime.h>

template <typename R, typename C>
__device__ inline void g_acc(R& gr, R& gi, R er, R ei, C bv) {
  gr = fma(er, (R)bv.x, gr);
  gr = fma(-ei, (R)bv.y, gr);
  gi = fma(er, (R)bv.y, gi);
  gi = fma(ei, (R)bv.x, gi);
}
template <typename R, typename C>
__device__ inline void e_acc(R& nr, R& ni, C av, R gr, R gi) {
  nr = fma((R)av.x, gr, nr);
  nr = fma((R)av.y, gi, nr);
  ni = fma((R)av.x, gi, ni);
  ni = fma(-(R)av.y, gr, ni);
}

// The FP64 epilogue of a pair, also with explicit fused operations so that
// every kernel that computes a pair (a tile kernel and the pass that
// recomputes marked pairs, or the large-bond kernel and its list pass)
// rounds it alike, whatever the compiler would fuse in each:
//   ln K_q = ln(Re a^2 + Im a^2) + 2 e ln 2 (Eqs. (7), (10); a rescaled by 2^-e)
//   ||x - y||^2 summed feature by feature (Eq. (3))
//   K = w K_q + (1 - w) K_c (Eq. (11))
__device__ inline double qk_ln_kq(double re, double im, int expo) {
  const double mag2 = fma(re, re, im * im);
  return mag2 > 0.0 ? fma(2.0 * (double)expo, 0.69314718055994530942, log(mag2)) : -INFINITY;
}
__device__ inline double qk_sq_dist(const double* xr, const double* xc, int d) {
  double d2 = 0.0;
  for (int f = 0; f < d; ++f) {
    const double df = xr[f] - xc[f];
    d2 = fma(df, df, d2);
  }
  return d2;
}
__device__ inline double qk_mix(double w, double kq, double kc) {
  return fma(w, kq, (1.0 - w) * kc);
}
