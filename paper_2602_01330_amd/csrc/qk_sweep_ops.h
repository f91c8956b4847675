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
