// Pre-processing of raw features (Section II-A): z-score standardisation,
// principal component analysis keeping the n leading components, and min-max
// scaling of each kept component to [0, 1], all in FP64 on the device.
//
// Fit (training rows X, N x D):
//   mu_c, sigma_c        column mean and population standard deviation
//                        (two passes: the mean, then the squared deviations);
//   Z = (X - mu) / sigma (0 for a constant column);
//   C = Z^T Z / (N - 1)  the sample covariance, D x D, 16 x 16 output tiles;
//   C = V diag(lambda) V^T by the cyclic two-sided Jacobi method: each sweep
//                        is D' - 1 rounds (D' = D rounded up to even) of D'/2
//                        disjoint plane rotations chosen by a round-robin
//                        tournament, applied as C <- J^T C J and V <- V J;
//                        sweeps until the off-diagonal Frobenius norm falls
//                        below 1e-12 of the whole (or stops shrinking below
//                        1e-8 of it, the rounding floor of degenerate
//                        eigenvalue clusters);
//   components           the eigenvectors of the n largest eigenvalues (ranked
//                        on the device, ties to the smaller index), each with
//                        its entry of largest magnitude positive;
//   Y = Z W^T, per component min m_j and max M_j over the training rows.
// Apply (any rows): z-score with the fitted mu, sigma; Y = Z W^T;
//   u = (Y - m) / (M - m) (0 where M = m), times a scale.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qk_internal.h"

namespace {

constexpr int kPpThreads = 256;
constexpr int kPpTile = 16;

// deterministic block sum: fixed per-thread strides, then a fixed tree
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < kPpThreads / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// one workgroup per column c
__global__ __launch_bounds__(kPpThreads) void pp_colstats_kernel(const double* __restrict__ x,
                                                                 int64_t n, int64_t ld, int d,
                                                                 double* __restrict__ mu,
                                                                 double* __restrict__ sigma) {
  __shared__ double red[kPpThreads / 64];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kPpThreads) s += x[r * ld + c];
  const double m = block_sum(s, red) / (double)n;
  double q = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kPpThreads) {
    const double dv = x[r * ld + c] - m;
    q = fma(dv, dv, q);
  }
  const double var = block_sum(q, red) / (double)n;
  if (threadIdx.x == 0) {
    mu[c] = m;
    sigma[c] = sqrt(var);
  }
}

__global__ void pp_standardize_kernel(const double* __restrict__ x, int64_t n, int64_t ld, int d,
                                      const double* __restrict__ mu,
                                      const double* __restrict__ sigma, double* __restrict__ z) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  const int64_t r = e / d;
  const int c = (int)(e - r * d);
  const double sg = sigma[c];
  z[e] = sg > 0.0 ? (x[r * ld + c] - mu[c]) / sg : 0.0;
}

// out[i][j] = scale * sum_r A[r][ia + i] * B[r][jb + j] for a 16 x 16 tile:
// A is n x lda (columns i), B is n x ldb (columns j); with transposed = 1
// the operands are A[i][r], B[j][r] (rows) instead. One thread per output.
template <bool kRows>
__global__ __launch_bounds__(kPpThreads) void pp_gemm_tile_kernel(
    const double* __restrict__ a, int64_t lda, int m_a, const double* __restrict__ b,
    int64_t ldb, int m_b, int64_t n, double scale, double* __restrict__ out, int64_t ld_out,
    int tiles_b, int symmetric) {
  __shared__ double sa[kPpTile][kPpTile + 1], sb[kPpTile][kPpTile + 1];
  const int ti = blockIdx.x / tiles_b, tj = blockIdx.x % tiles_b;
  if (symmetric && tj < ti) return;  // the mirror writes the lower tiles
  const int ly = threadIdx.x / kPpTile, lx = threadIdx.x % kPpTile;
  const int i = ti * kPpTile + ly, j = tj * kPpTile + lx;
  double acc = 0.0;
  for (int64_t r0 = 0; r0 < n; r0 += kPpTile) {
    // stage A[r0 + ly][ti*16 + lx] and B[r0 + ly][tj*16 + lx] (kRows: A[ti*16 + ly][r0 + lx])
    {
      const int64_t r = r0 + (kRows ? lx : ly);
      const int ci = ti * kPpTile + (kRows ? ly : lx), cj = tj * kPpTile + (kRows ? ly : lx);
      double va = 0.0, vb = 0.0;
      if (r < n && ci < m_a) va = kRows ? a[(int64_t)ci * lda + r] : a[r * lda + ci];
      if (r < n && cj < m_b) vb = kRows ? b[(int64_t)cj * ldb + r] : b[r * ldb + cj];
      if (kRows) {
        sa[lx][ly] = va;  // [r][column]
        sb[lx][ly] = vb;
      } else {
        sa[ly][lx] = va;
        sb[ly][lx] = vb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPpTile; ++k) acc = fma(sa[k][ly], sb[k][lx], acc);
    __syncthreads();
  }
  if (i < m_a && j < m_b) {
    out[(int64_t)i * ld_out + j] = scale * acc;
    if (symmetric && i != j) out[(int64_t)j * ld_out + i] = scale * acc;
  }
}

// round-robin tournament of m (even) players: the pairs of round r
__device__ inline void rr_pair(int r, int i, int m, int& p, int& q) {
  const int P = m - 1;
  if (i == 0) {
    p = 0;
    q = 1 + r;
  } else {
    int u = r + i, v = r - i + P;
    if (u >= P) u -= P;
    if (v >= P) v -= P;
    p = 1 + u;
    q = 1 + v;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// The rotation of each pair of round r: (cos, sin, new C_pp, new C_qq), or
// sin = 0 when none is needed. The new diagonal uses the stable update
// C_pp - t C_pq, C_qq + t C_pq (t = sin / cos), and the pair's own
// off-diagonal entries are set to zero, as in exact arithmetic.
__global__ void pp_jac_angles_kernel(const double* __restrict__ c, int d, int m, int r,
                                     double4* __restrict__ rot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m / 2) return;
  int p, q;
  rr_pair(r, i, m, p, q);
  double cs = 1.0, sn = 0.0, na = 0.0, nb = 0.0;
  if (q < d) {  // the padding player never rotates
    const double a = c[(int64_t)p * d + p], b = c[(int64_t)q * d + q];
    const double g = c[(int64_t)p * d + q];
    if (fabs(g) > 1e-300 && fabs(g) > 1e-17 * sqrt(fabs(a) * fabs(b))) {
      const double th = (b - a) / (2.0 * g);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(fma(th, th, 1.0)));
      cs = 1.0 / sqrt(fma(t, t, 1.0));
      sn = t * cs;
      na = fma(-t, g, a);
      nb = fma(t, g, b);
    }
  }
  rot[i] = make_double4(cs, sn, na, nb);
}

// (cp, cq) -> (cs cp - sn cq, sn cp + cs cq), one rounding order for every
// element, so the row update of (p, j) and the column update of (j, p)
// produce the same bits from the same inputs and C stays symmetric
__device__ inline void rotate(double cs, double sn, double& cp, double& cq) {
  const double u = sn * cq, v = cs * cq;
  const double np = fma(cs, cp, -u), nq = fma(sn, cp, v);
  cp = np;
  cq = nq;
}

// C <- J^T C: rows p, q of every pair; grid (column chunks, pairs)
__global__ void pp_jac_rows_kernel(double* __restrict__ c, int d, int m, int r,
                                   const double4* __restrict__ rot) {
  const int i = blockIdx.y;
  const double4 cr = rot[i];
  if (cr.y == 0.0) return;
  int p, q;
  rr_pair(r, i, m, p, q);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double cp = c[(int64_t)p * d + j], cq = c[(int64_t)q * d + j];
  rotate(cr.x, cr.y, cp, cq);
  c[(int64_t)p * d + j] = cp;
  c[(int64_t)q * d + j] = cq;
}

// C <- C J and V <- V J: columns p, q of every pair; the pair's own 2 x 2
// block takes the stable diagonal and exact zeros
__global__ void pp_jac_cols_kernel(double* __restrict__ c, double* __restrict__ v, int d, int m,
                                   int r, const double4* __restrict__ rot) {
  const int i = blockIdx.y;
  const double4 cr = rot[i];
  if (cr.y == 0.0) return;
  int p, q;
  rr_pair(r, i, m, p, q);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double cp = c[(int64_t)j * d + p], cq = c[(int64_t)j * d + q];
  rotate(cr.x, cr.y, cp, cq);
  if (j == p) {
    cp = cr.z;
    cq = 0.0;
  } else if (j == q) {
    cp = 0.0;
    cq = cr.w;
  }
  c[(int64_t)j * d + p] = cp;
  c[(int64_t)j * d + q] = cq;
  double vp = v[(int64_t)j * d + p], vq = v[(int64_t)j * d + q];
  rotate(cr.x, cr.y, vp, vq);
  v[(int64_t)j * d + p] = vp;
  v[(int64_t)j * d + q] = vq;
}

// off-diagonal and total squared mass: out[0] = sum_{i != j} c_ij^2, out[1] = sum c_ij^2
__global__ __launch_bounds__(kPpThreads) void pp_offdiag_kernel(const double* __restrict__ c,
                                                                int d, double* __restrict__ out) {
  __shared__ double red[kPpThreads / 64];
  double off = 0.0, tot = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)d * d; e += kPpThreads) {
    const double x = c[e];
    tot = fma(x, x, tot);
    if (e / d != e % d) off = fma(x, x, off);
  }
  off = block_sum(off, red);
  tot = block_sum(tot, red);
  if (threadIdx.x == 0) {
    out[0] = off;
    out[1] = tot;
  }
}

// eigenvalues (the diagonal) ranked in decreasing order, ties to the smaller
// index: perm[rank] = i; lam[rank] = lambda_i
__global__ void pp_rank_kernel(const double* __restrict__ c, int d, int* __restrict__ perm,
                               double* __restrict__ lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  const double li = c[(int64_t)i * d + i];
  int rank = 0;
  for (int j = 0; j < d; ++j) {
    const double lj = c[(int64_t)j * d + j];
    rank += (lj > li) || (lj == li && j < i);
  }
  perm[rank] = i;
  lam[rank] = li;
}

// component k = column perm[k] of V, with its entry of largest magnitude
// positive (the first such entry on ties): W[k][i]; one workgroup per k
__global__ __launch_bounds__(kPpThreads) void pp_components_kernel(const double* __restrict__ v,
                                                                   int d,
                                                                   const int* __restrict__ perm,
                                                                   double* __restrict__ w) {
  __shared__ double rv[kPpThreads / 64];
  __shared__ int ri[kPpThreads / 64];
  const int k = blockIdx.x;
  int col = perm[k];
  col = col < 0 ? 0 : (col >= d ? d - 1 : col);  // a ranking over non-finite values
  double best = -1.0;
  int bi = d;
  for (int i = threadIdx.x; i < d; i += kPpThreads) {
    const double a = fabs(v[(int64_t)i * d + col]);
    if (a > best) {  // strides visit i in increasing order: keeps the first
      best = a;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    rv[threadIdx.x >> 6] = best;
    ri[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  double b = rv[0];
  int bidx = ri[0];
  for (int u = 1; u < kPpThreads / 64; ++u)
    if (rv[u] > b || (rv[u] == b && ri[u] < bidx)) {
      b = rv[u];
      bidx = ri[u];
    }
  const double sgn = v[(int64_t)bidx * d + col] < 0.0 ? -1.0 : 1.0;
  for (int i = threadIdx.x; i < d; i += kPpThreads) w[(int64_t)k * d + i] = sgn * v[(int64_t)i * d + col];
}

// per column j of Y (n x k): minimum and maximum; one workgroup per column
__global__ __launch_bounds__(kPpThreads) void pp_minmax_kernel(const double* __restrict__ y,
                                                               int64_t n, int k,
                                                               double* __restrict__ ymin,
                                                               double* __restrict__ ymax) {
  __shared__ double r0[kPpThreads / 64], r1[kPpThreads / 64];
  const int j = blockIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t r = threadIdx.x; r < n; r += kPpThreads) {
    const double v = y[r * k + j];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = lo;
    r1[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kPpThreads / 64; ++w) {
      lo = fmin(lo, r0[w]);
      hi = fmax(hi, r1[w]);
    }
    lo = fmin(lo, r0[0]);
    hi = fmax(hi, r1[0]);
    ymin[j] = lo;
    ymax[j] = hi;
  }
}

__global__ void pp_scale_kernel(const double* __restrict__ y, int64_t n, int k,
                                const double* __restrict__ ymin, const double* __restrict__ ymax,
                                double scale, double* __restrict__ out, int64_t ld_out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t r = e / k;
  const int j = (int)(e - r * k);
  const double span = ymax[j] - ymin[j];
  out[r * ld_out + j] = span > 0.0 ? scale * ((y[e] - ymin[j]) / span) : 0.0;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t qk_launch_pp_colstats(const double* x, int64_t n, int64_t ld, int d, double* mu,
                                 double* sigma, hipStream_t s) {
  hipLaunchKernelGGL(pp_colstats_kernel, dim3(d), dim3(kPpThreads), 0, s, x, n, ld, d, mu, sigma);
  return hipGetLastError();
}

hipError_t qk_launch_pp_standardize(const double* x, int64_t n, int64_t ld, int d,
                                    const double* mu, const double* sigma, double* z,
                                    hipStream_t s) {
  if (n * d == 0) return hipSuccess;
  hipLaunchKernelGGL(pp_standardize_kernel, dim3(blocks_for(n * d, 256)), dim3(256), 0, s, x, n,
                     ld, d, mu, sigma, z);
  return hipGetLastError();
}

hipError_t qk_launch_pp_cov(const double* z, int64_t n, int d, double* c, hipStream_t s) {
  const int t = (d + kPpTile - 1) / kPpTile;
  hipLaunchKernelGGL(pp_gemm_tile_kernel<false>, dim3(t * t), dim3(kPpThreads), 0, s, z,
                     (int64_t)d, d, z, (int64_t)d, d, n, 1.0 / (double)(n - 1), c, (int64_t)d, t,
                     1);
  return hipGetLastError();
}

hipError_t qk_launch_pp_project(const double* z, int64_t n, int d, const double* w, int k,
                                double* y, hipStream_t s) {
  // y[r][j] = sum_i z[r][i] w[j][i]: rows of z against rows of w
  const int ta = (int)((n + kPpTile - 1) / kPpTile), tb = (k + kPpTile - 1) / kPpTile;
  hipLaunchKernelGGL(pp_gemm_tile_kernel<true>, dim3(ta * tb), dim3(kPpThreads), 0, s, z,
                     (int64_t)d, (int)n, w, (int64_t)d, k, (int64_t)d, 1.0, y, (int64_t)k, tb, 0);
  return hipGetLastError();
}

hipError_t qk_launch_pp_jacobi_round(double* c, double* v, int d, int m, int r, double4* rot,
                                     hipStream_t s) {
  const int pairs = m / 2;
  hipLaunchKernelGGL(pp_jac_angles_kernel, dim3(blocks_for(pairs, 128)), dim3(128), 0, s, c, d,
                     m, r, rot);
  const dim3 g(blocks_for(d, 128), pairs);
  hipLaunchKernelGGL(pp_jac_rows_kernel, g, dim3(128), 0, s, c, d, m, r, rot);
  hipLaunchKernelGGL(pp_jac_cols_kernel, g, dim3(128), 0, s, c, v, d, m, r, rot);
  return hipGetLastError();
}

hipError_t qk_launch_pp_offdiag(const double* c, int d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(pp_offdiag_kernel, dim3(1), dim3(kPpThreads), 0, s, c, d, out);
  return hipGetLastError();
}

hipError_t qk_launch_pp_components(const double* c, const double* v, int d, int k, int* perm,
                                   double* lam, double* w, hipStream_t s) {
  // every rank slot starts valid; with finite eigenvalues the ranking writes
  // each slot exactly once
  const hipError_t e = hipMemsetAsync(perm, 0, d * sizeof(int), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pp_rank_kernel, dim3(blocks_for(d, 128)), dim3(128), 0, s, c, d, perm, lam);
  hipLaunchKernelGGL(pp_components_kernel, dim3(k), dim3(kPpThreads), 0, s, v, d, perm, w);
  return hipGetLastError();
}

hipError_t qk_launch_pp_minmax(const double* y, int64_t n, int k, double* ymin, double* ymax,
                               hipStream_t s) {
  hipLaunchKernelGGL(pp_minmax_kernel, dim3(k), dim3(kPpThreads), 0, s, y, n, k, ymin, ymax);
  return hipGetLastError();
}

hipError_t qk_launch_pp_scale(const double* y, int64_t n, int k, const double* ymin,
                              const double* ymax, double scale, double* out, int64_t ld_out,
                              hipStream_t s) {
  if (n * k == 0) return hipSuccess;
  hipLaunchKernelGGL(pp_scale_kernel, dim3(blocks_for(n * k, 256)), dim3(256), 0, s, y, n, k,
                     ymin, ymax, scale, out, ld_out);
  return hipGetLastError();
}
