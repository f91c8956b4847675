// Classical RBF Gram matrix (Eq. (3)), the quantum-classical mix (Eq. (11))
// and the SVM decision values of kernel rows (Eqs. (4), (5)) as standalone
// kernels; FP64 throughout.
#include <hip/hip_runtime.h>

#include "qk_internal.h"

namespace {

constexpr int kT = 16;      // 16 x 16 outputs per workgroup
constexpr int kChunk = 64;  // features staged per LDS round

// K_c[i][j] = exp(-gamma * sum_t (x_it - y_jt)^2), by direct differences.
__global__ __launch_bounds__(256) void rbf_kernel(const double* __restrict__ x,
                                                  int64_t m, int64_t ld_x,
                                                  const double* __restrict__ y,
                                                  int64_t n, int64_t ld_y, int d,
                                                  double gamma,
                                                  double* __restrict__ kc,
                                                  int64_t ld_kc) {
  __shared__ double xs[kT][kChunk + 1];
  __shared__ double ys[kT][kChunk + 1];
  const int tr = threadIdx.x / kT, tc = threadIdx.x % kT;
  const int64_t i0 = (int64_t)blockIdx.y * kT, j0 = (int64_t)blockIdx.x * kT;
  double acc = 0.0;
  for (int f0 = 0; f0 < d; f0 += kChunk) {
    for (int e = threadIdx.x; e < kT * kChunk; e += 256) {
      int rr = e / kChunk, ff = e % kChunk;
      int64_t gi = i0 + rr, gj = j0 + rr;
      int f = f0 + ff;
      xs[rr][ff] = (gi < m && f < d) ? x[gi * ld_x + f] : 0.0;
      ys[rr][ff] = (gj < n && f < d) ? y[gj * ld_y + f] : 0.0;
    }
    __syncthreads();
    const int lim = (d - f0) < kChunk ? (d - f0) : kChunk;
    for (int ff = 0; ff < lim; ++ff) {
      double df = xs[tr][ff] - ys[tc][ff];
      acc += df * df;
    }
    __syncthreads();
  }
  const int64_t i = i0 + tr, j = j0 + tc;
  if (i < m && j < n) kc[i * ld_kc + j] = exp(-gamma * acc);
}

__global__ void mix_kernel(const double* __restrict__ kq, int64_t ld_kq,
                           const double* __restrict__ kc, int64_t ld_kc,
                           int64_t m, int64_t n, double w, double* k,
                           int64_t ld_k) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    k[i * ld_k + j] = w * kq[i * ld_kq + j] + (1.0 - w) * kc[i * ld_kc + j];
  }
}

// f[r] = sum_i coef[i] K[r][i] + b: one 256-thread workgroup per row, the
// columns strided over the threads (coalesced), a fixed reduction order.
__global__ __launch_bounds__(256) void svm_decision_kernel(const double* __restrict__ k,
                                                           int64_t ld_k, int64_t n,
                                                           const double* __restrict__ coef,
                                                           double b, double* __restrict__ f) {
  __shared__ double red[4];
  const int64_t r = blockIdx.x;
  const double* row = k + r * ld_k;
  double acc = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 256) acc = fma(coef[c], row[c], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) f[r] = ((red[0] + red[1]) + (red[2] + red[3])) + b;
}

}  // namespace

hipError_t qk_launch_svm_decision(const double* k, int64_t m, int64_t n, int64_t ld_k,
                                  const double* coef, double b, double* f, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(svm_decision_kernel, dim3((unsigned)m), dim3(256), 0, s, k, ld_k, n, coef,
                     b, f);
  return hipGetLastError();
}

hipError_t qk_launch_rbf(const double* x, int64_t m, int64_t ld_x,
                         const double* y, int64_t n, int64_t ld_y, int d,
                         double gamma, double* kc, int64_t ld_kc, hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  dim3 grid((unsigned)((n + kT - 1) / kT), (unsigned)((m + kT - 1) / kT));
  hipLaunchKernelGGL(rbf_kernel, grid, dim3(256), 0, s, x, m, ld_x, y, n, ld_y, d,
                     gamma, kc, ld_kc);
  return hipGetLastError();
}

hipError_t qk_launch_mix(const double* kq, int64_t ld_kq, const double* kc,
                         int64_t ld_kc, int64_t m, int64_t n, double w,
                         double* k, int64_t ld_k, hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  int64_t blocks = (m * n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(mix_kernel, dim3((unsigned)blocks), dim3(256), 0, s, kq, ld_kq,
                     kc, ld_kc, m, n, w, k, ld_k);
  return hipGetLastError();
}
