// Classical RBF Gram matrix (Eq. (3)) and the quantum-classical mix
// (Eq. (11)) as standalone kernels; FP64 throughout.
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

}  // namespace

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
