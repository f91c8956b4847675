// Complex-FP64 overlap sweep for padded bond dimensions 8..64 (circuits
// whose bonds exceed 4: more layers, or the truncating chi_max = 64 regime).
//
// Per pair (i, j) and site k:  E' = sum_s A_i^{s dagger} E B_j^s, E is
// T x T complex (Eqs. (7), (9), (10): the transfer-matrix form of the
// overlap <psi(x_i)|psi(x_j)>), with an exact power-of-two rescale every
// site and an int32 exponent, as in the other sweep forms.
//
// One workgroup per pair (a flat list of the pairs of every task; symmetric
// tasks list the upper triangle): 512 threads at T = 64, 256 at 32, one
// wavefront at 16 and 8. E and the intermediate G^s = E B^s sit in LDS
// (2 T^2 complex, rows padded by one element: 130 KB at T = 64). Each thread
// computes a KR x KC register tile of G^s and of E' (4 x 2 at T = 64, 2 x 2
// at 32 and 16, 1 x 1 at 8), so that every operand it loads (a row segment
// of B^s or A^s from memory, a column segment of E or G^s from LDS) serves
// several products; the tile columns of a wavefront read one contiguous row
// of B^s or G^s, and its tile rows share the E, A^s reads.
// Every entry follows the operation order of the FP64 tile kernel (G over b
// ascending, E' over s then a ascending).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qk_internal.h"
#include "qk_pairs.h"
#include "qk_sweep_ops.h"

namespace {

template <int T>
struct BigShape {
  static constexpr int KR = T == 64 ? 4 : (T == 8 ? 1 : 2);  // register tile rows
  static constexpr int KC = T == 8 ? 1 : 2;                  // register tile columns
  static constexpr int GR = T / KR, GC = T / KC;             // tiles per dimension
  static constexpr int kThreads = GR * GC;                   // 512, 256, 64, 64
  static constexpr int P = T + 1;                            // LDS row pitch
  // resident workgroups per CU (LDS: 2 T (T+1) x 16 B) and the waves per
  // SIMD that this asks the register allocation to leave room for
  static constexpr int kPerCu = T == 64 ? 1 : (T == 32 ? 4 : 16);
  static constexpr int kWavesPerEu = kThreads / 64 * kPerCu / 4;
};

template <int T>
struct BigSmem {
  double2 e[T * BigShape<T>::P];
  double2 g[T * BigShape<T>::P];
  double red[BigShape<T>::kThreads / 64];
};

__device__ inline double wave_max(double v) {
  for (int off = 1; off < 64; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int T>
__device__ void sweep_pair(const QkTask& t, int64_t i, int64_t j, BigSmem<T>& sm) {
  using S = BigShape<T>;
  constexpr int TT = T * T, kSlot = 2 * TT, KR = S::KR, KC = S::KC, P = S::P;
  constexpr int kThreads = S::kThreads;
  const int tid = threadIdx.x;
  const int r0 = (tid / S::GC) * KR;  // tile rows a (or a')
  const int c0 = (tid % S::GC) * KC;  // tile columns b'
  const double* ta = static_cast<const double*>(t.ta);
  const double* tb = static_cast<const double*>(t.tb);
  const int nq = t.nq;
  for (int e = tid; e < T * P; e += kThreads)
    sm.e[e] = make_double2(e == 0 ? 1.0 : 0.0, 0.0);
  int expo = 0;
  __syncthreads();
  for (int k = 0; k < nq; ++k) {
    const double2* A = reinterpret_cast<const double2*>(ta) + ((int64_t)k * t.na + i) * kSlot;
    const double2* B = reinterpret_cast<const double2*>(tb) + ((int64_t)k * t.nb + j) * kSlot;
    double nr[KR][KC], ni[KR][KC];
#pragma unroll
    for (int x = 0; x < KR; ++x)
#pragma unroll
      for (int y = 0; y < KC; ++y) nr[x][y] = ni[x][y] = 0.0;
    for (int s = 0; s < 2; ++s) {
      // G^s[a][b'] = sum_b E[a][b] B^s[b][b'], a in r0.., b' in c0..
      {
        double gr[KR][KC], gi[KR][KC];
#pragma unroll
        for (int x = 0; x < KR; ++x)
#pragma unroll
          for (int y = 0; y < KC; ++y) gr[x][y] = gi[x][y] = 0.0;
        for (int b = 0; b < T; ++b) {
          double2 ev[KR], bv[KC];
#pragma unroll
          for (int x = 0; x < KR; ++x) ev[x] = sm.e[(r0 + x) * P + b];
#pragma unroll
          for (int y = 0; y < KC; ++y) bv[y] = B[s * TT + b * T + c0 + y];
#pragma unroll
          for (int x = 0; x < KR; ++x)
#pragma unroll
            for (int y = 0; y < KC; ++y) g_acc(gr[x][y], gi[x][y], ev[x].x, ev[x].y, bv[y]);
        }
#pragma unroll
        for (int x = 0; x < KR; ++x)
#pragma unroll
          for (int y = 0; y < KC; ++y) sm.g[(r0 + x) * P + c0 + y] = make_double2(gr[x][y], gi[x][y]);
      }
      __syncthreads();
      // E'[a'][b'] += sum_a conj(A^s[a][a']) G^s[a][b'], a' in r0.., b' in c0..
      for (int a = 0; a < T; ++a) {
        double2 av[KR], gv[KC];
#pragma unroll
        for (int x = 0; x < KR; ++x) av[x] = A[s * TT + a * T + r0 + x];
#pragma unroll
        for (int y = 0; y < KC; ++y) gv[y] = sm.g[a * P + c0 + y];
#pragma unroll
        for (int x = 0; x < KR; ++x)
#pragma unroll
          for (int y = 0; y < KC; ++y) e_acc(nr[x][y], ni[x][y], av[x], gv[y].x, gv[y].y);
      }
      __syncthreads();
    }
    // exact power-of-two rescale: the exponent of the largest |entry|
    double mx = 0.0;
#pragma unroll
    for (int x = 0; x < KR; ++x)
#pragma unroll
      for (int y = 0; y < KC; ++y) mx = fmax(mx, fmax(fabs(nr[x][y]), fabs(ni[x][y])));
    mx = wave_max(mx);
    if ((tid & 63) == 0) sm.red[tid >> 6] = mx;
    __syncthreads();
    mx = sm.red[0];
    for (int w = 1; w < kThreads / 64; ++w) mx = fmax(mx, sm.red[w]);
    const int ex = mx > 0.0 ? (int)((__double_as_longlong(mx) >> 52) & 0x7ff) - 1022 : 0;
    const double sc = __longlong_as_double((long long)(1023 - ex) << 52);
    expo += ex;
#pragma unroll
    for (int x = 0; x < KR; ++x)
#pragma unroll
      for (int y = 0; y < KC; ++y)
        sm.e[(r0 + x) * P + c0 + y] = make_double2(nr[x][y] * sc, ni[x][y] * sc);
    __syncthreads();
  }
  // epilogue: ln K_q = 2 (ln|E[0][0]| + expo ln 2), K_q, fused RBF and mix
  double d2 = 0.0;
  if (t.fuse) {
    const double* xr = t.xr + i * t.ld_xr;
    const double* xc = t.xc + j * t.ld_xc;
    for (int f = tid; f < nq; f += kThreads) {
      const double df = xr[f] - xc[f];
      d2 = fma(df, df, d2);
    }
    d2 = wave_sum(d2);
    if ((tid & 63) == 0) sm.red[tid >> 6] = d2;
    __syncthreads();
    d2 = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) d2 += sm.red[w];
  }
  if (tid == 0) {
    const double lnk = qk_ln_kq(sm.e[0].x, sm.e[0].y, expo);
    const double kq = exp(lnk);  // 0 for an amplitude of 0
    qk_pair_put(t, t.kq, t.ld_kq, i, j, kq);
    qk_pair_put(t, t.lnkq, t.ld_ln, i, j, lnk);
    if (t.fuse) {
      const double kc = exp(-t.gamma * d2);
      const double w = t.w_rows ? t.w_rows[i] : t.w;
      qk_pair_put(t, t.kc, t.ld_kc, i, j, kc);
      qk_pair_put(t, t.k, t.ld_k, i, j, qk_mix(w, kq, kc));
    }
  }
  __syncthreads();  // E and the reduction slots are reused by the next pair
}

template <int T>
__global__ __launch_bounds__(BigShape<T>::kThreads, BigShape<T>::kWavesPerEu) void sweep_big_kernel(
    QkPairTable tab) {
  __shared__ BigSmem<T> sm;
  const int64_t total = tab.pair_begin[tab.n_tasks];
  for (int64_t p = blockIdx.x; p < total; p += gridDim.x) {
    int64_t i, j;
    const QkTask& t = qk_pair_lookup(tab, p, i, j);
    sweep_pair<T>(t, i, j, sm);
  }
}

template <int T>
__global__ __launch_bounds__(BigShape<T>::kThreads, BigShape<T>::kWavesPerEu) void sweep_big_list_kernel(
    QkPairTable tab, const int64_t* list, const int32_t* count) {
  __shared__ BigSmem<T> sm;
  const int32_t total = *count;
  for (int32_t q = blockIdx.x; q < total; q += gridDim.x) {
    int64_t i, j;
    const QkTask& t = qk_pair_lookup(tab, list[q], i, j);
    sweep_pair<T>(t, i, j, sm);
  }
}

int big_per_cu(int T) {
  return T == 64 ? BigShape<64>::kPerCu
                 : (T == 32 ? BigShape<32>::kPerCu
                            : (T == 16 ? BigShape<16>::kPerCu : BigShape<8>::kPerCu));
}

template <int T>
hipError_t launch_big(const QkPairTable& tab, int grid, hipStream_t s) {
  hipLaunchKernelGGL(sweep_big_kernel<T>, dim3(grid), dim3(BigShape<T>::kThreads), 0, s, tab);
  return hipGetLastError();
}

template <int T>
hipError_t launch_big_list(const QkPairTable& tab, const int64_t* list, const int32_t* count,
                           int grid, hipStream_t s) {
  hipLaunchKernelGGL(sweep_big_list_kernel<T>, dim3(grid), dim3(BigShape<T>::kThreads), 0, s,
                     tab, list, count);
  return hipGetLastError();
}

}  // namespace

bool qk_sweep_big_supports(int T) { return T == 8 || T == 16 || T == 32 || T == 64; }

hipError_t qk_launch_sweep_big(const QkTask* tasks, int n_tasks, int cus, hipStream_t s) {
  if (n_tasks < 1) return hipErrorInvalidValue;
  const int T = tasks[0].T;  // one launch per bond dimension
  QkPairTable tab{};
  const int64_t acc = qk_pair_table_fill(tasks, n_tasks, T, tab);
  if (acc < 0) return hipErrorInvalidValue;
  if (acc == 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(acc, (int64_t)cus * big_per_cu(T));
  switch (T) {
    case 8: return launch_big<8>(tab, grid, s);
    case 16: return launch_big<16>(tab, grid, s);
    case 32: return launch_big<32>(tab, grid, s);
    case 64: return launch_big<64>(tab, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t qk_launch_sweep_big_list(const QkTask* tasks, int n_tasks, const int64_t* list,
                                    const int32_t* count, int cus, hipStream_t s) {
  if (n_tasks < 1) return hipErrorInvalidValue;
  const int T = tasks[0].T;
  QkPairTable tab{};
  if (qk_pair_table_fill(tasks, n_tasks, T, tab) < 0) return hipErrorInvalidValue;
  const int grid = cus * big_per_cu(T);
  switch (T) {
    case 8: return launch_big_list<8>(tab, list, count, grid, s);
    case 16: return launch_big_list<16>(tab, list, count, grid, s);
    case 32: return launch_big_list<32>(tab, list, count, grid, s);
    case 64: return launch_big_list<64>(tab, list, count, grid, s);
    default: return hipErrorInvalidValue;
  }
}
