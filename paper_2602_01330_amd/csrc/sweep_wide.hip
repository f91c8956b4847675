// Complex-FP32 overlap sweep on the matrix cores for padded bond dimensions
// 8..64 (circuits whose bonds exceed 4: more layers, or the truncating
// chi_max = 64 regime).
//
// Per pair (i, j) and site k:  E' = sum_s A_i^{s dagger} E B_j^s, E is
// T x T complex (Eqs. (7), (9), (10): the transfer-matrix form of the overlap
// <psi(x_i)|psi(x_j)>), with an exact power-of-two rescale of E every eight
// sites and an int32 exponent, as in the other sweep forms.
//
// One workgroup per pair with T/16 wavefronts (T = 8 runs padded to 16).
// Both products are realified complex GEMMs on v_mfma_f32_16x16x4f32 whose A
// operand comes from registers and whose B operand is a site tensor:
//   R:  G^s[a][b']    = sum_b E[a][b] B^s[b][b']
//   L:  E'^T[b'][a']  = sum_a G^s[a][b'] conj(A^s[a][a'])
// An accumulator tile of that instruction holds column j = lane mod 16 and
// row 4 (lane / 16) + r in register r. Read as an A operand, register r of a
// tile is the 16 x 4 slice whose k = lane / 16 stands for row 4k + r of the
// tile's row block; the site tensor rows are read in the same permuted
// order, so every product consumes the previous product's accumulators
// without moving them. Wavefront w owns rows a in [16w, 16w + 16) of E (held
// transposed, as the L accumulators leave it) and of G^s; L contracts over
// all a, so each wavefront writes its G^s rows to LDS in the layout the
// others read them back (one 8-byte word per lane, consecutive lanes).
// The two s terms use separate LDS slots: two barriers per site.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qk_internal.h"
#include "qk_pairs.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWideRescaleEvery = 8;

template <int T>
struct WideShape {
  static constexpr int TP = T < 16 ? 16 : T;  // padded to whole 16-blocks
  static constexpr int NB = TP / 16;          // blocks per bond index = wavefronts
  static constexpr int kThreads = 64 * NB;
  static constexpr int64_t kSlotFloats = (int64_t)2 * T * T * kQkPackFloats;
};

template <int T>
struct WideSmem {
  static constexpr int NB = WideShape<T>::NB, TP = WideShape<T>::TP;
  // B^s rows padded by 4 elements: the four row groups of an operand read
  // fall on alternate halves of the banks
  static constexpr int kPitch = TP + 4;
  float2 g[NB][NB][4][64];  // G^s: [row block][column block][register][lane]
  float2 b[TP][kPitch];     // B^s as (Re, Im); zero outside T x T
  float red[NB];
  double d2[NB];
};

// Element (row, col) of one s-slice of a packed site tensor, as (-Im, Re,
// Im); zero in the padding of T = 8.
template <int T>
__device__ inline float3 ld_pk(const float* slice, int row, int col) {
  if (T < 16 && (row >= T || col >= T)) return make_float3(0.f, 0.f, 0.f);
  const float* p = slice + ((int64_t)row * T + col) * kQkPackFloats;
  return make_float3(p[0], p[1], p[2]);
}

__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline float wave_fmax(float v) {
  for (int off = 1; off < 64; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_dsum(double v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The workgroup's share of one B^s slice: (Re, Im) of elements
// tid + kThreads m, row-major over T x T.
template <int T>
struct BStage {
  static constexpr int kThreads = WideShape<T>::kThreads;
  static constexpr int kPer = (T * T + kThreads - 1) / kThreads;
  float2 v[kPer];
  __device__ void load(const float* slice) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kThreads * m;
      if (T * T % kThreads == 0 || e < T * T) {
        const float* p = slice + (int64_t)e * kQkPackFloats;
        v[m] = make_float2(p[1], p[2]);
      }
    }
  }
  __device__ void store(WideSmem<T>& sm) const {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kThreads * m;
      if (T * T % kThreads == 0 || e < T * T) sm.b[e / T][e % T] = v[m];
    }
  }
};

template <int T>
__device__ void wide_pair(const QkTask& t, int64_t i, int64_t j, WideSmem<T>& sm,
                          int64_t pair, double ln_tau, int64_t* list, int32_t* count) {
  using S = WideShape<T>;
  constexpr int NB = S::NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  // E[a = 16 w + c][b = 16 tb + 4 g + r] in (er, ei)[tb][r]; E_0 = [1]
  float er[NB][4], ei[NB][4];
#pragma unroll
  for (int tb = 0; tb < NB; ++tb)
#pragma unroll
    for (int r = 0; r < 4; ++r) er[tb][r] = ei[tb][r] = 0.f;
  if (threadIdx.x == 0) er[0][0] = 1.f;
  int expo = 0, ex_pend = 0;
  const float* ta = static_cast<const float*>(t.ta);
  const float* tb = static_cast<const float*>(t.tb);
  const int nq = t.nq;
  constexpr int64_t kS = (int64_t)T * T * kQkPackFloats;  // floats per s-slice
  auto bslice = [&](int k, int s) { return tb + ((int64_t)k * t.nb + j) * S::kSlotFloats + s * kS; };
  BStage<T> pf;
  pf.load(bslice(0, 0));
  for (int k = 0; k < nq; ++k) {
    const float* A = ta + ((int64_t)k * t.na + i) * S::kSlotFloats;
    f4 nr[NB], ni[NB];  // E'^T tiles (column block q of E', rows a' of this wavefront)
#pragma unroll
    for (int q = 0; q < NB; ++q) nr[q] = ni[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // B^s to LDS; the barrier also ends every wavefront's reads of G^{s-1}
      pf.store(sm);
      __syncthreads();
      if (s == 0) {
        pf.load(bslice(k, 1));
      } else if (k + 1 < nq) {
        pf.load(bslice(k + 1, 0));
      }
      if (s == 0 && k > 0 && k % kWideRescaleEvery == 0) {
        // the wavefront maxima of E_k, posted at the end of the previous site
        float mx = sm.red[0];
#pragma unroll
        for (int v = 1; v < NB; ++v) mx = fmaxf(mx, sm.red[v]);
        ex_pend = mx > 0.f ? (int)((__float_as_uint(mx) >> 23) & 0xff) - 126 : 0;
      }
      // R: rows a of this wavefront of G^s, every column block q
      f4 gr[NB], gi[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) gr[q] = gi[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < NB; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * kb + 4 * g + r;
          float2 bv[NB];
#pragma unroll
          for (int q = 0; q < NB; ++q) bv[q] = sm.b[row][16 * q + c];
          const float xr = er[kb][r], xi = ei[kb][r];
#pragma unroll
          for (int q = 0; q < NB; ++q) gr[q] = mma(xr, bv[q].x, gr[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) gi[q] = mma(xr, bv[q].y, gi[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) gr[q] = mma(xi, -bv[q].y, gr[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) gi[q] = mma(xi, bv[q].x, gi[q]);
        }
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.g[w][q][r][lane] = make_float2(gr[q][r], gi[q][r]);
      __syncthreads();  // G^s visible; every wavefront is done reading B^s
      // L: E'^T += G^{s T} conj(A^s), a' in this wavefront's block
      const float* As = A + s * kS;
#pragma unroll
      for (int kb = 0; kb < NB; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float3 p = ld_pk<T>(As, 16 * kb + 4 * g + r, 16 * w + c);
          float2 gv[NB];
#pragma unroll
          for (int q = 0; q < NB; ++q) gv[q] = sm.g[kb][q][r][lane];
#pragma unroll
          for (int q = 0; q < NB; ++q) nr[q] = mma(gv[q].x, p.y, nr[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) ni[q] = mma(gv[q].y, p.y, ni[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) nr[q] = mma(gv[q].y, p.z, nr[q]);
#pragma unroll
          for (int q = 0; q < NB; ++q) ni[q] = mma(gv[q].x, p.x, ni[q]);
        }
    }
    // E_{k+1}; the exponent found from E_k scales it exactly (the map is linear)
    const bool apply = k > 0 && k % kWideRescaleEvery == 0;
    const float sc = __uint_as_float((uint32_t)(127 - ex_pend) << 23);
    float mx = 0.f;
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        er[q][r] = apply ? nr[q][r] * sc : nr[q][r];
        ei[q][r] = apply ? ni[q][r] * sc : ni[q][r];
        mx = fmaxf(mx, fmaxf(fabsf(er[q][r]), fabsf(ei[q][r])));
      }
    if (apply) expo += ex_pend;
    if (k % kWideRescaleEvery == kWideRescaleEvery - 1) {
      mx = wave_fmax(mx);
      if (lane == 0) sm.red[w] = mx;
    }
  }
  // epilogue: ln K_q = 2 (ln|E[0][0]| + expo ln 2), K_q, fused RBF and mix
  double d2 = 0.0;
  if (t.fuse) {
    const double* xr = t.xr + i * t.ld_xr;
    const double* xc = t.xc + j * t.ld_xc;
    for (int f = threadIdx.x; f < nq; f += S::kThreads) {
      const double df = xr[f] - xc[f];
      d2 = fma(df, df, d2);
    }
    d2 = wave_dsum(d2);
    if (lane == 0) sm.d2[w] = d2;
    __syncthreads();
    d2 = 0.0;
#pragma unroll
    for (int v = 0; v < NB; ++v) d2 += sm.d2[v];
  }
  if (threadIdx.x == 0) {
    const double re = er[0][0], im = ei[0][0];
    const double mag2 = re * re + im * im;
    const double lnk = mag2 > 0.0 ? log(mag2) + 2.0 * (double)expo * 0.69314718055994530942
                                  : -INFINITY;
    const double kq = mag2 > 0.0 ? exp(lnk) : 0.0;
    if (list && lnk >= ln_tau) list[atomicAdd(count, 1)] = pair;  // for the FP64 pass
    qk_pair_put(t, t.kq, t.ld_kq, i, j, kq);
    qk_pair_put(t, t.lnkq, t.ld_ln, i, j, lnk);
    if (t.fuse) {
      const double kc = exp(-t.gamma * d2);
      const double wm = t.w_rows ? t.w_rows[i] : t.w;
      qk_pair_put(t, t.kc, t.ld_kc, i, j, kc);
      qk_pair_put(t, t.k, t.ld_k, i, j, wm * kq + (1.0 - wm) * kc);
    }
  }
  __syncthreads();  // LDS slots and reduction words are reused by the next pair
}

template <int T>
__global__ __launch_bounds__(WideShape<T>::kThreads, 2) void sweep_wide_kernel(QkPairTable tab,
                                                                           double ln_tau,
                                                                           int64_t* list,
                                                                           int32_t* count) {
  __shared__ WideSmem<T> sm;
  if (T < 16) {  // the staging writes only the T x T corner of B^s
    for (int e = threadIdx.x; e < WideShape<T>::TP * WideSmem<T>::kPitch; e += blockDim.x)
      (&sm.b[0][0])[e] = make_float2(0.f, 0.f);
  }
  const int64_t total = tab.pair_begin[tab.n_tasks];
  for (int64_t p = blockIdx.x; p < total; p += gridDim.x) {
    int64_t i, j;
    const QkTask& t = qk_pair_lookup(tab, p, i, j);
    wide_pair<T>(t, i, j, sm, p, ln_tau, list, count);
  }
}

template <int T>
hipError_t launch_wide(const QkPairTable& tab, int64_t pairs, int cus, int per_cu,
                       double ln_tau, int64_t* list, int32_t* count, hipStream_t s) {
  const int grid = (int)std::min<int64_t>(pairs, (int64_t)cus * per_cu);
  hipLaunchKernelGGL(sweep_wide_kernel<T>, dim3(grid), dim3(WideShape<T>::kThreads), 0, s, tab,
                     ln_tau, list, count);
  return hipGetLastError();
}

}  // namespace

bool qk_sweep_wide_supports(int T) { return T == 8 || T == 16 || T == 32 || T == 64; }

hipError_t qk_launch_sweep_wide(const QkTask* tasks, int n_tasks, int cus, double ln_tau,
                                bool refine, int64_t* list_scratch, hipStream_t s) {
  if (n_tasks < 1) return hipErrorInvalidValue;
  const int T = tasks[0].T;  // one launch per bond dimension
  QkPairTable tab{};
  const int64_t pairs = qk_pair_table_fill(tasks, n_tasks, T, tab);
  if (pairs < 0 || pairs > INT32_MAX) return hipErrorInvalidValue;
  if (pairs == 0) return hipSuccess;
  // refinement list: up to every pair's number, then the int32 count
  int64_t* list = nullptr;
  int32_t* count = nullptr;
  hipError_t e;
  if (refine) {
    if (list_scratch) {
      list = list_scratch;  // the caller sized it for pairs + 1 words
    } else {
      e = hipMallocAsync((void**)&list, pairs * sizeof(int64_t) + sizeof(int64_t), s);
      if (e != hipSuccess) return e;
    }
    count = reinterpret_cast<int32_t*>(list + pairs);
    e = qk_launch_zero_i32(count, 1, s);
    if (e != hipSuccess) {
      if (!list_scratch) (void)hipFreeAsync(list, s);
      return e;
    }
  }
  // T = 64: 65 KB of LDS and four wavefronts per workgroup, two per CU
  switch (T) {
    case 8: e = launch_wide<8>(tab, pairs, cus, 16, ln_tau, list, count, s); break;
    case 16: e = launch_wide<16>(tab, pairs, cus, 16, ln_tau, list, count, s); break;
    case 32: e = launch_wide<32>(tab, pairs, cus, 8, ln_tau, list, count, s); break;
    case 64: e = launch_wide<64>(tab, pairs, cus, 2, ln_tau, list, count, s); break;
    default: e = hipErrorInvalidValue;
  }
  if (e == hipSuccess && refine) {
    QkTask t64[QK_MAX_TASKS];
    for (int k = 0; k < n_tasks; ++k) {
      t64[k] = tasks[k];
      t64[k].ta = tasks[k].ta64;
      t64[k].tb = tasks[k].tb64;
    }
    e = qk_launch_sweep_big_list(t64, n_tasks, list, count, cus, s);
  }
  if (list && !list_scratch) (void)hipFreeAsync(list, s);
  return e;
}
