// Transfer-matrix overlap sweep on the vector ALUs: one pair per lane.
//
// For a pair (row sample i, column sample j) with site tensors A_k^s (row) and
// B_k^s (column), both chi x chi after padding to T:
//   E_0 = 1 (top-left entry),  E_{k+1} = sum_s A_k^{s dagger} E_k B_k^s,
// then <psi_i|psi_j> = E_n[0][0] and K_q = |E_n|^2 (Eq. (7)). After every site
// E is multiplied by 2^-e (e = frexp exponent of max|Re|,|Im|), which is exact,
// and e is added to an int32 exponent; ln K_q = 2 (ln|E_n| + e ln 2) in FP64.
//
// A workgroup of 256 lanes owns a 16 x 16 tile of pairs. The 16 row and 16
// column site tensors of the current site are staged in LDS (double-buffered:
// the next site's global loads are in flight while the current site is
// computed). Tiles of all tasks of a launch form one list walked with a static
// grid stride (persistent workgroups). The same template serves complex FP64
// (the plain comparator) and complex FP32.
#include <hip/hip_runtime.h>

#include "qk_internal.h"
#include "qk_sweep_ops.h"

namespace {

constexpr int kTile = 16;
constexpr int kThreads = kTile * kTile;

template <typename R>
struct Cx;
template <>
struct Cx<double> {
  using V = double2;
};
template <>
struct Cx<float> {
  using V = float2;
};

// Complex element idx of a site array: FP64 (Re, Im) pairs, or the packed
// FP32 (-Im, Re, Im) triples whose last two floats are (Re, Im).
__device__ inline double2 load_c(const double* base, int64_t idx) {
  return reinterpret_cast<const double2*>(base)[idx];
}
__device__ inline float2 load_c(const float* base, int64_t idx) {
  const float* e = base + idx * kQkPackFloats;
  return make_float2(e[1], e[2]);
}

// Exponent e with m = f * 2^e, f in [0.5, 1); m > 0 and normal.
__device__ inline int frexp_exp(double m) {
  return (int)((__double_as_longlong(m) >> 52) & 0x7ff) - 1022;
}
__device__ inline int frexp_exp(float m) {
  return (int)((__float_as_uint(m) >> 23) & 0xff) - 126;
}
__device__ inline double pow2(double, int e) {  // 2^e for -1022 <= e <= 1023
  return __longlong_as_double((long long)(e + 1023) << 52);
}
__device__ inline float pow2(float, int e) {  // 2^e for -126 <= e <= 127
  return __uint_as_float((unsigned)(e + 127) << 23);
}


template <typename R, int T>
struct SweepSmem {
  using C = typename Cx<R>::V;
  static constexpr int kSlot = 2 * T * T;       // complex per sample-site
  static constexpr int kStride = kSlot + 1;     // padded against bank conflicts
  C a[2][kTile * kStride];
  C b[2][kTile * kStride];
};

template <typename R, int T>
__device__ void run_tile(const QkTask& t, int ti, int tj, SweepSmem<R, T>& sm,
                         unsigned* mask_out, const uint32_t* mask_in, double ln_tau) {
  using C = typename Cx<R>::V;
  constexpr int kSlot = SweepSmem<R, T>::kSlot;
  constexpr int kStride = SweepSmem<R, T>::kStride;
  const int tid = threadIdx.x;
  const int r = tid / kTile, c = tid % kTile;
  const int64_t i0 = (int64_t)ti * kTile, j0 = (int64_t)tj * kTile;
  const int64_t i = i0 + r, j = j0 + c;
  const R* ta = static_cast<const R*>(t.ta);
  const R* tb = static_cast<const R*>(t.tb);
  const int nq = t.nq;

  // global -> register staging of one site for the whole tile
  constexpr int kPer = (2 * kTile * kSlot + kThreads - 1) / kThreads;
  C stage[kPer];
  auto load_site = [&](int k) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int e = tid + q * kThreads;
      C v;
      v.x = 0;
      v.y = 0;
      if (e < 2 * kTile * kSlot) {
        int side = e / (kTile * kSlot);
        int rem = e % (kTile * kSlot);
        int smp = rem / kSlot;
        if (side == 0) {
          if (i0 + smp < t.na) v = load_c(ta, ((int64_t)k * t.na + i0) * kSlot + rem);
        } else {
          if (j0 + smp < t.nb) v = load_c(tb, ((int64_t)k * t.nb + j0) * kSlot + rem);
        }
      }
      stage[q] = v;
    }
  };
  auto store_site = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int e = tid + q * kThreads;
      if (e < 2 * kTile * kSlot) {
        int side = e / (kTile * kSlot);
        int rem = e % (kTile * kSlot);
        int smp = rem / kSlot, o = rem % kSlot;
        if (side == 0) sm.a[buf][smp * kStride + o] = stage[q];
        else sm.b[buf][smp * kStride + o] = stage[q];
      }
    }
  };

  R er[T][T], ei[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      er[a][b] = (a == 0 && b == 0) ? R(1) : R(0);
      ei[a][b] = R(0);
    }
  int expo = 0;

  load_site(0);
  store_site(0);
  __syncthreads();
  for (int k = 0; k < nq; ++k) {
    const int buf = k & 1;
    if (k + 1 < nq) load_site(k + 1);
    const C* As = &sm.a[buf][r * kStride];
    const C* Bs = &sm.b[buf][c * kStride];
    R nr[T][T], ni[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) {
        nr[a][b] = R(0);
        ni[a][b] = R(0);
      }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // G = E B^s (T x T), then E' += A^{s dagger} G
      R gr[T][T], gi[T][T];
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int bb = 0; bb < T; ++bb) {
          gr[a][bb] = R(0);
          gi[a][bb] = R(0);
        }
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int bb = 0; bb < T; ++bb) {
          C bv = Bs[s * T * T + b * T + bb];
#pragma unroll
          for (int a = 0; a < T; ++a) g_acc(gr[a][bb], gi[a][bb], er[a][b], ei[a][b], bv);
        }
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int aa = 0; aa < T; ++aa) {
          C av = As[s * T * T + a * T + aa];  // A^s[a][aa]; dagger -> conj
#pragma unroll
          for (int bb = 0; bb < T; ++bb) e_acc(nr[aa][bb], ni[aa][bb], av, gr[a][bb], gi[a][bb]);
        }
    }
    // exact power-of-two rescale
    R m = R(0);
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) m = fmax(m, fmax(fabs(nr[a][b]), fabs(ni[a][b])));
    int e = m > R(0) ? frexp_exp(m) : 0;
    R sc = pow2(R(0), -e);
    expo += e;
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) {
        er[a][b] = nr[a][b] * sc;
        ei[a][b] = ni[a][b] * sc;
      }
    if (k + 1 < nq) store_site(buf ^ 1);
    __syncthreads();
  }

  // epilogue: ln K_q, K_q, optional RBF and mix; FP64
  const bool valid = i < t.na && j < t.nb && (!t.symmetric || j >= i);
  if (!valid) return;
  const int bit = r * kTile + c;
  // refinement pass: write only the pairs the reduced pass marked
  if (mask_in && !((mask_in[bit >> 5] >> (bit & 31)) & 1u)) return;
  const double lnk = qk_ln_kq((double)er[0][0], (double)ei[0][0], expo);
  if (mask_out && lnk > ln_tau) atomicOr(&mask_out[bit >> 5], 1u << (bit & 31));
  const double kq = exp(lnk);  // 0 for an amplitude of 0
  auto put = [&](double* p, int64_t ld, double v) {
    if (!p) return;
    p[i * ld + j] = v;
    if (t.symmetric && j != i) p[j * ld + i] = v;
  };
  put(t.kq, t.ld_kq, kq);
  put(t.lnkq, t.ld_ln, lnk);
  if (t.fuse) {
    const double kc = exp(-t.gamma * qk_sq_dist(t.xr + i * t.ld_xr, t.xc + j * t.ld_xc, nq));
    const double w = t.w_rows ? t.w_rows[i] : t.w;
    put(t.kc, t.ld_kc, kc);
    put(t.k, t.ld_k, qk_mix(w, kq, kc));
  }
}

// Largest T the persistent kernel instantiates for each real type.
template <typename R>
struct MaxT;
template <>
struct MaxT<double> {
  static constexpr int v = 4;
};
template <>
struct MaxT<float> {
  static constexpr int v = 4;
};

// One 16 x 16 tile of the task table: skipped when a refinement mask marks
// none of its pairs, else swept (and, for a reduced form, its mask written).
template <typename R>
__device__ void sweep_one_tile(const QkTaskTable& tt, int64_t q, const uint32_t* mask_in,
                               uint32_t* mask_out, double ln_tau, SweepSmem<R, MaxT<R>::v>& sm4,
                               unsigned* tile_mask) {
  const uint32_t* mi = mask_in ? mask_in + q * kQkMaskWords : nullptr;
  if (mi) {  // uniform per workgroup: skip tiles without a marked pair
    unsigned any = 0;
    for (int wd = 0; wd < kQkMaskWords; ++wd) any |= mi[wd];
    if (!any) return;
  }
  if (threadIdx.x < kQkMaskWords) tile_mask[threadIdx.x] = 0;
  __syncthreads();
  unsigned* tf = mask_out ? tile_mask : nullptr;
  int ti_task = 0;
  while (ti_task + 1 < tt.n_tasks && tt.t[ti_task + 1].tile_begin <= q) ++ti_task;
  const QkTask& t = tt.t[ti_task];
  int ti, tj;
  qk_tile_coords(t, q - t.tile_begin, ti, tj);
  switch (t.T) {
    case 1:
      run_tile<R, 1>(t, ti, tj, *reinterpret_cast<SweepSmem<R, 1>*>(&sm4), tf, mi, ln_tau);
      break;
    case 2:
      run_tile<R, 2>(t, ti, tj, *reinterpret_cast<SweepSmem<R, 2>*>(&sm4), tf, mi, ln_tau);
      break;
    default:
      run_tile<R, 4>(t, ti, tj, sm4, tf, mi, ln_tau);
      break;
  }
  __syncthreads();
  if (mask_out && threadIdx.x < kQkMaskWords)
    mask_out[q * kQkMaskWords + threadIdx.x] = tile_mask[threadIdx.x];
}

template <typename R>
__global__ __launch_bounds__(kThreads) void sweep_valu_kernel(QkTaskTable tt,
                                                              const uint32_t* mask_in,
                                                              uint32_t* mask_out,
                                                              double ln_tau) {
  __shared__ SweepSmem<R, MaxT<R>::v> sm4;
  __shared__ unsigned tile_mask[kQkMaskWords];
  for (int64_t rnd = 0; rnd * gridDim.x < tt.total_tiles; ++rnd) {
    const int64_t q = qk_tile_of(rnd, blockIdx.x, gridDim.x);
    if (q >= tt.total_tiles) continue;  // last round only; no barrier skipped
    sweep_one_tile<R>(tt, q, mask_in, mask_out, ln_tau, sm4, tile_mask);
  }
}

// Refinement: list the tiles holding marked pairs (in any order: each
// tile's result does not depend on it), so that the FP64 pass spreads them
// evenly over its workgroups instead of leaving a few workgroups with several.
__global__ void compact_marked_kernel(const uint32_t* __restrict__ mask, int64_t total_tiles,
                                      int32_t* __restrict__ list, int32_t* __restrict__ count) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= total_tiles) return;
  unsigned any = 0;
  for (int wd = 0; wd < kQkMaskWords; ++wd) any |= mask[q * kQkMaskWords + wd];
  if (any) list[atomicAdd(count, 1)] = (int32_t)q;
}

// Pair-level FP64 refinement: only the marked pairs of a marked tile are
// recomputed, 16 lanes per pair (lane (a', b') owns entry E[a'][b']) and 16
// pairs per 256-thread workgroup at a time. A site of a pair is staged in
// LDS by its own 16 lanes; G^s (lane (a, b') computes G^s[a][b'] from row a
// of E) and the new E (lane (a', b') from column b' of G^s) pass through the
// pair's LDS area. The 16 lanes of a pair sit in one wavefront, whose LDS
// operations complete in issue order, so no workgroup barrier is needed.
// Every entry follows the tile kernel's operation order (g_acc over b
// ascending, e_acc over s then a ascending, the same power-of-two rescale:
// a maximum is independent of the order it is taken in), so the refined
// value equals the tile kernel's bit for bit; a diagonal tile costs one pass
// of 16 pairs instead of 256.
constexpr int kRefPairs = kThreads / 16;

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt untouched
  __builtin_amdgcn_wave_barrier();
  __asm__ volatile("" ::: "memory");
}

// Per-pair areas sized for the largest bond dimension (4), whatever the
// tile's: the waves of a workgroup move on to the next listed tile without a
// barrier, and in a ragged launch that tile may have another bond dimension,
// so a pair's area must not move with it.
struct RefSmem {
  static constexpr int kSlotMax = 2 * 4 * 4, kTTMax = 4 * 4;
  double2 ab[2][kRefPairs][2][kSlotMax];  // [buffer][pair][A, B][s][a][b]
  double2 g[kRefPairs][2][kTTMax];        // G^s[a][b']
  double2 e[kRefPairs][kTTMax];           // E[a][b]
};

// max over the 16 lanes of a pair (aligned lane groups of 16)
__device__ inline double max16(double v) {
  v = fmax(v, __shfl_xor(v, 1, 64));
  v = fmax(v, __shfl_xor(v, 2, 64));
  v = fmax(v, __shfl_xor(v, 4, 64));
  v = fmax(v, __shfl_xor(v, 8, 64));
  return v;
}

template <int T>
__device__ void refine_tile_pairs(const QkTask& t, int ti, int tj, const uint32_t* mi,
                                  RefSmem& sm) {
  constexpr int TT = T * T, kSlot = 2 * TT;
  const int tid = threadIdx.x;
  const int p = tid >> 4, l = tid & 15, aa = l >> 2, bb = l & 3;
  const bool on = aa < T && bb < T;
  const double* ta = static_cast<const double*>(t.ta64);
  const double* tb = static_cast<const double*>(t.tb64);
  const int nq = t.nq;
  int total = 0;
  for (int wd = 0; wd < kQkMaskWords; ++wd) total += __popc(mi[wd]);
  for (int base = 0; base < total; base += kRefPairs) {
    // this pair slot takes the (base + p)-th marked bit of the tile
    int want = base + p, bit = -1;
    for (int wd = 0; wd < kQkMaskWords && bit < 0; ++wd) {
      unsigned m = mi[wd];
      const int cnt = __popc(m);
      if (want < cnt) {
        for (int q = 0; q < want; ++q) m &= m - 1;  // drop the lower set bits
        bit = wd * 32 + __ffs(m) - 1;
      } else {
        want -= cnt;
      }
    }
    const bool have = bit >= 0;
    const int64_t i = (int64_t)ti * kTile + (have ? bit / kTile : 0);
    const int64_t j = (int64_t)tj * kTile + (have ? bit % kTile : 0);
    auto load = [&](int k, double2 (&v)[2][2]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = l + 16 * h;
        v[h][0] = e < kSlot ? load_c(ta, ((int64_t)k * t.na + i) * kSlot + e) : make_double2(0, 0);
        v[h][1] = e < kSlot ? load_c(tb, ((int64_t)k * t.nb + j) * kSlot + e) : make_double2(0, 0);
      }
    };
    auto stage = [&](int buf, const double2 (&v)[2][2]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = l + 16 * h;
        if (e < kSlot) {
          sm.ab[buf][p][0][e] = v[h][0];
          sm.ab[buf][p][1][e] = v[h][1];
        }
      }
    };
    double er = (aa == 0 && bb == 0) ? 1.0 : 0.0, ei = 0.0;
    int expo = 0;
    if (on) sm.e[p][aa * T + bb] = make_double2(er, ei);
    double2 nxt[2][2];
    load(0, nxt);
    stage(0, nxt);
    wave_lds_sync();
    for (int k = 0; k < nq; ++k) {
      const int buf = k & 1;
      if (k + 1 < nq) load(k + 1, nxt);
      const double2* As = sm.ab[buf][p][0];
      const double2* Bs = sm.ab[buf][p][1];
      // G^s[a][b'] for a = aa, b' = bb
      if (on) {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          double gr = 0.0, gi = 0.0;
#pragma unroll
          for (int b = 0; b < T; ++b) {
            const double2 ev = sm.e[p][aa * T + b];
            g_acc(gr, gi, ev.x, ev.y, Bs[s2 * TT + b * T + bb]);
          }
          sm.g[p][s2][aa * T + bb] = make_double2(gr, gi);
        }
      }
      wave_lds_sync();
      // E'[a'][b'] for a' = aa, b' = bb
      double nr = 0.0, ni = 0.0;
      if (on) {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
          for (int a = 0; a < T; ++a) {
            const double2 gv = sm.g[p][s2][a * T + bb];
            e_acc(nr, ni, As[s2 * TT + a * T + aa], gv.x, gv.y);
          }
      }
      const double m = max16(fmax(fabs(nr), fabs(ni)));
      const int e = m > 0.0 ? frexp_exp(m) : 0;
      const double sc = pow2(0.0, -e);
      expo += e;
      er = nr * sc;
      ei = ni * sc;
      if (on) sm.e[p][aa * T + bb] = make_double2(er, ei);
      if (k + 1 < nq) stage(buf ^ 1, nxt);
      wave_lds_sync();
    }
    // epilogue on lane (0, 0) of the pair, as in the tile kernel
    if (have && l == 0) {
      const double lnk = qk_ln_kq(er, ei, expo);
      const double kq = exp(lnk);  // 0 for an amplitude of 0
      auto put = [&](double* ptr, int64_t ld, double v) {
        if (!ptr) return;
        ptr[i * ld + j] = v;
        if (t.symmetric && j != i) ptr[j * ld + i] = v;
      };
      put(t.kq, t.ld_kq, kq);
      put(t.lnkq, t.ld_ln, lnk);
      if (t.fuse) {
        const double kc = exp(-t.gamma * qk_sq_dist(t.xr + i * t.ld_xr, t.xc + j * t.ld_xc, nq));
        const double w = t.w_rows ? t.w_rows[i] : t.w;
        put(t.kc, t.ld_kc, kc);
        put(t.k, t.ld_k, qk_mix(w, kq, kc));
      }
    }
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(kThreads) void refine_pairs_kernel(QkTaskTable tt,
                                                                const uint32_t* mask_in,
                                                                const int32_t* list,
                                                                const int32_t* count) {
  __shared__ RefSmem sm;
  const int n = *count;
  for (int x = blockIdx.x; x < n; x += gridDim.x) {
    const int64_t q = list[x];
    int k = 0;
    while (k + 1 < tt.n_tasks && tt.t[k + 1].tile_begin <= q) ++k;
    const QkTask& t = tt.t[k];
    int ti, tj;
    qk_tile_coords(t, q - t.tile_begin, ti, tj);
    const uint32_t* mi = mask_in + q * kQkMaskWords;
    switch (t.T) {
      case 1: refine_tile_pairs<1>(t, ti, tj, mi, sm); break;
      case 2: refine_tile_pairs<2>(t, ti, tj, mi, sm); break;
      default: refine_tile_pairs<4>(t, ti, tj, mi, sm); break;
    }
  }
}

}  // namespace

int qk_sweep_valu_tile() { return kTile; }

hipError_t qk_launch_sweep_fp64(const QkTaskTable& tt, int grid, const uint32_t* mask_in,
                                hipStream_t s) {
  if (tt.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(sweep_valu_kernel<double>, dim3(grid), dim3(kThreads), 0, s, tt, mask_in,
                     (uint32_t*)nullptr, 0.0);
  return hipGetLastError();
}

namespace {
__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace

hipError_t qk_launch_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t qk_launch_refine_fp64(const QkTaskTable& tt, int grid, const uint32_t* mask,
                                 int32_t* list, int32_t* count, hipStream_t s) {
  if (tt.total_tiles == 0) return hipSuccess;
  const int64_t blocks = (tt.total_tiles + 255) / 256;
  hipLaunchKernelGGL(compact_marked_kernel, dim3((unsigned)blocks), dim3(256), 0, s, mask,
                     tt.total_tiles, list, count);
  hipLaunchKernelGGL(refine_pairs_kernel, dim3(grid), dim3(kThreads), 0, s, tt, mask,
                     (const int32_t*)list, (const int32_t*)count);
  return hipGetLastError();
}

hipError_t qk_launch_sweep_fp32(const QkTaskTable& tt, int grid, uint32_t* mask_out,
                                double ln_tau, hipStream_t s) {
  if (tt.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(sweep_valu_kernel<float>, dim3(grid), dim3(kThreads), 0, s, tt,
                     (const uint32_t*)nullptr, mask_out, ln_tau);
  return hipGetLastError();
}
