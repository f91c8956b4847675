// MPS build on the device: time-evolving block decimation of the encoding
// circuit of Eq. (6), FP64. Three kernels by padded bond bound W: eight
// samples per 64-lane wavefront for W <= 4 (mps_build8_kernel), one
// wavefront per sample for W = 8, 16 and single qubits (mps_build_kernel),
// one workgroup of 8 W threads per sample for W = 32, 64
// (mps_build_wg_kernel).
//
// Per layer: the single-qubit gates G_k = RZ(2 x_k) H on every site, then the
// RZZ(theta_k) chain as two-site steps, left to right on odd layers and right
// to left on even layers (the entanglers of one layer commute, and the
// orthogonality centre always sits on the merged pair). A step merges the two
// sites into Theta (2 chi_l x 2 chi_r), multiplies the diagonal RZZ phase,
// factors Theta = U S V^dagger with a one-sided (Hestenes) Jacobi SVD, keeps
// s_j > cutoff * s_0 (at most chi_max), renormalises the kept values and
// splits back. The site tensors live in the packed sweep layout
// [site][sample][s][a][b] (padded to T x T, zero outside the realized block),
// so the FP64 sweep reads the build's output directly.
//
// `entangle` is the entangler block size B (0: no entanglers): the chain acts
// on the pairs (k, k + 1) inside blocks of B consecutive qubits, as in the
// block-structured entangling layers of Section II-C; B >= n is the open
// chain over every qubit. A step across a block boundary applies no phase,
// so its Theta is a product across the cut and the cutoff keeps one singular
// value there.
#include <hip/hip_runtime.h>

#include "qk_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct cplx {
  double re, im;
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ inline double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}

// Sum of v over aligned groups of 2^lg lanes (lg <= 5), every lane receiving
// its group's sum. Within a 16-lane row the partners come from DPP (quad
// permutations, then the half-row and row mirrors, each pairing lanes of
// the two halves reduced so far), which keeps the data in VALU; only the
// 32-lane step crosses rows.
__device__ inline double dpp_f64(double v, int ctrl_sel) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  switch (ctrl_sel) {
    case 0: lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false); break;
    default: lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
             hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false); break;
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double group_sum(double v, int lg) {
  if (lg > 0) v += dpp_f64(v, 0);  // lane ^ 1
  if (lg > 1) v += dpp_f64(v, 1);  // lane ^ 2
  if (lg > 2) v += dpp_f64(v, 2);  // 7 - lane within 8
  if (lg > 3) v += dpp_f64(v, 3);  // 15 - lane within 16
  if (lg > 4) v += __shfl_xor(v, 16, 64);
  return v;
}

// Orders the LDS accesses of one wavefront's lanes: LDS operations of a wave
// execute in issue order, so waiting for this lane's own and keeping the
// compiler from moving memory accesses across suffices within a wave.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt untouched
  __builtin_amdgcn_wave_barrier();
  __asm__ volatile("" ::: "memory");
}

// One-sided Jacobi on the columns of X (R rows x C columns, column-major in
// LDS with leading dimension LD), accumulating V (C x C, column-major, LD).
// On return the columns of X are mutually orthogonal and X_in V = X_out.
// C must be even (a padded zero column is skipped). A pair is rotated while
// |x_p^H x_q| > 1e-14 |x_p| |x_q|; columns with |x|^2 <= floor2 are rounding
// noise of a rank-deficient X and are left alone. Returns false if the sweep
// limit was reached.
template <int LD>
__device__ bool jacobi_columns(double2* X, double2* V, int R, int C, double floor2,
                               int max_sweeps) {
  const int lane = threadIdx.x;
  const int npairs = C >> 1;
  // lanes per pair: the smallest power of two covering the rows (so the
  // dot-product reductions take log2(rows) shuffle steps), but no more than
  // the wave can give every pair
  int cap = 64 / npairs;
  cap = cap >= 32 ? 32 : (cap >= 16 ? 16 : (cap >= 8 ? 8 : (cap >= 4 ? 4 : (cap >= 2 ? 2 : 1))));
  int g = 1, lg = 0;
  while (g < R && g < cap) {
    g <<= 1;
    ++lg;
  }
  const int pair = lane >> lg;
  const int sub = lane & (g - 1);
  const bool active = pair < npairs;
  const int players = C - 1;
  const double tol = 1e-14;

  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < players; ++r) {
      int p = 0, q = 0;
      if (active) {
        // round-robin tournament: r, pair < players, so one conditional
        // subtraction reduces each index
        if (pair == 0) {
          p = 0;
          q = 1 + r;
        } else {
          int u = r + pair, v = r - pair + players;
          if (u >= players) u -= players;
          if (v >= players) v -= players;
          p = 1 + u;
          q = 1 + v;
        }
      }
      double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
      if (active) {
        for (int row = sub; row < R; row += g) {
          double2 xp = X[p * LD + row];
          double2 xq = X[q * LD + row];
          al += xp.x * xp.x + xp.y * xp.y;
          be += xq.x * xq.x + xq.y * xq.y;
          gr += xp.x * xq.x + xp.y * xq.y;  // conj(xp) * xq
          gi += xp.x * xq.y - xp.y * xq.x;
        }
      }
      al = group_sum(al, lg);
      be = group_sum(be, lg);
      gr = group_sum(gr, lg);
      gi = group_sum(gi, lg);
      const double gabs2 = gr * gr + gi * gi;
      const bool do_rot =
          active && al > floor2 && be > floor2 && gabs2 > tol * tol * (al * be);
      if (do_rot) {
        const double inv_gabs = rsqrt(gabs2);
        const double zeta = 0.5 * (be - al) * inv_gabs;
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = rsqrt(1.0 + t * t);
        const double s = c * t;
        // e^{-i phi} = conj(gamma) / |gamma|
        const double2 ph = make_double2(gr * inv_gabs, -gi * inv_gabs);
        for (int row = sub; row < R; row += g) {
          double2 xp = X[p * LD + row];
          double2 xq = cmul(ph, X[q * LD + row]);
          X[p * LD + row] = make_double2(c * xp.x - s * xq.x, c * xp.y - s * xq.y);
          X[q * LD + row] = make_double2(s * xp.x + c * xq.x, s * xp.y + c * xq.y);
        }
        for (int row = sub; row < C; row += g) {
          double2 vp = V[p * LD + row];
          double2 vq = cmul(ph, V[q * LD + row]);
          V[p * LD + row] = make_double2(c * vp.x - s * vq.x, c * vp.y - s * vq.y);
          V[q * LD + row] = make_double2(s * vp.x + c * vq.x, s * vp.y + c * vq.y);
        }
      }
      rotated |= do_rot ? 1 : 0;
      __syncthreads();
    }
    if (!__any(rotated)) return true;
  }
  return false;
}

// LDS layout per workgroup, D = 2 * W (largest Theta dimension).
template <int W>
struct BuildSmem {
  static constexpr int D = 2 * W;
  double2 X[D * D];
  double2 V[D * D];
  double2 sa[2 * W * W];  // site k copy   [s][a][b], padded to W x W
  double2 sb[2 * W * W];  // site k+1 copy
  double S[D];
  int perm[D];
};
template <int W>
__global__ __launch_bounds__(64) void mps_build_kernel(
    const double* __restrict__ x, int64_t ld_x, int64_t N, int nq, int n_layers,
    int chi_max, int entangle, double cutoff, double2* __restrict__ t64,
    int32_t* __restrict__ chi_tab, int32_t* __restrict__ status, double* __restrict__ disc_out,
    int max_sweeps) {
  constexpr int D = 2 * W;
  __shared__ BuildSmem<W> sm;
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  double2* X = sm.X;
  double2* V = sm.V;
  double2* sa = sm.sa;
  double2* sb = sm.sb;
  // the packed bond block is W x W (W is the batch's padded bond dimension),
  // so every layout index below is a compile-time shift or mask
  constexpr int T = W, TT = W * W, slot = 2 * TT;
  const double* xi = x + i * ld_x;
  int32_t* chi = chi_tab + i * (int64_t)(nq + 1);
  auto site = [&](int k) -> double2* { return t64 + ((int64_t)k * N + i) * slot; };

  // product state |0...0>, every bond 1; reject non-finite features
  int bad = 0;
  for (int k = lane; k < nq; k += 64) bad |= !isfinite(xi[k]);
  if (__any(bad) && lane == 0) atomicOr(status, QK_FLAG_NONFINITE);
  for (int64_t e = lane; e < (int64_t)nq * slot; e += 64) {
    int k = (int)(e / slot), r = (int)(e % slot);
    site(k)[r] = make_double2(r == 0 ? 1.0 : 0.0, 0.0);
  }
  for (int b = lane; b <= nq; b += 64) chi[b] = 1;
  __syncthreads();

  const double inv_sqrt2 = 0.70710678118654752440;
  int chi_seen = 1;
  double disc = 0.0;  // discarded weight, summed over the truncations (lane 0)
  for (int layer = 0; layer < n_layers; ++layer) {
    // 1. single-qubit layer: A'[0] = e^{-ix}(A0 + A1)/sqrt2, A'[1] = e^{ix}(A0 - A1)/sqrt2
    for (int64_t e = lane; e < (int64_t)nq * TT; e += 64) {
      int k = (int)(e / TT), r = (int)(e % TT);
      double sn, cs;
      sincos(xi[k], &sn, &cs);
      double2* A = site(k);
      double2 a0 = A[r], a1 = A[TT + r];
      double2 u = cscale(cadd(a0, a1), inv_sqrt2);
      double2 v = cscale(make_double2(a0.x - a1.x, a0.y - a1.y), inv_sqrt2);
      A[r] = cmul(make_double2(cs, -sn), u);
      A[TT + r] = cmul(make_double2(cs, sn), v);
    }
    __syncthreads();
    if (nq == 1) continue;

    // 2. entangler chain
    const bool l2r = (layer % 2) == 0;
    for (int step = 0; step < nq - 1; ++step) {
      const int k = l2r ? step : (nq - 2 - step);
      const int cl = chi[k], cm = chi[k + 1], cr = chi[k + 2];
      double theta = 0.0;
      if (entangle && (k + 1) % entangle != 0) theta = 2.0 * (kPi - xi[k]) * (kPi - xi[k + 1]);
      // stage the two sites (realized blocks) in LDS, W x W padded
      for (int e = lane; e < 2 * W * W; e += 64) {
        int s = e / (W * W), r = e % (W * W), a = r / W, b = r % W;
        sa[e] = (a < T && b < T) ? site(k)[s * TT + a * T + b] : make_double2(0, 0);
        sb[e] = (a < T && b < T) ? site(k + 1)[s * TT + a * T + b] : make_double2(0, 0);
      }
      __syncthreads();
      // Theta[(s,a)][(t,c)], rows s*cl + a, cols t*cr + c
      const int R = 2 * cl, C = 2 * cr;
      const bool transpose = C > R;  // factor Theta^dagger when it is wide
      const int XR = transpose ? C : R, XC = transpose ? R : C;
      double sh, ch;
      sincos(0.5 * theta, &sh, &ch);
      double fro = 0.0;
      // lanes walk the padded (s, a) x (t, c) index space (compile-time
      // strides) and skip the padding, placing each entry at its compact
      // position row = s * cl + a, col = t * cr + c
      for (int e = lane; e < 4 * W * W; e += 64) {
        const int rp = e % (2 * W), cp = e / (2 * W);
        const int s = rp / W, a = rp % W, t = cp / W, c = cp % W;
        if (a >= cl || c >= cr) continue;
        const int row = s * cl + a, col = t * cr + c;
        double2 acc = make_double2(0, 0);
        for (int b = 0; b < cm; ++b)
          acc = cadd(acc, cmul(sa[s * W * W + a * W + b], sb[t * W * W + b * W + c]));
        // exp(-i theta/2 sigma_s sigma_t)
        double2 ph = (s == t) ? make_double2(ch, -sh) : make_double2(ch, sh);
        acc = cmul(ph, acc);
        fro += acc.x * acc.x + acc.y * acc.y;
        if (!transpose) X[col * D + row] = acc;
        else X[row * D + col] = make_double2(acc.x, -acc.y);
      }
      const int XCe = XC + (XC & 1);  // even column count
      for (int e = lane; e < D * D; e += 64) {
        int col = e / D, row = e % D;
        if (col >= XC && col < XCe) X[e] = make_double2(0, 0);
        V[e] = make_double2((col == row && col < XCe) ? 1.0 : 0.0, 0.0);
      }
      __syncthreads();
      for (int off = 1; off < 64; off <<= 1) fro += __shfl_xor(fro, off, 64);
      const bool conv = jacobi_columns<D>(X, V, XR, XCe, 1e-30 * fro, max_sweeps);
      if (!conv && lane == 0) atomicOr(status, QK_FLAG_NOCONV);
      // singular values = column norms; rank them (descending, stable)
      for (int cc = lane; cc < XCe; cc += 64) {
        double s2 = 0.0;
        for (int row = 0; row < XR; ++row) {
          double2 v = X[cc * D + row];
          s2 += v.x * v.x + v.y * v.y;
        }
        sm.S[cc] = sqrt(s2);
      }
      __syncthreads();
      for (int cc = lane; cc < XCe; cc += 64) {
        double mine = sm.S[cc];
        int rank = 0;
        for (int j = 0; j < XCe; ++j) {
          double o = sm.S[j];
          rank += (o > mine) || (o == mine && j < cc);
        }
        sm.perm[rank] = cc;
      }
      __syncthreads();
      const double s0 = sm.S[sm.perm[0]];
      int keep = 0;
      double norm2 = 0.0;
      const int kmax = XC < chi_max ? XC : chi_max;
      for (int j = 0; j < kmax; ++j) {
        double sj = sm.S[sm.perm[j]];
        if (j == 0 || sj > cutoff * s0) {
          ++keep;
          norm2 += sj * sj;
        } else {
          break;
        }
      }
      if (keep > W) {
        if (lane == 0) atomicOr(status, QK_FLAG_CHI_OVER);
        keep = W;
        norm2 = 0.0;
        for (int j = 0; j < keep; ++j) norm2 += sm.S[sm.perm[j]] * sm.S[sm.perm[j]];
      }
      if (lane == 0) {  // weight of the dropped singular values, in rank order
        double tot = 0.0, tail = 0.0;
        for (int j = 0; j < XCe; ++j) {
          const double s2 = sm.S[sm.perm[j]] * sm.S[sm.perm[j]];
          tot += s2;
          if (j >= keep) tail += s2;
        }
        if (tot > 0.0) disc += tail / tot;
      }
      const double inv_norm = norm2 > 0.0 ? 1.0 / sqrt(norm2) : 0.0;
      if (keep > chi_seen) chi_seen = keep;
      // Left factor Lf (R x keep) and right factor Rf (keep x C) of Theta:
      //   no transpose: Lf[:,j] = X[:,pj]/S_pj, Rf[j,:] = conj(V[:,pj])
      //   transpose   : Lf[:,j] = V[:,pj],     Rf[j,:] = conj(X[:,pj])/S_pj
      // with S absorbed right (l2r) or left (r2l), renormalised.
      for (int e = lane; e < 2 * TT; e += 64) {
        int s = e / TT, r = e % TT, a = r / T, j = r % T;
        double2 v = make_double2(0, 0);
        if (a < cl && j < keep) {
          int pj = sm.perm[j], row = s * cl + a;
          double Sj = sm.S[pj];
          double2 u;
          if (!transpose) u = Sj > 0.0 ? cscale(X[pj * D + row], 1.0 / Sj) : make_double2(0, 0);
          else u = V[pj * D + row];
          v = l2r ? u : cscale(u, Sj * inv_norm);
        }
        site(k)[e] = v;
      }
      for (int e = lane; e < 2 * TT; e += 64) {
        int t = e / TT, r = e % TT, j = r / T, c = r % T;
        double2 v = make_double2(0, 0);
        if (j < keep && c < cr) {
          int pj = sm.perm[j], col = t * cr + c;
          double Sj = sm.S[pj];
          double2 h;
          if (!transpose) {
            double2 q = V[pj * D + col];
            h = make_double2(q.x, -q.y);
          } else {
            double2 q = X[pj * D + col];
            h = Sj > 0.0 ? make_double2(q.x / Sj, -q.y / Sj) : make_double2(0, 0);
          }
          v = l2r ? cscale(h, Sj * inv_norm) : h;
        }
        site(k + 1)[e] = v;
      }
      if (lane == 0) chi[k + 1] = keep;
      __syncthreads();
    }
  }
  if (lane == 0) {
    atomicMax(status + 1, chi_seen);
    if (disc_out) disc_out[i] = disc;
  }
}

// ---------------------------------------------------------------------------
// The TEBD build for bond bounds 32 and 64 (deep, truncating circuits): one
// workgroup of 8 W threads per sample. The merged matrix X = Theta (R = 2
// chi_l rows, C = 2 chi_r columns, up to 2W x 2W complex: 256 KB at W = 64)
// lives in registers: column pair slot p (C / 2 of them) is held by the 8
// threads 8p .. 8p + 7, thread `sub` holding rows sub + 8i of both columns.
// A one-sided Jacobi round rotates every slot's pair with 8-lane sums and
// then moves the columns one place along a round-robin tournament through
// LDS (column 0 stays in slot 0; the others circulate), so that in C - 1
// rounds every pair of columns meets once and the columns return to their
// starting slots. V is not accumulated: with U the normalised kept columns
// of X V = U S, the right factor S V^dagger is U^dagger Theta, formed from a
// copy of Theta kept in a per-sample global workspace. Rotation rule,
// tolerance, sweep limit, cutoff, chi cap, renormalisation and status flags
// are those of mps_build_kernel.
template <int W>
struct BuildWgShape {
  static constexpr int D = 2 * W;               // largest Theta dimension
  static constexpr int kSub = 8;                // threads per column pair
  static constexpr int kThreads = kSub * W;     // W column pairs
  static constexpr int kRows = D / kSub;        // rows per thread
  static constexpr int kHalf = kRows / 2;       // rows moved per exchange phase
  static constexpr int kPitch = W + 1;          // staged site row pitch
};

template <int W>
struct BuildWgSmem {
  using S = BuildWgShape<W>;
  union {
    double2 site[2 * W * S::kPitch];                   // site k: [s][a][b], pitch W + 1
    double2 xb[2 * S::kHalf * W * S::kSub];            // exchange: [side][row][slot][sub]
    double2 u[S::D * W];                               // kept left vectors: [row][rank]
  };
  double sv[S::D];     // column norms
  int rnk[S::D];       // rank of column c
  int perm[S::D];      // column of rank j
  double red[S::kThreads / 64];
};

template <int W>
constexpr int64_t kBuildWgWsPerSample = (int64_t)(2 * W) * (2 * W);  // Theta, row-major

template <int W>
__global__ __launch_bounds__(BuildWgShape<W>::kThreads) void mps_build_wg_kernel(
    const double* __restrict__ x, int64_t ld_x, int64_t N, int nq, int n_layers,
    int chi_max, int entangle, double cutoff, double2* __restrict__ t64,
    int32_t* __restrict__ chi_tab, int32_t* __restrict__ status, double2* __restrict__ ws,
    double* __restrict__ disc_out, int max_sweeps) {
  using Sh = BuildWgShape<W>;
  constexpr int D = Sh::D, kR = Sh::kRows, kH = Sh::kHalf, kP = Sh::kPitch;
  constexpr int T = W, TT = W * W, slot = 2 * TT;
  __shared__ BuildWgSmem<W> sm;
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  const int ps = tid >> 3, sub = tid & 7;  // column-pair slot, row group
  const double* xi = x + i * ld_x;
  int32_t* chi = chi_tab + i * (int64_t)(nq + 1);
  double2* th = ws + i * kBuildWgWsPerSample<W>;
  auto site = [&](int k) -> double2* { return t64 + ((int64_t)k * N + i) * slot; };

  // product state |0...0>, every bond 1; reject non-finite features
  int bad = 0;
  for (int k = tid; k < nq; k += Sh::kThreads) bad |= !isfinite(xi[k]);
  if (__syncthreads_or(bad) && tid == 0) atomicOr(status, QK_FLAG_NONFINITE);
  for (int64_t e = tid; e < (int64_t)nq * slot; e += Sh::kThreads) {
    const int k = (int)(e / slot), r = (int)(e % slot);
    site(k)[r] = make_double2(r == 0 ? 1.0 : 0.0, 0.0);
  }
  for (int b = tid; b <= nq; b += Sh::kThreads) chi[b] = 1;
  __syncthreads();

  const double inv_sqrt2 = 0.70710678118654752440;
  int chi_seen = 1;
  double disc = 0.0;  // discarded weight, summed over the truncations (thread 0)
  for (int layer = 0; layer < n_layers; ++layer) {
    // 1. single-qubit layer on the realized blocks:
    //    A'[0] = e^{-ix}(A0 + A1)/sqrt2, A'[1] = e^{ix}(A0 - A1)/sqrt2
    for (int64_t e = tid; e < (int64_t)nq * TT; e += Sh::kThreads) {
      const int k = (int)(e / TT), r = (int)(e % TT), a = r / T, b = r % T;
      if (a >= chi[k] || b >= chi[k + 1]) continue;
      double sn, cs;
      sincos(xi[k], &sn, &cs);
      double2* A = site(k);
      const double2 a0 = A[r], a1 = A[TT + r];
      const double2 uu = cscale(cadd(a0, a1), inv_sqrt2);
      const double2 vv = cscale(make_double2(a0.x - a1.x, a0.y - a1.y), inv_sqrt2);
      A[r] = cmul(make_double2(cs, -sn), uu);
      A[TT + r] = cmul(make_double2(cs, sn), vv);
    }
    __syncthreads();
    if (nq == 1) continue;

    // 2. entangler chain
    const bool l2r = (layer % 2) == 0;
    for (int step = 0; step < nq - 1; ++step) {
      const int k = l2r ? step : (nq - 2 - step);
      const int cl = chi[k], cm = chi[k + 1], cr = chi[k + 2];
      const int R = 2 * cl, C = 2 * cr, P = cr;  // rows, columns, column pairs
      const bool live = ps < P;
      double theta = 0.0;
      if (entangle && (k + 1) % entangle != 0) theta = 2.0 * (kPi - xi[k]) * (kPi - xi[k + 1]);
      double sh, ch;
      sincos(0.5 * theta, &sh, &ch);
      // stage site k (realized block) in LDS, rows padded to W + 1
      for (int e = tid; e < 2 * TT; e += Sh::kThreads) {
        const int s = e / TT, r = e % TT, a = r / T, b = r % T;
        if (a < cl && b < cm) sm.site[(s * W + a) * kP + b] = site(k)[e];
      }
      __syncthreads();
      // Theta[(s,a)][(t,c)] = ph(s,t) sum_b A_k^s[a][b] A_{k+1}^t[b][c], rows
      // s cl + a, columns t cr + c; this slot's columns are p = ps, q = C-1-ps
      double2 xp[kR], xq[kR];
      int rs[kR], ra[kR];
#pragma unroll
      for (int m = 0; m < kR; ++m) {
        xp[m] = xq[m] = make_double2(0.0, 0.0);
        const int row = sub + 8 * m;
        rs[m] = row < R ? row / cl : 0;
        ra[m] = row < R ? row - rs[m] * cl : 0;
      }
      const int colp = ps, colq = C - 1 - ps;
      const int tp = live ? colp / cr : 0, cp = live ? colp - tp * cr : 0;
      const int tq = live ? colq / cr : 0, cq = live ? colq - tq * cr : 0;
      if (live) {
        const double2* B = site(k + 1);
        for (int b = 0; b < cm; ++b) {
          const double2 bp = B[tp * TT + b * T + cp];
          const double2 bq = B[tq * TT + b * T + cq];
#pragma unroll
          for (int m = 0; m < kR; ++m) {
            if (sub + 8 * m < R) {
              const double2 av = sm.site[(rs[m] * W + ra[m]) * kP + b];
              xp[m] = cadd(xp[m], cmul(av, bp));
              xq[m] = cadd(xq[m], cmul(av, bq));
            }
          }
        }
      }
      double fro = 0.0;
#pragma unroll
      for (int m = 0; m < kR; ++m) {
        const int row = sub + 8 * m;
        if (live && row < R) {
          // exp(-i theta/2 sigma_s sigma_t)
          xp[m] = cmul(rs[m] == tp ? make_double2(ch, -sh) : make_double2(ch, sh), xp[m]);
          xq[m] = cmul(rs[m] == tq ? make_double2(ch, -sh) : make_double2(ch, sh), xq[m]);
          th[row * D + colp] = xp[m];
          th[row * D + colq] = xq[m];
          fro += xp[m].x * xp[m].x + xp[m].y * xp[m].y + xq[m].x * xq[m].x + xq[m].y * xq[m].y;
        }
      }
      for (int off = 1; off < 64; off <<= 1) fro += __shfl_xor(fro, off, 64);
      if ((tid & 63) == 0) sm.red[tid >> 6] = fro;
      __syncthreads();  // also: every thread is done reading the staged site
      fro = 0.0;
#pragma unroll
      for (int v = 0; v < Sh::kThreads / 64; ++v) fro += sm.red[v];
      const double floor2 = 1e-30 * fro;

      // one-sided Jacobi over the C columns
      const double tol = 1e-14;
      bool conv = false;
      for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0;
        for (int rnd = 0; rnd < C - 1; ++rnd) {
          double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
          for (int m = 0; m < kR; ++m) {
            al += xp[m].x * xp[m].x + xp[m].y * xp[m].y;
            be += xq[m].x * xq[m].x + xq[m].y * xq[m].y;
            gr += xp[m].x * xq[m].x + xp[m].y * xq[m].y;  // conj(xp) * xq
            gi += xp[m].x * xq[m].y - xp[m].y * xq[m].x;
          }
          al = group_sum(al, 3);
          be = group_sum(be, 3);
          gr = group_sum(gr, 3);
          gi = group_sum(gi, 3);
          const double gabs2 = gr * gr + gi * gi;
          const bool do_rot = live && al > floor2 && be > floor2 && gabs2 > tol * tol * (al * be);
          if (do_rot) {
            const double inv_gabs = rsqrt(gabs2);
            const double zeta = 0.5 * (be - al) * inv_gabs;
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = rsqrt(1.0 + tt * tt);
            const double s = c * tt;
            // e^{-i phi} = conj(gamma) / |gamma|
            const double2 ph = make_double2(gr * inv_gabs, -gi * inv_gabs);
#pragma unroll
            for (int m = 0; m < kR; ++m) {
              const double2 a0 = xp[m];
              const double2 b0 = cmul(ph, xq[m]);
              xp[m] = make_double2(c * a0.x - s * b0.x, c * a0.y - s * b0.y);
              xq[m] = make_double2(s * a0.x + c * b0.x, s * a0.y + c * b0.y);
            }
          }
          rotated |= do_rot ? 1 : 0;
          if (P < 2) continue;  // a single pair: nothing moves
          // tournament move, half of the rows at a time: slot 1 takes slot
          // 0's q column, slots p >= 2 take slot p-1's p column; slots p <
          // P-1 take slot p+1's q column, slot P-1 its own p column
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (live) {
#pragma unroll
              for (int m = 0; m < kH; ++m) {
                sm.xb[((0 * kH + m) * W + ps) * 8 + sub] = xp[h * kH + m];
                sm.xb[((1 * kH + m) * W + ps) * 8 + sub] = xq[h * kH + m];
              }
            }
            __syncthreads();
            if (live) {
              const int srcp_side = ps == 1 ? 1 : 0, srcp = ps == 1 ? 0 : ps - 1;
              const int srcq_side = ps == P - 1 ? 0 : 1, srcq = ps == P - 1 ? ps : ps + 1;
#pragma unroll
              for (int m = 0; m < kH; ++m) {
                if (ps != 0) xp[h * kH + m] = sm.xb[((srcp_side * kH + m) * W + srcp) * 8 + sub];
                xq[h * kH + m] = sm.xb[((srcq_side * kH + m) * W + srcq) * 8 + sub];
              }
            }
            __syncthreads();
          }
        }
        if (!__syncthreads_or(rotated)) {
          conv = true;
          break;
        }
      }
      if (!conv && tid == 0) atomicOr(status, QK_FLAG_NOCONV);
      // singular values = column norms (columns are back in their slots)
      double np = 0.0, nqq = 0.0;
#pragma unroll
      for (int m = 0; m < kR; ++m) {
        np += xp[m].x * xp[m].x + xp[m].y * xp[m].y;
        nqq += xq[m].x * xq[m].x + xq[m].y * xq[m].y;
      }
      np = group_sum(np, 3);
      nqq = group_sum(nqq, 3);
      if (live && sub == 0) {
        sm.sv[colp] = sqrt(np);
        sm.sv[colq] = sqrt(nqq);
      }
      __syncthreads();
      for (int cc = tid; cc < C; cc += Sh::kThreads) {
        const double mine = sm.sv[cc];
        int rank = 0;
        for (int j = 0; j < C; ++j) {
          const double o = sm.sv[j];
          rank += (o > mine) || (o == mine && j < cc);
        }
        sm.rnk[cc] = rank;
        sm.perm[rank] = cc;
      }
      __syncthreads();
      const double s0 = sm.sv[sm.perm[0]];
      int keep = 0;
      double norm2 = 0.0;
      const int xc = R < C ? R : C;
      const int kmax = xc < chi_max ? xc : chi_max;
      for (int j = 0; j < kmax; ++j) {
        const double sj = sm.sv[sm.perm[j]];
        if (j == 0 || sj > cutoff * s0) {
          ++keep;
          norm2 += sj * sj;
        } else {
          break;
        }
      }
      if (keep > W) {
        if (tid == 0) atomicOr(status, QK_FLAG_CHI_OVER);
        keep = W;
        norm2 = 0.0;
        for (int j = 0; j < keep; ++j) norm2 += sm.sv[sm.perm[j]] * sm.sv[sm.perm[j]];
      }
      if (tid == 0) {  // weight of the dropped singular values, in rank order
        double tot = 0.0, tail = 0.0;
        for (int j = 0; j < C; ++j) {
          const double s2 = sm.sv[sm.perm[j]] * sm.sv[sm.perm[j]];
          tot += s2;
          if (j >= keep) tail += s2;
        }
        if (tot > 0.0) disc += tail / tot;
      }
      const double inv_norm = norm2 > 0.0 ? 1.0 / sqrt(norm2) : 0.0;
      if (keep > chi_seen) chi_seen = keep;
      // kept left singular vectors U[:, j] = X[:, perm j] / S to LDS
      if (live) {
        const int jp = sm.rnk[colp], jq = sm.rnk[colq];
        const double sp = sm.sv[colp], sq = sm.sv[colq];
#pragma unroll
        for (int m = 0; m < kR; ++m) {
          const int row = sub + 8 * m;
          if (row < R) {
            if (jp < keep) sm.u[row * W + jp] = sp > 0.0 ? cscale(xp[m], 1.0 / sp) : make_double2(0, 0);
            if (jq < keep) sm.u[row * W + jq] = sq > 0.0 ? cscale(xq[m], 1.0 / sq) : make_double2(0, 0);
          }
        }
      }
      __syncthreads();
      // left site k: U (l2r) or U S / norm (r2l), zero outside the kept block
      for (int e = tid; e < 2 * TT; e += Sh::kThreads) {
        const int s = e / TT, r = e % TT, a = r / T, j = r % T;
        double2 v = make_double2(0, 0);
        if (a < cl && j < keep) {
          v = sm.u[(s * cl + a) * W + j];
          if (!l2r) v = cscale(v, sm.sv[sm.perm[j]] * inv_norm);
        }
        site(k)[e] = v;
      }
      // right site k+1: U^dagger Theta = S V^dagger, scaled by 1/norm (l2r)
      // or 1/S (r2l); thread (t, c) = tid mod 2W, ranks j = tid / 2W + 4 n
      {
        constexpr int kJ = W / 4;  // ranks per thread
        const int tc = tid % (2 * W), jg = tid / (2 * W);
        const int t = tc / W, c = tc % W;
        double2 acc[kJ];
#pragma unroll
        for (int n = 0; n < kJ; ++n) acc[n] = make_double2(0, 0);
        if (c < cr) {
          for (int row = 0; row < R; ++row) {
            const double2 tv = th[row * D + t * cr + c];
#pragma unroll
            for (int n = 0; n < kJ; ++n) {
              const int j = jg + 4 * n;
              if (j < keep) acc[n] = cadd(acc[n], cmulc(sm.u[row * W + j], tv));
            }
          }
        }
#pragma unroll
        for (int n = 0; n < kJ; ++n) {
          const int j = jg + 4 * n;
          double2 v = make_double2(0, 0);
          if (j < keep && c < cr) {
            const double sj = sm.sv[sm.perm[j]];
            v = l2r ? cscale(acc[n], inv_norm) : (sj > 0.0 ? cscale(acc[n], 1.0 / sj) : make_double2(0, 0));
          }
          site(k + 1)[t * TT + j * T + c] = v;
        }
      }
      if (tid == 0) chi[k + 1] = keep;
      __syncthreads();
    }
  }
  if (tid == 0) {
    atomicMax(status + 1, chi_seen);
    if (disc_out) disc_out[i] = disc;
  }
}

// ---------------------------------------------------------------------------
// The same TEBD build for padded bond dimensions W <= 4, eight samples per
// wavefront: the eight lanes of a sample each hold one row of the merged
// matrix X (at most 2W <= 8 rows) and one row of V in registers. A Jacobi
// rotation of a column pair then touches only the lane's own registers, and
// the column dot products are 8-lane DPP sums, so a round needs no LDS
// traffic and no barrier; every lane computes the rotation parameters of its
// sample. One wave advances eight samples per instruction, where the
// one-sample-per-wave kernel kept most lanes idle and ran several waves per
// SIMD, each waiting for issue.
//
// Per sample the two sites of a step sit in LDS (two padded W x W x 2
// buffers). The site carried over from the previous step stays there; the
// next fresh site is loaded from memory one step ahead. A site gets its
// single-qubit gate G_k = RZ(2 x_k) H when it is first loaded in a layer:
// gates on other sites commute with the entangler of the merged pair and are
// unitaries on one side of its cut, so the singular values, and hence the
// truncation, are those of the gate-first order. The rotation rule,
// tolerance, sweep limit, cutoff, chi cap, renormalisation and status flags
// are those of mps_build_kernel.
constexpr int kB8Lanes = 8;      // lanes per sample
constexpr int kB8Samples = 8;    // samples per 64-lane workgroup

template <int W>
struct Build8Smem {
  static constexpr int kSlot = 2 * W * W;  // [s][a][b]
  double2 site[kB8Samples][2][kSlot];
};

// round-robin tournament of nc columns: pair k of round r
__device__ constexpr int rr_p(int r, int k, int players) {
  return k == 0 ? 0 : 1 + (r + k) % players;
}
__device__ constexpr int rr_q(int r, int k, int players) {
  return k == 0 ? 1 + r : 1 + (r - k + players) % players;
}

// One-sided Jacobi over the nc (even) columns of X, rows in the 8 lanes of
// each sample (lane holds xr[col]); V rows likewise (vr[col]). Returns
// whether the sweeps converged for this lane's sample.
template <int D, int NC>
__device__ bool jacobi_rows(double2 (&xr)[D], double2 (&vr)[D], double floor2, int max_sweeps) {
  constexpr int P = NC - 1, NP = NC / 2;
  const double tol = 1e-14;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      double al[NP], be[NP], gr[NP], gi[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const double2 xp = xr[rr_p(r, k, P)], xq = xr[rr_q(r, k, P)];
        al[k] = xp.x * xp.x + xp.y * xp.y;
        be[k] = xq.x * xq.x + xq.y * xq.y;
        gr[k] = xp.x * xq.x + xp.y * xq.y;  // conj(xp) * xq
        gi[k] = xp.x * xq.y - xp.y * xq.x;
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        al[k] = group_sum(al[k], 3);
        be[k] = group_sum(be[k], 3);
        gr[k] = group_sum(gr[k], 3);
        gi[k] = group_sum(gi[k], 3);
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const int p = rr_p(r, k, P), q = rr_q(r, k, P);
        const double gabs2 = gr[k] * gr[k] + gi[k] * gi[k];
        const bool do_rot =
            al[k] > floor2 && be[k] > floor2 && gabs2 > tol * tol * (al[k] * be[k]);
        if (do_rot) {
          const double inv_gabs = rsqrt(gabs2);
          const double zeta = 0.5 * (be[k] - al[k]) * inv_gabs;
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = rsqrt(1.0 + t * t);
          const double sn = c * t;
          const double2 ph = make_double2(gr[k] * inv_gabs, -gi[k] * inv_gabs);
          const double2 xp = xr[p], xq = cmul(ph, xr[q]);
          xr[p] = make_double2(c * xp.x - sn * xq.x, c * xp.y - sn * xq.y);
          xr[q] = make_double2(sn * xp.x + c * xq.x, sn * xp.y + c * xq.y);
          const double2 vp = vr[p], vq = cmul(ph, vr[q]);
          vr[p] = make_double2(c * vp.x - sn * vq.x, c * vp.y - sn * vq.y);
          vr[q] = make_double2(sn * vp.x + c * vq.x, sn * vp.y + c * vq.y);
          rotated = 1;
        }
      }
    }
    if (!__any(rotated)) return true;
    if (sweep == max_sweeps - 1) return !rotated;
  }
  return false;  // a limit of 0 sweeps: nothing was verified
}

// Per step after X (rows in lanes) and V = I are formed: the Jacobi
// rotations over the wave's NC columns, the singular values and their
// descending stable order, the kept count (cutoff, chi cap, padded bound) and
// the two factors written back into the padded LDS buffers Lo (left site
// [s][a][j]) and Ro (right site [t][j][c]), S absorbed to the right (l2r) or
// left and renormalised:
//   no transpose: Lf[:,j] = X[:,pj]/S_pj, Rf[j,:] = conj(V[:,pj])
//   transpose   : Lf[:,j] = V[:,pj],     Rf[j,:] = conj(X[:,pj])/S_pj
// Returns the kept count.
template <int W, int NC>
__device__ int b8_factor(double2 (&xr)[2 * W], double2 (&vr)[2 * W], double floor2, int r,
                         int XC, int cl, int cr, bool tr, bool l2r, int chi_max, double cutoff,
                         double2* Lo, double2* Ro, int& noconv, int& over, double& dw,
                         int max_sweeps) {
  constexpr int D = 2 * W, TT = W * W;
  const bool conv = jacobi_rows<D, NC>(xr, vr, floor2, max_sweeps);
  noconv |= conv ? 0 : 1;
  // singular values = column norms (every lane); rank descending, stable
  double S[NC], inv_S[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    S[j] = sqrt(group_sum(xr[j].x * xr[j].x + xr[j].y * xr[j].y, 3));
    inv_S[j] = S[j] > 0.0 ? 1.0 / S[j] : 0.0;
  }
  int rk[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    int ahead = 0;
#pragma unroll
    for (int o = 0; o < NC; ++o) ahead += (S[o] > S[j]) || (S[o] == S[j] && o < j);
    rk[j] = (j < XC) ? ahead : D;  // padding columns are never kept
  }
  double s_at[NC];  // singular values in rank order
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) v = rk[j] == q ? S[j] : v;
    s_at[q] = v;
  }
  const int kmax = XC < chi_max ? XC : chi_max;
  int keep = 0;
  double norm2 = 0.0;
  bool run = true;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    if (run && q < kmax && (q == 0 || s_at[q] > cutoff * s_at[0])) {
      ++keep;
      norm2 += s_at[q] * s_at[q];
    } else {
      run = false;
    }
  }
  if (keep > W) {
    over = 1;
    keep = W;
    norm2 = 0.0;
#pragma unroll
    for (int q = 0; q < (NC < W ? NC : W); ++q) norm2 += s_at[q] * s_at[q];
  }
  {  // weight of the dropped singular values (same value in every lane)
    double tot = 0.0, tail = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const double s2 = s_at[q] * s_at[q];
      tot += s2;
      if (q >= keep) tail += s2;
    }
    if (tot > 0.0) dw += tail / tot;
  }
  const double inv_norm = norm2 > 0.0 ? 1.0 / sqrt(norm2) : 0.0;
  const int R = 2 * cl, C = 2 * cr;
  // padding rows (a >= cl) of the left site and padding columns (c >= cr) of
  // the right site, zeroed by the lane of that padded index
  if (r < D) {
    const int sp = r >= W ? 1 : 0, ap = r - sp * W;
    if (ap >= cl)
#pragma unroll
      for (int j = 0; j < W; ++j) Lo[sp * TT + ap * W + j] = make_double2(0.0, 0.0);
    if (ap >= cr)
#pragma unroll
      for (int j = 0; j < W; ++j) Ro[sp * TT + j * W + ap] = make_double2(0.0, 0.0);
  }
  if (r < R) {  // row r of Lf: lane r holds X row r (or V row r)
    const int s = r >= cl ? 1 : 0, a = r - s * cl;
    double2* row = Lo + s * TT + a * W;
    for (int j = keep; j < W; ++j) row[j] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = rk[c];
      if (j < keep) {
        const double2 u = tr ? vr[c] : cscale(xr[c], inv_S[c]);
        row[j] = l2r ? u : cscale(u, S[c] * inv_norm);
      }
    }
  }
  if (r < C) {  // column r of Rf: lane r holds V row r (or X row r)
    const int t = r >= cr ? 1 : 0, c = r - t * cr;
    double2* colp = Ro + t * TT + c;
    for (int j = keep; j < W; ++j) colp[j * W] = make_double2(0.0, 0.0);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int j = rk[cc];
      if (j < keep) {
        const double2 h = tr ? make_double2(xr[cc].x * inv_S[cc], -xr[cc].y * inv_S[cc])
                             : make_double2(vr[cc].x, -vr[cc].y);
        colp[j * W] = l2r ? cscale(h, S[cc] * inv_norm) : h;
      }
    }
  }
  return keep;
}

// The parts of one launch: part p takes workgroups [wg_begin[p], wg_begin[p+1]).
struct B8Table {
  QkBuildPart p[QK_MAX_BUILD_PARTS];
  int64_t wg_begin[QK_MAX_BUILD_PARTS + 1];
  int n_parts;
};

template <int W>
__global__ __launch_bounds__(64) void mps_build8_kernel(B8Table tab, int nq, int n_layers,
                                                        int chi_max, int entangle,
                                                        double cutoff, int max_sweeps) {
  constexpr int D = 2 * W, TT = W * W, slot = 2 * TT;
  __shared__ Build8Smem<W> sm;
  int part = 0;
  while (part + 1 < tab.n_parts && tab.wg_begin[part + 1] <= (int64_t)blockIdx.x) ++part;
  const QkBuildPart& P = tab.p[part];
  const double* __restrict__ x = P.x;
  const int64_t ld_x = P.ld_x, N = P.n;
  double2* __restrict__ t64 = P.t64;
  int32_t* __restrict__ chi_tab = P.chi;
  int32_t* __restrict__ status = P.status;
  const int lane = threadIdx.x;
  const int g = lane >> 3, r = lane & 7;
  const int64_t i0 = ((int64_t)blockIdx.x - tab.wg_begin[part]) * kB8Samples + g;
  const bool live = i0 < N;
  const int64_t i = live ? i0 : N - 1;  // idle groups shadow the last sample, writing nothing
  const double* xi = x + i * ld_x;
  int32_t* chi = chi_tab + i * (int64_t)(nq + 1);
  auto site = [&](int k) -> double2* { return t64 + ((int64_t)k * N + i) * slot; };
  double2 (*buf)[slot] = sm.site[g];

  int bad = 0;
  for (int k = r; k < nq; k += kB8Lanes) bad |= !isfinite(xi[k]);
  if (live && bad) atomicOr(status, QK_FLAG_NONFINITE);
  if (live)
    for (int b = r; b <= nq; b += kB8Lanes) chi[b] = 1;
  __syncthreads();

  const double inv_sqrt2 = 0.70710678118654752440;
  // lane r holds elements e = r + 8 m (m < ceil(TT / 8)) of both s of a site
  constexpr int kPer = (TT + kB8Lanes - 1) / kB8Lanes;
  double2 fresh[2][kPer];
  auto load_site = [&](int k, int layer) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = r + kB8Lanes * m;
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        double2 v = make_double2(0.0, 0.0);
        if (e < TT) {
          if (layer == 0) v = make_double2((s2 == 0 && e == 0) ? 1.0 : 0.0, 0.0);  // |0>
          else v = site(k)[s2 * TT + e];
        }
        fresh[s2][m] = v;
      }
    }
  };
  // G_k on the loaded site, into buffer b
  auto put_site = [&](int b, double sn, double cs) {  // sincos of the site's feature
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = r + kB8Lanes * m;
      if (e < TT) {
        const double2 a0 = fresh[0][m], a1 = fresh[1][m];
        const double2 u = cscale(cadd(a0, a1), inv_sqrt2);
        const double2 v = cscale(make_double2(a0.x - a1.x, a0.y - a1.y), inv_sqrt2);
        buf[b][e] = cmul(make_double2(cs, -sn), u);
        buf[b][TT + e] = cmul(make_double2(cs, sn), v);
      }
    }
  };

  int chi_seen = 1, noconv = 0, over = 0;
  double disc = 0.0;  // discarded weight, summed over the truncations
  for (int layer = 0; layer < n_layers; ++layer) {
    const bool l2r = (layer % 2) == 0;
    // bond dimension before this layer's step rewrote it (all 1 before the
    // first layer; the boundary bonds are always 1)
    auto old_chi = [&](int b) -> int { return (layer == 0 || b <= 0 || b >= nq) ? 1 : chi[b]; };
    // the site that a step loads fresh, and its feature
    auto fresh_of = [&](int k) -> int { return l2r ? k + 2 : k - 1; };
    // buffer lb holds the step's left site, 1 - lb its right site
    int lb = 0;
    const int k0 = l2r ? 0 : nq - 2;
    double xl = xi[k0], xrr = xi[k0 + 1];  // features of the step's two sites
    {
      double sn, cs;
      load_site(k0, layer);
      sincos(xl, &sn, &cs);
      put_site(0, sn, cs);
      load_site(k0 + 1, layer);
      sincos(xrr, &sn, &cs);
      put_site(1, sn, cs);
    }
    // bonds of a step: `carry` (the near side, rewritten by the previous
    // step), `mid` (the merged bond) and `far`, both from the previous layer
    int carry = 1;
    int mid = old_chi(k0 + 1);
    int far = old_chi(l2r ? k0 + 2 : k0);
    (void)mid;  // bond entries past the merged bond are zero in the buffers
    // the entangler phase of a step and the feature of its fresh site are
    // known a step ahead, so their sines and cosines overlap other work
    double sh = 0.0, ch = 1.0;
    if (entangle && (k0 + 1) % entangle != 0)
      sincos((kPi - xl) * (kPi - xrr), &sh, &ch);  // theta / 2
    double xq = nq > 2 ? xi[fresh_of(k0)] : 0.0;
    wave_lds_sync();
    for (int step = 0; step < nq - 1; ++step) {
      const int k = l2r ? step : (nq - 2 - step);
      const bool more = step + 1 < nq - 1;
      const int cl = l2r ? carry : far, cr = l2r ? far : carry;
      // next step's fresh site (loaded during this step), its gate and the
      // next entangler phase; the feature of the fresh site after that
      const int kf = fresh_of(k);
      int far_next = 1;
      double g_sn = 0.0, g_cs = 1.0, n_sh = 0.0, n_ch = 1.0, xq_next = 0.0;
      if (more) {
        load_site(kf, layer);
        far_next = old_chi(l2r ? k + 3 : k - 1);
        if (step + 2 < nq - 1) xq_next = xi[fresh_of(l2r ? k + 1 : k - 1)];
        sincos(xq, &g_sn, &g_cs);
        if (entangle && ((l2r ? k + 1 : k - 1) + 1) % entangle != 0) {
          const double xa = l2r ? xrr : xq, xb = l2r ? xq : xl;
          sincos((kPi - xa) * (kPi - xb), &n_sh, &n_ch);
        }
      }

      double2* Lo = buf[lb];
      double2* Ro = buf[1 - lb];
      const int R = 2 * cl, C = 2 * cr;
      const bool tr = C > R;  // factor Theta^dagger when it is wide
      const int XR = tr ? C : R, XC = tr ? R : C;
      // lane r forms row r of X: X = Theta, or X = Theta^dagger, where
      // Theta[(s,a)][(t,c)] = exp(-i theta/2 sigma_s sigma_t) sum_b L[s][a][b] R[t][b][c]
      double2 xr[D], vr[D];
      double fro = 0.0;
#pragma unroll
      for (int col = 0; col < D; ++col) {
        double2 acc = make_double2(0.0, 0.0);
        if (r < XR && col < XC) {
          const int rs = tr ? col : r, cs2 = tr ? r : col;  // Theta row, column
          const int s = rs >= cl ? 1 : 0, a = rs - s * cl;
          const int t = cs2 >= cr ? 1 : 0, c = cs2 - t * cr;
#pragma unroll
          for (int b = 0; b < W; ++b)
            acc = cadd(acc, cmul(Lo[s * TT + a * W + b], Ro[t * TT + b * W + c]));
          acc = cmul((s == t) ? make_double2(ch, -sh) : make_double2(ch, sh), acc);
          if (tr) acc.y = -acc.y;
        }
        xr[col] = acc;
        fro += acc.x * acc.x + acc.y * acc.y;
        vr[col] = make_double2((col == r && col < XC) ? 1.0 : 0.0, 0.0);
      }
      fro = group_sum(fro, 3);
      // column count over the wave's samples, rounded to a compiled width
      int nc = XC;
      nc = max(nc, __shfl_xor(nc, 8, 64));
      nc = max(nc, __shfl_xor(nc, 16, 64));
      nc = max(nc, __shfl_xor(nc, 32, 64));
      const double floor2 = 1e-30 * fro;
      int keep;
      if (nc <= 2)
        keep = b8_factor<W, 2>(xr, vr, floor2, r, XC, cl, cr, tr, l2r, chi_max, cutoff, Lo, Ro, noconv, over, disc, max_sweeps);
      else if (nc <= 4 || D <= 4)
        keep = b8_factor<W, (D < 4 ? D : 4)>(xr, vr, floor2, r, XC, cl, cr, tr, l2r, chi_max, cutoff, Lo, Ro, noconv, over, disc, max_sweeps);
      else if (nc <= 6 || D <= 6)
        keep = b8_factor<W, (D < 6 ? D : 6)>(xr, vr, floor2, r, XC, cl, cr, tr, l2r, chi_max, cutoff, Lo, Ro, noconv, over, disc, max_sweeps);
      else
        keep = b8_factor<W, D>(xr, vr, floor2, r, XC, cl, cr, tr, l2r, chi_max, cutoff, Lo, Ro, noconv, over, disc, max_sweeps);
      if (keep > chi_seen) chi_seen = keep;
      wave_lds_sync();
      // The finished site goes to memory (the carried one too on the layer's
      // last step). Its LDS values are read first, then the fresh site takes
      // its buffer, then the stores issue: waiting for the fresh site's loads
      // never has to wait for stores.
      const int kdone = l2r ? k : k + 1;
      const double2* done = l2r ? Lo : Ro;
      const double2* kept = l2r ? Ro : Lo;
      constexpr int kOut = (slot + kB8Lanes - 1) / kB8Lanes;
      double2 vd[kOut], vk[kOut];
#pragma unroll
      for (int m = 0; m < kOut; ++m) {
        const int e = r + kB8Lanes * m;
        vd[m] = e < slot ? done[e] : make_double2(0.0, 0.0);
        vk[m] = (!more && e < slot) ? kept[e] : make_double2(0.0, 0.0);
      }
      wave_lds_sync();
      if (more) {
        if (l2r) {
          put_site(lb, g_sn, g_cs);  // site k is done: fresh site k+2 in its buffer
          lb = 1 - lb;               // site k+1 (old right) is the new left site
          xl = xrr;
          xrr = xq;
        } else {
          put_site(1 - lb, g_sn, g_cs);  // site k+1 is done: fresh site k-1 there
          lb = 1 - lb;                   // ... as the new left; site k is the right one
          xrr = xl;
          xl = xq;
        }
        carry = keep;
        far = far_next;
        sh = n_sh;
        ch = n_ch;
        xq = xq_next;
      }
      if (live) {
        double2* gd = site(kdone);
        double2* gk = site(l2r ? k + 1 : k);
#pragma unroll
        for (int m = 0; m < kOut; ++m) {
          const int e = r + kB8Lanes * m;
          if (e < slot) {
            gd[e] = vd[m];
            if (!more) gk[e] = vk[m];
          }
        }
        if (r == 0) chi[k + 1] = keep;
      }
      wave_lds_sync();
    }
    // the next layer reads this layer's sites and bonds from memory
    __syncthreads();
  }
  if (live && r == 0) {
    if (noconv) atomicOr(status, QK_FLAG_NOCONV);
    if (over) atomicOr(status, QK_FLAG_CHI_OVER);
    atomicMax(status + 1, chi_seen);
    if (P.disc) P.disc[i] = disc;
  }
}

// FP64 complex -> packed FP32 (-Im, Re, Im)
__global__ void pack32_kernel(const double2* __restrict__ a, float* __restrict__ b,
                              int64_t count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) {
    const double2 v = a[i];
    const float re = (float)v.x, im = (float)v.y;
    float* o = b + i * kQkPackFloats;
    o[0] = -im;
    o[1] = re;
    o[2] = im;
  }
}

}  // namespace

hipError_t qk_launch_build(const double* x, int64_t ld_x, int64_t n, int nq,
                           int n_layers, int chi_max, int entangle,
                           double cutoff, int chi_ws, int T, double2* t64,
                           int32_t* chi, int32_t* status, double* disc, int max_sweeps,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nq >= 2 && (T == 1 || T == 2 || T == 4)) {
    const QkBuildPart part{x, ld_x, n, t64, chi, status, disc};
    return qk_launch_build_many(&part, 1, nq, n_layers, chi_max, entangle, cutoff, chi_ws, T,
                                max_sweeps, s);
  }
  // bond bounds of 32 and 64: one workgroup per sample, Theta of each
  // sample in a stream-ordered global workspace for the duration of the build
  if (T == 32 || T == 64) {
    const int64_t per = T == 32 ? kBuildWgWsPerSample<32> : kBuildWgWsPerSample<64>;
    double2* ws = nullptr;
    const hipError_t ea = hipMallocAsync((void**)&ws, n * per * sizeof(double2), s);
    if (ea != hipSuccess) return ea;
    if (T == 32)
      hipLaunchKernelGGL(mps_build_wg_kernel<32>, dim3((unsigned)n),
                         dim3(BuildWgShape<32>::kThreads), 0, s, x, ld_x, n, nq, n_layers,
                         chi_max, entangle, cutoff, t64, chi, status, ws, disc, max_sweeps);
    else
      hipLaunchKernelGGL(mps_build_wg_kernel<64>, dim3((unsigned)n),
                         dim3(BuildWgShape<64>::kThreads), 0, s, x, ld_x, n, nq, n_layers,
                         chi_max, entangle, cutoff, t64, chi, status, ws, disc, max_sweeps);
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ws, s);  // stream-ordered: after the build
    return e;
  }
  dim3 grid((unsigned)n), block(64);
#define QK_BUILD_CASE(WV)                                                     \
  case WV:                                                                    \
    hipLaunchKernelGGL(mps_build_kernel<WV>, grid, block, 0, s, x, ld_x, n,   \
                       nq, n_layers, chi_max, entangle, cutoff, t64, chi,     \
                       status, disc, max_sweeps);                             \
    break;
  switch (T) {
    QK_BUILD_CASE(1)  // a single qubit (every multi-qubit bound <= 4 takes the 8-sample kernel)
    QK_BUILD_CASE(8)
    QK_BUILD_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
#undef QK_BUILD_CASE
  return hipGetLastError();
}

hipError_t qk_launch_build_many(const QkBuildPart* parts, int n_parts, int nq, int n_layers,
                                int chi_max, int entangle, double cutoff, int chi_ws, int T,
                                int max_sweeps, hipStream_t s) {
  if (n_parts < 1 || n_parts > QK_MAX_BUILD_PARTS) return hipErrorInvalidValue;
  if (nq < 2 || !(T == 1 || T == 2 || T == 4)) {
    // one launch per part with the one-sample-per-wave kernel
    for (int k = 0; k < n_parts; ++k) {
      const QkBuildPart& p = parts[k];
      const hipError_t e = qk_launch_build(p.x, p.ld_x, p.n, nq, n_layers, chi_max, entangle,
                                           cutoff, chi_ws, T, p.t64, p.chi, p.status, p.disc,
                                           max_sweeps, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  B8Table tab{};
  int64_t wg = 0;
  int m = 0;
  for (int k = 0; k < n_parts; ++k) {
    if (parts[k].n == 0) continue;
    tab.p[m] = parts[k];
    tab.wg_begin[m] = wg;
    wg += (parts[k].n + kB8Samples - 1) / kB8Samples;
    ++m;
  }
  tab.wg_begin[m] = wg;
  tab.n_parts = m;
  if (wg == 0) return hipSuccess;
  const dim3 grid8((unsigned)wg), block8(64);
  switch (T) {
    case 1:
      hipLaunchKernelGGL(mps_build8_kernel<1>, grid8, block8, 0, s, tab, nq, n_layers, chi_max, entangle, cutoff, max_sweeps);
      break;
    case 2:
      hipLaunchKernelGGL(mps_build8_kernel<2>, grid8, block8, 0, s, tab, nq, n_layers, chi_max, entangle, cutoff, max_sweeps);
      break;
    default:
      hipLaunchKernelGGL(mps_build8_kernel<4>, grid8, block8, 0, s, tab, nq, n_layers, chi_max, entangle, cutoff, max_sweeps);
      break;
  }
  (void)chi_ws;
  return hipGetLastError();
}

hipError_t qk_launch_pack32(const double2* t64, float* t32, int64_t count,
                            hipStream_t s) {
  if (count == 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pack32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, t64, t32, count);
  return hipGetLastError();
}
