// Exact path-sum evaluation of the quantum kernel for circuits of one to
// three layers, an alternative to building MPS and sweeping them.
//
// Every gate of the encoding circuit except H is diagonal in the
// computational basis (Eq. (6)). Expanding each Hadamard layer over basis
// states writes <psi(x)|psi(y)> (Eqs. (7), (10)) as a sum over basis
// histories: one history u for x, one v for y, sharing the last layer z.
// With the per-site state c = (u^(1..L-1), v^(1..L-1), z), 2^(2L-1) values,
// the sum is a chain over the qubits k = 0 .. d-1 of
//   a site weight   w_k(c) = 2^-L (-1)^(layer-to-layer bit products)
//                            exp(i x_k sum_l s(u^l) - i y_k sum_l s(v^l)),
//   a bond factor   J_k(c, c') = prod over lines of exp(+-i theta_k / 2 s s'),
// with s = 1 - 2 bit and theta_k = 2 (pi - x_k)(pi - x_{k+1}). J_k is the
// Kronecker product of one 2 x 2 matrix [[p, conj p], [conj p, p]] per line
// (p = e^{i theta_k(x) / 2} on x's lines, e^{-i theta_k(y) / 2} on y's, their
// product on the shared line), so applying it costs one butterfly per line.
//
// L = 2: c = 4 u1 + 2 v1 + z and, with q = e^{2 i x_k}, r = e^{2 i y_k},
//   w_k = 1/4 (q conj r, 1, q, -r, conj r, -conj q, 1, conj q r).
// L = 1: c = z and, with q = e^{i x_k}, r = e^{i y_k},
//   w_k = 1/2 (q conj r, conj q r).
// L = 3: c = 16 u1 + 8 u2 + 4 v1 + 2 v2 + z (32 states, 5 lines), with
//   q = e^{i x_k}, r = e^{i y_k}: w_k(c) = 1/8 (-1)^(u1 u2 + u2 z + v1 v2 + v2 z)
//   q^{su} conj(r)^{sv}, su = s(u1) + s(u2) + s(z), sv likewise; the 16
//   products q^a conj(r)^b (a, b in {3, 1, -1, -3}) are formed once per site.
// The 2^-L factors go into the base-2 exponent, and the chain vector is
// rescaled by an exact power of two every 8 sites, so ln K_q is exact in
// range. One pair per lane, a 16 x 16 pair tile per 256-thread workgroup;
// lanes share nothing, so the kernel has no barrier. Per sample and qubit a
// table holds q and p (precomputed once per call, site-major, so the 16
// samples of a tile row or column are contiguous).
#include <hip/hip_runtime.h>

#include <cmath>

#include "qk_internal.h"
#include "qk_sweep_ops.h"

namespace {

constexpr int kPsTile = 16;
constexpr int kPsThreads = kPsTile * kPsTile;
constexpr int kPsRescale = 8;  // sites between exact rescales

// tab[k * n + s] = (Re q, Im q, Re p, Im p) of sample s at qubit k
__global__ void pathsum_table_kernel(const double* __restrict__ x, int64_t n, int64_t ld_x,
                                     int d, int n_layers, int entangle,
                                     double4* __restrict__ tab) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  const int64_t s = e % n;
  const int k = (int)(e / n);
  const double* xs = x + s * ld_x;
  const double xk = xs[k];
  double qs, qc, ps = 0.0, pc = 1.0;
  sincos(n_layers == 2 ? 2.0 * xk : xk, &qs, &qc);
  if (entangle && k + 1 < d && (k + 1) % entangle != 0) {
    const double th = 2.0 * (M_PI - xk) * (M_PI - xs[k + 1]);
    sincos(0.5 * th, &ps, &pc);
  }
  tab[(int64_t)k * n + s] = make_double4(qc, qs, pc, ps);
}

struct Cd {
  double re, im;
};
__device__ inline Cd cmul(Cd a, Cd b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ inline Cd cmulc(Cd a, Cd b) {  // a conj(b)
  return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -a.re * b.im)};
}
// (t, o) <- (p t + conj(p) o, conj(p) t + p o)
__device__ inline void butterfly(Cd& t, Cd& o, Cd p) {
  const double sr = t.re + o.re, si = t.im + o.im;
  const double dr = t.re - o.re, di = t.im - o.im;
  const double a = p.re * sr, b = p.re * si;
  t = {fma(-p.im, di, a), fma(p.im, dr, b)};
  o = {fma(p.im, di, a), fma(-p.im, dr, b)};
}

template <int L>
struct PsState {
  static constexpr int S = 1 << (2 * L - 1);
  Cd v[S];
};

// v <- v * w_k (without the 2^-L factor)
template <int L>
__device__ inline void apply_weight(PsState<L>& st, Cd q, Cd r) {
  if constexpr (L == 1) {
    const Cd g = cmulc(q, r);  // q conj r
    st.v[0] = cmul(st.v[0], g);
    st.v[1] = cmulc(st.v[1], g);
  } else if constexpr (L == 2) {
    const Cd t = cmulc(q, r);  // q conj r
    st.v[0] = cmul(st.v[0], t);
    st.v[2] = cmul(st.v[2], q);
    const Cd v3 = cmul(st.v[3], r);
    st.v[3] = {-v3.re, -v3.im};
    st.v[4] = cmulc(st.v[4], r);
    const Cd v5 = cmulc(st.v[5], q);
    st.v[5] = {-v5.re, -v5.im};
    st.v[7] = cmulc(st.v[7], t);
  } else {
    // powers q^a, a = 3, 1, -1, -3 (index (3 - a) / 2), and conj(r)^b
    const Cd q3 = cmul(cmul(q, q), q), r3 = cmul(cmul(r, r), r);
    const Cd qa[4] = {q3, q, {q.re, -q.im}, {q3.re, -q3.im}};  // q^a
    const Cd rb[4] = {{r3.re, -r3.im}, {r.re, -r.im}, r, r3};    // conj(r)^b
    Cd w[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) w[a][b] = cmul(qa[a], rb[b]);
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int u1 = (c >> 4) & 1, u2 = (c >> 3) & 1, v1 = (c >> 2) & 1, v2 = (c >> 1) & 1,
                z = c & 1;
      const int su = 3 - 2 * (u1 + u2 + z), sv = 3 - 2 * (v1 + v2 + z);
      const bool neg = ((u1 & u2) ^ (u2 & z) ^ (v1 & v2) ^ (v2 & z)) != 0;
      const Cd p = cmul(st.v[c], w[(3 - su) / 2][(3 - sv) / 2]);
      st.v[c] = neg ? Cd{-p.re, -p.im} : p;
    }
  }
}

// v <- v J_k
template <int L>
__device__ inline void apply_bond(PsState<L>& st, Cd px, Cd py) {
  const Cd pz = cmulc(px, py);  // shared line: e^{i (theta_x - theta_y) / 2}
  if constexpr (L == 1) {
    butterfly(st.v[0], st.v[1], pz);
  } else if constexpr (L == 3) {
    const Cd pyc = {py.re, -py.im};
    // lines u1, u2 (bits 4, 3) take px; v1, v2 (bits 2, 1) conj(py); z pz
#pragma unroll
    for (int bit = 4; bit >= 0; --bit) {
      const Cd p = bit >= 3 ? px : (bit >= 1 ? pyc : pz);
#pragma unroll
      for (int c = 0; c < 32; ++c)
        if (!((c >> bit) & 1)) butterfly(st.v[c], st.v[c | (1 << bit)], p);
    }
  } else {
    const Cd pyc = {py.re, -py.im};
#pragma unroll
    for (int c = 0; c < 4; ++c) butterfly(st.v[c], st.v[c + 4], px);  // u1 line
    butterfly(st.v[0], st.v[2], pyc);  // v1 line
    butterfly(st.v[1], st.v[3], pyc);
    butterfly(st.v[4], st.v[6], pyc);
    butterfly(st.v[5], st.v[7], pyc);
#pragma unroll
    for (int c = 0; c < 8; c += 2) butterfly(st.v[c], st.v[c + 1], pz);  // z line
  }
}

template <int L>
__device__ inline void rescale(PsState<L>& st, int& expo) {
  double m = 0.0;
#pragma unroll
  for (int c = 0; c < PsState<L>::S; ++c) m = fmax(m, fmax(fabs(st.v[c].re), fabs(st.v[c].im)));
  if (m > 0.0) {
    int e;
    (void)frexp(m, &e);
    expo += e;
    const double sc = ldexp(1.0, -e);
#pragma unroll
    for (int c = 0; c < PsState<L>::S; ++c) st.v[c] = {st.v[c].re * sc, st.v[c].im * sc};
  }
}

template <int L>
__global__ __launch_bounds__(kPsThreads) void pathsum_kernel(
    const double4* __restrict__ tr, int64_t m, const double4* __restrict__ tc, int64_t n,
    int d, int symmetric, int64_t ntc, double* __restrict__ kq, int64_t ld_kq,
    double* __restrict__ lnkq, int64_t ld_ln, qk_fuse_desc f, int use_fuse) {
  // tile coordinates: the upper triangle row by row (symmetric) or row-major
  int64_t q = blockIdx.x, ti = 0, tj;
  if (symmetric) {
    while (q >= ntc - ti) {
      q -= ntc - ti;
      ++ti;
    }
    tj = ti + q;
  } else {
    ti = q / ntc;
    tj = q % ntc;
  }
  const int r = threadIdx.x / kPsTile, c = threadIdx.x % kPsTile;
  const int64_t i = ti * kPsTile + r, j = tj * kPsTile + c;
  const bool valid = i < m && j < n && (!symmetric || j >= i);
  // lanes past the edge shadow the last row / column (loads stay in bounds)
  const int64_t ii = i < m ? i : m - 1, jj = j < n ? j : n - 1;

  PsState<L> st;
  int expo = -L * d;  // the 2^-L of every site weight
  double4 a = tr[ii], b = tc[jj];
#pragma unroll
  for (int s = 0; s < PsState<L>::S; ++s) st.v[s] = {1.0, 0.0};
  apply_weight<L>(st, Cd{a.x, a.y}, Cd{b.x, b.y});
  for (int k = 1; k < d; ++k) {
    const double4 an = tr[(int64_t)k * m + ii], bn = tc[(int64_t)k * n + jj];
    apply_bond<L>(st, Cd{a.z, a.w}, Cd{b.z, b.w});
    apply_weight<L>(st, Cd{an.x, an.y}, Cd{bn.x, bn.y});
    if (k % kPsRescale == 0) rescale<L>(st, expo);
    a = an;
    b = bn;
  }
  rescale<L>(st, expo);
  Cd amp = {0.0, 0.0};
#pragma unroll
  for (int s = 0; s < PsState<L>::S; ++s) amp = {amp.re + st.v[s].re, amp.im + st.v[s].im};
  if (!valid) return;
  const double lnk = qk_ln_kq(amp.re, amp.im, expo);
  const double kqv = exp(lnk);
  auto put = [&](double* p, int64_t ld, double v) {
    if (!p) return;
    p[i * ld + j] = v;
    if (symmetric && j != i) p[j * ld + i] = v;
  };
  put(kq, ld_kq, kqv);
  put(lnkq, ld_ln, lnk);
  if (use_fuse) {
    const double kc = exp(-f.gamma * qk_sq_dist(f.x_rows_dev + i * f.ld_xr,
                                                 f.x_cols_dev + j * f.ld_xc, d));
    const double w = f.w_rows_dev ? f.w_rows_dev[i] : f.w;
    put(f.kc_dev, f.ld_kc, kc);
    put(f.k_dev, f.ld_k, qk_mix(w, kqv, kc));
  }
}

}  // namespace

hipError_t qk_launch_pathsum_table(const double* x, int64_t n, int64_t ld_x, int d, int n_layers,
                                   int entangle, double4* tab, hipStream_t s) {
  const int64_t total = n * (int64_t)d;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(pathsum_table_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     x, n, ld_x, d, n_layers, entangle, tab);
  return hipGetLastError();
}

hipError_t qk_launch_pathsum(const double4* tr, int64_t m, const double4* tc, int64_t n, int d,
                             int n_layers, int symmetric, double* kq, int64_t ld_kq,
                             double* lnkq, int64_t ld_ln, const qk_fuse_desc* fuse,
                             hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  const int64_t ntr = (m + kPsTile - 1) / kPsTile, ntc = (n + kPsTile - 1) / kPsTile;
  const int64_t tiles = symmetric ? ntr * (ntr + 1) / 2 : ntr * ntc;
  qk_fuse_desc f{};
  if (fuse) f = *fuse;
  const int use_fuse = fuse ? 1 : 0;
  if (n_layers == 1)
    hipLaunchKernelGGL(pathsum_kernel<1>, dim3((unsigned)tiles), dim3(kPsThreads), 0, s, tr, m, tc,
                       n, d, symmetric, ntc, kq, ld_kq, lnkq, ld_ln, f, use_fuse);
  else if (n_layers == 3)
    hipLaunchKernelGGL(pathsum_kernel<3>, dim3((unsigned)tiles), dim3(kPsThreads), 0, s, tr, m, tc,
                       n, d, symmetric, ntc, kq, ld_kq, lnkq, ld_ln, f, use_fuse);
  else
    hipLaunchKernelGGL(pathsum_kernel<2>, dim3((unsigned)tiles), dim3(kPsThreads), 0, s, tr, m, tc,
                       n, d, symmetric, ntc, kq, ld_kq, lnkq, ld_ln, f, use_fuse);
  return hipGetLastError();
}
