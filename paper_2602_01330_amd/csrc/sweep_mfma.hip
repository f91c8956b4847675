// Matrix-core (MFMA) forms of the transfer-matrix overlap sweep, chi_pad <= 4.
//
// Per pair (i, j) and site k:  E' = sum_s A_i^{s dagger} E B_j^s  (E is 4 x 4
// complex). Complex products are realified, [Re C | Im C] = [Re X | Im X] .
// [[Re Y, Im Y], [-Im Y, Re Y]]. Two kernels:
//
// * FP32 (sweep_m4_kernel, further below): both steps of a site on the
//   4 x 4 x 1 block MFMA, one block per pair, E and G kept in registers; see
//   the comment above that kernel.
//
// * Split BF16 (sweep_mfma_kernel): each site is two GEMM-shaped steps on
//   16 x 16 MFMAs,
//   step R (right multiply, shared by the pairs of one column j):
//     G[(p,a)][(s,c,b')] = sum_{(c_in,b)} E[(p,a)][(c_in,b)] Bhat_j[(c_in,b)][(s,c,b')]
//     16 x 16 x 8 per column of four pairs, every lane busy;
//   step L (left multiply, shared by the pairs of one row i):
//     E'[(c',a')][(q,b')] = sum_{(s,c_in,a)} Ahat_i[(c',a')][(s,c_in,a)] G[(s,c_in,a)][(q,b')]
//     8 x 16 x 16 per row of four pairs, whose rows 8..15 are zero: chi = 4
//     gives only 8 realified output rows, so this step runs the matrix cores
//     at half width (the ceiling of this kernel is 2/3 of the MFMA peak).
//   A wavefront owns a 4 x 4 block of pairs and runs its whole chain of
//   sites without workgroup barriers. Every lane loads its own operand values
//   of the next site with buffer loads (prefetched one site ahead, straight
//   into the operand registers; the 16 waves of a workgroup share the 16 row
//   and 16 column samples of a 16 x 16 tile, so repeats hit the CU's L1). The
//   two re-layouts between the steps (MFMA output -> operand of the other
//   step) go through a per-wave LDS area. Every packed element holds z and
//   i z (one extra float), each lane loads the form its output part needs,
//   and E enters step R as (Im E, Re E) so that the one negated entry of the
//   realified product falls on the i z form.
//   The operands are split into BF16 pieces for v_mfma_f32_16x16x32_bf16
//   with FP32 accumulation -- BF16x2: x = h + l with round-to-nearest pieces
//   (|x - h - l| <= 2^-18 |x|), the products hh, hl, lh, ll; BF16x3:
//   x = h + m + l exactly (8+8+8 bits), the products of total order <= 2 plus
//   m*l and l*m (8 per real product). The split is folded into the
//   contraction index, so one MFMA K of 32 covers four (BF16x2) or eight
//   (BF16x3) products of each FP32 term.
//
// Common to both: addresses come from a per-site buffer descriptor (scalar)
// plus constant per-lane offsets; offsets past a site array's end read as
// zero in hardware, which pads bond blocks smaller than 4 x 4 without any
// per-element select. On gfx950 plain VALU instructions do not overlap the
// FP32 MFMAs of the same SIMD, so the site loops keep VALU work small. Each
// pair's E is scaled by an exact power of two every kRescaleEvery sites
// (per-pair int32 exponent), at the same sites for every pair.
//
// Reduced-precision forms mark every pair whose K_q exceeds a threshold;
// the FP64 sweep (the refinement pass with the masks) recomputes the tiles
// holding marked pairs and writes exactly those pairs, so that entries near
// 1 carry FP64 accuracy.
#include <hip/hip_runtime.h>

#include "qk_tune.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum Form { kBF16x2 = 1, kBF16x3 = 2 };  // split-BF16 forms of the 16 x 16 kernel

// A wave owns kColBlocks 4 x 4 pair blocks side by side (same four rows):
// the row operands and their forms are loaded and built once for all of them.
// Two blocks per wave halve the row operand work but need more than 128
// registers, i.e. two waves per SIMD instead of four; one block per wave
// measured faster on the 784-qubit image workload.
constexpr int kColBlocks = 1;
constexpr int kWavesPerRow = 4 / kColBlocks;
constexpr int kWaves = 16 / kColBlocks;  // waves per 16 x 16 pair tile
constexpr int kThreads = 64 * kWaves;
constexpr int kTile = 16;
// Per-wave LDS areas (floats). Strides are chosen so that the accesses of
// each half-wave (b32, 32 lanes) or lane octet (b128) fall in distinct banks
// of a 32-bank LDS:
//   G[p][q][a][b'][(s,c)] = p*336 + q*80 + a*16 + b'*4 + (s,c)
//     written b32 by lanes (p, (s,c,b')), read b128 by lanes (a, (q,b'));
//   E[q][p][a][(b,c)]     = q*136 + p*34 + a*8 + b*2 + c
//     written b32 by lanes (c, (q,b)), read b64 by lanes (b, (p,a)).
constexpr int kGp = 336, kGq = 80, kGa = 16;
constexpr int kEq = 136, kEp = 34;
// Sites between exact rescales. The transfer map of two normalised
// left-canonical MPS is a contraction, so E never overflows; between two
// rescales its largest entry (in [1/2, 1) after a rescale) must not fall
// below the FP32 normal range, i.e. shrink by 2^126 within this many sites,
// which only pairs whose overlap is already negligible can do.
constexpr int kRescaleEvery = 8;

// Feature rows staged for the fused RBF distances after the sweep, over the
// (then idle) G areas: 32 samples x kXChunk doubles, padded rows.
constexpr int kXChunk = 256;
constexpr int kXStride = kXChunk + 2;

struct MfmaSmem {
  alignas(16) float g[16][4 * kGp];  // per 4 x 4 pair block
  float e[16][4 * kEq];
  int ex[16][16];
  unsigned mask[kQkMaskWords];
};
static_assert(32 * kXStride * sizeof(double) <= sizeof(float) * 16 * 4 * kGp,
              "feature staging fits in the G areas");

// max over lanes l ^ 1 and l ^ 2 (DPP quad permutations) and l ^ 16
// (swizzle) of the bit patterns of non-negative floats, whose unsigned order
// is their numeric order
__device__ inline unsigned umax_xor_1_2_16(unsigned m) {
  // old value 0 is the identity of the max, so each permute folds into the
  // max as a DPP operand
  m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0xB1, 0xF, 0xF, false));
  m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x4E, 0xF, 0xF, false));
  m = max(m, (unsigned)__builtin_amdgcn_ds_swizzle((int)m, 0x401F));
  return m;
}

// Scale for a pair whose largest |entry| has the bit pattern m: 2^(126 - ex)
// with ex the biased exponent of m, which brings that entry into [1/2, 1).
// ex = 0 (zero or subnormal maximum) scales by 2^126, leaving zeros at zero;
// ex = 255 (inf / NaN) gives a huge negative factor, so non-finite values
// stay non-finite; ex <= 253 always holds for finite E, whose entries never
// exceed 1 (the transfer map is a contraction).
__device__ inline float rescale_factor(unsigned ex) { return __uint_as_float((253u - ex) << 23); }

// Buffer descriptor over one site's packed sample array: loads at byte
// offsets at or beyond `bytes` return zero, which pads bond blocks smaller
// than 4 x 4 and the unused operand rows without any per-element select.
__device__ inline __amdgpu_buffer_rsrc_t site_rsrc(const char* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ inline float2 ld2(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

__device__ inline __bf16 bf16_trunc(float x) {
  unsigned short h = (unsigned short)(__float_as_uint(x) >> 16);
  return __builtin_bit_cast(__bf16, h);
}
__device__ inline float bf16_trunc_f(float x) { return __uint_as_float(__float_as_uint(x) & 0xffff0000u); }

// pieces of x: BF16x2 -> (h, l), BF16x3 -> (h, m, l)
template <int F>
struct Split;
template <>
struct Split<kBF16x2> {
  __bf16 p[2];
  __device__ Split(float x) {
    // round-to-nearest pieces: |x - h - l| <= 2^-18 |x|
    p[0] = (__bf16)x;
    p[1] = (__bf16)(x - (float)p[0]);
  }
};
template <>
struct Split<kBF16x3> {
  __bf16 p[3];
  __device__ Split(float x) {
    float h = bf16_trunc_f(x);
    float r = x - h;
    float m = bf16_trunc_f(r);
    p[0] = bf16_trunc(x);
    p[1] = bf16_trunc(r);
    p[2] = (__bf16)(r - m);
  }
};

// piece index of the left / right factor for product term t
__device__ constexpr int lhs_piece2(int t) { return t >> 1; }       // h h l l
__device__ constexpr int rhs_piece2(int t) { return t & 1; }        // h l h l
__device__ constexpr int lhs_piece3(int t) {                        // 0 0 1 0 1 2 1 2
  return t == 0 ? 0 : t == 1 ? 0 : t == 2 ? 1 : t == 3 ? 0 : t == 4 ? 1 : t == 5 ? 2 : t == 6 ? 1 : 2;
}
__device__ constexpr int rhs_piece3(int t) {                        // 0 1 0 2 1 0 2 1
  return t == 0 ? 0 : t == 1 ? 1 : t == 2 ? 0 : t == 3 ? 2 : t == 4 ? 1 : t == 5 ? 0 : t == 6 ? 2 : 1;
}

// acc[x] += sum over NC chunks of a[x][c] * b[x][c] for four independent
// products x, issued chunk-major so consecutive MFMAs never depend on each
// other.
template <int F, int NC>
__device__ inline void mma4(const float (*a)[NC], const float (*b)[NC], f4* acc) {
  if constexpr (F == kBF16x2) {
#pragma unroll
    for (int c0 = 0; c0 < NC; c0 += 2) {
      bf8 va[4], vb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          Split<kBF16x2> sa(a[x][c0 + h]), sb(b[x][c0 + h]);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            va[x][h * 4 + t] = sa.p[lhs_piece2(t)];
            vb[x][h * 4 + t] = sb.p[rhs_piece2(t)];
          }
        }
#pragma unroll
      for (int x = 0; x < 4; ++x)
        acc[x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va[x], vb[x], acc[x], 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bf8 va[4], vb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        Split<kBF16x3> sa(a[x][c]), sb(b[x][c]);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          va[x][t] = sa.p[lhs_piece3(t)];
          vb[x][t] = sb.p[rhs_piece3(t)];
        }
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
        acc[x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va[x], vb[x], acc[x], 0, 0, 0);
    }
  }
}


#define QK_LDS_FENCE() __asm__ volatile("" ::: "memory")

template <int F>
__device__ void run_tile(const QkTask& t, int ti, int tj, MfmaSmem& sm, uint32_t* mask,
                         int64_t tile_id, double ln_tau) {
  constexpr int NB = kColBlocks;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index: scalar
  const int lane = tid & 63;
  const int g = lane >> 4, n = lane & 15;
  const int wr = w / kWavesPerRow, wc0 = (w % kWavesPerRow) * NB;
  const int64_t i0 = (int64_t)ti * kTile + 4 * wr;
  int64_t j0[NB];
  float* gb[NB];
  float* eb[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    j0[x] = (int64_t)tj * kTile + 4 * (wc0 + x);
    gb[x] = sm.g[wr * 4 + wc0 + x];
    eb[x] = sm.e[wr * 4 + wc0 + x];
  }
  const int T = t.T, TT = T * T, slotT = 2 * TT;
  const int nq = t.nq;

  // ---- per-lane byte offsets into a site's packed sample array (constant
  // over the sites). Samples past the end are clamped to the last one: those
  // pairs compute garbage that is never written, and every pair's E is
  // independent. Elements outside the T x T bond block, and the A values of
  // the zero rows of step L, take the out-of-range offset and load as zero.
  // step R, column q: B^s[b = g][b' = n&3], s = n>>3
  const int rs = n >> 3, rcout = (n >> 2) & 1, rbp = n & 3;
  // step L, row p: A^s[a = g][a' = n&3] for s = 0, 1 (lanes n < 8)
  const int lcp = n >> 2, lap = n & 3;
  constexpr int kEB = kQkPackFloats * 4;  // bytes per packed complex element
  const unsigned bbytes = (unsigned)((int64_t)t.nb * slotT * kEB);
  const unsigned abytes = (unsigned)((int64_t)t.na * slotT * kEB);
  const bool bin = g < T && rbp < T;
  const bool ain = g < T && lap < T && n < 8;
  unsigned boff[NB][4], aoff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int x = 0; x < NB; ++x) {
      const int64_t j = (j0[x] + q) < t.nb ? (j0[x] + q) : (t.nb - 1);
      // the lane's operand pair is z = (x, y) (packed bytes 4..11) or
      // i z = (-y, x) (bytes 0..7): output part c = 0 (Im of G) takes z,
      // c = 1 (Re of G) takes i z
      boff[x][q] = bin ? (unsigned)((j * slotT + rs * TT + g * T + rbp) * kEB + (rcout ? 0 : 4))
                       : bbytes;
    }
    const int64_t i = (i0 + q) < t.na ? (i0 + q) : (t.na - 1);
    // rows c' = 0 (Re of E') take z, rows c' = 1 (Im of E') take i z
    aoff[q] = ain ? (unsigned)((i * slotT + g * T + lap) * kEB + (lcp ? 0 : 4)) : abytes;
  }
  const unsigned a1off = (unsigned)(TT * kEB);
  const char* bbase = static_cast<const char*>(t.tb);
  const char* abase = static_cast<const char*>(t.ta);
  const int64_t bstride = bbytes, astride = abytes;

  struct Ops {
    float2 b[NB][4];
    float2 a[4][2];
  };
  // the loads land straight in the operand registers and stay in flight
  // until their first use one step later
  auto fetch_b = [&](int k, Ops& o) {
    const __amdgpu_buffer_rsrc_t r = site_rsrc(bbase + (int64_t)k * bstride, bbytes);
#pragma unroll
    for (int x = 0; x < NB; ++x)
#pragma unroll
      for (int q = 0; q < 4; ++q) o.b[x][q] = ld2(r, boff[x][q]);
  };
  auto fetch_a = [&](int k, Ops& o) {
    const __amdgpu_buffer_rsrc_t r = site_rsrc(abase + (int64_t)k * astride, abytes);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o.a[q][0] = ld2(r, aoff[q]);
      o.a[q][1] = ld2(r, aoff[q] + a1off);
    }
  };

  // E in step-R operand form: lane (p = n>>2, a = n&3, b = g) holds
  // (Im E[a][b], Re E[a][b]) as the contraction parts (0, 1). Against the B
  // forms z = (x, y) and i z = (-y, x) this gives Im(E B) = Im E x + Re E y
  // and Re(E B) = Re E x - Im E y with no sign work.
  float eR[NB][4][2];
  int expo[NB][4];
#pragma unroll
  for (int x = 0; x < NB; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      eR[x][q][0] = 0.f;
      eR[x][q][1] = ((n & 3) == 0 && g == 0) ? 1.f : 0.f;
      expo[x][q] = 0;
    }

  // one site; each operand set is refetched for the next site right after
  // its last use
  Ops cur;
  auto site_step = [&](int k) {
    const bool more = k + 1 < nq;
    const int kn = more ? k + 1 : k;
    // ---- step R: G = E Bhat_j for each block's four columns (four
    // independent chains per block, issued chunk-major)
    {
      f4 acc[NB][4];
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        float bop[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bop[q][0] = cur.b[x][q].x;
          bop[q][1] = cur.b[x][q].y;
          acc[x][q] = f4{0.f, 0.f, 0.f, 0.f};
        }
        mma4<F, 2>(eR[x], bop, acc[x]);
      }
      fetch_b(kn, cur);  // in flight until the next step R
      // lane holds G[(p=g, a=r)][(s, c, b')] of pair (g, q), c = 0 the
      // imaginary and c = 1 the real part; stored as (s, Re / Im)
#pragma unroll
      for (int x = 0; x < NB; ++x)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float* gw = &gb[x][g * kGp + q * kGq + rbp * 4 + (rs * 2 + (rcout ^ 1))];
#pragma unroll
          for (int r = 0; r < 4; ++r) gw[r * kGa] = acc[x][q][r];
        }
    }
    QK_LDS_FENCE();
    // keep the step-L operand work (which waits for the A loads) below this
    // point, so step R waits only for the B loads issued one site earlier
    __builtin_amdgcn_sched_barrier(0);
    // ---- step L: E' = Ahat_i^dagger G for the wave's four rows (the row
    // operand built once for all blocks), then the exact power-of-two rescale
    // every few sites (pair (p, q) lives on lanes g in {0,1}, n>>2 == q: 4
    // lanes b' x 4 registers), then E' to LDS
    {
      const int q = n >> 2, bp = n & 3;  // output column (q, b')
      float aop[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        // z or i z of A^s[a][a'] (zero on rows n >= 8): against (Re G, Im G)
        // this gives Re(conj(A) G) on rows c' = 0 and Im(conj(A) G) on c' = 1
        const float2 a0 = cur.a[p][0], a1 = cur.a[p][1];
        aop[p][0] = a0.x;  // s = 0, c_in = 0
        aop[p][1] = a0.y;  // s = 0, c_in = 1
        aop[p][2] = a1.x;  // s = 1, c_in = 0
        aop[p][3] = a1.y;  // s = 1, c_in = 1
      }
      f4 acc[NB][4];
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        float bop[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const f4 gv = *reinterpret_cast<const f4*>(&gb[x][p * kGp + q * kGq + g * kGa + bp * 4]);
          bop[p][0] = gv[0];
          bop[p][1] = gv[1];
          bop[p][2] = gv[2];
          bop[p][3] = gv[3];
          acc[x][p] = f4{0.f, 0.f, 0.f, 0.f};
        }
        mma4<F, 4>(aop, bop, acc[x]);
      }
      fetch_a(kn, cur);  // in flight until the next step L
      // every pair rescales at the same sites: a power-of-two scale is exact
      // except where entries enter the subnormal range, so a schedule that
      // depended on the wave would make a pair's last bits depend on its
      // position in the launch
      const bool rescale = (k % kRescaleEvery) == kRescaleEvery - 1;
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        if (rescale) {
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            // largest |entry| of the lane (NaN-propagating maximum, no
            // canonicalising), then over the pair's lanes as bit patterns
            const float lm = __builtin_elementwise_maximum(
                __builtin_elementwise_maximum(fabsf(acc[x][p][0]), fabsf(acc[x][p][1])),
                __builtin_elementwise_maximum(fabsf(acc[x][p][2]), fabsf(acc[x][p][3])));
            const unsigned m = umax_xor_1_2_16(__float_as_uint(lm));
            const unsigned ex = m >> 23;
            const float sc = rescale_factor(ex);
            expo[x][p] += (int)ex - 126;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[x][p][r] *= sc;
          }
        }
        if (g < 2) {
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              eb[x][q * kEq + p * kEp + r * 8 + bp * 2 + g] = acc[x][p][r];
        }
      }
    }
    QK_LDS_FENCE();
    {
      const int p = n >> 2, a = n & 3;
#pragma unroll
      for (int x = 0; x < NB; ++x)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float2 ev =
              *reinterpret_cast<const float2*>(&eb[x][q * kEq + p * kEp + a * 8 + g * 2]);
          eR[x][q][0] = ev.y;  // Im
          eR[x][q][1] = ev.x;  // Re
        }
    }
    QK_LDS_FENCE();
  };

  // Drain the previous tile's output stores first: with stores and loads
  // both outstanding the vector memory counter no longer counts in order, and
  // every operand use in the loop would wait for all loads. Then B before A,
  // as inside the loop, so that each use waits only for its own loads.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt / lgkmcnt untouched
  fetch_b(0, cur);
  __builtin_amdgcn_sched_barrier(0);
  fetch_a(0, cur);
  __builtin_amdgcn_sched_barrier(0);
  for (int k = 0; k < nq; ++k) site_step(k);

  // ---- epilogue: pair (p, q) = (pi >> 2, pi & 3) of each block, four lanes
  // per pair
  if (g == 0 && (n & 3) == 0) {
#pragma unroll
    for (int x = 0; x < NB; ++x)
#pragma unroll
      for (int p = 0; p < 4; ++p) sm.ex[wr * 4 + wc0 + x][p * 4 + (n >> 2)] = expo[x][p];
  }
  if (tid < kQkMaskWords) sm.mask[tid] = 0;
  const int pi = lane & 15, part = lane >> 4;
  const int p = pi >> 2, q = pi & 3;
  const int64_t i = i0 + p;
  // final E[0][0] and exponent of each pair to registers (the wave's own LDS
  // areas), then every wave is done with the G areas
  float2 efin[NB];
  int xfin[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    efin[x] = *reinterpret_cast<const float2*>(&eb[x][q * kEq + p * kEp]);
    xfin[x] = sm.ex[wr * 4 + wc0 + x][pi];
  }
  __syncthreads();
  // fused RBF: squared distances by direct difference, the tile's 16 row and
  // 16 column feature vectors staged through LDS in chunks (each feature
  // element is read from memory once per tile); lane `part` of a pair sums
  // the features f = part mod 4 of each chunk
  double d2[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) d2[x] = 0.0;
  if (t.fuse) {
    double* xs = reinterpret_cast<double*>(&sm.g[0][0]);
    const int64_t ti0 = (int64_t)ti * kTile, tj0 = (int64_t)tj * kTile;
    for (int f0 = 0; f0 < nq; f0 += kXChunk) {
      const int nf = min(kXChunk, nq - f0);
      for (int e = tid; e < 32 * nf; e += kThreads) {
        const int smp = e / nf, f = e - smp * nf;
        double v = 0.0;
        if (smp < 16) {
          const int64_t r = ti0 + smp;
          if (r < t.na) v = t.xr[r * t.ld_xr + f0 + f];
        } else {
          const int64_t c = tj0 + smp - 16;
          if (c < t.nb) v = t.xc[c * t.ld_xc + f0 + f];
        }
        xs[smp * kXStride + f] = v;
      }
      __syncthreads();
      const double* xrow = xs + (4 * wr + p) * kXStride;
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const double* xcol = xs + (16 + 4 * (wc0 + x) + q) * kXStride;
        double acc = 0.0;
        for (int f = part; f < nf; f += 4) {
          const double df = xrow[f] - xcol[f];
          acc += df * df;
        }
        d2[x] += acc;
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    const int64_t j = j0[x] + q;
    const bool valid = i < t.na && j < t.nb && (!t.symmetric || j >= i);
    const double re = (double)efin[x].x, im = (double)efin[x].y;
    const double mag2 = re * re + im * im;
    const double lnk =
        mag2 > 0.0 ? log(mag2) + 2.0 * (double)xfin[x] * 0.69314718055994530942 : -INFINITY;
    const double kq = mag2 > 0.0 ? exp(lnk) : 0.0;
    double d2x = d2[x];
    d2x += __shfl_xor(d2x, 16, 64);
    d2x += __shfl_xor(d2x, 32, 64);
    if (valid && part == 0) {
      auto put = [&](double* ptr, int64_t ld, double v) {
        if (!ptr) return;
        ptr[i * ld + j] = v;
        if (t.symmetric && j != i) ptr[j * ld + i] = v;
      };
      put(t.kq, t.ld_kq, kq);
      put(t.lnkq, t.ld_ln, lnk);
      if (t.fuse) {
        const double kc = exp(-t.gamma * d2x);
        const double wgt = t.w_rows ? t.w_rows[i] : t.w;
        put(t.kc, t.ld_kc, kc);
        put(t.k, t.ld_k, wgt * kq + (1.0 - wgt) * kc);
      }
      if (mask && lnk > ln_tau) {
        const int bit = (int)(i - (int64_t)ti * kTile) * kTile + (int)(j - (int64_t)tj * kTile);
        atomicOr(&sm.mask[bit >> 5], 1u << (bit & 31));
      }
    }
  }
  __syncthreads();
  if (mask && tid < kQkMaskWords) mask[tile_id * kQkMaskWords + tid] = sm.mask[tid];
}

template <int F>
__global__ __launch_bounds__(kThreads) void sweep_mfma_kernel(QkTaskTable tt, uint32_t* flags,
                                                              double ln_tau) {
  __shared__ MfmaSmem sm;
  for (int64_t rnd = 0; rnd * gridDim.x < tt.total_tiles; ++rnd) {
    const int64_t q = qk_tile_of(rnd, blockIdx.x, gridDim.x);
    if (q >= tt.total_tiles) break;  // only the last round is partial
    int k = 0;
    while (k + 1 < tt.n_tasks && tt.t[k + 1].tile_begin <= q) ++k;
    const QkTask& t = tt.t[k];
    int ti, tj;
    qk_tile_coords(t, q - t.tile_begin, ti, tj);
    run_tile<F>(t, ti, tj, sm, flags, q, ln_tau);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// FP32 form on the 4x4x1 block MFMA (v_mfma_f32_4x4x1_16b_f32: sixteen
// independent 4 x 4 outer-product accumulations per instruction, at the
// same FLOP rate as the 16 x 16 x 4 shape). Block b of an instruction is one
// pair of the wave's 4 x 4 pair block, so neither step wastes a row:
//
//   step R, per pair:  G^s[a][(c,b')] = sum_(c_in,b) E[a][(c_in,b)] Bhat^s[(c_in,b)][(c,b')]
//     four chains (s, c) of eight K steps; A operand: lane a of the block
//     holds row a of E (Re and Im for b = 0..3); B operand: lane b' holds
//     column b' of Bhat. The output leaves lane b' holding column b' of
//     G^s_c (rows a in the four accumulator registers).
//   step L, per pair (transposed):  E'^T[b'][(c',a')] = sum_(s,c_in,a) G^s_(c_in)[a][b'] Ahat^s[(c_in,a)][(c',a')]
//     two chains c' of sixteen K steps; A operand: lane b' holds column b'
//     of G -- exactly what step R left there; B operand: lane a' holds
//     column a' of Ahat. The output leaves lane a' holding row a' of E' --
//     exactly the A operand of the next step R.
//
// E and G never leave the registers: no LDS and no lane exchange per site.
// The column operand Bhat_j depends only on the pair's column, and pairs
// (p, q) sit in block 4 p + q, so the four 16-lane groups (rows p) need the
// same values: each group loads one quarter (bond row b = its group index)
// and every step R instruction broadcasts the group holding its b to all
// four groups (BLGP = 4 + b). The row operand Ahat_i is loaded whole by the
// four lanes of every block. Both come from the packed (-Im, Re, Im)
// elements, three floats per lane and element, which hold every sign the
// realified products take.
// soff is a wave-uniform constant (the element's offset from the lane's
// base): it travels in the instruction's scalar offset, not in a VGPR
__device__ inline float3 ld3(__amdgpu_buffer_rsrc_t r, unsigned off, int soff = 0) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, soff, 0);
  return make_float3(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]));
}

// packed element (-Im z, Re z, Im z) -> entry of the realified right factor
// [[Re, Im], [-Im, Re]] at (c_in, c): (0,0) Re, (1,0) -Im, (0,1) Im, (1,1) Re
__device__ inline float rhat(const float3& v, int c, int c_in) {
  return c == c_in ? v.y : (c_in ? v.x : v.z);
}
// entry of the realified conj(A) factor at (c_in, c'): Re(conj(a) g) =
// Re a Re g + Im a Im g, Im(conj(a) g) = Re a Im g - Im a Re g
__device__ inline float lhat(const float3& v, int cp, int c_in) {
  return cp == c_in ? v.y : (c_in ? v.z : v.x);
}

template <int BQ>
__device__ inline void m4_step_r_b(const float (&e)[2][4], const float3 (&wb)[2], f4 (&g)[2][2]) {
#pragma unroll
  for (int cin = 0; cin < 2; ++cin)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        g[s][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(e[cin][BQ], rhat(wb[s], c, cin), g[s][c], 0, 0,
                                                     4 + BQ);
}

// Per-wave staging slot of the row operand: 4 rows x 32 elements (s, a, x)
// of one site, each element padded to 16 bytes for aligned b128 reads. Rows
// are 64 bytes further apart than their 512 bytes, so the four rows' elements
// that one read instruction gathers (row pp, element x, for every pp and x)
// start on different LDS banks.
constexpr int kM4StRow = 32 * 4 + 16;  // floats per staged row
struct M4Smem {
  union {
    alignas(16) double xs[32 * kXStride];   // feature rows of the tile (fused RBF, after the sweep)
    alignas(16) float st[16][4 * kM4StRow];  // row-operand staging, one slot per wave (during it)
  } u;
  unsigned mask[kQkMaskWords];
};

// A wave owns NB 4 x 4 pair blocks side by side (same four rows): the row
// operand is loaded once for all of them, which halves the load traffic per
// MFMA at NB = 2; a 16 x 16 tile then takes 16 / NB waves.
template <int NB, int T>
__device__ void run_tile_m4(const QkTask& t, int ti, int tj, M4Smem& sm, uint32_t* mask,
                            int64_t tile_id, double ln_tau) {
  constexpr int kThr = kThreads / NB;
  constexpr int TT = T * T, slotT = 2 * TT;
  constexpr int kEB = kQkPackFloats * 4;  // bytes per packed element
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index: scalar
  const int lane = tid & 63;
  const int x = lane & 3, qq = (lane >> 2) & 3, pp = lane >> 4;
  const int wr = w / (4 / NB), wc0 = (w % (4 / NB)) * NB;
  const int64_t i = (int64_t)ti * kTile + 4 * wr + pp;
  int64_t j[NB];
#pragma unroll
  for (int y = 0; y < NB; ++y) j[y] = (int64_t)tj * kTile + 4 * (wc0 + y) + qq;
  // samples past the end are clamped to the last one: their pairs compute
  // values that are never written
  const int64_t ic = i < t.na ? i : t.na - 1;
  const int nq = t.nq;
  const unsigned bbytes = (unsigned)((int64_t)t.nb * slotT * kEB);
  const unsigned abytes = (unsigned)((int64_t)t.na * slotT * kEB);
  // Per-lane base offsets; the element (s, a) adds a constant scalar offset.
  // Lanes whose bond index lies outside the T x T block start at the
  // out-of-range offset and load zeros (whether or not the range check counts
  // the scalar part: valid elements lie inside the array, and the library
  // keeps n * slot + 4 KiB below 2^32); bond rows a >= T are not loaded.
  unsigned boff[NB];
#pragma unroll
  for (int y = 0; y < NB; ++y) {
    const int64_t jc = j[y] < t.nb ? j[y] : t.nb - 1;
    boff[y] = (pp < T && x < T) ? (unsigned)((jc * slotT + pp * T + x) * kEB) : bbytes;
  }
  const char* bbase = static_cast<const char*>(t.tb);
  const char* abase = static_cast<const char*>(t.ta);
  const int64_t bstride = bbytes, astride = abytes;
  // The row operand is staged through the wave's own LDS slot: the wave's
  // 4 rows x 32 elements of a site are loaded from memory once (two
  // elements per lane, rows contiguous in memory) and every lane then reads
  // the 8 elements it needs; direct loads would return each element to all
  // four lanes of a row (one per column of the block), and load data return
  // is the sweep's other bottleneck next to the matrix cores. One wave writes
  // and reads its slot, and LDS operations of one wave complete in order, so
  // no barrier is needed.
  float* st = sm.u.st[w];
  unsigned soff[2];
  int sdst[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int el = lane + 64 * h, r = el >> 5, e = el & 31;
    const int s = e >> 4, a = (e >> 2) & 3, xx = e & 3;
    int64_t ir = (int64_t)ti * kTile + 4 * wr + r;
    ir = ir < t.na ? ir : t.na - 1;
    soff[h] = (a < T && xx < T) ? (unsigned)((ir * slotT + s * TT + a * T + xx) * kEB) : abytes;
    sdst[h] = r * kM4StRow + 4 * e;
  }

  float3 wb[NB][2];  // column operands: element [s][b = pp][x] of sample j
  float3 stg[2];     // staged row-operand elements in flight
  float3 va[2][4];   // row operand: elements [s][a][x] of sample i
  auto fetch_b = [&](int k) {
    const __amdgpu_buffer_rsrc_t r = site_rsrc(bbase + (int64_t)k * bstride, bbytes);
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int s = 0; s < 2; ++s) wb[y][s] = ld3(r, boff[y], s * TT * kEB);
  };
  auto fetch_stage = [&](int k) {
    const __amdgpu_buffer_rsrc_t r = site_rsrc(abase + (int64_t)k * astride, abytes);
#pragma unroll
    for (int h = 0; h < 2; ++h) stg[h] = ld3(r, soff[h]);
  };
  auto put_stage = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      *reinterpret_cast<f4*>(st + sdst[h]) = f4{stg[h].x, stg[h].y, stg[h].z, 0.f};
  };
  auto read_a = [&]() {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const f4 v = *reinterpret_cast<const f4*>(st + pp * kM4StRow + 4 * (s * 16 + a * 4 + x));
        va[s][a] = make_float3(v[0], v[1], v[2]);
      }
  };

  // lane x of a block holds row a = x of the pair's E: e[c][b] = (Re, Im) E[x][b]
  float e[NB][2][4];
#pragma unroll
  for (int y = 0; y < NB; ++y)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) e[y][c][b] = (c == 0 && b == 0 && x == 0) ? 1.f : 0.f;
  int expo[NB];
#pragma unroll
  for (int y = 0; y < NB; ++y) expo[y] = 0;

  __builtin_amdgcn_s_waitcnt(0x0F70);  // drain the previous tile's stores (vmcnt(0))
  fetch_stage(0);
  __builtin_amdgcn_sched_barrier(0);
  fetch_b(0);
  __builtin_amdgcn_sched_barrier(0);
  // one site: E <- sum_s A^{s dagger} E B^s for every pair of the wave
  auto site = [&](int k) {
    const int kn = k + 1 < nq ? k + 1 : k;
    // this site's row operand: staged elements to the slot, the next site's
    // staging loads in flight over the whole site, the lane's 8 elements
    // read back (their latency hidden behind step R)
    put_stage();
    fetch_stage(kn);
    read_a();
    __builtin_amdgcn_sched_barrier(0);
    f4 g[NB][2][2];
#pragma unroll
    for (int y = 0; y < NB; ++y) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 2; ++c) g[y][s][c] = f4{0.f, 0.f, 0.f, 0.f};
      m4_step_r_b<0>(e[y], wb[y], g[y]);
      m4_step_r_b<1>(e[y], wb[y], g[y]);
      m4_step_r_b<2>(e[y], wb[y], g[y]);
      m4_step_r_b<3>(e[y], wb[y], g[y]);
    }
    fetch_b(kn);  // in flight until the next step R
    __builtin_amdgcn_sched_barrier(0);
    f4 en[NB][2];
#pragma unroll
    for (int y = 0; y < NB; ++y) en[y][0] = en[y][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cin = 0; cin < 2; ++cin)
#pragma unroll
          for (int y = 0; y < NB; ++y)
#pragma unroll
            for (int cp = 0; cp < 2; ++cp)
              en[y][cp] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[y][s][cin][a],
                                                             lhat(va[s][a], cp, cin), en[y][cp],
                                                             0, 0, 0);
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) e[y][c][b] = en[y][c][b];
  };
  // power-of-two rescale of each pair (a block's four lanes), after every
  // kRescaleEvery-th site and at the same sites for every pair, so that a
  // pair's result does not depend on its position in the launch (the scale
  // is exact except for entries in the subnormal range)
  auto rescale = [&]() {
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      float lm = 0.f;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) lm = __builtin_elementwise_maximum(lm, fabsf(e[y][c][b]));
      unsigned m = __float_as_uint(lm);
      m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0xB1, 0xF, 0xF, false));
      m = max(m, (unsigned)__builtin_amdgcn_update_dpp(0, (int)m, 0x4E, 0xF, 0xF, false));
      const unsigned ex = m >> 23;
      const float sc = rescale_factor(ex);
      expo[y] += (int)ex - 126;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) e[y][c][b] *= sc;
    }
  };
  // whole groups of kRescaleEvery sites, each followed by the rescale, then
  // the remainder without it: the site body carries no VALU work (which
  // would not overlap the matrix-core instructions of the same SIMD)
  const int nfull = nq - nq % kRescaleEvery;
  for (int k0 = 0; k0 < nfull; k0 += kRescaleEvery) {
    for (int k = k0; k < k0 + kRescaleEvery; ++k) site(k);
    rescale();
  }
  for (int k = nfull; k < nq; ++k) site(k);

  // ---- epilogue: lane x = 0 of a block holds E[0][0] of its pair
  if (tid < kQkMaskWords) sm.mask[tid] = 0;
  double d2[NB];
#pragma unroll
  for (int y = 0; y < NB; ++y) d2[y] = 0.0;
  if (t.fuse) {
    // fused RBF: squared distances by direct difference, the tile's 16 row
    // and 16 column feature vectors staged through LDS in chunks; lane x of
    // a pair sums the features f = x mod 4 of each chunk
    const int64_t ti0 = (int64_t)ti * kTile, tj0 = (int64_t)tj * kTile;
    for (int f0 = 0; f0 < nq; f0 += kXChunk) {
      const int nf = min(kXChunk, nq - f0);
      __syncthreads();
      for (int el = tid; el < 32 * nf; el += kThr) {
        const int smp = el / nf, f = el - smp * nf;
        double v = 0.0;
        if (smp < 16) {
          const int64_t r = ti0 + smp;
          if (r < t.na) v = t.xr[r * t.ld_xr + f0 + f];
        } else {
          const int64_t c = tj0 + smp - 16;
          if (c < t.nb) v = t.xc[c * t.ld_xc + f0 + f];
        }
        sm.u.xs[smp * kXStride + f] = v;
      }
      __syncthreads();
      const double* xrow = sm.u.xs + (4 * wr + pp) * kXStride;
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const double* xcol = sm.u.xs + (16 + 4 * (wc0 + y) + qq) * kXStride;
        double acc = 0.0;
        for (int f = x; f < nf; f += 4) {
          const double df = xrow[f] - xcol[f];
          acc += df * df;
        }
        d2[y] += acc;
      }
    }
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      d2[y] += __shfl_xor(d2[y], 1, 64);
      d2[y] += __shfl_xor(d2[y], 2, 64);
    }
  }
  __syncthreads();  // mask words cleared
#pragma unroll
  for (int y = 0; y < NB; ++y) {
    const bool valid = x == 0 && i < t.na && j[y] < t.nb && (!t.symmetric || j[y] >= i);
    const double re = (double)e[y][0][0], im = (double)e[y][1][0];
    const double mag2 = re * re + im * im;
    const double lnk =
        mag2 > 0.0 ? log(mag2) + 2.0 * (double)expo[y] * 0.69314718055994530942 : -INFINITY;
    const double kq = mag2 > 0.0 ? exp(lnk) : 0.0;
    if (valid) {
      const int64_t jj = j[y];
      auto put = [&](double* ptr, int64_t ld, double v) {
        if (!ptr) return;
        ptr[i * ld + jj] = v;
        if (t.symmetric && jj != i) ptr[jj * ld + i] = v;
      };
      put(t.kq, t.ld_kq, kq);
      put(t.lnkq, t.ld_ln, lnk);
      if (t.fuse) {
        const double kc = exp(-t.gamma * d2[y]);
        const double wgt = t.w_rows ? t.w_rows[i] : t.w;
        put(t.kc, t.ld_kc, kc);
        put(t.k, t.ld_k, wgt * kq + (1.0 - wgt) * kc);
      }
      if (mask && lnk > ln_tau) {
        const int bit = (int)(i - (int64_t)ti * kTile) * kTile + (int)(jj - (int64_t)tj * kTile);
        atomicOr(&sm.mask[bit >> 5], 1u << (bit & 31));
      }
    }
  }
  __syncthreads();
  if (mask && tid < kQkMaskWords) mask[tile_id * kQkMaskWords + tid] = sm.mask[tid];
}

// Pair blocks per wave of the FP32 form: a 16 x 16 tile is 8 waves, up to
// two workgroups per CU, four waves per SIMD (the register budget of 128
// VGPRs). (HIP's second launch bound is the minimum number of waves per SIMD)
constexpr int kM4Blocks = 2;

__global__ __launch_bounds__(kThreads / kM4Blocks, 4) void sweep_m4_kernel(QkTaskTable tt,
                                                                            uint32_t* flags,
                                                                            double ln_tau) {
  constexpr int NB = kM4Blocks;
  __shared__ M4Smem sm;
  for (int64_t rnd = 0; rnd * gridDim.x < tt.total_tiles; ++rnd) {
    const int64_t q = qk_tile_of(rnd, blockIdx.x, gridDim.x);
    if (q >= tt.total_tiles) break;  // only the last round is partial
    int k = 0;
    while (k + 1 < tt.n_tasks && tt.t[k + 1].tile_begin <= q) ++k;
    const QkTask& t = tt.t[k];
    int ti, tj;
    qk_tile_coords(t, q - t.tile_begin, ti, tj);
    if (t.T == 4) run_tile_m4<NB, 4>(t, ti, tj, sm, flags, q, ln_tau);
    else if (t.T == 2) run_tile_m4<NB, 2>(t, ti, tj, sm, flags, q, ln_tau);
    else run_tile_m4<NB, 1>(t, ti, tj, sm, flags, q, ln_tau);
    __syncthreads();
  }
}

}  // namespace

bool qk_mfma_supports(qk_precision p, int T) {
  const bool form = p == QK_PREC_FP32_MFMA || p == QK_PREC_BF16X2 || p == QK_PREC_BF16X3;
  return form && (T == 1 || T == 2 || T == 4);
}

int qk_mfma_tile(qk_precision) { return kTile; }

hipError_t qk_launch_sweep_mfma(const QkTaskTable& tt, qk_precision p, int cus, int wg_per_cu,
                                uint32_t* flags, double ln_tau, hipStream_t s) {
  if (tt.total_tiles == 0) return hipSuccess;
  const int grid = (int)(tt.total_tiles < (int64_t)cus ? tt.total_tiles : cus);
  switch (p) {
    case QK_PREC_FP32_MFMA: {
      const int64_t g4 = (int64_t)cus * (wg_per_cu >= 2 ? 2 : 1);
      hipLaunchKernelGGL(sweep_m4_kernel, dim3((int)(tt.total_tiles < g4 ? tt.total_tiles : g4)),
                         dim3(kThreads / kM4Blocks), 0, s, tt, flags, ln_tau);
      break;
    }
    case QK_PREC_BF16X2:
      hipLaunchKernelGGL(sweep_mfma_kernel<kBF16x2>, dim3(grid), dim3(kThreads), 0, s, tt, flags, ln_tau);
      break;
    case QK_PREC_BF16X3:
      hipLaunchKernelGGL(sweep_mfma_kernel<kBF16x3>, dim3(grid), dim3(kThreads), 0, s, tt, flags, ln_tau);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
