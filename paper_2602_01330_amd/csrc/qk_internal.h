// Internal declarations shared by the host side of libqk and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/qk.h"

// Device status word bits latched by the build kernel.
enum : int32_t {
  QK_FLAG_NONFINITE = 1,   // a feature was NaN or Inf
  QK_FLAG_CHI_OVER = 2,    // a kept bond exceeded the bound chi_ws
  QK_FLAG_NOCONV = 4       // a Jacobi SVD hit its sweep limit
};

// Packed FP32 complex element z = x + i y, stored as (-y, x, y): bytes 4..11
// hold z = (x, y) and bytes 0..7 hold i z = (-y, x), so a matrix-core lane
// takes either realified operand form with one 8-byte load and no arithmetic.
constexpr int kQkPackFloats = 3;

struct qk_mps_batch {
  int device = 0;
  int64_t n = 0;          // samples
  int32_t nq = 0;         // qubits (sites)
  int32_t n_layers = 0;
  int32_t chi_ws = 1;     // bond bound used by the build
  int32_t T = 1;          // padded bond dimension of the packed tensors
  double2* t64 = nullptr; // [nq][n][2][T][T] complex FP64
  float* t32 = nullptr;   // [nq][n][2][T][T] complex FP32, kQkPackFloats floats each
  int32_t* chi = nullptr; // [n][nq+1] realized bond dimensions
  int32_t* status = nullptr;  // [0] flag bits, [1] max realized chi
  double* disc = nullptr;     // [n] discarded weight per sample (0 when nothing is cut)
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  int64_t bytes = 0;
};

// Shared host helpers (qk_api.cpp).
#include <string>
qk_status qk_fail(qk_status s, const std::string& msg);
// Frees a batch without draining the device; the caller guarantees that no
// enqueued work still reads it. Memory returns to the pool in stream order.
void qk_mps_release_nosync(qk_mps_batch* b, hipStream_t s);

// Jacobi sweeps a two-site SVD of the build may take before it latches
// QK_FLAG_NOCONV (default), and the largest limit the setter accepts.
constexpr int kQkDefaultSvdSweeps = 60;
constexpr int kQkMaxSvdSweeps = 1000;

// Text of the build's status flag bits ("" when none is set).
std::string qk_flag_text(int32_t flags);
// Jacobi sweep limit of the build's two-site SVDs (qk_set_svd_sweep_limit).
int qk_svd_sweep_limit();

// Kernel launchers (build.hip). A two-site SVD that has not converged after
// max_sweeps Jacobi sweeps latches QK_FLAG_NOCONV.
hipError_t qk_launch_build(const double* x, int64_t ld_x, int64_t n, int nq,
                           int n_layers, int chi_max, int entangle,
                           double cutoff, int chi_ws, int T, double2* t64,
                           int32_t* chi, int32_t* status, double* disc, int max_sweeps,
                           hipStream_t s);
// Several feature matrices of one circuit built in one launch (bond bound
// up to 4): one part per batch.
struct QkBuildPart {
  const double* x;
  int64_t ld_x;
  int64_t n;
  double2* t64;
  int32_t* chi;
  int32_t* status;
  double* disc;  // per-sample discarded weight (may be NULL)
};
constexpr int QK_MAX_BUILD_PARTS = 8;
hipError_t qk_launch_build_many(const QkBuildPart* parts, int n_parts, int nq, int n_layers,
                                int chi_max, int entangle, double cutoff, int chi_ws, int T,
                                int max_sweeps, hipStream_t s);
hipError_t qk_launch_pack32(const double2* t64, float* t32, int64_t count,
                            hipStream_t s);

// One Gram block of a (possibly multi-task) sweep launch (sweep kernels).
struct QkTask {
  const void* ta;        // row tensors (double2* or float2*), [nq][na][2][T][T]
  const void* tb;        // column tensors
  const void* ta64;      // FP64 forms, used by the refinement pass (may be null)
  const void* tb64;
  int64_t na, nb;        // sample counts
  int32_t nq, T;
  int32_t symmetric;
  int32_t tiles_c;       // column tiles
  int64_t tile_begin;    // first global tile index of this task
  int64_t n_tiles;
  double* kq; int64_t ld_kq;
  double* lnkq; int64_t ld_ln;
  const double* xr; int64_t ld_xr;
  const double* xc; int64_t ld_xc;
  double gamma, w;
  const double* w_rows;  // per-row mixing weight (overrides w) or null
  double* kc; int64_t ld_kc;
  double* k; int64_t ld_k;
  int32_t fuse;
  int32_t band;          // tile rows per band of the tile order (0: kQkBand)
};

constexpr int QK_MAX_TASKS = 16;

// Tile processed by persistent workgroup `wg` (of `grid`) in round `round`.
// Workgroups are dispatched round-robin over the 8 XCDs (wg % 8), each with
// its own L2; when the grid is a multiple of 8, XCD x takes the contiguous
// slice [x * grid/8, (x+1) * grid/8) of each round's tiles, so the tiles an
// XCD runs together share their row samples (and different XCDs work on
// different column samples). A bijection of [0, grid) in every round.
__device__ inline int64_t qk_tile_of(int64_t round, int wg, int grid) {
  const int64_t base = round * (int64_t)grid;
  if (grid % 8) return base + wg;
  return base + (int64_t)(wg % 8) * (grid / 8) + wg / 8;
}

// Task-local tile index -> (tile row, tile column). Tiles are enumerated in
// bands of B = t.band tile rows (kQkBand when 0): within a band column by
// column, within a column row by row (symmetric tasks: upper triangle incl.
// the diagonal). A run of consecutive tiles -- what one XCD holds at a time
// under qk_tile_of -- then covers B row blocks x (run / B) column blocks,
// whose sample blocks the XCD's L2 serves to all of its workgroups; B trades
// row-block reuse against column-block reuse and is a tuning parameter.
// Shared by every sweep kernel, so a refinement pass finds the tiles its
// mask words were written for (both passes read the same task table).
constexpr int kQkBand = 4;

__device__ inline void qk_tile_coords(const QkTask& t, int64_t lt, int& ti, int& tj) {
  const int64_t B = t.band > 0 ? t.band : kQkBand;
  const int64_t nc = t.tiles_c;
  if (!t.symmetric) {
    const int64_t nr = t.n_tiles / nc;
    const int64_t band = lt / (B * nc);
    const int64_t l = lt - band * (B * nc);
    const int64_t r0 = band * B;
    const int64_t h = nr - r0 < B ? nr - r0 : B;
    ti = (int)(r0 + l % h);
    tj = (int)(l / h);
    return;
  }
  // full bands before band R hold C(R) = B n R + B R / 2 - B^2 R^2 / 2 tiles
  // (B (B - 1) / 2 in the band's partial first columns, B per later column)
  const int64_t n = nc;
  const int64_t nb = (n + B - 1) / B;
  auto before = [&](int64_t r) { return B * n * r + (B * r - B * B * r * r) / 2; };
  const double bq = (double)B * (double)n + 0.5 * (double)B;
  const double disc = bq * bq - 2.0 * (double)(B * B) * (double)lt;
  int64_t R = (int64_t)((bq - sqrt(disc > 0.0 ? disc : 0.0)) / (double)(B * B));
  if (R < 0) R = 0;
  if (R > nb - 1) R = nb - 1;
  while (R > 0 && before(R) > lt) --R;
  while (R + 1 < nb && before(R + 1) <= lt) ++R;
  const int64_t l = lt - before(R);
  const int64_t r0 = B * R;
  const int64_t h = n - r0 < B ? n - r0 : B;
  const int64_t part = h * (h - 1) / 2;  // the band's first h-1 columns are partial
  if (l < part) {
    int64_t c = 0;
    while ((c + 1) * (c + 2) / 2 <= l) ++c;
    ti = (int)(r0 + (l - c * (c + 1) / 2));
    tj = (int)(r0 + c);
  } else {
    const int64_t l2 = l - part;
    ti = (int)(r0 + l2 % h);
    tj = (int)(r0 + h - 1 + l2 / h);
  }
}

struct QkTaskTable {
  QkTask t[QK_MAX_TASKS];
  int32_t n_tasks;
  int64_t total_tiles;
};

// Sweep launchers (sweep_valu.hip / sweep_mfma.hip). Every sweep kernel uses
// 16 x 16 pair tiles with the same tile numbering. A reduced-precision pass
// writes, per tile, a 256-bit mask (8 words) of the pairs whose K_q exceeds
// the refinement threshold (bit (i % 16) * 16 + (j % 16)); the FP64 pass then
// visits only tiles with a set bit and writes only those pairs.
// Complex-FP64 sweep for padded bond dimensions 8..64 (sweep_big.hip): one
// launch per bond dimension, every pair of the given tasks.
bool qk_sweep_big_supports(int T);
hipError_t qk_launch_sweep_big(const QkTask* tasks, int n_tasks, int cus, hipStream_t s);
// The same FP64 sweep over only the listed pairs: list[0 .. *count) holds
// global pair numbers of the table made from `tasks` (whose ta/tb must be
// the FP64 tensors); the count is read on the device.
hipError_t qk_launch_sweep_big_list(const QkTask* tasks, int n_tasks, const int64_t* list,
                                    const int32_t* count, int cus, hipStream_t s);
// Complex-FP32 matrix-core sweep for the same bond dimensions (sweep_wide.hip):
// packed FP32 tensors, one launch per bond dimension, every pair. With
// `refine`, pairs whose ln K_q >= ln_tau are then recomputed by the FP64
// list sweep from the tasks' ta64/tb64. The list (pairs + 1 int64 words) is
// a stream-ordered allocation, or list_scratch when that is not NULL.
bool qk_sweep_wide_supports(int T);
hipError_t qk_launch_sweep_wide(const QkTask* tasks, int n_tasks, int cus, double ln_tau,
                                bool refine, int64_t* list_scratch, hipStream_t s);

constexpr int kQkMaskWords = 8;
hipError_t qk_launch_sweep_fp64(const QkTaskTable& tt, int grid, const uint32_t* mask_in,
                                hipStream_t s);
// Zero-fill of n int32 words by a kernel (no memset node in captured graphs).
hipError_t qk_launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
// FP64 recomputation of exactly the tiles whose mask words mark a pair:
// lists them in `list` (total_tiles entries; *count must be 0 on entry),
// then sweeps the listed tiles spread over `grid` workgroups.
hipError_t qk_launch_refine_fp64(const QkTaskTable& tt, int grid, const uint32_t* mask,
                                 int32_t* list, int32_t* count, hipStream_t s);
hipError_t qk_launch_sweep_fp32(const QkTaskTable& tt, int grid, uint32_t* mask_out,
                                double ln_tau, hipStream_t s);
int qk_sweep_valu_tile();

hipError_t qk_launch_rbf(const double* x, int64_t m, int64_t ld_x,
                         const double* y, int64_t n, int64_t ld_y, int d,
                         double gamma, double* kc, int64_t ld_kc, hipStream_t s);
hipError_t qk_launch_mix(const double* kq, int64_t ld_kq, const double* kc,
                         int64_t ld_kc, int64_t m, int64_t n, double w,
                         double* k, int64_t ld_k, hipStream_t s);
hipError_t qk_launch_svm_decision(const double* k, int64_t m, int64_t n, int64_t ld_k,
                                  const double* coef, double b, double* f, hipStream_t s);
// Path-sum evaluation for one- and two-layer circuits (pathsum.hip): the
// per-sample tables (site-major, n x d entries of (q, p)), then one pair per
// lane over 16 x 16 tiles, the upper triangle only when symmetric.
hipError_t qk_launch_pathsum_table(const double* x, int64_t n, int64_t ld_x, int d, int n_layers,
                                   int entangle, double4* tab, hipStream_t s);
hipError_t qk_launch_pathsum(const double4* tr, int64_t m, const double4* tc, int64_t n, int d,
                             int n_layers, int symmetric, double* kq, int64_t ld_kq,
                             double* lnkq, int64_t ld_ln, const qk_fuse_desc* fuse,
                             hipStream_t s);
// SVM training by SMO, one workgroup per binary problem p: samples
// idx[off[p] .. off[p+1]) (global rows of the symmetric kernel k), labels
// y = +1/-1 alongside; alpha / grad / diag are scratch of the same length;
// writes coef row p (n_all entries, a_t y_t at the problem's samples), b[p]
// and the step count iters[p] (svm.hip).
hipError_t qk_launch_svm_smo(const double* k, int64_t ld_k, const int32_t* idx, const double* y,
                             const int64_t* off, int n_problems, double C, double eps,
                             int64_t max_iter, double* alpha, double* grad, double* diag,
                             double* coef, int64_t ld_coef, int64_t n_all, double* b,
                             int64_t* iters, hipStream_t s);
// One-against-one decision values (m x n_problems, optional) and voted
// labels (optional) of m kernel rows (svm.hip).
hipError_t qk_launch_svm_predict(const double* k, int64_t m, int64_t n, int64_t ld_k,
                                 const double* coef, int64_t ld_coef, const double* b,
                                 int n_classes, double* f, int64_t ld_f, int32_t* labels,
                                 hipStream_t s);
