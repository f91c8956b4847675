// Host side of the libqk C ABI: argument checks, batch ownership, task
// tables and launch configuration. Every step of the computation runs in the
// HIP kernels of this library; nothing here touches sample data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qk_internal.h"
#include "qk_tune.h"

namespace {

thread_local std::string g_last_error;

qk_status fail(qk_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

void free_batch_memory(qk_mps_batch* b, hipStream_t s) {
  if (b->t64) (void)hipFreeAsync(b->t64, s);
  if (b->t32) (void)hipFreeAsync(b->t32, s);
  if (b->chi) (void)hipFreeAsync(b->chi, s);
  if (b->status) (void)hipFreeAsync(b->status, s);
  if (b->disc) (void)hipFreeAsync(b->disc, s);
  b->disc = nullptr;
  b->t64 = nullptr;
  b->t32 = nullptr;
  b->chi = nullptr;
  b->status = nullptr;
}

qk_status hip_fail(hipError_t e, const char* what) {
  return fail(QK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define QK_HIP(call, what)                      \
  do {                                          \
    hipError_t e__ = (call);                    \
    if (e__ != hipSuccess) return hip_fail(e__, what); \
  } while (0)

int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

// Device scratch of qk_overlap_gram_noalloc: refinement masks of the tile
// sweeps and pair lists of the large-bond sweep. Every GPU the library runs
// on holds its own copy until the process ends. In host code the name is a
// host-side stand-in, so launches use the address that hipGetSymbolAddress
// reports for each device.
constexpr int64_t kNoAllocScratchBytes = QK_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchAddr {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchAddr g_scratch_addr[kMaxDevices];

// The current device's copy of `scratch` (looked up once per device, with
// that device current).
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  ScratchAddr& a = g_scratch_addr[dev];
  std::call_once(a.once, [&a] {
    a.err = hipGetSymbolAddress(&a.ptr, HIP_SYMBOL(scratch));
    if (a.err == hipSuccess && !a.ptr) a.err = hipErrorInvalidSymbol;
  });
  *out = a.ptr;
  return a.err;
}

qk_status check_desc(const qk_circuit_desc* c) {
  if (!c) return fail(QK_ERR_INVALID_ARG, "circuit descriptor is NULL");
  if (c->n_qubits < 1) return fail(QK_ERR_INVALID_ARG, "n_qubits must be >= 1");
  if (c->n_layers < 1) return fail(QK_ERR_INVALID_ARG, "n_layers must be >= 1");
  if (c->chi_max < 1) return fail(QK_ERR_INVALID_ARG, "chi_max must be >= 1");
  if (c->entangle < 0)
    return fail(QK_ERR_INVALID_ARG, "entangle must be 0 (none), 1 (chain) or a block size >= 2");
  if (!(c->cutoff_rel >= 0.0) || !std::isfinite(c->cutoff_rel))
    return fail(QK_ERR_INVALID_ARG, "cutoff_rel must be finite and >= 0");
  return QK_OK;
}

// Entangler block size the kernels take: 0 (none), the qubit count for the
// open chain (entangle = 1), else the block size.
int ent_block(const qk_circuit_desc* c) {
  if (!c->entangle) return 0;
  return c->entangle == 1 ? std::max(c->n_qubits, 1) : c->entangle;
}

// Exact bond bound of this circuit family: each layer's RZZ chain multiplies
// the Schmidt rank across a cut by at most 2, no cut of n qubits has rank
// above 2^floor(n/2), and with entangler blocks of B qubits no cut inside a
// block has rank above 2^floor(B/2) (and a cut between blocks has rank 1).
int chi_bound(const qk_circuit_desc* c) {
  const int blk = std::min(ent_block(c), c->n_qubits);
  if (blk < 2 || c->n_qubits == 1) return 1;
  const int e = std::min(c->n_layers, blk / 2);
  int64_t b = 1;
  for (int l = 0; l < e && b < c->chi_max; ++l) b *= 2;
  return (int)std::min<int64_t>(b, c->chi_max);
}

qk_status alloc_batch(const qk_circuit_desc* c, int64_t n, int T, uint32_t store,
                      hipStream_t s, qk_mps_batch** out) {
  auto* b = new qk_mps_batch();
  (void)hipGetDevice(&b->device);
  b->n = n;
  b->nq = c->n_qubits;
  b->n_layers = c->n_layers;
  b->T = T;
  b->stream = s;
  const int64_t elems = (int64_t)c->n_qubits * n * 2 * T * T;
  auto cleanup = [&](qk_status st, const char* what) {
    free_batch_memory(b, s);
    delete b;
    return fail(st, what);
  };
  // stream-ordered allocations: no device-wide synchronisation on alloc/free.
  // The FP64 form is the build's workspace, so it is always allocated.
  if (hipMallocAsync((void**)&b->t64, std::max<int64_t>(elems, 1) * sizeof(double2), s) != hipSuccess)
    return cleanup(QK_ERR_OUT_OF_MEMORY, "device allocation of FP64 site tensors failed");
  if ((store & QK_STORE_FP32) &&
      hipMallocAsync((void**)&b->t32, std::max<int64_t>(elems, 1) * kQkPackFloats * sizeof(float), s) != hipSuccess)
    return cleanup(QK_ERR_OUT_OF_MEMORY, "device allocation of FP32 site tensors failed");
  if (hipMallocAsync((void**)&b->chi, std::max<int64_t>(n * (c->n_qubits + 1), 1) * sizeof(int32_t), s) != hipSuccess)
    return cleanup(QK_ERR_OUT_OF_MEMORY, "device allocation of the bond table failed");
  if (hipMallocAsync((void**)&b->status, 2 * sizeof(int32_t), s) != hipSuccess)
    return cleanup(QK_ERR_OUT_OF_MEMORY, "device allocation of the status word failed");
  if (hipMemsetAsync(b->status, 0, 2 * sizeof(int32_t), s) != hipSuccess)
    return cleanup(QK_ERR_HIP, "status reset failed");
  // discarded weight per sample: written by the build, zero for imports
  if (hipMallocAsync((void**)&b->disc, std::max<int64_t>(n, 1) * sizeof(double), s) != hipSuccess)
    return cleanup(QK_ERR_OUT_OF_MEMORY, "device allocation of the discarded weights failed");
  if (hipMemsetAsync(b->disc, 0, std::max<int64_t>(n, 1) * sizeof(double), s) != hipSuccess)
    return cleanup(QK_ERR_HIP, "discarded-weight reset failed");
  if (hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess)
    return cleanup(QK_ERR_HIP, "event creation failed");
  b->bytes = elems * (int64_t)sizeof(double2) +
             ((store & QK_STORE_FP32) ? elems * (int64_t)(kQkPackFloats * sizeof(float)) : 0) +
             n * (c->n_qubits + 1) * (int64_t)sizeof(int32_t);
  *out = b;
  return QK_OK;
}

// Drops the FP64 form after packing when the caller did not ask to keep it.
qk_status finish_batch(qk_mps_batch* b, uint32_t store) {
  const int64_t elems = (int64_t)b->nq * b->n * 2 * b->T * b->T;
  if (b->t32) QK_HIP(qk_launch_pack32(b->t64, b->t32, elems, b->stream), "pack to FP32");
  QK_HIP(hipEventRecord(b->ready, b->stream), "event record");
  if (!(store & QK_STORE_FP64)) {
    QK_HIP(hipFreeAsync(b->t64, b->stream), "free of the FP64 workspace");
    b->t64 = nullptr;
    b->bytes -= elems * (int64_t)sizeof(double2);
  }
  return QK_OK;
}

qk_status fill_task(QkTask& t, const qk_mps_batch* rows, const qk_mps_batch* cols,
                    int32_t symmetric, bool fp64, bool refine, double* kq, int64_t ld_kq,
                    double* lnkq, int64_t ld_ln, const qk_fuse_desc* fuse, int tile) {
  if (!rows || !cols) return fail(QK_ERR_INVALID_ARG, "batch is NULL");
  if (rows->nq != cols->nq) return fail(QK_ERR_INVALID_ARG, "qubit counts differ");
  if (rows->T != cols->T)
    return fail(QK_ERR_UNSUPPORTED, "row and column batches have different chi_pad");
  if (symmetric && rows != cols)
    return fail(QK_ERR_INVALID_ARG, "symmetric mode needs rows == cols");
  const bool work = rows->n > 0 && cols->n > 0;
  if (work && !kq && !lnkq && !(fuse && (fuse->kc_dev || fuse->k_dev)))
    return fail(QK_ERR_INVALID_ARG, "no output requested");
  if (kq && ld_kq < cols->n) return fail(QK_ERR_INVALID_ARG, "ld_kq < number of columns");
  if (lnkq && ld_ln < cols->n) return fail(QK_ERR_INVALID_ARG, "ld_ln < number of columns");
  if (fp64 && (!rows->t64 || !cols->t64))
    return fail(QK_ERR_INVALID_ARG, "FP64 sweep needs batches built with QK_STORE_FP64");
  if (!fp64 && (!rows->t32 || !cols->t32))
    return fail(QK_ERR_INVALID_ARG, "this sweep needs batches built with QK_STORE_FP32");
  if (!fp64 && refine && (!rows->t64 || !cols->t64))
    return fail(QK_ERR_INVALID_ARG,
                "FP64 refinement of large entries needs batches built with QK_STORE_FP64 "
                "(or disable it with qk_set_refine_threshold)");
  memset(&t, 0, sizeof(t));
  t.ta = fp64 ? (const void*)rows->t64 : (const void*)rows->t32;
  t.tb = fp64 ? (const void*)cols->t64 : (const void*)cols->t32;
  t.ta64 = rows->t64;
  t.tb64 = cols->t64;
  t.na = rows->n;
  t.nb = cols->n;
  t.nq = rows->nq;
  t.T = rows->T;
  t.symmetric = symmetric ? 1 : 0;
  const int64_t tr = (rows->n + tile - 1) / tile, tc = (cols->n + tile - 1) / tile;
  t.tiles_c = (int32_t)tc;
  t.n_tiles = symmetric ? tr * (tr + 1) / 2 : tr * tc;
  t.kq = kq;
  t.ld_kq = ld_kq;
  t.lnkq = lnkq;
  t.ld_ln = ld_ln;
  if (fuse && work) {
    if (!fuse->x_rows_dev || !fuse->x_cols_dev)
      return fail(QK_ERR_INVALID_ARG, "fusion needs the feature matrices");
    if (fuse->ld_xr < rows->nq || fuse->ld_xc < cols->nq)
      return fail(QK_ERR_INVALID_ARG, "feature leading dimension < qubit count");
    if (!(fuse->w >= 0.0 && fuse->w <= 1.0)) return fail(QK_ERR_INVALID_ARG, "w must be in [0, 1]");
    if (!(fuse->gamma >= 0.0) || !std::isfinite(fuse->gamma))
      return fail(QK_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    if (fuse->kc_dev && fuse->ld_kc < cols->n) return fail(QK_ERR_INVALID_ARG, "ld_kc too small");
    if (fuse->k_dev && fuse->ld_k < cols->n) return fail(QK_ERR_INVALID_ARG, "ld_k too small");
    t.fuse = 1;
    t.xr = fuse->x_rows_dev;
    t.ld_xr = fuse->ld_xr;
    t.xc = fuse->x_cols_dev;
    t.ld_xc = fuse->ld_xc;
    t.gamma = fuse->gamma;
    t.w = fuse->w;
    t.w_rows = fuse->w_rows_dev;
    t.kc = fuse->kc_dev;
    t.ld_kc = fuse->ld_kc;
    t.k = fuse->k_dev;
    t.ld_k = fuse->ld_k;
  }
  return QK_OK;
}

bool supported_T(qk_precision p, int T) {
  switch (p) {
    case QK_PREC_FP64:
      return T == 1 || T == 2 || T == 4 || qk_sweep_big_supports(T);
    case QK_PREC_FP32:
      return T == 1 || T == 2 || T == 4;
    case QK_PREC_FP32_MFMA:
      return qk_mfma_supports(p, T) || qk_sweep_wide_supports(T);
    default:
      return qk_mfma_supports(p, T);
  }
}

// Refinement thresholds on K_q per form (<= 0 disables refinement).
double g_refine_tau[6] = {0.0, 1e-2, 1e-3, 1e-2, 0.0, 1e-2};
std::mutex g_refine_mu;

double refine_tau(qk_precision p) {
  std::lock_guard<std::mutex> lk(g_refine_mu);
  return (p >= 0 && p < 6) ? g_refine_tau[p] : 0.0;
}

// Optional launch timing (HIP events on the launch stream).
struct LaunchTiming {
  std::mutex mu;
  bool enabled = false, recorded = false, refined = false;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
} g_timing;

void timing_mark(int which, hipStream_t s) {
  if (g_timing.enabled) (void)hipEventRecord(g_timing.ev[which], s);
}

// Caller-provided device scratch (the allocation-free entry point): the
// refinement masks and lists then live there instead of in stream-ordered
// allocations. Launches of one call run in stream order, so they reuse it.
struct Scratch {
  void* ptr = nullptr;
  int64_t bytes = 0;
};

qk_status run_tasks(std::vector<QkTask>& tasks_in, qk_precision prec, double tau, hipStream_t s,
                    int64_t max_tiles = -1, const Scratch* scratch = nullptr) {
  // tasks with bonds above 4 go to the per-pair kernels (one workgroup per
  // pair: complex FP64 on VALU, or complex FP32 on the matrix cores); the
  // tile kernels take the others
  std::vector<QkTask> tasks, big;
  for (const QkTask& t : tasks_in) (t.T > 4 ? big : tasks).push_back(t);
  // longest-processing-time order: per-tile cost ~ nq * T^3
  std::stable_sort(tasks.begin(), tasks.end(), [](const QkTask& a, const QkTask& b) {
    return (double)a.nq * a.T * a.T * a.T > (double)b.nq * b.T * b.T * b.T;
  });
  // launch shape: the tuning entry of the dominant (first) task when it was
  // tuned for this form, else the defaults; one launch has one shape, which
  // decides only the order and placement of tiles, never a pair's arithmetic
  QkTuneEntry te;
  const bool tuned =
      !tasks.empty() && qk_tune_lookup(tasks[0].T, tasks[0].nq, &te) && te.form == prec;
  const int band = tuned ? te.band : kQkBand;
  QkTaskTable tt;
  memset(&tt, 0, sizeof(tt));
  int64_t acc = 0;
  for (size_t k = 0; k < tasks.size(); ++k) {
    tasks[k].tile_begin = acc;
    tasks[k].band = band;
    acc += tasks[k].n_tiles;
    tt.t[k] = tasks[k];
  }
  tt.n_tasks = (int32_t)tasks.size();
  if (max_tiles >= 0 && acc > max_tiles) acc = max_tiles;  // autotuning slice
  tt.total_tiles = acc;
  std::lock_guard<std::mutex> tlk(g_timing.mu);
  g_timing.recorded = false;  // set once this call's events are all recorded
  g_timing.refined = false;
  if (acc == 0 && big.empty()) return QK_OK;
  if (scratch) {
    // everything this call keeps on the device, checked before any launch
    int64_t need = 0;
    if (prec != QK_PREC_FP64 && tau > 0.0 && acc > 0)
      need = (acc * (kQkMaskWords + 1) + 1) * (int64_t)sizeof(uint32_t);
    if (prec == QK_PREC_FP32_MFMA && tau > 0.0)
      for (int T : {64, 32, 16, 8}) {
        int64_t pairs = 0;
        for (const QkTask& t : big)
          if (t.T == T) pairs += t.symmetric ? t.na * (t.na + 1) / 2 : t.na * t.nb;
        if (pairs > 0) need = std::max<int64_t>(need, (pairs + 1) * (int64_t)sizeof(int64_t));
      }
    if (need > scratch->bytes)
      return fail(QK_ERR_INVALID_ARG,
                  "the call needs " + std::to_string(need) + " bytes of refinement scratch; the "
                  "allocation-free entry point has " + std::to_string(scratch->bytes));
  }
  // persistent workgroups per CU: from the tuning table, else per form
  const int grid64 = (int)std::min<int64_t>(
      acc, (int64_t)device_cus() * (tuned && prec == QK_PREC_FP64 ? te.wg_per_cu : 2));
  timing_mark(0, s);
  for (int T : {64, 32, 16, 8}) {  // one launch per bond dimension, largest first
    std::vector<QkTask> group;
    for (const QkTask& t : big)
      if (t.T == T) group.push_back(t);
    if (group.empty()) continue;
    if (prec == QK_PREC_FP64)
      QK_HIP(qk_launch_sweep_big(group.data(), (int)group.size(), device_cus(), s),
             "large-bond sweep launch");
    else if (prec == QK_PREC_FP32_MFMA)
      QK_HIP(qk_launch_sweep_wide(group.data(), (int)group.size(), device_cus(),
                                  tau > 0.0 ? std::log(tau) : 0.0, tau > 0.0,
                                  scratch ? static_cast<int64_t*>(scratch->ptr) : nullptr, s),
             "large-bond matrix-core sweep launch");
    else
      return fail(QK_ERR_UNSUPPORTED, "no sweep of this form for bonds above 4");
  }
  if (prec == QK_PREC_FP64 || acc == 0) {
    if (prec == QK_PREC_FP64 && acc > 0)
      QK_HIP(qk_launch_sweep_fp64(tt, grid64, nullptr, s), "sweep launch");
    timing_mark(1, s);
    timing_mark(2, s);
    g_timing.recorded = g_timing.enabled;
    return QK_OK;
  }
  // the reduced-precision sweeps address one site's packed sample array with
  // 32-bit byte offsets
  for (const QkTask& t : tasks) {
    const int64_t slot_bytes = (int64_t)2 * t.T * t.T * kQkPackFloats * 4;
    if (std::max(t.na, t.nb) * slot_bytes + 4096 > (int64_t)UINT32_MAX)
      return fail(QK_ERR_UNSUPPORTED, "batch too large for a 32-bit packed site array");
  }
  const bool refine = tau > 0.0;
  // refinement scratch: mask words per tile, then the list of marked tiles
  // and its length
  uint32_t* flags = nullptr;
  int32_t* marked = nullptr;
  int32_t* n_marked = nullptr;
  if (refine) {
    if (scratch)
      flags = static_cast<uint32_t*>(scratch->ptr);
    else
      QK_HIP(hipMallocAsync((void**)&flags, (acc * (kQkMaskWords + 1) + 1) * sizeof(uint32_t), s),
             "refinement mask allocation");
    marked = reinterpret_cast<int32_t*>(flags + acc * kQkMaskWords);
    n_marked = marked + acc;
    QK_HIP(qk_launch_zero_i32(n_marked, 1, s), "refinement counter reset");
  }
  const double ln_tau = refine ? std::log(tau) : 0.0;
  hipError_t e;
  if (prec == QK_PREC_FP32) {
    int grid = (int)std::min<int64_t>(
        acc, (int64_t)device_cus() * (tuned ? te.wg_per_cu : 3));
    e = qk_launch_sweep_fp32(tt, grid, flags, ln_tau, s);
  } else {
    e = qk_launch_sweep_mfma(tt, prec, device_cus(), tuned ? te.wg_per_cu : 2, flags, ln_tau, s);
  }
  timing_mark(1, s);
  if (e == hipSuccess && refine) {
    g_timing.refined = true;
    // FP64 pass over the flagged tiles only, same tile numbering
    QkTaskTable t64 = tt;
    for (int k = 0; k < t64.n_tasks; ++k) {
      t64.t[k].ta = t64.t[k].ta64;
      t64.t[k].tb = t64.t[k].tb64;
    }
    e = qk_launch_refine_fp64(t64, grid64, flags, marked, n_marked, s);
  }
  timing_mark(2, s);
  if (refine && !scratch) (void)hipFreeAsync(flags, s);
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  g_timing.recorded = g_timing.enabled;
  return QK_OK;
}

int tile_for(qk_precision p) {
  return (p == QK_PREC_FP64 || p == QK_PREC_FP32) ? qk_sweep_valu_tile() : qk_mfma_tile(p);
}

}  // namespace

qk_status qk_fail(qk_status s, const std::string& msg) { return fail(s, msg); }

std::string qk_flag_text(int32_t flags) {
  if (!flags) return "";
  std::string m = "build latched:";
  if (flags & QK_FLAG_NONFINITE) m += " non-finite feature;";
  if (flags & QK_FLAG_CHI_OVER) m += " bond above the padded bound;";
  if (flags & QK_FLAG_NOCONV) m += " Jacobi SVD sweep limit reached;";
  return m;
}

namespace {
std::atomic<int> g_svd_sweeps{kQkDefaultSvdSweeps};
}  // namespace

int qk_svd_sweep_limit() { return g_svd_sweeps.load(std::memory_order_relaxed); }

void qk_mps_release_nosync(qk_mps_batch* b, hipStream_t s) {
  if (!b) return;
  free_batch_memory(b, s);
  if (b->ready) (void)hipEventDestroy(b->ready);
  delete b;
}

extern "C" {

qk_status qk_set_launch_timing(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (enable && !g_timing.ev[0]) {
    for (auto& e : g_timing.ev) QK_HIP(hipEventCreate(&e), "event creation");
  }
  g_timing.enabled = enable != 0;
  g_timing.recorded = false;
  return QK_OK;
}

qk_status qk_last_launch_ms(float* sweep_ms, float* refine_ms) {
  if (!sweep_ms || !refine_ms) return fail(QK_ERR_INVALID_ARG, "null output");
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (!g_timing.enabled || !g_timing.recorded)
    return fail(QK_ERR_INVALID_ARG, "launch timing is off or no timed call was made");
  QK_HIP(hipEventSynchronize(g_timing.ev[2]), "event wait");
  float a = 0.f, b = 0.f;
  QK_HIP(hipEventElapsedTime(&a, g_timing.ev[0], g_timing.ev[1]), "elapsed time");
  if (g_timing.refined) QK_HIP(hipEventElapsedTime(&b, g_timing.ev[1], g_timing.ev[2]), "elapsed time");
  *sweep_ms = a;
  *refine_ms = b;
  return QK_OK;
}

const char* qk_status_string(qk_status s) {
  switch (s) {
    case QK_OK: return "ok";
    case QK_ERR_INVALID_ARG: return "invalid argument";
    case QK_ERR_OUT_OF_MEMORY: return "out of device memory";
    case QK_ERR_HIP: return "HIP runtime error";
    case QK_ERR_UNSUPPORTED: return "unsupported configuration";
    case QK_ERR_BUSY: return "busy";
    case QK_ERR_CANCELLED: return "cancelled";
    case QK_ERR_DEVICE: return "device-side check failed";
    case QK_ERR_NOT_FOUND: return "not found";
  }
  return "unknown status";
}

const char* qk_last_error(void) { return g_last_error.c_str(); }

qk_status qk_mps_build(const qk_circuit_desc* c, const double* x_dev,
                       int64_t n_samples, int64_t ld_x, uint32_t store,
                       void* hip_stream, qk_mps_batch** out) {
  qk_status st = check_desc(c);
  if (st != QK_OK) return st;
  if (!out) return fail(QK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_samples < 0) return fail(QK_ERR_INVALID_ARG, "n_samples < 0");
  if (n_samples > 0 && !x_dev) return fail(QK_ERR_INVALID_ARG, "x_dev is NULL");
  if (ld_x < c->n_qubits) return fail(QK_ERR_INVALID_ARG, "ld_x < n_qubits");
  if (store == 0 || (store & ~(uint32_t)QK_STORE_ALL))
    return fail(QK_ERR_INVALID_ARG, "store must be a non-empty QK_STORE_* mask");
  const int ws = chi_bound(c);
  const int T = pow2_ceil(ws);
  if (T > 64) return fail(QK_ERR_UNSUPPORTED, "bond bound above 64 is not supported by the build");
  hipStream_t s = (hipStream_t)hip_stream;
  qk_mps_batch* b = nullptr;
  st = alloc_batch(c, n_samples, T, store, s, &b);
  if (st != QK_OK) return st;
  b->chi_ws = ws;
  hipError_t e = qk_launch_build(x_dev, ld_x, n_samples, c->n_qubits, c->n_layers,
                                 c->chi_max, ent_block(c), c->cutoff_rel, ws, T,
                                 b->t64, b->chi, b->status, b->disc, qk_svd_sweep_limit(), s);
  if (e != hipSuccess) {
    qk_mps_release(b);
    return hip_fail(e, "build launch");
  }
  st = finish_batch(b, store);
  if (st != QK_OK) {
    qk_mps_release(b);
    return st;
  }
  *out = b;
  return QK_OK;
}

qk_status qk_mps_build_many(const qk_circuit_desc* c, int32_t n_inputs,
                            const double* const* x_devs, const int64_t* n_samples,
                            const int64_t* ld_x, uint32_t store, void* hip_stream,
                            qk_mps_batch** out) {
  qk_status st = check_desc(c);
  if (st != QK_OK) return st;
  if (n_inputs < 1 || n_inputs > QK_MAX_BUILD_PARTS)
    return fail(QK_ERR_INVALID_ARG, "n_inputs must be in [1, 8]");
  if (!x_devs || !n_samples || !ld_x || !out) return fail(QK_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < n_inputs; ++k) out[k] = nullptr;
  for (int k = 0; k < n_inputs; ++k) {
    if (n_samples[k] < 0) return fail(QK_ERR_INVALID_ARG, "n_samples < 0");
    if (n_samples[k] > 0 && !x_devs[k]) return fail(QK_ERR_INVALID_ARG, "x_dev is NULL");
    if (ld_x[k] < c->n_qubits) return fail(QK_ERR_INVALID_ARG, "ld_x < n_qubits");
  }
  if (store == 0 || (store & ~(uint32_t)QK_STORE_ALL))
    return fail(QK_ERR_INVALID_ARG, "store must be a non-empty QK_STORE_* mask");
  const int ws = chi_bound(c);
  const int T = pow2_ceil(ws);
  if (T > 64) return fail(QK_ERR_UNSUPPORTED, "bond bound above 64 is not supported by the build");
  hipStream_t s = (hipStream_t)hip_stream;
  qk_mps_batch* b[QK_MAX_BUILD_PARTS] = {};
  QkBuildPart parts[QK_MAX_BUILD_PARTS];
  auto release_all = [&]() {
    for (int k = 0; k < n_inputs; ++k)
      if (b[k]) qk_mps_release(b[k]);
  };
  for (int k = 0; k < n_inputs; ++k) {
    st = alloc_batch(c, n_samples[k], T, store, s, &b[k]);
    if (st != QK_OK) {
      release_all();
      return st;
    }
    b[k]->chi_ws = ws;
    parts[k] = QkBuildPart{x_devs[k], ld_x[k], n_samples[k], b[k]->t64, b[k]->chi, b[k]->status,
                           b[k]->disc};
  }
  hipError_t e = qk_launch_build_many(parts, n_inputs, c->n_qubits, c->n_layers, c->chi_max,
                                      ent_block(c), c->cutoff_rel, ws, T, qk_svd_sweep_limit(), s);
  if (e != hipSuccess) {
    release_all();
    return hip_fail(e, "build launch");
  }
  for (int k = 0; k < n_inputs; ++k) {
    st = finish_batch(b[k], store);
    if (st != QK_OK) {
      release_all();
      return st;
    }
  }
  for (int k = 0; k < n_inputs; ++k) out[k] = b[k];
  return QK_OK;
}

qk_status qk_mps_import(const qk_circuit_desc* c, int64_t n_samples,
                        int32_t chi_pad, const int32_t* chi_host,
                        const double* tensors_host, uint32_t store,
                        void* hip_stream, qk_mps_batch** out) {
  qk_status st = check_desc(c);
  if (st != QK_OK) return st;
  if (!out) return fail(QK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_samples < 0) return fail(QK_ERR_INVALID_ARG, "n_samples < 0");
  if (chi_pad < 1 || chi_pad > 64 || (chi_pad & (chi_pad - 1)))
    return fail(QK_ERR_INVALID_ARG, "chi_pad must be a power of two <= 64");
  if (n_samples > 0 && (!chi_host || !tensors_host))
    return fail(QK_ERR_INVALID_ARG, "host arrays are NULL");
  if (store == 0 || (store & ~(uint32_t)QK_STORE_ALL))
    return fail(QK_ERR_INVALID_ARG, "store must be a non-empty QK_STORE_* mask");
  int mx = 1;
  for (int64_t i = 0; i < n_samples * (c->n_qubits + 1); ++i) {
    if (chi_host[i] < 1 || chi_host[i] > chi_pad)
      return fail(QK_ERR_INVALID_ARG, "bond dimension outside [1, chi_pad]");
    mx = std::max(mx, chi_host[i]);
  }
  hipStream_t s = (hipStream_t)hip_stream;
  qk_mps_batch* b = nullptr;
  st = alloc_batch(c, n_samples, chi_pad, store, s, &b);
  if (st != QK_OK) return st;
  b->chi_ws = chi_pad;
  const int64_t elems = (int64_t)c->n_qubits * n_samples * 2 * chi_pad * chi_pad;
  const int32_t stat[2] = {0, mx};
  hipError_t e = hipStreamSynchronize(s);  // the stream-ordered allocations exist
  if (e == hipSuccess) e = hipMemcpy(b->t64, tensors_host, elems * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->chi, chi_host, n_samples * (c->n_qubits + 1) * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(b->status, stat, sizeof(stat), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    qk_mps_release(b);
    return hip_fail(e, "import copy");
  }
  st = finish_batch(b, store);
  if (st != QK_OK) {
    qk_mps_release(b);
    return st;
  }
  *out = b;
  return QK_OK;
}

qk_status qk_mps_info(const qk_mps_batch* b, int64_t* n_samples, int32_t* n_qubits,
                      int32_t* chi_pad, int32_t* chi_realized_max, int64_t* device_bytes) {
  if (!b) return fail(QK_ERR_INVALID_ARG, "batch is NULL");
  QK_HIP(hipEventSynchronize(b->ready), "batch synchronisation");
  int32_t st[2] = {0, 0};
  QK_HIP(hipMemcpy(st, b->status, sizeof(st), hipMemcpyDeviceToHost), "status read");
  if (n_samples) *n_samples = b->n;
  if (n_qubits) *n_qubits = b->nq;
  if (chi_pad) *chi_pad = b->T;
  if (chi_realized_max) *chi_realized_max = st[1];
  if (device_bytes) *device_bytes = b->bytes;
  if (st[0]) return fail(QK_ERR_DEVICE, qk_flag_text(st[0]));
  return QK_OK;
}

qk_status qk_mps_chi(const qk_mps_batch* b, int32_t* chi_host) {
  if (!b || !chi_host) return fail(QK_ERR_INVALID_ARG, "NULL argument");
  QK_HIP(hipEventSynchronize(b->ready), "batch synchronisation");
  QK_HIP(hipMemcpy(chi_host, b->chi, b->n * (b->nq + 1) * sizeof(int32_t),
                   hipMemcpyDeviceToHost),
         "bond table read");
  return QK_OK;
}

qk_status qk_mps_discarded(const qk_mps_batch* b, double* disc_host) {
  if (!b || !disc_host) return fail(QK_ERR_INVALID_ARG, "NULL argument");
  QK_HIP(hipEventSynchronize(b->ready), "batch synchronisation");
  QK_HIP(hipMemcpy(disc_host, b->disc, b->n * sizeof(double), hipMemcpyDeviceToHost),
         "discarded-weight read");
  return QK_OK;
}

qk_status qk_mps_release(qk_mps_batch* b) {
  if (!b) return QK_OK;
  // sweeps on any stream may still read the batch: drain the device first
  (void)hipDeviceSynchronize();
  free_batch_memory(b, nullptr);
  (void)hipStreamSynchronize(nullptr);
  if (b->ready) (void)hipEventDestroy(b->ready);
  delete b;
  return QK_OK;
}

qk_status qk_overlap_gram(const qk_mps_batch* rows, const qk_mps_batch* cols,
                          int32_t symmetric, qk_precision prec, double* kq_dev,
                          int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                          const qk_fuse_desc* fuse, void* hip_stream) {
  qk_gram_task task;
  memset(&task, 0, sizeof(task));
  task.rows = rows;
  task.cols = cols;
  task.symmetric = symmetric;
  task.kq_dev = kq_dev;
  task.ld_kq = ld_kq;
  task.lnkq_dev = lnkq_dev;
  task.ld_ln = ld_ln;
  if (fuse) {
    task.fuse = *fuse;
    task.use_fuse = 1;
  }
  return qk_overlap_gram_multi(&task, 1, prec, hip_stream);
}

qk_status qk_overlap_gram_multi(const qk_gram_task* tasks, int32_t n_tasks,
                                qk_precision prec, void* hip_stream) {
  if (!tasks || n_tasks < 1 || n_tasks > QK_MAX_TASKS)
    return fail(QK_ERR_INVALID_ARG, "need 1..16 tasks");
  hipStream_t s = (hipStream_t)hip_stream;
  if (prec == QK_PREC_AUTO) {
    // every task takes the form tuned for its own shape, so a task's result
    // does not depend on the tasks it is batched with; tasks that share a form
    // share one launch, the groups run back to back on the stream
    qk_precision form[QK_MAX_TASKS];
    for (int k = 0; k < n_tasks; ++k) {
      if (!tasks[k].rows || !tasks[k].cols) return fail(QK_ERR_INVALID_ARG, "batch is NULL");
      qk_status st = qk_resolve_precision(tasks[k].rows, tasks[k].cols, &form[k]);
      if (st != QK_OK) return st;
    }
    bool done[QK_MAX_TASKS] = {};
    for (int k = 0; k < n_tasks; ++k) {
      if (done[k]) continue;
      qk_gram_task group[QK_MAX_TASKS];
      int n = 0;
      for (int j = k; j < n_tasks; ++j)
        if (!done[j] && form[j] == form[k]) {
          group[n++] = tasks[j];
          done[j] = true;
        }
      qk_status st = qk_overlap_gram_multi(group, n, form[k], hip_stream);
      if (st != QK_OK) return st;
    }
    return QK_OK;
  }
  if (prec < QK_PREC_FP64 || prec > QK_PREC_FP32_MFMA)
    return fail(QK_ERR_INVALID_ARG, "unknown precision");
  std::vector<QkTask> tv(n_tasks);
  const int tile = tile_for(prec);
  const double tau = prec == QK_PREC_FP64 ? 0.0 : refine_tau(prec);
  for (int k = 0; k < n_tasks; ++k) {
    const qk_gram_task& g = tasks[k];
    qk_status st = fill_task(tv[k], g.rows, g.cols, g.symmetric, prec == QK_PREC_FP64,
                             tau > 0.0, g.kq_dev, g.ld_kq, g.lnkq_dev, g.ld_ln,
                             g.use_fuse ? &g.fuse : nullptr, tile);
    if (st != QK_OK) return st;
    if (!supported_T(prec, tv[k].T))
      return fail(QK_ERR_UNSUPPORTED, "chi_pad " + std::to_string(tv[k].T) +
                                          " is not supported by this sweep form");
  }
  // the sweep reads the batches: order it after their builds
  for (int k = 0; k < n_tasks; ++k) {
    QK_HIP(hipStreamWaitEvent(s, tasks[k].rows->ready, 0), "wait for row batch");
    QK_HIP(hipStreamWaitEvent(s, tasks[k].cols->ready, 0), "wait for column batch");
  }
  return run_tasks(tv, prec, tau, s);
}

qk_status qk_overlap_gram_noalloc(const qk_mps_batch* rows, const qk_mps_batch* cols,
                                  int32_t symmetric, qk_precision prec, double* kq_dev,
                                  int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                                  const qk_fuse_desc* fuse, void* hip_stream) {
  if (!rows || !cols) return fail(QK_ERR_INVALID_ARG, "batch is NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  if (prec == QK_PREC_AUTO) {
    qk_status st = qk_resolve_precision(rows, cols, &prec);
    if (st != QK_OK) return st;
  }
  if (prec < QK_PREC_FP64 || prec > QK_PREC_FP32_MFMA || prec == QK_PREC_AUTO)
    return fail(QK_ERR_INVALID_ARG, "unknown precision");
  std::vector<QkTask> tv(1);
  const double tau = prec == QK_PREC_FP64 ? 0.0 : refine_tau(prec);
  qk_status st = fill_task(tv[0], rows, cols, symmetric, prec == QK_PREC_FP64, tau > 0.0, kq_dev,
                           ld_kq, lnkq_dev, ld_ln, fuse, tile_for(prec));
  if (st != QK_OK) return st;
  if (!supported_T(prec, tv[0].T))
    return fail(QK_ERR_UNSUPPORTED, "chi_pad " + std::to_string(tv[0].T) +
                                        " is not supported by this sweep form");
  Scratch scr;
  QK_HIP(noalloc_scratch(&scr.ptr), "address of the device scratch");
  scr.bytes = kNoAllocScratchBytes;
  QK_HIP(hipStreamWaitEvent(s, rows->ready, 0), "wait for row batch");
  QK_HIP(hipStreamWaitEvent(s, cols->ready, 0), "wait for column batch");
  return run_tasks(tv, prec, tau, s, -1, &scr);
}

qk_status qk_autotune(const qk_mps_batch* rows, const qk_mps_batch* cols, int32_t symmetric,
                      int32_t max_tiles, void* hip_stream, qk_precision* chosen) {
  if (!rows || !cols || max_tiles < 1) return fail(QK_ERR_INVALID_ARG, "bad autotune arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  // Candidates: the forms that meet the stated tolerance, each with the launch
  // shapes it admits. Where the FP32 matrix-core form applies (bonds up to
  // 4), every key of a large job resolves to it (or to BF16x3 if that were
  // faster), so that AUTO gives all tasks of a mixed batch one form and the
  // batch runs as one launch: the FP32 VALU form stays available by name
  // only, and the complex-FP64 form competes only when the whole job fits
  // in the timed slice, i.e. a small job, where the reduced forms' FP64
  // refinement pass has a fixed cost that can exceed what they save.
  struct Cand {
    qk_precision p;
    int wg, band;
  };
  std::vector<Cand> cands;
  const bool mfma = qk_mfma_supports(QK_PREC_FP32_MFMA, rows->T);
  int64_t job_tiles = 0;
  {
    const int64_t tr = (rows->n + 15) / 16, tc = (cols->n + 15) / 16;
    job_tiles = symmetric ? tr * (tr + 1) / 2 : tr * tc;
  }
  const bool small_job = job_tiles <= max_tiles;
  if (rows->t64 && cols->t64 && (!mfma || small_job || !(rows->t32 && cols->t32)))
    for (int wg : {1, 2}) cands.push_back({QK_PREC_FP64, wg, kQkBand});
  if (rows->t32 && cols->t32) {
    if (mfma) {
      for (int band : {2, 4, 8})
        for (int wg : {2, 1}) cands.push_back({QK_PREC_FP32_MFMA, wg, band});
      cands.push_back({QK_PREC_BF16X3, 1, kQkBand});
    } else if (rows->T <= 4) {
      for (int wg : {2, 3, 4}) cands.push_back({QK_PREC_FP32, wg, kQkBand});
    }
  }
  if (cands.empty()) return fail(QK_ERR_UNSUPPORTED, "no sweep form applies to these batches");
  double* scratch = nullptr;
  QK_HIP(hipMallocAsync((void**)&scratch, std::max<int64_t>(rows->n * cols->n, 1) * sizeof(double), s),
         "autotune scratch");
  hipEvent_t e0, e1;
  QK_HIP(hipEventCreate(&e0), "event");
  QK_HIP(hipEventCreate(&e1), "event");
  QK_HIP(hipStreamWaitEvent(s, rows->ready, 0), "wait");
  QK_HIP(hipStreamWaitEvent(s, cols->ready, 0), "wait");
  double best = 1e300;
  Cand win = cands[0];
  int64_t tiles = 1;
  qk_status st = QK_OK;
  for (const Cand& c : cands) {
    std::vector<QkTask> tv(1);
    // When the slice is the whole job, a reduced form is timed with its FP64
    // refinement pass (part of what AUTO runs; on small jobs its fixed cost can
    // decide). On a partial slice it is not: the first tiles lie next to the
    // diagonal, where far more pairs exceed tau than in the whole job, and the
    // pass's fixed cost is not spread over the job's tiles.
    const double tau = c.p == QK_PREC_FP64 ? 0.0 : refine_tau(c.p);
    bool ref = tau > 0.0 && rows->t64 && cols->t64;
    st = fill_task(tv[0], rows, cols, symmetric, c.p == QK_PREC_FP64, ref, nullptr, 0,
                   scratch, cols->n, nullptr, tile_for(c.p));
    if (st != QK_OK) break;
    if (ref && tv[0].n_tiles > max_tiles) {
      ref = false;
      st = fill_task(tv[0], rows, cols, symmetric, false, false, nullptr, 0, scratch, cols->n,
                     nullptr, tile_for(c.p));
      if (st != QK_OK) break;
    }
    tiles = std::min<int64_t>(tv[0].n_tiles, max_tiles);
    qk_tune_store(rows->T, rows->nq, QkTuneEntry{c.p, c.wg, c.band, 0.0});
    st = run_tasks(tv, c.p, ref ? tau : 0.0, s, max_tiles);  // warm-up
    if (st != QK_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(QK_ERR_HIP, "event"); break; }
    for (int rep = 0; rep < 3 && st == QK_OK; ++rep)
      st = run_tasks(tv, c.p, ref ? tau : 0.0, s, max_tiles);
    if (st != QK_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(QK_ERR_HIP, "autotune timing");
      break;
    }
    const double us_tile = 1e3 * ms / 3.0 / (double)std::max<int64_t>(tiles, 1);
    if (us_tile < best) {
      best = us_tile;
      win = c;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipFreeAsync(scratch, s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != QK_OK) return st;
  qk_tune_store(rows->T, rows->nq, QkTuneEntry{win.p, win.wg, win.band, best});
  if (chosen) *chosen = win.p;
  return QK_OK;
}

qk_status qk_tune_export(char* buf, int64_t cap, int64_t* len) {
  const std::string t = qk_tune_export_text();
  if (len) *len = (int64_t)t.size() + 1;
  if (buf && cap > 0) {
    const int64_t n = std::min<int64_t>(cap - 1, (int64_t)t.size());
    memcpy(buf, t.data(), n);
    buf[n] = 0;
  }
  return QK_OK;
}

qk_status qk_tune_import(const char* text) {
  if (!text) return fail(QK_ERR_INVALID_ARG, "NULL text");
  if (!qk_tune_import_text(text)) return fail(QK_ERR_INVALID_ARG, "malformed tuning table");
  return QK_OK;
}

qk_status qk_set_svd_sweep_limit(int32_t sweeps) {
  if (sweeps < 0 || sweeps > kQkMaxSvdSweeps)
    return fail(QK_ERR_INVALID_ARG, "sweep limit must be in [0, 1000]");
  g_svd_sweeps.store(sweeps, std::memory_order_relaxed);
  return QK_OK;
}

qk_status qk_set_refine_threshold(qk_precision prec, double tau) {
  if (prec <= QK_PREC_FP64 || prec > QK_PREC_FP32_MFMA || prec == QK_PREC_AUTO)
    return fail(QK_ERR_INVALID_ARG, "refinement applies to the reduced-precision forms");
  if (!std::isfinite(tau)) return fail(QK_ERR_INVALID_ARG, "tau must be finite");
  std::lock_guard<std::mutex> lk(g_refine_mu);
  g_refine_tau[prec] = tau;
  return QK_OK;
}

qk_status qk_rbf_gram(const double* x_dev, int64_t m, int64_t ld_x, const double* y_dev,
                      int64_t n, int64_t ld_y, int32_t d, double gamma, double* kc_dev,
                      int64_t ld_kc, void* hip_stream) {
  if (m < 0 || n < 0 || d < 1) return fail(QK_ERR_INVALID_ARG, "bad sizes");
  if ((m > 0 && !x_dev) || (n > 0 && !y_dev) || (m > 0 && n > 0 && !kc_dev))
    return fail(QK_ERR_INVALID_ARG, "NULL pointer");
  if (ld_x < d || ld_y < d || ld_kc < n) return fail(QK_ERR_INVALID_ARG, "leading dimension too small");
  if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(QK_ERR_INVALID_ARG, "gamma must be finite and >= 0");
  hipError_t e = qk_launch_rbf(x_dev, m, ld_x, y_dev, n, ld_y, d, gamma, kc_dev, ld_kc,
                               (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "rbf launch");
  return QK_OK;
}

qk_status qk_dual_mix(const double* kq_dev, int64_t ld_kq, const double* kc_dev,
                      int64_t ld_kc, int64_t m, int64_t n, double w, double* k_dev,
                      int64_t ld_k, void* hip_stream) {
  if (m < 0 || n < 0) return fail(QK_ERR_INVALID_ARG, "bad sizes");
  if (m > 0 && n > 0 && (!kq_dev || !kc_dev || !k_dev)) return fail(QK_ERR_INVALID_ARG, "NULL pointer");
  if (ld_kq < n || ld_kc < n || ld_k < n) return fail(QK_ERR_INVALID_ARG, "leading dimension too small");
  if (!(w >= 0.0 && w <= 1.0)) return fail(QK_ERR_INVALID_ARG, "w must be in [0, 1]");
  hipError_t e = qk_launch_mix(kq_dev, ld_kq, kc_dev, ld_kc, m, n, w, k_dev, ld_k,
                               (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mix launch");
  return QK_OK;
}

qk_status qk_svm_decision(const double* k_dev, int64_t m, int64_t n, int64_t ld_k,
                          const double* coef_dev, double intercept, double* f_dev,
                          void* hip_stream) {
  if (m < 0 || n < 0) return fail(QK_ERR_INVALID_ARG, "bad sizes");
  if (m > INT32_MAX) return fail(QK_ERR_INVALID_ARG, "more than 2^31 - 1 rows");
  if (m > 0 && (!f_dev || (n > 0 && (!k_dev || !coef_dev))))
    return fail(QK_ERR_INVALID_ARG, "NULL pointer");
  if (ld_k < n) return fail(QK_ERR_INVALID_ARG, "leading dimension too small");
  if (!std::isfinite(intercept)) return fail(QK_ERR_INVALID_ARG, "intercept must be finite");
  hipError_t e = qk_launch_svm_decision(k_dev, m, n, ld_k, coef_dev, intercept, f_dev,
                                        (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "decision launch");
  return QK_OK;
}

qk_status qk_pathsum_gram(const double* x_rows_dev, int64_t m, int64_t ld_xr,
                          const double* x_cols_dev, int64_t n, int64_t ld_xc, int32_t d,
                          int32_t n_layers, int32_t entangle, int32_t symmetric, double* kq_dev,
                          int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                          const qk_fuse_desc* fuse, void* hip_stream) {
  if (m < 0 || n < 0 || m > INT32_MAX || n > INT32_MAX)
    return fail(QK_ERR_INVALID_ARG, "sample counts must be in [0, 2^31 - 1]");
  if (d < 1) return fail(QK_ERR_INVALID_ARG, "d < 1");
  if (n_layers < 1 || n_layers > 3)
    return fail(QK_ERR_UNSUPPORTED, "the path-sum evaluator covers one to three layers");
  if (entangle < 0)
    return fail(QK_ERR_INVALID_ARG, "entangle must be 0 (none), 1 (chain) or a block size >= 2");
  if (symmetric && (m != n || x_rows_dev != x_cols_dev || ld_xr != ld_xc))
    return fail(QK_ERR_INVALID_ARG, "symmetric mode needs the same rows and columns");
  if ((m > 0 && !x_rows_dev) || (n > 0 && !x_cols_dev))
    return fail(QK_ERR_INVALID_ARG, "features are NULL");
  if (ld_xr < d || ld_xc < d) return fail(QK_ERR_INVALID_ARG, "feature leading dimension < d");
  if ((kq_dev && ld_kq < n) || (lnkq_dev && ld_ln < n))
    return fail(QK_ERR_INVALID_ARG, "output leading dimension < n");
  qk_fuse_desc f{};
  if (fuse) {
    f = *fuse;
    f.x_rows_dev = x_rows_dev;  // the RBF uses the same features
    f.ld_xr = ld_xr;
    f.x_cols_dev = x_cols_dev;
    f.ld_xc = ld_xc;
    if (!(f.gamma >= 0.0) || !std::isfinite(f.gamma))
      return fail(QK_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    if (!f.w_rows_dev && !(f.w >= 0.0 && f.w <= 1.0))
      return fail(QK_ERR_INVALID_ARG, "w must be in [0, 1]");
    if ((f.kc_dev && f.ld_kc < n) || (f.k_dev && f.ld_k < n))
      return fail(QK_ERR_INVALID_ARG, "fused output leading dimension < n");
  }
  if (!kq_dev && !lnkq_dev && !(fuse && (f.kc_dev || f.k_dev)))
    return fail(QK_ERR_INVALID_ARG, "no output requested");
  if (m == 0 || n == 0) return QK_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t rows_tab = m * (int64_t)d, cols_tab = symmetric ? 0 : n * (int64_t)d;
  double4* tab = nullptr;
  QK_HIP(hipMallocAsync((void**)&tab, (rows_tab + cols_tab) * sizeof(double4), s),
         "path-sum table allocation");
  double4* tc = symmetric ? tab : tab + rows_tab;
  const int blk = entangle == 1 ? d : entangle;  // entangler block size (0: none)
  hipError_t e = qk_launch_pathsum_table(x_rows_dev, m, ld_xr, d, n_layers, blk, tab, s);
  if (e == hipSuccess && !symmetric)
    e = qk_launch_pathsum_table(x_cols_dev, n, ld_xc, d, n_layers, blk, tc, s);
  if (e == hipSuccess)
    e = qk_launch_pathsum(tab, m, tc, n, d, n_layers, symmetric, kq_dev, ld_kq, lnkq_dev, ld_ln,
                          fuse ? &f : nullptr, s);
  (void)hipFreeAsync(tab, s);
  if (e != hipSuccess) return hip_fail(e, "path-sum launch");
  return QK_OK;
}

qk_status qk_svm_fit_ovo(const double* k_dev, int64_t n, int64_t ld_k, const int32_t* labels_host,
                         int32_t n_classes, double C, double eps, int64_t max_iter,
                         double* coef_dev, int64_t ld_coef, double* intercept_dev,
                         int64_t* n_iter_dev, void* hip_stream) {
  if (n < 1 || n > INT32_MAX) return fail(QK_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  if (!k_dev || !labels_host || !coef_dev || !intercept_dev || !n_iter_dev)
    return fail(QK_ERR_INVALID_ARG, "NULL pointer");
  if (ld_k < n || ld_coef < n) return fail(QK_ERR_INVALID_ARG, "leading dimension too small");
  if (n_classes < 2 || n_classes > QK_SVM_MAX_CLASSES)
    return fail(QK_ERR_INVALID_ARG, "n_classes must be in [2, 64]");
  if (!(C > 0.0) || !std::isfinite(C)) return fail(QK_ERR_INVALID_ARG, "C must be positive");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(QK_ERR_INVALID_ARG, "eps must be positive");
  if (max_iter < 1) return fail(QK_ERR_INVALID_ARG, "max_iter must be positive");
  std::vector<std::vector<int32_t>> by_class(n_classes);
  for (int64_t t = 0; t < n; ++t) {
    const int32_t c = labels_host[t];
    if (c < -1 || c >= n_classes) return fail(QK_ERR_INVALID_ARG, "label outside [-1, n_classes)");
    if (c >= 0) by_class[c].push_back((int32_t)t);  // -1: left out of training
  }
  // problem (a, b), a < b, in lexicographic order: the samples of both
  // classes in increasing order, y = +1 for class a
  const int P = n_classes * (n_classes - 1) / 2;
  std::vector<int64_t> off(P + 1, 0);
  std::vector<int32_t> idx;
  std::vector<double> yv;
  idx.reserve((size_t)(n_classes - 1) * n);
  yv.reserve((size_t)(n_classes - 1) * n);
  int p = 0;
  for (int a = 0; a < n_classes; ++a)
    for (int b = a + 1; b < n_classes; ++b, ++p) {
      const auto& A = by_class[a];
      const auto& B = by_class[b];
      size_t ia = 0, ib = 0;
      while (ia < A.size() || ib < B.size()) {
        if (ib == B.size() || (ia < A.size() && A[ia] < B[ib])) {
          idx.push_back(A[ia++]);
          yv.push_back(1.0);
        } else {
          idx.push_back(B[ib++]);
          yv.push_back(-1.0);
        }
      }
      off[p + 1] = (int64_t)idx.size();
    }
  const int64_t tot = (int64_t)idx.size();
  hipStream_t s = (hipStream_t)hip_stream;
  // one stream-ordered block: off | y | alpha | grad | diag | idx
  const int64_t bytes = (int64_t)(P + 1) * 8 + tot * 8 * 4 + tot * 4 + 16;
  char* dbuf = nullptr;
  QK_HIP(hipMallocAsync((void**)&dbuf, bytes, s), "SVM scratch allocation");
  int64_t* d_off = reinterpret_cast<int64_t*>(dbuf);
  double* d_y = reinterpret_cast<double*>(dbuf + (int64_t)(P + 1) * 8);
  double* d_alpha = d_y + tot;
  double* d_grad = d_alpha + tot;
  double* d_diag = d_grad + tot;
  int32_t* d_idx = reinterpret_cast<int32_t*>(d_diag + tot);
  // tables go up through pinned staging; the call waits for the upload so
  // the staging can be freed before returning
  const int64_t hbytes = (int64_t)(P + 1) * 8 + tot * 8 + tot * 4;
  char* hbuf = nullptr;
  if (hipHostMalloc((void**)&hbuf, hbytes, 0) != hipSuccess) {
    (void)hipFreeAsync(dbuf, s);
    return fail(QK_ERR_OUT_OF_MEMORY, "SVM staging allocation failed");
  }
  std::memcpy(hbuf, off.data(), (P + 1) * 8);
  std::memcpy(hbuf + (P + 1) * 8, yv.data(), tot * 8);
  std::memcpy(hbuf + (P + 1) * 8 + tot * 8, idx.data(), tot * 4);
  hipError_t e = hipMemcpyAsync(d_off, hbuf, (P + 1) * 8 + tot * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_idx, hbuf + (P + 1) * 8 + tot * 8, tot * 4, hipMemcpyHostToDevice, s);
  const hipError_t es = hipStreamSynchronize(s);
  (void)hipHostFree(hbuf);
  if (e == hipSuccess) e = es;
  if (e == hipSuccess)
    e = qk_launch_svm_smo(k_dev, ld_k, d_idx, d_y, d_off, P, C, eps, max_iter, d_alpha, d_grad,
                          d_diag, coef_dev, ld_coef, n, intercept_dev, n_iter_dev, s);
  (void)hipFreeAsync(dbuf, s);
  if (e != hipSuccess) return hip_fail(e, "SVM training");
  return QK_OK;
}

qk_status qk_svm_predict_ovo(const double* k_dev, int64_t m, int64_t n, int64_t ld_k,
                             const double* coef_dev, int64_t ld_coef, const double* intercept_dev,
                             int32_t n_classes, double* f_dev, int64_t ld_f, int32_t* labels_dev,
                             void* hip_stream) {
  if (m < 0 || m > INT32_MAX) return fail(QK_ERR_INVALID_ARG, "m must be in [0, 2^31 - 1]");
  if (n < 1) return fail(QK_ERR_INVALID_ARG, "n < 1");
  if (n_classes < 2 || n_classes > QK_SVM_MAX_CLASSES)
    return fail(QK_ERR_INVALID_ARG, "n_classes must be in [2, 64]");
  const int64_t P = (int64_t)n_classes * (n_classes - 1) / 2;
  if (ld_k < n || ld_coef < n || (f_dev && ld_f < P))
    return fail(QK_ERR_INVALID_ARG, "leading dimension too small");
  if (!f_dev && !labels_dev) return fail(QK_ERR_INVALID_ARG, "no output requested");
  if (m > 0 && (!k_dev || !coef_dev || !intercept_dev)) return fail(QK_ERR_INVALID_ARG, "NULL pointer");
  hipError_t e = qk_launch_svm_predict(k_dev, m, n, ld_k, coef_dev, ld_coef, intercept_dev,
                                       n_classes, f_dev, ld_f, labels_dev,
                                       (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "SVM prediction launch");
  return QK_OK;
}

qk_status qk_resolve_precision(const qk_mps_batch* rows, const qk_mps_batch* cols,
                               qk_precision* out) {
  if (!rows || !cols || !out) return fail(QK_ERR_INVALID_ARG, "NULL argument");
  *out = qk_tune_choose(rows->T, rows->nq, rows->t32 != nullptr, rows->t64 != nullptr);
  return QK_OK;
}

}  // extern "C"
