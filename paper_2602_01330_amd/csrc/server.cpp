// Serving: continuous batching of kernel-row requests against resident
// support sets (the qk_server_* declarations in qk.h describe the contract).
//
// One worker thread owns all device work of the server. Its loop:
//   1. retire finished iterations (event query): mark their requests DONE,
//      stamp the time, return their budget, free their device buffers;
//   2. if a stream slot is free, admit queued requests in arrival order while
//      the HBM budget and the per-iteration row cap allow;
//   3. launch the admitted rows as one iteration on that slot's stream: per
//      feature dimension d, stage the rows and weights, build their MPS, then
//      ONE multi-task sweep launch (one task per d) with the fused RBF and
//      per-row mix; where the support set carries a trained SVM, the decision
//      values of the new rows follow on the same stream; copy each request's
//      rows (and decision values) and each build's status words to pinned
//      host memory. A request whose build latched a device check retires as
//      FAILED with the check's text.
// Submissions only touch host memory and the queue, so they never wait for
// the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qk_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Support {
  qk_circuit_desc desc{};
  qk_mps_batch* mps = nullptr;
  double* x = nullptr;  // n x d, library-owned copy of the features
  int64_t n = 0;
  double* coef = nullptr;  // n SVM coefficients alpha_i y_i on the device, or NULL
  double intercept = 0.0;
};

struct Request {
  int64_t id = 0;
  int32_t d = 0;
  int64_t n_rows = 0;
  double w = 0.5;
  std::vector<double> x;
  int32_t state = QK_REQ_QUEUED;
  std::string err;
  bool cancel = false;
  int64_t n_support = 0;
  int64_t bytes = 0;           // budget reservation while admitted
  double* out_host = nullptr;  // pinned n_rows x n_support, filled by the D2H copy
  double* f_host = nullptr;    // pinned n_rows decision values (admitted with a model)
  bool want_ln = false;        // also return ln K_q rows
  double* ln_host = nullptr;   // pinned n_rows x n_support ln K_q (want_ln)
  int group = -1;              // the iteration's d group (index of its build's status words)
};

struct Iteration {
  int slot = 0;
  hipEvent_t done = nullptr;
  std::vector<Request*> reqs;
  std::map<int32_t, Support> sups;  // support sets used, copied under the lock
  std::vector<qk_mps_batch*> batches;
  std::vector<void*> dev;     // stream-ordered device buffers
  std::vector<void*> pinned;  // host staging of features and weights
  int32_t* status_host = nullptr;  // pinned: each d group's build status words (2 int32)
};

}  // namespace

struct qk_server {
  qk_server_config cfg{};
  int device = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;       // wakes the worker
  std::condition_variable cv_done;  // wakes waiters on request state
  std::deque<Request*> pending;
  std::unordered_map<int64_t, Request*> reqs;
  std::unordered_map<int64_t, std::array<double, 3>> times;  // submit, admit, done
  std::map<int32_t, Support> supports;
  std::vector<double*> old_coefs;  // replaced models, freed at destroy (iterations may hold them)
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::deque<Iteration*> inflight;
  int64_t next_id = 1;
  int64_t budget_used = 0, peak = 0;
  int64_t n_done = 0, n_iters = 0, entries = 0;
  bool stop = false;
  std::thread worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int64_t request_bytes(const Request& r, const Support& sup) {
  const int64_t T = sup.mps->T, d = r.d, rows = r.n_rows, ns = sup.n;
  const int64_t tiles = ((rows + 15) / 16) * ((ns + 15) / 16);
  return rows * d * 2 * T * T * (int64_t)(sizeof(double2) + kQkPackFloats * sizeof(float))  // MPS forms
         + rows * (d + 1) * 4                                                 // bond table
         + rows * d * 8 + rows * 8                                            // features, w
         + rows * ns * 8                                                      // K rows
         + tiles * 32                                                         // refinement masks
         + (sup.coef ? rows * 8 : 0)                                          // decision values
         + (r.want_ln ? rows * ns * 8 : 0);                                   // ln K_q rows
}

void free_host(Request* r) {
  if (r->out_host) (void)hipHostFree(r->out_host);
  if (r->f_host) (void)hipHostFree(r->f_host);
  if (r->ln_host) (void)hipHostFree(r->ln_host);
  r->out_host = nullptr;
  r->f_host = nullptr;
  r->ln_host = nullptr;
}

void finish(qk_server* s, Request* r, int32_t state, const std::string& err = "") {
  r->state = state;
  r->err = err;
  s->times[r->id][2] = s->now();
  if (state == QK_REQ_DONE) {
    ++s->n_done;
    s->entries += r->n_rows * r->n_support;
  }
}

void retire(qk_server* s, Iteration* it) {
  for (Request* r : it->reqs) {
    s->budget_used -= r->bytes;
    r->bytes = 0;
    // the build of the request's rows latched a device check (sweep limit,
    // bond bound, non-finite input): its rows are not valid kernel values
    const int32_t flags =
        (it->status_host && r->group >= 0) ? it->status_host[2 * r->group] : 0;
    if (r->cancel) {
      free_host(r);
      finish(s, r, QK_REQ_CANCELLED);
    } else if (flags) {
      free_host(r);
      finish(s, r, QK_REQ_FAILED, qk_flag_text(flags));
    } else {
      finish(s, r, QK_REQ_DONE);
    }
  }
  hipStream_t st = s->streams[it->slot];
  for (qk_mps_batch* b : it->batches) qk_mps_release_nosync(b, st);
  for (void* p : it->dev) (void)hipFreeAsync(p, st);
  for (void* p : it->pinned) (void)hipHostFree(p);
  if (it->status_host) (void)hipHostFree(it->status_host);
  (void)hipEventDestroy(it->done);
  s->slot_busy[it->slot] = false;
  delete it;
}

// Enqueues one iteration on the slot's stream. Called without the lock held;
// the requests are already RUNNING and owned by the iteration.
std::string launch(qk_server* s, Iteration* it) {
  hipStream_t st = s->streams[it->slot];
  std::map<int32_t, std::vector<Request*>> by_d;
  for (Request* r : it->reqs) by_d[r->d].push_back(r);
  std::vector<qk_gram_task> tasks;
  struct Out {
    Request* r;
    double* k;
    double* f;   // decision values of the d group, or NULL
    double* ln;  // ln K_q rows of the d group, or NULL
    int64_t row0;
  };
  struct Decision {
    const double* k;
    int64_t rows, n;
    const double* coef;
    double b;
    double* f;
  };
  std::vector<Decision> decisions;
  std::vector<Out> outs;
  if (hipHostMalloc((void**)&it->status_host, 2 * by_d.size() * sizeof(int32_t), 0) != hipSuccess)
    return "pinned status allocation failed";
  int group = 0;
  for (auto& kv : by_d) {
    const Support& sup = it->sups.at(kv.first);
    const int32_t d = kv.first;
    int64_t rows = 0;
    bool any_ln = false;
    for (Request* r : kv.second) {
      rows += r->n_rows;
      any_ln = any_ln || r->want_ln;
    }
    double *hx = nullptr, *hw = nullptr, *dx = nullptr, *dw = nullptr, *dk = nullptr;
    double* dln = nullptr;
    if (hipHostMalloc((void**)&hx, rows * d * sizeof(double), 0) != hipSuccess ||
        hipHostMalloc((void**)&hw, rows * sizeof(double), 0) != hipSuccess)
      return "pinned staging allocation failed";
    it->pinned.push_back(hx);
    it->pinned.push_back(hw);
    int64_t off = 0;
    for (Request* r : kv.second) {
      std::memcpy(hx + off * d, r->x.data(), r->n_rows * d * sizeof(double));
      for (int64_t q = 0; q < r->n_rows; ++q) hw[off + q] = r->w;
      off += r->n_rows;
    }
    if (hipMallocAsync((void**)&dx, rows * d * sizeof(double), st) != hipSuccess ||
        hipMallocAsync((void**)&dw, rows * sizeof(double), st) != hipSuccess ||
        hipMallocAsync((void**)&dk, rows * sup.n * sizeof(double), st) != hipSuccess)
      return "device allocation for an iteration failed";
    it->dev.push_back(dx);
    it->dev.push_back(dw);
    it->dev.push_back(dk);
    if (any_ln) {
      if (hipMallocAsync((void**)&dln, rows * sup.n * sizeof(double), st) != hipSuccess)
        return "device allocation for an iteration failed";
      it->dev.push_back(dln);
    }
    if (hipMemcpyAsync(dx, hx, rows * d * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dw, hw, rows * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
      return "feature upload failed";
    qk_mps_batch* mb = nullptr;
    qk_status bs = qk_mps_build(&sup.desc, dx, rows, d, QK_STORE_ALL, st, &mb);
    if (bs != QK_OK) return std::string("request encoding failed: ") + qk_last_error();
    it->batches.push_back(mb);
    qk_gram_task t;
    std::memset(&t, 0, sizeof(t));
    t.rows = mb;
    t.cols = sup.mps;
    t.symmetric = 0;
    t.lnkq_dev = dln;
    t.ld_ln = sup.n;
    t.use_fuse = 1;
    t.fuse.x_rows_dev = dx;
    t.fuse.ld_xr = d;
    t.fuse.x_cols_dev = sup.x;
    t.fuse.ld_xc = d;
    t.fuse.gamma = s->cfg.gamma_scale / d;
    t.fuse.w = 0.5;
    t.fuse.w_rows_dev = dw;
    t.fuse.k_dev = dk;
    t.fuse.ld_k = sup.n;
    tasks.push_back(t);
    double* df = nullptr;
    if (sup.coef) {
      if (hipMallocAsync((void**)&df, rows * sizeof(double), st) != hipSuccess)
        return "device allocation for an iteration failed";
      it->dev.push_back(df);
      decisions.push_back({dk, rows, sup.n, sup.coef, sup.intercept, df});
    }
    off = 0;
    for (Request* r : kv.second) {
      outs.push_back({r, dk, df, r->want_ln ? dln : nullptr, off});
      r->group = group;
      off += r->n_rows;
    }
    ++group;
  }
  qk_status gs = qk_overlap_gram_multi(tasks.data(), (int32_t)tasks.size(), s->cfg.prec, st);
  if (gs != QK_OK) return std::string("sweep launch failed: ") + qk_last_error();
  for (const Decision& dc : decisions)
    if (qk_launch_svm_decision(dc.k, dc.rows, dc.n, dc.n, dc.coef, dc.b, dc.f, st) != hipSuccess)
      return "decision launch failed";
  // each group's build status, read at retirement (the build runs on this stream)
  for (size_t g = 0; g < it->batches.size(); ++g)
    if (hipMemcpyAsync(it->status_host + 2 * g, it->batches[g]->status, 2 * sizeof(int32_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      return "status download failed";
  for (const Out& o : outs) {
    const int64_t bytes = o.r->n_rows * o.r->n_support * (int64_t)sizeof(double);
    if (hipMemcpyAsync(o.r->out_host, o.k + o.row0 * o.r->n_support, bytes,
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      return "result download failed";
    // the request's pinned buffer exists iff its support set had a model at admission
    if (o.f && o.r->f_host &&
        hipMemcpyAsync(o.r->f_host, o.f + o.row0, o.r->n_rows * sizeof(double),
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      return "result download failed";
    if (o.ln && hipMemcpyAsync(o.r->ln_host, o.ln + o.row0 * o.r->n_support, bytes,
                               hipMemcpyDeviceToHost, st) != hipSuccess)
      return "result download failed";
  }
  if (hipEventCreateWithFlags(&it->done, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(it->done, st) != hipSuccess)
    return "event record failed";
  return "";
}

void worker_main(qk_server* s) {
  (void)hipSetDevice(s->device);
  const int64_t budget = s->cfg.budget_bytes;
  const int64_t max_rows = s->cfg.max_rows_per_iter;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // 1. retire finished iterations, oldest first
    bool retired = false;
    while (!s->inflight.empty()) {
      Iteration* it = s->inflight.front();
      if (hipEventQuery(it->done) != hipSuccess) break;
      s->inflight.pop_front();
      retire(s, it);
      retired = true;
    }
    if (retired) s->cv_done.notify_all();
    if (s->stop && s->pending.empty() && s->inflight.empty()) break;
    // 2. admit into a free slot
    int slot = -1;
    for (size_t k = 0; k < s->slot_busy.size(); ++k)
      if (!s->slot_busy[k]) {
        slot = (int)k;
        break;
      }
    Iteration* it = nullptr;
    if (slot >= 0 && !s->pending.empty()) {
      int64_t rows = 0;
      while (!s->pending.empty()) {
        Request* r = s->pending.front();
        if (r->cancel) {
          s->pending.pop_front();
          finish(s, r, QK_REQ_CANCELLED);
          s->cv_done.notify_all();
          continue;
        }
        const Support& sup = s->supports.at(r->d);
        const int64_t need = request_bytes(*r, sup);
        if (need > budget || r->n_rows > max_rows) {
          s->pending.pop_front();
          finish(s, r, QK_REQ_FAILED, "request exceeds the HBM budget or the row cap");
          s->cv_done.notify_all();
          continue;
        }
        if (s->budget_used + need > budget || rows + r->n_rows > max_rows) break;
        // one sweep task per d: at most QK_MAX_TASKS distinct d per iteration
        if (it && !it->sups.count(r->d) && (int)it->sups.size() >= QK_MAX_TASKS) break;
        if ((!r->out_host &&
             hipHostMalloc((void**)&r->out_host, r->n_rows * sup.n * sizeof(double), 0) != hipSuccess) ||
            (sup.coef && !r->f_host &&
             hipHostMalloc((void**)&r->f_host, r->n_rows * sizeof(double), 0) != hipSuccess) ||
            (r->want_ln && !r->ln_host &&
             hipHostMalloc((void**)&r->ln_host, r->n_rows * sup.n * sizeof(double), 0) != hipSuccess)) {
          free_host(r);
          s->pending.pop_front();
          finish(s, r, QK_REQ_FAILED, "pinned result allocation failed");
          s->cv_done.notify_all();
          continue;
        }
        s->pending.pop_front();
        r->bytes = need;
        r->n_support = sup.n;
        s->budget_used += need;
        s->peak = std::max(s->peak, s->budget_used);
        rows += r->n_rows;
        r->state = QK_REQ_RUNNING;
        s->times[r->id][1] = s->now();
        if (!it) {
          it = new Iteration();
          it->slot = slot;
        }
        it->sups[r->d] = sup;
        it->reqs.push_back(r);
      }
    }
    if (it) {
      s->slot_busy[slot] = true;
      ++s->n_iters;
      lk.unlock();
      std::string err = launch(s, it);
      lk.lock();
      if (!err.empty()) {
        // device work already enqueued drains before the buffers are freed
        (void)hipStreamSynchronize(s->streams[slot]);
        if (!it->done) (void)hipEventCreateWithFlags(&it->done, hipEventDisableTiming);
        for (Request* r : it->reqs) {
          s->budget_used -= r->bytes;
          r->bytes = 0;
          free_host(r);  // the stream has drained: no copy still targets them
          finish(s, r, QK_REQ_FAILED, err);
        }
        it->reqs.clear();
        retire(s, it);
        s->cv_done.notify_all();
      } else {
        s->inflight.push_back(it);
      }
      continue;
    }
    // 3. nothing to launch: sleep until a submission or poll the in-flight events
    if (s->inflight.empty())
      s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    else
      s->cv.wait_for(lk, std::chrono::microseconds(100));
  }
}

}  // namespace

extern "C" {

qk_status qk_server_create(const qk_server_config* cfg, qk_server** out) {
  if (!out) return qk_fail(QK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  qk_server_config c{};
  if (cfg) c = *cfg;
  if (c.budget_bytes < 0 || c.max_rows_per_iter < 0 || c.n_streams < 0 || c.n_streams > 4)
    return qk_fail(QK_ERR_INVALID_ARG, "bad server configuration");
  if (c.budget_bytes == 0) c.budget_bytes = (int64_t)1 << 30;
  if (c.max_rows_per_iter == 0) c.max_rows_per_iter = 512;
  if (c.n_streams == 0) c.n_streams = 2;
  if (c.gamma_scale == 0.0) c.gamma_scale = 1.0;
  if (!(c.gamma_scale > 0.0) || !std::isfinite(c.gamma_scale))
    return qk_fail(QK_ERR_INVALID_ARG, "gamma_scale must be positive");
  if (c.prec < QK_PREC_FP64 || c.prec > QK_PREC_FP32_MFMA)
    return qk_fail(QK_ERR_INVALID_ARG, "unknown precision");
  auto* s = new qk_server();
  s->cfg = c;
  s->t0 = Clock::now();
  (void)hipGetDevice(&s->device);
  for (int k = 0; k < c.n_streams; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return qk_fail(QK_ERR_HIP, "stream creation failed");
    }
    s->streams.push_back(st);
    s->slot_busy.push_back(false);
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return QK_OK;
}

qk_status qk_server_load_support(qk_server* s, const qk_circuit_desc* c, const double* x_dev,
                                 int64_t n, int64_t ld_x) {
  if (!s || !c || !x_dev || n < 1) return qk_fail(QK_ERR_INVALID_ARG, "bad support arguments");
  const int32_t d = c->n_qubits;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->supports.count(d)) return qk_fail(QK_ERR_INVALID_ARG, "support set for this d exists");
  }
  if (ld_x < d) return qk_fail(QK_ERR_INVALID_ARG, "ld_x < d");
  hipStream_t st = s->streams[0];
  Support sup;
  sup.desc = *c;
  sup.n = n;
  if (hipMalloc((void**)&sup.x, n * d * sizeof(double)) != hipSuccess)
    return qk_fail(QK_ERR_OUT_OF_MEMORY, "support feature allocation failed");
  if (hipMemcpy2DAsync(sup.x, d * sizeof(double), x_dev, ld_x * sizeof(double), d * sizeof(double),
                       n, hipMemcpyDeviceToDevice, st) != hipSuccess) {
    (void)hipFree(sup.x);
    return qk_fail(QK_ERR_HIP, "support feature copy failed");
  }
  qk_status bs = qk_mps_build(c, sup.x, n, d, QK_STORE_ALL, st, &sup.mps);
  if (bs != QK_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(sup.x);
    return bs;
  }
  bs = qk_mps_info(sup.mps, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (bs != QK_OK) {
    std::string m = qk_last_error();
    qk_mps_release(sup.mps);
    (void)hipFree(sup.x);
    return qk_fail(bs, m);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->supports[d] = sup;
  return QK_OK;
}

qk_status qk_server_set_model(qk_server* s, int32_t d, const double* coef_host, int64_t n,
                              double intercept) {
  if (!s) return qk_fail(QK_ERR_INVALID_ARG, "NULL server");
  if (!std::isfinite(intercept)) return qk_fail(QK_ERR_INVALID_ARG, "intercept must be finite");
  int64_t ns = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto f = s->supports.find(d);
    if (f == s->supports.end()) return qk_fail(QK_ERR_NOT_FOUND, "no support set loaded for this d");
    ns = f->second.n;
  }
  if (!coef_host) {
    // removes the model: requests admitted from now on return kernel rows only
    std::lock_guard<std::mutex> lk(s->mu);
    Support& sup = s->supports.at(d);
    if (sup.coef) s->old_coefs.push_back(sup.coef);
    sup.coef = nullptr;
    sup.intercept = 0.0;
    return QK_OK;
  }
  if (n != ns) return qk_fail(QK_ERR_INVALID_ARG, "coefficient count differs from the support size");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(coef_host[i])) return qk_fail(QK_ERR_INVALID_ARG, "non-finite coefficient");
  double* dc = nullptr;
  if (hipMalloc((void**)&dc, n * sizeof(double)) != hipSuccess)
    return qk_fail(QK_ERR_OUT_OF_MEMORY, "model allocation failed");
  if (hipMemcpy(dc, coef_host, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dc);
    return qk_fail(QK_ERR_HIP, "model upload failed");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  Support& sup = s->supports.at(d);
  if (sup.coef) s->old_coefs.push_back(sup.coef);
  sup.coef = dc;
  sup.intercept = intercept;
  return QK_OK;
}

qk_status qk_server_submit(qk_server* s, const double* x_host, int64_t n_rows, int32_t d,
                           double w, int64_t* id) {
  return qk_server_submit_ex(s, x_host, n_rows, d, w, 0u, id);
}

qk_status qk_server_submit_ex(qk_server* s, const double* x_host, int64_t n_rows, int32_t d,
                              double w, uint32_t outputs, int64_t* id) {
  if (!s || !x_host || !id || n_rows < 1) return qk_fail(QK_ERR_INVALID_ARG, "bad request");
  if (outputs & ~(uint32_t)QK_OUT_LNKQ) return qk_fail(QK_ERR_INVALID_ARG, "unknown output flag");
  if (!(w >= 0.0 && w <= 1.0)) return qk_fail(QK_ERR_INVALID_ARG, "w must be in [0, 1]");
  for (int64_t k = 0; k < n_rows * (int64_t)d; ++k)
    if (!std::isfinite(x_host[k])) return qk_fail(QK_ERR_INVALID_ARG, "non-finite feature");
  auto* r = new Request();
  r->d = d;
  r->n_rows = n_rows;
  r->w = w;
  r->want_ln = (outputs & QK_OUT_LNKQ) != 0;
  r->x.assign(x_host, x_host + n_rows * (int64_t)d);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->supports.count(d)) {
      delete r;
      return qk_fail(QK_ERR_NOT_FOUND, "no support set loaded for this d");
    }
    if (s->stop) {
      delete r;
      return qk_fail(QK_ERR_BUSY, "server is shutting down");
    }
    r->id = s->next_id++;
    s->reqs[r->id] = r;
    s->times[r->id] = {s->now(), -1.0, -1.0};
    s->pending.push_back(r);
    *id = r->id;
  }
  s->cv.notify_one();
  return QK_OK;
}

qk_status qk_server_poll_decision(qk_server* s, int64_t id, double* rows_host, int64_t ld_rows,
                                  double* f_host, int32_t* state) {
  return qk_server_poll_ex(s, id, rows_host, ld_rows, f_host, nullptr, 0, state);
}

qk_status qk_server_poll_ex(qk_server* s, int64_t id, double* rows_host, int64_t ld_rows,
                            double* f_host, double* ln_host, int64_t ld_ln, int32_t* state) {
  if (!s || !state) return qk_fail(QK_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return qk_fail(QK_ERR_NOT_FOUND, "unknown or released request");
  Request* r = f->second;
  *state = r->state;
  if (r->state == QK_REQ_FAILED) return qk_fail(QK_OK, r->err);
  const bool fetch = rows_host || f_host || ln_host;
  if (r->state == QK_REQ_DONE && fetch) {
    if (rows_host && ld_rows < r->n_support)
      return qk_fail(QK_ERR_INVALID_ARG, "ld_rows < support size");
    if (ln_host && ld_ln < r->n_support)
      return qk_fail(QK_ERR_INVALID_ARG, "ld_ln < support size");
    if (f_host && !r->f_host)
      return qk_fail(QK_ERR_INVALID_ARG, "the request was admitted without a model");
    if (ln_host && !r->ln_host)
      return qk_fail(QK_ERR_INVALID_ARG, "the request did not ask for ln K_q rows");
    if (rows_host)
      for (int64_t q = 0; q < r->n_rows; ++q)
        std::memcpy(rows_host + q * ld_rows, r->out_host + q * r->n_support,
                    r->n_support * sizeof(double));
    if (ln_host)
      for (int64_t q = 0; q < r->n_rows; ++q)
        std::memcpy(ln_host + q * ld_ln, r->ln_host + q * r->n_support,
                    r->n_support * sizeof(double));
    if (f_host) std::memcpy(f_host, r->f_host, r->n_rows * sizeof(double));
    free_host(r);
    s->reqs.erase(f);
    delete r;
  } else if (r->state == QK_REQ_CANCELLED && fetch) {
    s->reqs.erase(f);
    delete r;
  }
  return QK_OK;
}

qk_status qk_server_poll(qk_server* s, int64_t id, double* rows_host, int64_t ld_rows,
                         int32_t* state) {
  return qk_server_poll_decision(s, id, rows_host, ld_rows, nullptr, state);
}

qk_status qk_server_wait(qk_server* s, int64_t id, int32_t timeout_ms, int32_t* state) {
  if (!s || !state) return qk_fail(QK_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto active = [&] {
    auto f = s->reqs.find(id);
    return f != s->reqs.end() &&
           (f->second->state == QK_REQ_QUEUED || f->second->state == QK_REQ_RUNNING);
  };
  if (!s->reqs.count(id)) return qk_fail(QK_ERR_NOT_FOUND, "unknown or released request");
  if (timeout_ms < 0) s->cv_done.wait(lk, [&] { return !active(); });
  else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !active(); });
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return qk_fail(QK_ERR_NOT_FOUND, "request released");
  *state = f->second->state;
  return QK_OK;
}

qk_status qk_server_cancel(qk_server* s, int64_t id) {
  if (!s) return qk_fail(QK_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto f = s->reqs.find(id);
  if (f == s->reqs.end()) return qk_fail(QK_ERR_NOT_FOUND, "unknown or released request");
  Request* r = f->second;
  if (r->state == QK_REQ_QUEUED) {
    auto p = std::find(s->pending.begin(), s->pending.end(), r);
    if (p != s->pending.end()) s->pending.erase(p);
    finish(s, r, QK_REQ_CANCELLED);
    s->cv_done.notify_all();
  } else if (r->state == QK_REQ_RUNNING) {
    r->cancel = true;
  }
  return QK_OK;
}

qk_status qk_server_request_times(qk_server* s, int64_t id, double* t_submit, double* t_admit,
                                  double* t_done) {
  if (!s) return qk_fail(QK_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto f = s->times.find(id);
  if (f == s->times.end()) return qk_fail(QK_ERR_NOT_FOUND, "unknown request");
  if (t_submit) *t_submit = f->second[0];
  if (t_admit) *t_admit = f->second[1];
  if (t_done) *t_done = f->second[2];
  return QK_OK;
}

qk_status qk_server_stats(qk_server* s, int64_t* n_done, int64_t* n_iters,
                          int64_t* peak_budget_bytes, int64_t* entries_done) {
  if (!s) return qk_fail(QK_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (n_done) *n_done = s->n_done;
  if (n_iters) *n_iters = s->n_iters;
  if (peak_budget_bytes) *peak_budget_bytes = s->peak;
  if (entries_done) *entries_done = s->entries;
  return QK_OK;
}

qk_status qk_server_destroy(qk_server* s) {
  if (!s) return QK_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipDeviceSynchronize();
  for (auto& kv : s->reqs) {
    free_host(kv.second);
    delete kv.second;
  }
  for (auto& kv : s->supports) {
    qk_mps_release(kv.second.mps);
    (void)hipFree(kv.second.x);
    if (kv.second.coef) (void)hipFree(kv.second.coef);
  }
  for (double* c : s->old_coefs) (void)hipFree(c);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return QK_OK;
}

}  // extern "C"
