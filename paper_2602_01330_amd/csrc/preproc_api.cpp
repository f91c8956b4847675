// Host side of the pre-processing entry points (qk_preproc_*): argument
// checks, the fitted statistics' ownership, and the Jacobi sweep loop (one
// host check of the off-diagonal mass per sweep). The arithmetic runs in the
// kernels of preprocess.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>

#include "qk_internal.h"

hipError_t qk_launch_pp_colstats(const double* x, int64_t n, int64_t ld, int d, double* mu,
                                 double* sigma, hipStream_t s);
hipError_t qk_launch_pp_standardize(const double* x, int64_t n, int64_t ld, int d,
                                    const double* mu, const double* sigma, double* z,
                                    hipStream_t s);
hipError_t qk_launch_pp_cov(const double* z, int64_t n, int d, double* c, hipStream_t s);
hipError_t qk_launch_pp_project(const double* z, int64_t n, int d, const double* w, int k,
                                double* y, hipStream_t s);
hipError_t qk_launch_pp_jacobi_round(double* c, double* v, int d, int m, int r, double4* rot,
                                     hipStream_t s);
hipError_t qk_launch_pp_offdiag(const double* c, int d, double* out, hipStream_t s);
hipError_t qk_launch_pp_components(const double* c, const double* v, int d, int k, int* perm,
                                   double* lam, double* w, hipStream_t s);
hipError_t qk_launch_pp_minmax(const double* y, int64_t n, int k, double* ymin, double* ymax,
                               hipStream_t s);
hipError_t qk_launch_pp_scale(const double* y, int64_t n, int k, const double* ymin,
                              const double* ymax, double scale, double* out, int64_t ld_out,
                              hipStream_t s);

struct qk_preproc {
  int d = 0, k = 0, sweeps = 0;
  double* mu = nullptr;     // d
  double* sigma = nullptr;  // d
  double* w = nullptr;      // k x d components
  double* ymin = nullptr;   // k
  double* ymax = nullptr;   // k
  double* lam = nullptr;    // d eigenvalues, decreasing
};

namespace {

constexpr int kMaxSweeps = 40;

void release(qk_preproc* p) {
  if (!p) return;
  for (double* q : {p->mu, p->sigma, p->w, p->ymin, p->ymax, p->lam})
    if (q) (void)hipFree(q);
  delete p;
}

#define PP_HIP(call, what)                                                   \
  do {                                                                       \
    hipError_t e__ = (call);                                                 \
    if (e__ != hipSuccess) {                                                 \
      st = qk_fail(QK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e__)); \
      goto done;                                                             \
    }                                                                        \
  } while (0)

}  // namespace

extern "C" {

qk_status qk_preproc_fit(const double* x_dev, int64_t n, int64_t ld_x, int32_t d,
                         int32_t n_components, void* hip_stream, qk_preproc** out) {
  if (!out) return qk_fail(QK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!x_dev) return qk_fail(QK_ERR_INVALID_ARG, "x_dev is NULL");
  if (n < 2) return qk_fail(QK_ERR_INVALID_ARG, "need at least two training rows");
  if (d < 1 || d > 8192) return qk_fail(QK_ERR_INVALID_ARG, "d must be in [1, 8192]");
  if (ld_x < d) return qk_fail(QK_ERR_INVALID_ARG, "ld_x < d");
  if (n_components < 1 || n_components > d)
    return qk_fail(QK_ERR_INVALID_ARG, "n_components must be in [1, d]");
  if (n > (int64_t)INT32_MAX) return qk_fail(QK_ERR_INVALID_ARG, "more than 2^31 - 1 rows");
  hipStream_t s = (hipStream_t)hip_stream;
  qk_status st = QK_OK;
  auto* p = new qk_preproc();
  p->d = d;
  p->k = n_components;
  const int m = d + (d & 1);  // tournament players (a padding index when d is odd)
  double *z = nullptr, *c = nullptr, *v = nullptr, *y = nullptr, *od = nullptr;
  double4* rot = nullptr;
  int* perm = nullptr;
  double od_h[2] = {0.0, 0.0};
  double prev_off = INFINITY;
  bool converged = false;
  PP_HIP(hipMalloc((void**)&p->mu, d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&p->sigma, d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&p->w, (int64_t)n_components * d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&p->ymin, n_components * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&p->ymax, n_components * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&p->lam, d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&z, n * d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&c, (int64_t)d * d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&v, (int64_t)d * d * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&y, n * n_components * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&od, 2 * sizeof(double)), "allocation");
  PP_HIP(hipMalloc((void**)&rot, (m / 2) * sizeof(double4)), "allocation");
  PP_HIP(hipMalloc((void**)&perm, d * sizeof(int)), "allocation");
  PP_HIP(qk_launch_pp_colstats(x_dev, n, ld_x, d, p->mu, p->sigma, s), "column statistics");
  {
    // a non-finite feature makes a column statistic non-finite: refuse
    std::string buf((size_t)2 * d * sizeof(double), '\0');
    double* h = reinterpret_cast<double*>(&buf[0]);
    PP_HIP(hipMemcpyAsync(h, p->mu, d * sizeof(double), hipMemcpyDeviceToHost, s), "read back");
    PP_HIP(hipMemcpyAsync(h + d, p->sigma, d * sizeof(double), hipMemcpyDeviceToHost, s),
           "read back");
    PP_HIP(hipStreamSynchronize(s), "synchronise");
    for (int i = 0; i < 2 * d; ++i)
      if (!std::isfinite(h[i])) {
        st = qk_fail(QK_ERR_INVALID_ARG, "non-finite feature in the training rows");
        goto done;
      }
  }
  PP_HIP(qk_launch_pp_standardize(x_dev, n, ld_x, d, p->mu, p->sigma, z, s), "standardise");
  PP_HIP(qk_launch_pp_cov(z, n, d, c, s), "covariance");
  {
    // V = I
    std::string eye((size_t)d * d * sizeof(double), '\0');
    double* e = reinterpret_cast<double*>(&eye[0]);
    for (int i = 0; i < d; ++i) e[(int64_t)i * d + i] = 1.0;
    PP_HIP(hipMemcpyAsync(v, e, (size_t)d * d * sizeof(double), hipMemcpyHostToDevice, s),
           "identity upload");
    PP_HIP(hipStreamSynchronize(s), "synchronise");
  }
  // Converged when the off-diagonal Frobenius norm is below 1e-12 of the
  // whole (squared: 1e-24), or when it has stopped shrinking below 1e-8 of it
  // (clusters of equal eigenvalues, such as the null space of a covariance
  // of fewer rows than features, only trade rounding noise between
  // themselves; the components of separated eigenvalues are then accurate to
  // about 1e-8 of the norm over the gap).
  for (int sweep = 0; sweep < kMaxSweeps && d > 1; ++sweep) {
    PP_HIP(qk_launch_pp_offdiag(c, d, od, s), "off-diagonal mass");
    PP_HIP(hipMemcpyAsync(od_h, od, sizeof(od_h), hipMemcpyDeviceToHost, s), "read back");
    PP_HIP(hipStreamSynchronize(s), "synchronise");
    if (!(od_h[0] > 1e-24 * od_h[1]) ||
        (od_h[0] <= 1e-16 * od_h[1] && od_h[0] > 0.25 * prev_off)) {
      converged = true;
      break;
    }
    prev_off = od_h[0];
    for (int r = 0; r < m - 1; ++r)
      PP_HIP(qk_launch_pp_jacobi_round(c, v, d, m, r, rot, s), "Jacobi round");
    p->sweeps = sweep + 1;
  }
  if (d == 1) converged = true;
  if (!converged) {
    PP_HIP(qk_launch_pp_offdiag(c, d, od, s), "off-diagonal mass");
    PP_HIP(hipMemcpyAsync(od_h, od, sizeof(od_h), hipMemcpyDeviceToHost, s), "read back");
    PP_HIP(hipStreamSynchronize(s), "synchronise");
    if (!(od_h[0] <= 1e-16 * od_h[1])) {
      char msg[160];
      snprintf(msg, sizeof msg,
               "the Jacobi eigensolver reached its sweep limit (off-diagonal mass %.3e of "
               "the total after %d sweeps; previous sweep %.3e)",
               od_h[0] / od_h[1], kMaxSweeps, prev_off / od_h[1]);
      st = qk_fail(QK_ERR_DEVICE, msg);
      goto done;
    }
  }
  PP_HIP(qk_launch_pp_components(c, v, d, n_components, perm, p->lam, p->w, s), "components");
  PP_HIP(qk_launch_pp_project(z, n, d, p->w, n_components, y, s), "projection");
  PP_HIP(qk_launch_pp_minmax(y, n, n_components, p->ymin, p->ymax, s), "min / max");
  PP_HIP(hipStreamSynchronize(s), "synchronise");
done:
  for (void* q : {(void*)z, (void*)c, (void*)v, (void*)y, (void*)od, (void*)rot, (void*)perm})
    if (q) (void)hipFree(q);
  if (st != QK_OK) {
    release(p);
    return st;
  }
  *out = p;
  return QK_OK;
}

qk_status qk_preproc_apply(const qk_preproc* p, const double* x_dev, int64_t n, int64_t ld_x,
                           double scale, double* out_dev, int64_t ld_out, void* hip_stream) {
  if (!p) return qk_fail(QK_ERR_INVALID_ARG, "pre-processing handle is NULL");
  if (n < 0) return qk_fail(QK_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return QK_OK;
  if (!x_dev || !out_dev) return qk_fail(QK_ERR_INVALID_ARG, "NULL pointer");
  if (ld_x < p->d) return qk_fail(QK_ERR_INVALID_ARG, "ld_x < d");
  if (ld_out < p->k) return qk_fail(QK_ERR_INVALID_ARG, "ld_out < n_components");
  if (!std::isfinite(scale)) return qk_fail(QK_ERR_INVALID_ARG, "scale must be finite");
  hipStream_t s = (hipStream_t)hip_stream;
  qk_status st = QK_OK;
  double *z = nullptr, *y = nullptr;
  PP_HIP(hipMallocAsync((void**)&z, n * p->d * sizeof(double), s), "allocation");
  PP_HIP(hipMallocAsync((void**)&y, n * p->k * sizeof(double), s), "allocation");
  PP_HIP(qk_launch_pp_standardize(x_dev, n, ld_x, p->d, p->mu, p->sigma, z, s), "standardise");
  PP_HIP(qk_launch_pp_project(z, n, p->d, p->w, p->k, y, s), "projection");
  PP_HIP(qk_launch_pp_scale(y, n, p->k, p->ymin, p->ymax, scale, out_dev, ld_out, s), "scale");
done:
  if (z) (void)hipFreeAsync(z, s);
  if (y) (void)hipFreeAsync(y, s);
  return st;
}

qk_status qk_preproc_info(const qk_preproc* p, int32_t* d, int32_t* n_components,
                          int32_t* sweeps, double* eigvals_host) {
  if (!p) return qk_fail(QK_ERR_INVALID_ARG, "pre-processing handle is NULL");
  if (d) *d = p->d;
  if (n_components) *n_components = p->k;
  if (sweeps) *sweeps = p->sweeps;
  if (eigvals_host &&
      hipMemcpy(eigvals_host, p->lam, p->d * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return qk_fail(QK_ERR_HIP, "eigenvalue read");
  return QK_OK;
}

qk_status qk_preproc_release(qk_preproc* p) {
  if (p) (void)hipDeviceSynchronize();
  release(p);
  return QK_OK;
}

}  // extern "C"
