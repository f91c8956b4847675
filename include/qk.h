/*
 * qk.h -- C ABI of libqk: MPS quantum kernels, the RBF kernel and their
 * linear mix on one AMD Instinct MI355X (gfx950).
 *
 * Operations (paper: "Scalable Tensor Network Simulation for
 * Quantum-Classical Dual Kernel"):
 *   - encode every sample as a matrix-product state of the feature state
 *     |psi(x)> = U(x)|0...0> (Eq. (6), Section II-C);
 *   - fill Gram matrices of the quantum kernel K_q = |<psi(x)|psi(y)>|^2
 *     (Eq. (7); equivalently |<0|U^dagger(y)U(x)|0>|^2, Eqs. (8)-(10)),
 *     block by block (Section II-D, blockwise construction);
 *   - the classical RBF kernel K_c = exp(-gamma ||x - y||^2) (Eq. (3));
 *   - the dual kernel K = w K_q + (1 - w) K_c (Eq. (11); the paper's alpha).
 *
 * Conventions shared by every entry point:
 *   - Every function returns a qk_status; no C++ exception crosses the ABI.
 *     On failure qk_last_error() returns a thread-local message.
 *   - Pointers named *_dev are device pointers (HIP device memory of the
 *     current device); *_host are host pointers. Caller-owned buffers stay
 *     owned by the caller and must stay alive until the stream has finished
 *     the enqueued work. The library never frees or retains them.
 *   - Matrices are row-major with an explicit leading dimension in elements.
 *   - hip_stream is a hipStream_t (NULL = the default stream). Work is
 *     enqueued on it and the call returns; argument checks are synchronous
 *     and a rejected call enqueues nothing.
 *   - Errors found on the device (non-finite input, a bond dimension above
 *     the bound) are latched in the batch and reported by qk_mps_info().
 *   - Calls on different streams may run concurrently; an MPS batch is
 *     read-only after qk_mps_build() returns.
 */
#ifndef QK_H
#define QK_H

#include <stdint.h>

#if defined(__GNUC__)
#define QK_API __attribute__((visibility("default")))
#else
#define QK_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QK_OK = 0,
  QK_ERR_INVALID_ARG = -1,
  QK_ERR_OUT_OF_MEMORY = -2,
  QK_ERR_HIP = -3,
  QK_ERR_UNSUPPORTED = -4,
  QK_ERR_BUSY = -5,
  QK_ERR_CANCELLED = -6,
  QK_ERR_DEVICE = -7, /* a check latched on the device failed */
  QK_ERR_NOT_FOUND = -8
} qk_status;

/* Number format / engine of the overlap sweep. */
typedef enum {
  QK_PREC_FP64 = 0,      /* complex FP64 on VALU: the plain comparator     */
  QK_PREC_FP32 = 1,      /* complex FP32 on VALU                           */
  QK_PREC_BF16X2 = 2,    /* split BF16 (h+l, 4 products) on MFMA, FP32 acc  */
  QK_PREC_BF16X3 = 3,    /* split BF16 (exact h+m+l, 8 products) on MFMA    */
  QK_PREC_AUTO = 4,      /* tuned/default form at bonds <= 4; FP64 at 8..64 */
  QK_PREC_FP32_MFMA = 5  /* complex FP32 on v_mfma_f32_4x4x1_16b_f32       */
} qk_precision;

/* Which packed forms a batch keeps after qk_mps_build (bit mask). */
enum {
  QK_STORE_FP64 = 1, /* complex FP64 site tensors (needed by QK_PREC_FP64) */
  QK_STORE_FP32 = 2, /* complex FP32 site tensors (all other forms)        */
  QK_STORE_ALL = 3
};

/*
 * Encoding circuit (the block-structured feature map of Section II-C,
 * Fig. 1(B): single-qubit encoding layers interleaved with locally
 * restricted entangling layers); per layer:
 *   H on every qubit, RZ(2 x_k) on qubit k, then RZZ(theta_k) on (k, k+1),
 *   theta_k = 2 (pi - x_k)(pi - x_{k+1}), for every k = 0..n-2 whose pair
 *   lies inside one entangler block; repeated n_layers times with the same x.
 *   RZ(p) = exp(-i p Z/2), RZZ(t) = exp(-i t ZZ/2).
 * Entangler blocks: entangle = 1 is one block (the open chain over all
 * qubits); entangle = B >= 2 cuts the chain into blocks of B consecutive
 * qubits (pairs with (k + 1) % B == 0 get no gate), a block product state;
 * entangle = 0 drops every entangler.
 */
typedef struct {
  int32_t n_qubits;   /* = number of features d, >= 1                      */
  int32_t n_layers;   /* L >= 1                                             */
  int32_t chi_max;    /* bond-dimension cap, >= 1                           */
  int32_t entangle;   /* 0: none; 1: open chain; B >= 2: blocks of B qubits */
  double cutoff_rel;  /* keep singular values s_j > cutoff_rel * s_0, >= 0  */
} qk_circuit_desc;

typedef struct qk_mps_batch qk_mps_batch; /* opaque, device-resident, library-owned */

/*
 * qk_mps_build -- one MPS per sample (Eq. (6)).
 * Time-evolving block decimation in FP64 on the device (eight samples per
 * wavefront for chi_pad <= 4, one per wavefront at 8 and 16, one workgroup
 * of 8 chi_pad threads per sample at 32 and 64): per layer, the
 * single-qubit gates, then the RZZ chain as two-site
 * steps (merge, phase, one-sided Jacobi SVD, truncate at s_j > cutoff*s_0 and
 * chi_max, renormalise), sweeping left to right on odd and right to left on
 * even layers. Then the tensors are packed for the overlap sweep.
 *   c        circuit; the library bounds every bond by chi_ws =
 *            min(chi_max, 2^min(n_layers, floor(b/2))) with b the qubits of
 *            an entangler block (n_qubits for the open chain; chi_ws = 1
 *            when entangle = 0), the exact bond bound of this circuit family;
 *            tensors are padded to chi_pad = the power of two >= chi_ws;
 *            chi_ws <= 64 is supported (from 32 on, the build keeps a copy
 *            of each sample's merged matrix in a temporary device
 *            workspace of (2 chi_pad)^2 complex: 256 KB per sample at 64).
 *   x_dev    n_samples x n_qubits FP64 features, row-major, leading dim ld_x.
 *            Must be finite (checked on the device, reported by qk_mps_info).
 *   store    QK_STORE_* mask of packed forms to keep.
 *   out      receives a new batch; release it with qk_mps_release.
 * Errors: INVALID_ARG (bad desc, null pointers, ld_x < n_qubits),
 *         UNSUPPORTED (chi_ws > 64), OUT_OF_MEMORY, HIP.
 */
QK_API qk_status qk_mps_build(const qk_circuit_desc* c, const double* x_dev,
                       int64_t n_samples, int64_t ld_x, uint32_t store,
                       void* hip_stream, qk_mps_batch** out);

/*
 * qk_mps_build_many -- qk_mps_build for n_inputs feature matrices of the
 * same circuit (for example a training and a test set) in one device launch
 * where chi_pad <= 4, so the builds share the GPU without one launch
 * waiting behind the other. Input k: x_devs[k] (n_samples[k] x n_qubits
 * FP64, leading dimension ld_x[k]); out[k] receives its batch, the same
 * batch qk_mps_build would return for that input alone. 1 <= n_inputs <= 8;
 * x_devs, n_samples, ld_x and out are host arrays of n_inputs entries.
 * On error no batch is returned (every out[k] is NULL).
 * Errors as qk_mps_build; INVALID_ARG also for n_inputs outside [1, 8].
 */
QK_API qk_status qk_mps_build_many(const qk_circuit_desc* c, int32_t n_inputs,
                                   const double* const* x_devs, const int64_t* n_samples,
                                   const int64_t* ld_x, uint32_t store, void* hip_stream,
                                   qk_mps_batch** out);

/*
 * qk_mps_import -- test hook: upload MPS built elsewhere (e.g. on the host).
 *   chi_host     n_samples x (n_qubits+1) bond dimensions (chi_0 = chi_n = 1).
 *   tensors_host complex FP64 (re, im interleaved), layout
 *                [site k][sample i][s][a][b], a, b < chi_pad, zero outside
 *                the realized (chi_k, chi_{k+1}) block; chi_pad a power of 2,
 *                at most 64.
 * The copy is synchronous. Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
QK_API qk_status qk_mps_import(const qk_circuit_desc* c, int64_t n_samples,
                        int32_t chi_pad, const int32_t* chi_host,
                        const double* tensors_host, uint32_t store,
                        void* hip_stream, qk_mps_batch** out);

/*
 * qk_mps_info -- synchronises the batch's build stream, then reports the
 * sample count, qubit count, padded and largest realized bond dimension and
 * the device bytes held. Returns QK_ERR_DEVICE if the build latched an error
 * (non-finite input, a bond above chi_ws, or a two-site SVD that reached the
 * Jacobi sweep limit); qk_last_error() says which.
 * Any output pointer may be NULL.
 */
QK_API qk_status qk_mps_info(const qk_mps_batch* b, int64_t* n_samples,
                      int32_t* n_qubits, int32_t* chi_pad,
                      int32_t* chi_realized_max, int64_t* device_bytes);

/* Copies the realized bond table (n_samples x (n_qubits+1) int32) to host. */
QK_API qk_status qk_mps_chi(const qk_mps_batch* b, int32_t* chi_host);

/* Copies the per-sample discarded weight (n_samples FP64, host) of the
 * build: the sum over the sample's truncations of sum_{j >= keep} s_j^2 /
 * sum_j s_j^2, the singular values s of each merged two-site matrix in
 * descending order (cutoff and chi_max decide keep). The paper contracts the
 * overlap network exactly (Section II-C, Eqs. (8)-(10)); truncating the bonds
 * is this library's choice for circuits whose exact bonds exceed chi_max,
 * and this weight measures it. The state's squared error against the
 * untruncated circuit state is
 * bounded by about twice this sum, so it says how far a truncating build is
 * from the exact kernel. 0 for batches from qk_mps_import and for samples no
 * truncation touched beyond rounding noise. Synchronises the build stream. */
QK_API qk_status qk_mps_discarded(const qk_mps_batch* b, double* disc_host);

/* Frees the batch after waiting for all work on the device (sweeps on any
 * stream may read it). NULL is accepted. */
QK_API qk_status qk_mps_release(qk_mps_batch* b);

/*
 * Optional fusion of the RBF kernel (Eq. (3)) and the mix (Eq. (11)) into
 * the epilogue of the overlap sweep. x_rows_dev / x_cols_dev are the FP64
 * features the batches were built from (row-major, leading dims ld_xr,
 * ld_xc, d = n_qubits columns). kc_dev and k_dev are FP64 outputs laid out
 * like kq (either may be NULL to skip it). w_rows_dev (may be NULL) holds one
 * mixing weight per row sample and then overrides w: rows of different
 * requests batched into one launch keep their own weights.
 */
typedef struct {
  const double* x_rows_dev;
  int64_t ld_xr;
  const double* x_cols_dev;
  int64_t ld_xc;
  double gamma;
  double w;
  const double* w_rows_dev;
  double* kc_dev;
  int64_t ld_kc;
  double* k_dev;
  int64_t ld_k;
} qk_fuse_desc;

/*
 * qk_overlap_gram -- K_q for every pair (row sample i, column sample j)
 * (Eq. (7)) by the transfer-matrix sweep E_{k+1} = sum_s A_k^{s dagger} E_k
 * B_k^s, E_0 = 1, with an exact power-of-two rescale of E (after every site
 * in the VALU forms, every 8 sites in the matrix-core forms; a power of two
 * is exact, so the period does not change a normal value) and an int32
 * exponent; ln K_q = 2 (ln|E_n| + e ln 2) in FP64 and
 * K_q = exp(ln K_q) (0 once below the FP64 range).
 *   rows, cols   batches with the same qubit count and chi_pad.
 *   symmetric    1: rows == cols; only j >= i is contracted and both
 *                triangles are written (train x train); 0: full rectangle.
 *   prec         QK_PREC_*; QK_PREC_FP64 needs QK_STORE_FP64 in both batches.
 *                chi_pad 1, 2, 4: every form (tile kernels); chi_pad 8..64:
 *                QK_PREC_FP64 and QK_PREC_FP32_MFMA (one workgroup per
 *                pair; the FP32 form recomputes pairs with K_q above its
 *                refinement threshold in FP64).
 *   kq_dev       FP64 rows->n_samples x cols->n_samples output, ld_kq (may be
 *                NULL if lnkq_dev is given).
 *   lnkq_dev     FP64 ln K_q output, ld_ln (NULL to skip).
 *   fuse         NULL, or RBF + mix outputs as above.
 * Errors: INVALID_ARG, UNSUPPORTED (chi_pad not supported by prec), HIP.
 */
QK_API qk_status qk_overlap_gram(const qk_mps_batch* rows, const qk_mps_batch* cols,
                          int32_t symmetric, qk_precision prec, double* kq_dev,
                          int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                          const qk_fuse_desc* fuse, void* hip_stream);

/*
 * qk_overlap_gram_noalloc -- qk_overlap_gram for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, results and errors as
 * qk_overlap_gram (the same kernels run), but the refinement masks and pair
 * lists live in a static device array of QK_NOALLOC_SCRATCH_BYTES per GPU
 * (held from the first call on that GPU until the process ends) instead of
 * stream-ordered allocations; the call makes no hipMalloc / hipFree.
 * The scratch needed is 4 (9 t + 1) bytes for t 16 x 16 pair tiles under a
 * reduced form at chi_pad <= 4 (t = T(T+1)/2 of T = ceil(n/16) tile rows when
 * symmetric, else the product of the two tile counts), 8 (pairs + 1) bytes
 * for QK_PREC_FP32_MFMA at chi_pad 8..64, none for QK_PREC_FP64. A call that
 * needs more returns INVALID_ARG before anything is enqueued. All calls on
 * one GPU share its array, and the scratch is fully written before it is
 * read within a call, so calls in stream order are independent; calls that
 * overlap on one GPU (different streams, or host threads) race on it and
 * must be serialised by the caller. The stream must belong to the current
 * device.
 */
#define QK_NOALLOC_SCRATCH_BYTES (16 << 20)
QK_API qk_status qk_overlap_gram_noalloc(const qk_mps_batch* rows, const qk_mps_batch* cols,
                                         int32_t symmetric, qk_precision prec, double* kq_dev,
                                         int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                                         const qk_fuse_desc* fuse, void* hip_stream);

/*
 * One Gram block in a ragged multi-task launch: uneven qubit counts and
 * bond dimensions share one persistent launch. Fields as in
 * qk_overlap_gram.
 */
typedef struct {
  const qk_mps_batch* rows;
  const qk_mps_batch* cols;
  int32_t symmetric;
  double* kq_dev;
  int64_t ld_kq;
  double* lnkq_dev;
  int64_t ld_ln;
  qk_fuse_desc fuse;   /* used when use_fuse != 0 */
  int32_t use_fuse;
} qk_gram_task;

/*
 * qk_overlap_gram_multi -- all tasks in one persistent launch; tiles of all
 * tasks form one list in longest-processing-time order (cost n * chi^3).
 * QK_PREC_AUTO resolves every task on its own (as qk_resolve_precision), so
 * a task's result does not depend on the other tasks; tasks that resolve to
 * the same form share one launch, one launch per form in order of first
 * appearance. At most 16 tasks. Errors as qk_overlap_gram.
 */
QK_API qk_status qk_overlap_gram_multi(const qk_gram_task* tasks, int32_t n_tasks,
                                qk_precision prec, void* hip_stream);

/*
 * qk_rbf_gram -- K_c[i][j] = exp(-gamma sum_t (x_it - y_jt)^2) (Eq. (3)),
 * FP64, direct differences. x_dev: m x d (ld_x), y_dev: n x d (ld_y),
 * kc_dev: m x n (ld_kc). Errors: INVALID_ARG, HIP.
 */
QK_API qk_status qk_rbf_gram(const double* x_dev, int64_t m, int64_t ld_x,
                      const double* y_dev, int64_t n, int64_t ld_y, int32_t d,
                      double gamma, double* kc_dev, int64_t ld_kc,
                      void* hip_stream);

/*
 * qk_dual_mix -- K = w K_q + (1 - w) K_c elementwise (Eq. (11)), FP64,
 * m x n with separate leading dimensions; k_dev may alias kq_dev or kc_dev
 * when the leading dimensions agree. Errors: INVALID_ARG, HIP.
 */
QK_API qk_status qk_dual_mix(const double* kq_dev, int64_t ld_kq, const double* kc_dev,
                      int64_t ld_kc, int64_t m, int64_t n, double w,
                      double* k_dev, int64_t ld_k, void* hip_stream);

/*
 * qk_svm_decision -- decision values of an SVM on precomputed kernel rows
 * (Eqs. (4), (5)): f[r] = sum_i coef[i] K[r][i] + intercept, with coef[i] =
 * alpha_i y_i of the training samples (zero off the support vectors) and K
 * rows against the training set (for example the rows a serving request
 * returns). The predicted label of row r is sign(f[r]). FP64.
 *   k_dev      m x n kernel rows, leading dimension ld_k >= n.
 *   coef_dev   n coefficients (device).
 *   f_dev      m outputs (device).
 * Errors: INVALID_ARG (negative sizes, NULL pointers, ld_k < n, m >= 2^31,
 *         non-finite intercept), HIP.
 */
QK_API qk_status qk_svm_decision(const double* k_dev, int64_t m, int64_t n, int64_t ld_k,
                                 const double* coef_dev, double intercept, double* f_dev,
                                 void* hip_stream);

/*
 * qk_pathsum_gram -- the quantum kernel (Eqs. (7), (10)) of encoding
 * circuits (Eq. (6)) of one to three layers by exact path-sum evaluation, with
 * no MPS build and no truncation: every gate but H is diagonal, so the
 * overlap is a sum over computational-basis histories, evaluated as a chain
 * over the qubits of 2^(2L-1) states (2, 8 or 32) whose bond
 * factor splits into one 2 x 2 factor per history line. Complex FP64, one
 * pair per lane; exact power-of-two rescaling, so ln K_q is exact in range.
 * Equal, to rounding, to the MPS route wherever that route does not
 * truncate (chi_max >= 2^L); it costs about 150 FP64 operations per pair and
 * qubit at L = 2 against 2048 for the bond-4 sweep.
 *   x_rows_dev  m x d features (leading dimension ld_xr >= d); x_cols_dev
 *               n x d. symmetric = 1 needs the same pointer, m = n and
 *               ld_xr = ld_xc, contracts the upper triangle and mirrors it.
 *   n_layers    1, 2 or 3 (QK_ERR_UNSUPPORTED otherwise); entangle as in
 *               qk_circuit_desc (0 none, 1 open chain, B >= 2 blocks of B).
 *   kq_dev, lnkq_dev  optional m x n outputs (leading dimensions >= n).
 *   fuse        optional RBF (Eq. (3)) and mix (Eq. (11)) outputs as in
 *               qk_overlap_gram; its x fields are ignored (the RBF uses
 *               x_rows_dev / x_cols_dev).
 * Device scratch: (m + n) d 32 bytes of tables (m d when symmetric) from the
 * stream-ordered pool. Features must be finite. Errors: INVALID_ARG,
 * UNSUPPORTED, OUT_OF_MEMORY, HIP.
 */
QK_API qk_status qk_pathsum_gram(const double* x_rows_dev, int64_t m, int64_t ld_xr,
                                 const double* x_cols_dev, int64_t n, int64_t ld_xc, int32_t d,
                                 int32_t n_layers, int32_t entangle, int32_t symmetric,
                                 double* kq_dev, int64_t ld_kq, double* lnkq_dev, int64_t ld_ln,
                                 const qk_fuse_desc* fuse, void* hip_stream);

/*
 * qk_svm_fit_ovo -- trains the SVMs of Eqs. (1)-(2) on a precomputed kernel
 * matrix, one binary problem per pair of classes (one-against-one, Section
 * II-B), all problems in one launch (one workgroup each).
 *   k_dev       n x n symmetric kernel matrix of the training samples
 *               (device, leading dimension ld_k >= n), e.g. the dual kernel
 *               from qk_overlap_gram in symmetric mode.
 *   labels_host n class labels in [0, n_classes) (host, read before return);
 *               -1 leaves a sample out of training (its coefficients are 0),
 *               so the folds of a cross-validation train on one resident
 *               kernel matrix without copying submatrices.
 *   n_classes   2..64; P = n_classes (n_classes - 1) / 2 problems, ordered
 *               (0,1), (0,2), ..., (0,n_classes-1), (1,2), ...
 *   C           the box bound of Eq. (2); eps the stopping tolerance on the
 *               maximal KKT violation (LIBSVM's default is 1e-3); max_iter
 *               caps the SMO steps per problem.
 *   coef_dev    P x n output (device, leading dimension ld_coef >= n): row p
 *               holds alpha_t y_t at the samples of problem p (y = +1 for
 *               its first class) and 0 elsewhere, so qk_svm_decision with
 *               row p gives f_p = K_row . coef_p + b_p.
 *   intercept_dev  P biases b_p of Eq. (5) (device output).
 *   n_iter_dev  P SMO step counts (device output, int64); a count equal to
 *               max_iter means the problem stopped unconverged.
 * Method: SMO with the second-order pair selection of Fan, Chen and Lin
 * (2005), ties to the smallest sample index, each FP64 operation rounded
 * separately; b from the KKT conditions (mean over the free multipliers,
 * else the midpoint of the bounded interval). A problem's samples are those
 * of its two classes in increasing order. Device scratch (about 36 bytes
 * per sample per problem) comes from the stream-ordered pool. The call
 * blocks until the stream has reached the upload of the problem tables (it
 * waits for the work enqueued before it); training itself is asynchronous.
 * The kernel matrix must be finite. Errors: INVALID_ARG (sizes, NULL
 * pointers, labels outside [-1, n_classes), C / eps not positive and finite,
 * max_iter < 1), OUT_OF_MEMORY, HIP.
 */
#define QK_SVM_MAX_CLASSES 64
QK_API qk_status qk_svm_fit_ovo(const double* k_dev, int64_t n, int64_t ld_k,
                                const int32_t* labels_host, int32_t n_classes, double C,
                                double eps, int64_t max_iter, double* coef_dev, int64_t ld_coef,
                                double* intercept_dev, int64_t* n_iter_dev, void* hip_stream);

/*
 * qk_svm_predict_ovo -- one-against-one prediction from m kernel rows
 * against the n training samples (k_dev m x n, leading dimension ld_k >= n),
 * with the P coefficient rows and biases of qk_svm_fit_ovo. Writes the
 * decision values f (m x P, leading dimension ld_f >= P; NULL to skip) and
 * the voted labels (m int32; NULL to skip): problem (a, b) votes a when
 * f > 0, else b; the label is the class with most votes, ties to the
 * smaller class. One workgroup per row. FP64. Errors: INVALID_ARG (sizes,
 * NULL pointers, both outputs NULL), HIP.
 */
QK_API qk_status qk_svm_predict_ovo(const double* k_dev, int64_t m, int64_t n, int64_t ld_k,
                                    const double* coef_dev, int64_t ld_coef,
                                    const double* intercept_dev, int32_t n_classes, double* f_dev,
                                    int64_t ld_f, int32_t* labels_dev, void* hip_stream);

/*
 * Reduced-precision forms (QK_PREC_FP32, _FP32_MFMA, _BF16X2, _BF16X3) carry
 * a relative error of ~1e-5 (FP32-class) or ~2e-4 (BF16X2) in K_q after
 * hundreds of sites, which exceeds 1e-5 absolute only where K_q is large.
 * After such a sweep every pair whose K_q exceeds tau is recomputed by the
 * FP64 sweep (this needs QK_STORE_FP64 in the batches). The decision depends
 * only on that pair's own value, so a pair's result does not depend on which
 * other samples share its launch.
 * Defaults: tau = 1e-2 (FP32-class forms), 1e-3 (BF16X2). tau <= 0
 * disables refinement for that form. Process-wide setting.
 */
QK_API qk_status qk_set_refine_threshold(qk_precision prec, double tau);

/*
 * Jacobi sweep limit of the build's two-site SVDs (one-sided Jacobi: the
 * factorisation behind the bond truncation of each two-qubit gate step). A
 * build whose SVD has not converged after `sweeps` sweeps latches the
 * non-convergence flag, which qk_mps_info reports and the server turns into
 * a failed request. Default 60 (converged builds take 2 to 4 sweeps per SVD
 * at bond bounds <= 4; a host replay of the rotation rule on a 784-qubit,
 * 8-layer image counts up to 38 at bond 64, where the merged matrices are
 * strongly graded);
 * accepted range [0, 1000]; 0 makes every SVD report non-convergence.
 * Process-wide; applies to builds launched after the call.
 * Errors: INVALID_ARG.
 */
QK_API qk_status qk_set_svd_sweep_limit(int32_t sweeps);

/*
 * Pre-processing of raw features (Section II-A): z-score standardisation,
 * principal component analysis keeping the n leading components, min-max
 * scaling of each component to [0, 1]; the statistics are fitted on training
 * rows and applied to any rows. FP64 on the device.
 *
 * qk_preproc_fit -- fits on x_dev (n >= 2 training rows x d raw features,
 * row-major, leading dim ld_x >= d, caller-owned device memory):
 *   mu, sigma    column means and population standard deviations;
 *   components   the eigenvectors of the sample covariance Z^T Z / (n - 1) of
 *                the standardised rows Z for its n_components largest
 *                eigenvalues (cyclic two-sided Jacobi, FP64; ties in the
 *                ranking go to the smaller index), each with its entry of
 *                largest magnitude positive;
 *   min, max     of each projected component over the training rows.
 * Synchronous (the eigensolver checks convergence on the host each sweep).
 * d <= 8192, 1 <= n_components <= d. Device memory: the fitted statistics
 * (library-owned, (2 d + n_components (d + 2) + d) doubles), plus n d +
 * 2 d^2 + n n_components doubles of temporaries during the call.
 * Errors: INVALID_ARG, HIP, DEVICE (eigensolver sweep limit).
 */
typedef struct qk_preproc qk_preproc;
QK_API qk_status qk_preproc_fit(const double* x_dev, int64_t n, int64_t ld_x, int32_t d,
                                int32_t n_components, void* hip_stream, qk_preproc** out);

/* Applies a fit to n rows x_dev (leading dim ld_x >= d): z-score with the
 * fitted statistics (0 for constant training columns), projection on the
 * components, u = (y - min) / (max - min) (0 where max = min), times scale
 * (1 for the paper's [0, 1] angles, pi for [0, pi]); writes n x n_components
 * FP64 to out_dev (leading dim ld_out >= n_components). Rows other than the
 * training rows may fall outside [0, scale]. Asynchronous on hip_stream;
 * temporaries from the stream-ordered pool. Errors: INVALID_ARG, HIP. */
QK_API qk_status qk_preproc_apply(const qk_preproc* p, const double* x_dev, int64_t n,
                                  int64_t ld_x, double scale, double* out_dev, int64_t ld_out,
                                  void* hip_stream);

/* Sizes of a fit, the Jacobi sweeps it took, and (eigvals_host, d doubles,
 * nullable) the covariance eigenvalues in decreasing order. */
QK_API qk_status qk_preproc_info(const qk_preproc* p, int32_t* d, int32_t* n_components,
                                 int32_t* sweeps, double* eigvals_host);

/* Frees a fit after waiting for the device. NULL is accepted. */
QK_API qk_status qk_preproc_release(qk_preproc* p);

/*
 * qk_autotune -- times the sweep forms that meet the stated tolerance, each
 * at the launch shapes it admits, on the first max_tiles 16 x 16 tiles of
 * rows x cols (when these are all the tiles, each reduced form with its FP64
 * refinement pass as AUTO would run it, provided both batches hold FP64
 * tensors; on a partial slice the sweep alone), and records the fastest
 * (form, workgroups per CU, band height of the tile order) under the key
 * (chi_pad, ceil(log2 n_qubits)); QK_PREC_AUTO then resolves to that form
 * for every batch pair with that key, and launches of that form whose
 * dominant task has the key use that shape. Candidates where complex FP32
 * on the matrix cores applies: that form at bands of 2, 4 and 8 tile rows
 * with one or two workgroups per CU, and split BF16x3; complex FP64 (one or
 * two workgroups per CU) only when the slice is the whole job. Elsewhere:
 * complex FP64, and complex FP32 on VALU with 2..4 workgroups per CU at
 * chi_pad <= 4. The launch shape changes which workgroup computes which
 * tile, never a result. Synchronises the stream. Writes the winner to
 * *chosen (may be NULL).
 */
QK_API qk_status qk_autotune(const qk_mps_batch* rows, const qk_mps_batch* cols,
                             int32_t symmetric, int32_t max_tiles, void* hip_stream,
                             qk_precision* chosen);

/* Tuning table as text, one entry per line: "chi_pad bucket form wg_per_cu
 * band us_per_tile" (an entry without the band, five fields, imports with
 * band 4). Export writes at most cap bytes (NUL-terminated) and the needed
 * size to *len; import merges a table (INVALID_ARG if malformed, or a band
 * outside 1..64). */
QK_API qk_status qk_tune_export(char* buf, int64_t cap, int64_t* len);
QK_API qk_status qk_tune_import(const char* text);

/*
 * Launch timing for measurement. qk_set_launch_timing(1) makes every later
 * qk_overlap_gram / qk_overlap_gram_multi call record HIP events on its
 * stream around its sweep launch and around its FP64 refinement pass;
 * qk_last_launch_ms waits for the most recent such call's last event and
 * writes the two elapsed times in milliseconds (refine_ms = 0 when no
 * refinement ran). Process-wide, for one caller at a time; returns
 * QK_ERR_INVALID_ARG when timing is off or no timed call has been made.
 */
QK_API qk_status qk_set_launch_timing(int32_t enable);
QK_API qk_status qk_last_launch_ms(float* sweep_ms, float* refine_ms);

/* Resolves QK_PREC_AUTO for a batch pair: writes the form the library
 * would run (from the tuning table, else the built-in default). */
QK_API qk_status qk_resolve_precision(const qk_mps_batch* rows,
                               const qk_mps_batch* cols, qk_precision* out);

QK_API const char* qk_status_string(qk_status s);
QK_API const char* qk_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving: kernel rows of test requests against resident support sets.
 *
 * The blockwise Gram construction of Section II-D, run as a service: the
 * support samples of each feature dimension d are encoded once and stay in
 * device memory; each request carries 1..n test samples and a mixing weight
 * w and returns its rows of K = w K_q + (1 - w) K_c (Eqs. (3), (7), (11);
 * gamma = gamma_scale / d) against the support set of its d.
 *
 * Continuous batching: a worker thread admits queued requests in arrival
 * order while the HBM budget allows (per-request state: FP64 build workspace,
 * packed MPS, feature and output rows) and the row cap of an iteration is not
 * exceeded. One iteration encodes the admitted rows (one build per d) and
 * runs ONE persistent sweep launch over all of them (one task per d, per-row
 * w), then copies each request's rows to pinned host memory. Up to n_streams
 * iterations are in flight, so requests arriving while others run are
 * admitted as soon as a stream slot and budget free up. A pair's result does
 * not depend on the other rows of its iteration (per-pair arithmetic and
 * per-pair refinement), so a request's rows are identical alone and in a mix.
 * --------------------------------------------------------------------------- */
typedef struct qk_server qk_server;

typedef struct {
  int64_t budget_bytes;       /* device bytes for per-request state; 0 -> 1 GiB     */
  int32_t max_rows_per_iter;  /* rows admitted into one iteration; 0 -> 512        */
  int32_t n_streams;          /* iterations in flight, 1..4; 0 -> 2                 */
  qk_precision prec;          /* sweep form (QK_PREC_AUTO recommended)              */
  double gamma_scale;         /* gamma = gamma_scale / d; 0 -> 1                    */
} qk_server_config;

enum { QK_REQ_QUEUED = 0, QK_REQ_RUNNING = 1, QK_REQ_DONE = 2, QK_REQ_FAILED = 3,
       QK_REQ_CANCELLED = 4 };

/* Starts the worker thread on the current device. Errors: INVALID_ARG, HIP. */
QK_API qk_status qk_server_create(const qk_server_config* cfg, qk_server** out);

/* Encodes a support set for circuit c (keyed by c->n_qubits; one per d) and
 * keeps its MPS and a copy of its FP64 features (n x d, device rows x_dev,
 * leading dim ld_x) until qk_server_destroy. Synchronous. Support memory is
 * outside the budget. Errors: INVALID_ARG (duplicate d, bad desc), and those
 * of qk_mps_build. */
QK_API qk_status qk_server_load_support(qk_server* s, const qk_circuit_desc* c,
                                        const double* x_dev, int64_t n, int64_t ld_x);

/* Attaches a trained binary SVM (Eqs. (4), (5)) to the support set of
 * dimension d: coef_host holds n = support-size FP64 coefficients
 * alpha_i y_i (host, copied before the call returns; zero off the support
 * vectors), intercept is b. Requests admitted after the call also get their
 * decision values f[r] = sum_i coef[i] K[r][i] + b, computed on the device
 * from the iteration's kernel rows in the same stream (qk_server_poll_decision
 * returns them); requests already admitted keep the model they were admitted
 * with. coef_host NULL removes the model. Replaced coefficient arrays stay on
 * the device until qk_server_destroy. Errors: NOT_FOUND (no support set for
 * d), INVALID_ARG (n differs from the support size, non-finite value),
 * OUT_OF_MEMORY, HIP. */
QK_API qk_status qk_server_set_model(qk_server* s, int32_t d, const double* coef_host,
                                     int64_t n, double intercept);

/* Queues a request: n_rows x d FP64 features on the host (copied before the
 * call returns), mixing weight w in [0, 1]. Never waits for the GPU. Writes
 * the request id. Errors: NOT_FOUND (no support set for d), INVALID_ARG
 * (n_rows < 1, w outside [0, 1], non-finite feature). */
QK_API qk_status qk_server_submit(qk_server* s, const double* x_host, int64_t n_rows,
                                  int32_t d, double w, int64_t* id);

/* Output flags of qk_server_submit_ex. QK_OUT_LNKQ: the request also returns
 * its rows of ln K_q (FP64, -inf where the overlap amplitude is 0), the
 * faithful form of K_q for many qubits, where K_q itself falls below the
 * FP64 range (Eq. (7) at d = 784 reaches 1e-300 and less on these inputs). */
enum { QK_OUT_LNKQ = 1 };

/* As qk_server_submit, with extra outputs requested by `outputs` (QK_OUT_*
 * bits). The ln K_q rows count against the budget like the K rows and are
 * fetched with qk_server_poll_ex. Errors: those of qk_server_submit, and
 * INVALID_ARG for an unknown flag. */
QK_API qk_status qk_server_submit_ex(qk_server* s, const double* x_host, int64_t n_rows,
                                     int32_t d, double w, uint32_t outputs, int64_t* id);

/* Writes the request state (QK_REQ_*). When DONE and rows_host is not NULL,
 * copies its n_rows x n_support FP64 rows (leading dim ld_rows >= n_support)
 * and releases them; a later poll of that id returns NOT_FOUND. FAILED
 * carries the reason in qk_last_error(). */
QK_API qk_status qk_server_poll(qk_server* s, int64_t id, double* rows_host,
                                int64_t ld_rows, int32_t* state);

/* As qk_server_poll, and when DONE also copies the request's n_rows FP64
 * decision values to f_host if it is not NULL. Either output may be NULL; a
 * non-NULL one releases the request. Errors: INVALID_ARG (f_host given for a
 * request admitted while its support set had no model; nothing is released)
 * and those of qk_server_poll. */
QK_API qk_status qk_server_poll_decision(qk_server* s, int64_t id, double* rows_host,
                                         int64_t ld_rows, double* f_host, int32_t* state);

/* As qk_server_poll_decision, and when DONE also copies the request's
 * n_rows x n_support ln K_q rows (leading dim ld_ln >= n_support) to ln_host
 * if it is not NULL. Any non-NULL output releases the request. Errors:
 * INVALID_ARG (ln_host given for a request submitted without QK_OUT_LNKQ, or
 * ld_ln too small; nothing is released) and those of qk_server_poll_decision. */
QK_API qk_status qk_server_poll_ex(qk_server* s, int64_t id, double* rows_host,
                                   int64_t ld_rows, double* f_host, double* ln_host,
                                   int64_t ld_ln, int32_t* state);

/* Blocks until the request leaves QUEUED/RUNNING or timeout_ms passes
 * (< 0: no limit); writes the state. */
QK_API qk_status qk_server_wait(qk_server* s, int64_t id, int32_t timeout_ms, int32_t* state);

/* Cancels a queued or running request (running work completes on the device
 * and is discarded). Errors: NOT_FOUND. */
QK_API qk_status qk_server_cancel(qk_server* s, int64_t id);

/* Times of a request in seconds since qk_server_create: submitted, admitted
 * into an iteration, rows on the host (-1 if not reached). */
QK_API qk_status qk_server_request_times(qk_server* s, int64_t id, double* t_submit,
                                         double* t_admit, double* t_done);

/* Counters: requests done, iterations launched, peak budget bytes in use,
 * kernel entries (row x support pairs) delivered. Any pointer may be NULL. */
QK_API qk_status qk_server_stats(qk_server* s, int64_t* n_done, int64_t* n_iters,
                                 int64_t* peak_budget_bytes, int64_t* entries_done);

/* Stops admitting, drains in-flight iterations, frees everything. */
QK_API qk_status qk_server_destroy(qk_server* s);

#ifdef __cplusplus
}
#endif

#endif /* QK_H */
