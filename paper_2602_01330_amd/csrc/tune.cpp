// Resolution of QK_PREC_AUTO.
#include "qk_tune.h"

qk_precision qk_tune_choose(int T, int nq, bool have_fp32, bool have_fp64) {
  (void)nq;
  if (have_fp32 && (T == 1 || T == 2 || T == 4)) return QK_PREC_FP32;
  (void)have_fp64;
  return QK_PREC_FP64;
}
