// Matrix-core (MFMA) forms of the overlap sweep.
#include <hip/hip_runtime.h>

#include "qk_tune.h"

bool qk_mfma_supports(qk_precision, int) { return false; }
int qk_mfma_tile(qk_precision) { return 16; }
hipError_t qk_launch_sweep_mfma(const QkTaskTable&, qk_precision, int, hipStream_t) {
  return hipErrorInvalidValue;
}
