// Sweep-form selection and the MFMA sweep launcher.
#pragma once

#include "qk_internal.h"

// True if the MFMA sweep of form p is instantiated for padded bond T.
bool qk_mfma_supports(qk_precision p, int T);
// Pair-tile edge (rows = columns) the MFMA sweep of form p uses.
int qk_mfma_tile(qk_precision p);
hipError_t qk_launch_sweep_mfma(const QkTaskTable& tt, qk_precision p, int cus,
                                uint32_t* mask, double ln_tau, hipStream_t s);

// QK_PREC_AUTO: the form to run for batches with padded bond T and nq sites.
qk_precision qk_tune_choose(int T, int nq, bool have_fp32, bool have_fp64);
