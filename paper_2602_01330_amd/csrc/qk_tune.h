// Sweep-form selection and the MFMA sweep launcher.
#pragma once

#include <string>

#include "qk_internal.h"

// True if the MFMA sweep of form p is instantiated for padded bond T.
bool qk_mfma_supports(qk_precision p, int T);
// Pair-tile edge (rows = columns) the MFMA sweep of form p uses.
int qk_mfma_tile(qk_precision p);
// FP32 form: wg_per_cu persistent workgroups per CU (1 or 2).
hipError_t qk_launch_sweep_mfma(const QkTaskTable& tt, qk_precision p, int cus, int wg_per_cu,
                                uint32_t* mask, double ln_tau, hipStream_t s);

// QK_PREC_AUTO: the form to run for batches with padded bond T and nq sites.
qk_precision qk_tune_choose(int T, int nq, bool have_fp32, bool have_fp64);

// Tuning table: (T, ceil(log2(nq))) -> fastest form and its launch shape
// measured by qk_autotune: persistent workgroups per CU and tile rows per
// band of the tile order (the shape of the block of tiles one XCD works on).
struct QkTuneEntry {
  qk_precision form;
  int wg_per_cu;
  int band;
  double us_per_tile;
};
int qk_tune_bucket(int nq);
bool qk_tune_lookup(int T, int nq, QkTuneEntry* e);
void qk_tune_store(int T, int nq, const QkTuneEntry& e);
std::string qk_tune_export_text();
bool qk_tune_import_text(const std::string& text);
