// Resolution of QK_PREC_AUTO and the tuning table filled by qk_autotune.
//
// The table maps (padded bond dimension T, site-count bucket ceil(log2 nq))
// to the fastest measured sweep form and persistent workgroups per CU.
// Without an entry, AUTO takes complex FP32 on MFMA for T <= 4 (the fastest
// form meeting the stated tolerance on MI355X in the measurements), else
// complex FP64.
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "qk_tune.h"

namespace {
std::mutex g_mu;
std::map<std::pair<int, int>, QkTuneEntry> g_table;
}  // namespace

int qk_tune_bucket(int nq) {
  int b = 0;
  while ((1 << b) < nq) ++b;
  return b;
}

bool qk_tune_lookup(int T, int nq, QkTuneEntry* e) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto f = g_table.find({T, qk_tune_bucket(nq)});
  if (f == g_table.end()) return false;
  *e = f->second;
  return true;
}

void qk_tune_store(int T, int nq, const QkTuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[{T, qk_tune_bucket(nq)}] = e;
}

std::string qk_tune_export_text() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  o.precision(6);
  for (auto& kv : g_table)
    o << kv.first.first << " " << kv.first.second << " " << (int)kv.second.form << " "
      << kv.second.wg_per_cu << " " << kv.second.band << " " << kv.second.us_per_tile << "\n";
  return o.str();
}

// One line per key: "T bucket form wg_per_cu band us_per_tile", or the older
// "T bucket form wg_per_cu us_per_tile" (band 4).
bool qk_tune_import_text(const std::string& text) {
  std::istringstream in(text);
  std::map<std::pair<int, int>, QkTuneEntry> t;
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::vector<double> v;
    double x;
    while (ls >> x) v.push_back(x);
    if (!ls.eof()) return false;
    if (v.empty()) continue;
    if (v.size() != 5 && v.size() != 6) return false;
    const int T = (int)v[0], b = (int)v[1], f = (int)v[2], wg = (int)v[3];
    const int band = v.size() == 6 ? (int)v[4] : 4;
    const double us = v.back();
    if (T < 1 || b < 0 || f < QK_PREC_FP64 || f > QK_PREC_FP32_MFMA || f == QK_PREC_AUTO ||
        wg < 1 || wg > 8 || band < 1 || band > 64)
      return false;
    t[{T, b}] = QkTuneEntry{(qk_precision)f, wg, band, us};
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : t) g_table[kv.first] = kv.second;
  return true;
}

qk_precision qk_tune_choose(int T, int nq, bool have_fp32, bool have_fp64) {
  QkTuneEntry e;
  if (qk_tune_lookup(T, nq, &e)) {
    if (e.form == QK_PREC_FP64 ? have_fp64 : have_fp32) return e.form;
  }
  if (have_fp32 && have_fp64 && (T == 1 || T == 2 || T == 4)) return QK_PREC_FP32_MFMA;
  if (have_fp32 && (T == 1 || T == 2 || T == 4)) return QK_PREC_FP32;
  return QK_PREC_FP64;
}
