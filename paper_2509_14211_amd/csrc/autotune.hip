// Autotuner for the fused PageRank pass.
//
// The paper's runtime keys its compiled-kernel cache by a method signature
// and picks algorithms with cheap estimators that never change results
// (Section III-C, III-D).  Here the choice is the tile plan of the fused
// pass (workgroup or wavefront tiles, LDS hot slice, degree relabeling,
// grid size): candidates are timed on the matrix itself, the fastest is
// installed for it, and the result is remembered in a small text file keyed
// by the matrix signature (size, entries, largest and mean row length,
// value type), so a later process reuses it without timing again.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.h"

using namespace nbgrb;

namespace {

std::string signature(const MatP& A, int type) {
  // row-length sketch from the row pointers (host copy; one pass)
  std::vector<int> rp((size_t)A->nrows + 1);
  Ctx& c = ctx();
  hip_check(hipMemcpyAsync(rp.data(), A->rowptr->p, sizeof(int) * rp.size(), hipMemcpyDeviceToHost, c.stream),
            "copy row pointers");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  int64_t maxlen = 0;
  for (int64_t i = 0; i < A->nrows; ++i) maxlen = std::max<int64_t>(maxlen, rp[i + 1] - rp[i]);
  std::ostringstream s;
  s << "pr-fused t" << type << " n" << A->nrows << " m" << A->nnz << " max" << maxlen << " cus"
    << c.cus;
  return s.str();
}

bool read_cache(const std::string& path, const std::string& key, GrM_PlanConfig* out) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    // key|kernel lds_entries lds_rows long_row chunk grid hot relabel xcd_split|us
    const size_t a = line.find('|');
    const size_t b = line.rfind('|');
    if (a == std::string::npos || b == a) continue;
    if (line.substr(0, a) != key) continue;
    std::istringstream v(line.substr(a + 1, b - a - 1));
    GrM_PlanConfig c{};
    if (v >> c.kernel >> c.lds_entries >> c.lds_rows >> c.long_row >> c.chunk >> c.grid >> c.hot >> c.relabel) {
      if (!(v >> c.xcd_split)) c.xcd_split = 0;  // entries written before the field existed
      *out = c;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

void append_cache(const std::string& path, const std::string& key, const GrM_PlanConfig& c, double us) {
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << key << "|" << c.kernel << " " << c.lds_entries << " " << c.lds_rows << " " << c.long_row << " " << c.chunk
    << " " << c.grid << " " << c.hot << " " << c.relabel << " " << c.xcd_split << "|" << us << "\n";
}

PlanConfig to_plan(const GrM_PlanConfig& g) {
  PlanConfig p;
  p.kernel = g.kernel;
  p.lds_entries = g.lds_entries;
  p.lds_rows = g.lds_rows;
  p.long_row = g.long_row;
  p.chunk = g.chunk;
  p.grid = g.grid;
  p.hot = g.hot;
  p.relabel = g.relabel;
  p.xcd = g.xcd_split;
  return p;
}

}  // namespace

extern "C" {

GrB_Info GrM_autotune_pagerank(GrM_PlanConfig* chosen, double* us_per_pass, GrB_Matrix AT, GrB_Vector outdeg,
                               GrB_Type type, const char* cache_path) {
  try {
    require_init();
    if (!chosen || !AT || !outdeg || !type) fail(GrB_NULL_POINTER, "NULL argument");
    if (AT->magic != MAGIC_MAT || outdeg->magic != MAGIC_VEC) fail(GrB_UNINITIALIZED_OBJECT, "bad handle");
    const int T = type->code;
    if (T != T_FP32 && T != T_FP64) fail(GrB_DOMAIN_MISMATCH, "type must be FP32 or FP64");
    Ctx& c = ctx();
    const MatP A = AT->data;
    const std::string key = signature(A, T);
    GrM_PlanConfig best{};
    if (cache_path && *cache_path && read_cache(cache_path, key, &best)) {
      c.tuned[{A->id, T}] = to_plan(best);
      *chosen = best;
      if (us_per_pass) *us_per_pass = -1.0;
      return GrB_SUCCESS;
    }
    const int hmax = wave_hot_max(T);
    std::vector<GrM_PlanConfig> cands;
    for (int relabel = 0; relabel < 2; ++relabel) {
      cands.push_back({0, 2048, 1024, 2048, 2048, 0, 0, relabel, 0});
      cands.push_back({0, 2048, 1024, 2048, 2048, c.cus * 16, 0, relabel, 0});
      cands.push_back({0, 2048, 1024, 2048, 2048, c.cus * 16, 0, relabel, 1});
      cands.push_back({1, 512, 256, 512, 512, 0, 0, relabel, 0});
      cands.push_back({1, 512, 256, 512, 512, 0, hmax, relabel, 0});
      cands.push_back({1, 512, 256, 512, 512, 0, hmax, relabel, 1});
      cands.push_back({1, 512, 256, 128, 512, 0, hmax, relabel, 0});
      // stripe plans (FP32 ranks; the layout addresses < 2^30 columns and < 2^31 entries)
      if (T == T_FP32 && A->ncols < ((int64_t)1 << 30) && A->nnz < ((int64_t)1 << 31)) {
        cands.push_back({2, 0, 0, 1024, 0, 0, 0, relabel, 0});
        cands.push_back({2, 0, 0, 2048, 0, 0, 0, relabel, 0});
        // past the L2 of all XCDs (32 MiB of gathered values), also with the
        // packed entries read nontemporally
        if (A->ncols * 4 > ((int64_t)32 << 20)) cands.push_back({2, 0, 0, 1024, 1, 0, 0, relabel, 0});
        // two-phase: the entries outside the LDS blocks are filled by a
        // streaming phase instead of gathered
        cands.push_back({3, 0, 0, 1024, 0, 0, 0, relabel, 0});
        cands.push_back({3, 0, 0, 1024, 1, 0, 0, relabel, 0});
        cands.push_back({3, 0, 0, 2048, 0, 0, 0, relabel, 0});
        cands.push_back({3, 0, 0, 2048, 1, 0, 0, relabel, 0});
        cands.push_back({3, 0, 0, 4096, 0, 0, 0, relabel, 0});
      }
    }
    // Time k1 and k2 fused passes in one batch each (tol 0, no early stop);
    // the difference divided by k2 - k1 is the time of one pass.
    const int k1 = 3, k2 = 11;
    GrB_Vector rv = nullptr;
    GrB_Info info = GrB_Vector_new(&rv, type, (GrB_Index)A->nrows);
    if (info != GrB_SUCCESS) return info;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    double best_us = 1e300;
    bool any = false;
    // Each candidate's plan (some are as large as the matrix) is dropped
    // once it is timed, so only one is held at a time; a candidate whose
    // layout does not fit in memory is skipped.
    auto drop_plans = [&]() {
      hip_check(hipStreamSynchronize(c.stream), "sync");
      A->plans.clear();
      if (A->relabeled) A->relabeled->A->plans.clear();
    };
    for (const GrM_PlanConfig& cand : cands) {
      c.tuned[{A->id, T}] = to_plan(cand);
      double t[2] = {0, 0};
      int it = 0;
      double res = 0;
      // warm-up builds the plan (and the relabeled copy) outside the timing
      info = GrM_pagerank(rv, &it, &res, AT, outdeg, 0.85, 0.0, 2, GrM_DANGLING_UNIFORM, nullptr, 2);
      for (int j = 0; j < 2 && info == GrB_SUCCESS; ++j) {
        const int k = j == 0 ? k1 : k2;
        hip_check(hipEventRecord(e0, c.stream), "record");
        info = GrM_pagerank(rv, &it, &res, AT, outdeg, 0.85, 0.0, k, GrM_DANGLING_UNIFORM, nullptr, k);
        if (info != GrB_SUCCESS) break;
        hip_check(hipEventRecord(e1, c.stream), "record");
        hip_check(hipEventSynchronize(e1), "sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t[j] = ms;
      }
      drop_plans();
      if (info == GrB_OUT_OF_MEMORY) {
        info = GrB_SUCCESS;
        continue;
      }
      if (info != GrB_SUCCESS) break;
      const double us = (t[1] - t[0]) * 1e3 / (k2 - k1);
      if (!any || us < best_us) {
        best_us = us;
        best = cand;
        any = true;
      }
    }
    if (info == GrB_SUCCESS && !any) {
      info = GrB_OUT_OF_MEMORY;
      set_error_text("no candidate plan fits in memory");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    GrB_Vector_free(&rv);
    if (info != GrB_SUCCESS) return info;
    c.tuned[{A->id, T}] = to_plan(best);
    // The candidates' tile plans and layouts stay cached with the matrix
    // (some are as large as the matrix itself); drop them, and the
    // renumbered copy when the choice does not use it.  The chosen plan is
    // rebuilt on first use.
    hip_check(hipStreamSynchronize(c.stream), "sync");
    A->plans.clear();
    if (A->relabeled) {
      A->relabeled->A->plans.clear();
      if (!best.relabel) A->relabeled.reset();
    }
    if (cache_path && *cache_path) append_cache(cache_path, key, best, best_us);
    *chosen = best;
    if (us_per_pass) *us_per_pass = best_us;
    return GrB_SUCCESS;
  } catch (const GrbError& e) {
    set_error_text(e.msg);
    return e.info;
  } catch (const std::exception& e) {
    set_error_text(e.what());
    return GrB_PANIC;
  }
}

}  // extern "C"
