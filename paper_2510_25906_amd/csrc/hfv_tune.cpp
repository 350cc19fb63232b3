// Launch-configuration autotuner (a project addition, not part of the paper's
// method): times the residual on the caller's own state for candidate launch
// configurations and keeps the fastest.  Every configuration computes the
// same states up to the order of floating-point sums, so tuning changes
// speed only.
//
// Search, coordinate by coordinate (each phase keeps the best of the previous):
//   1. the linear + NAD kernel's mapping: variables (1, 2 in 2D, nvar lanes),
//      stencil members or unknowns (2, 4, 8 lanes) per cell;
//   2. the class-list kernels: lanes per cell x block x grid (capped and
//      striding, or one list entry per lane group), in hybrid mode jointly
//      with whether CWENOZ reuses the linear pass's central fits and whether
//      the MUSCL and first-order lists ride in the CWENOZ launch (the best
//      lane count depends on both: FP64 on the 85k-cell mesh, two lanes
//      refitting and four lanes reusing are each best for their own setting)
//      (skipped when no cell can reach a class list's kernels in numbers,
//      i.e. in all-linear mode, where only first-order cells use them);
//   3. the fused (owner-computes) residual kernel against face fluxes + gather;
//   4. XCD-contiguous block order against plain block order;
//   5. in hybrid mode, when the MUSCL lists keep a launch of their own, its
//      lane count;
//   6. in the modes with class lists, the list kernels' tables read from
//      their cell-major copies against the [entry][cell] tables;
//   7. the four fastest configurations timed so far are timed again and the
//      fastest of that second timing is kept (among ~100 candidates the
//      fastest first timing is as likely a fast outlier as a fast launch).
// Each candidate runs once untimed, then three batches of `reps` calls back
// to back between HIP events; its score is the median batch's time per call.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hfv_internal.hpp"

namespace {

struct Tuner {
  hfv_ctx *ctx;
  const void *U;
  void *R;
  hipStream_t s;
  int reps;
  hipEvent_t ea, eb;
  std::vector<hfv_tune_record> rec;

  // residual time of configuration c in ms: three batches of `reps` calls
  // back to back (as a time loop runs them), the median batch's time per
  // call; +inf when c is rejected
  double time(const hfv_launch &c) {
    if (hfv_set_launch(ctx, &c) != HFV_OK) return INFINITY;
    if (hfv_residual(ctx, U, R, nullptr, nullptr, s) != HFV_OK) return INFINITY;
    if (hipStreamSynchronize(s) != hipSuccess) return INFINITY;
    std::vector<float> t;
    for (int i = 0; i < 3; ++i) {
      float ms = 0;
      if (hipEventRecord(ea, s) != hipSuccess) return INFINITY;
      for (int j = 0; j < reps; ++j)
        if (hfv_residual(ctx, U, R, nullptr, nullptr, s) != HFV_OK) return INFINITY;
      if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
          hipEventElapsedTime(&ms, ea, eb) != hipSuccess)
        return INFINITY;
      t.push_back(ms / reps);
    }
    std::sort(t.begin(), t.end());
    const double med = t[1];
    rec.push_back(hfv_tune_record{c, med});
    return med;
  }

  // best of the candidates (the earlier one on ties); `best` is updated in place
  void pick(const std::vector<hfv_launch> &cands, hfv_launch &best, double &best_ms) {
    for (const hfv_launch &c : cands) {
      const double ms = time(c);
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
};

}  // namespace

extern "C" hfv_status hfv_autotune(hfv_ctx *ctx, const void *U, int32_t reps, hfv_launch *best_out,
                                   hfv_tune_record *records, int32_t max_records, int32_t *n_records,
                                   void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  if (reps < 1 || reps > 1000) return ctx->err = "reps must be in [1, 1000]", HFV_ERR_PARAM;
  if (max_records < 0 || (max_records > 0 && !records)) return ctx->err = "bad record buffer", HFV_ERR_PARAM;
  hipStream_t s = (hipStream_t)stream;
  hfv_launch start;
  hfv_get_launch(ctx, &start);
  const int prof_mask = ctx->prof_mask;
  ctx->prof_mask = 0;  // tuning runs do not consume timing slots

  Tuner tu{ctx, U, nullptr, s, reps, nullptr, nullptr, {}};
  const size_t rbytes = (size_t)(ctx->prec == 64 ? 8 : 4) * ctx->nvar * ctx->N;
  hfv_status st = HFV_OK;
  if (hipMalloc(&tu.R, rbytes) != hipSuccess) {
    ctx->err = "autotune: residual buffer allocation failed";
    st = HFV_ERR_OOM;
  } else if (hipEventCreateWithFlags(&tu.ea, hipEventDisableSystemFence) != hipSuccess ||
             hipEventCreateWithFlags(&tu.eb, hipEventDisableSystemFence) != hipSuccess) {
    // timing-only events (no cache write-back and invalidation at each record)
    ctx->err = "autotune: event creation failed";
    st = HFV_ERR_HIP;
  }
  hfv_launch best = start;
  double best_ms = INFINITY;
  if (st == HFV_OK) {
    best_ms = tu.time(start);
    if (!std::isfinite(best_ms)) {
      ctx->err = "autotune: the starting configuration failed";
      st = HFV_ERR_HIP;
    }
  }
  if (st == HFV_OK) {
    std::vector<int> var_lanes = {1, ctx->nvar};
    if (ctx->dim == 2) var_lanes.push_back(2);
    // 1. linear kernel mapping
    std::vector<hfv_launch> cands;
    for (int l : var_lanes) {
      hfv_launch c = best;
      c.linear_split = 0;
      c.linear_lanes = l;
      cands.push_back(c);
    }
    for (int split = 1; split <= 2; ++split)
      for (int l : {2, 4, 8}) {
        hfv_launch c = best;
        c.linear_split = split;
        c.linear_lanes = l;
        cands.push_back(c);
      }
    tu.pick(cands, best, best_ms);
    // 2. class-list kernels and block size (with fit reuse and merged lists
    // in hybrid mode)
    if (ctx->p.mode != HFV_ALL_LINEAR) {
      const bool hyb = ctx->p.mode == HFV_HYBRID;
      cands.clear();
      for (int reuse = 0; reuse <= (hyb ? 1 : 0); ++reuse)
        for (int merged = 0; merged <= (hyb ? 1 : 0); ++merged)
          for (int l : var_lanes)
            for (int b : {128, 256})
              for (int lb : {0, 4, 8, 16}) {
                hfv_launch c = best;
                c.lanes_per_cell = l;
                c.block = b;
                c.list_blocks = lb * ctx->n_cu;
                if (hyb) {
                  c.cwenoz_reuse = reuse;
                  c.merged_lists = merged;
                }
                cands.push_back(c);
              }
      tu.pick(cands, best, best_ms);
    }
    // 3. residual kernel(s)
    {
      hfv_launch c = best;
      c.fused_residual = 1 - best.fused_residual;
      tu.pick({c}, best, best_ms);
    }
    // 4. block order
    {
      hfv_launch c = best;
      c.xcd_remap = 1 - best.xcd_remap;
      tu.pick({c}, best, best_ms);
    }
    // 5. MUSCL lanes (0 = as the other class-list kernels)
    if (ctx->p.mode == HFV_HYBRID && !best.merged_lists) {
      cands.clear();
      for (int l : var_lanes)
        if (l != best.lanes_per_cell) {
          hfv_launch c = best;
          c.muscl_lanes = l;
          cands.push_back(c);
        }
      tu.pick(cands, best, best_ms);
    }
    // 6. layout of the class-list kernels' table reads
    if (ctx->p.mode != HFV_ALL_LINEAR) {
      hfv_launch c = best;
      c.lists_cell_major = 1 - best.lists_cell_major;
      tu.pick({c}, best, best_ms);
    }
    // 7. confirmation of the fastest few
    {
      std::vector<hfv_tune_record> top(tu.rec);
      std::sort(top.begin(), top.end(),
                [](const hfv_tune_record &x, const hfv_tune_record &y) { return x.ms < y.ms; });
      std::vector<hfv_launch> few;
      for (const hfv_tune_record &r : top) {
        bool seen = false;
        for (const hfv_launch &c : few) seen = seen || std::memcmp(&c, &r.cfg, sizeof c) == 0;
        if (!seen) few.push_back(r.cfg);
        if (few.size() == 4) break;
      }
      double again_ms = INFINITY;
      hfv_launch again = best;
      for (const hfv_launch &c : few) {
        const double ms = tu.time(c);
        if (ms < again_ms) {
          again_ms = ms;
          again = c;
        }
      }
      if (std::isfinite(again_ms)) {
        best = again;
        best_ms = again_ms;
      }
    }
    if (hfv_set_launch(ctx, &best) != HFV_OK) st = HFV_ERR_PARAM;
  } else {
    (void)hfv_set_launch(ctx, &start);
  }
  if (tu.ea) (void)hipEventDestroy(tu.ea);
  if (tu.eb) (void)hipEventDestroy(tu.eb);
  if (tu.R) (void)hipFree(tu.R);
  ctx->prof_mask = prof_mask;
  if (best_out) *best_out = best;
  const int n = std::min<int>((int)tu.rec.size(), max_records);
  for (int i = 0; i < n; ++i) records[i] = tu.rec[i];
  if (n_records) *n_records = (int32_t)tu.rec.size();
  return st;
}
