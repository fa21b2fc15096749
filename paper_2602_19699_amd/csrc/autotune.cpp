// Autotuner: times every candidate schedule on the caller's own problem (the
// lanes-per-instance widths of the lane schedule, one or two instances per
// compute unit of the workgroup schedule) and keeps the fastest per problem
// class in the context, where solves that leave the choice to the library
// (group_lanes, or wg_per_cu, 0) find it.
#include <cmath>
#include <cstdio>
#include <vector>

#include "runtime.hpp"

namespace cbic {

std::string tune_key(const cbic_system* sys, int B, int Tmax, const cbic_solve_opts* o) {
  int b2 = 1;
  while (b2 < B) b2 <<= 1;
  char k[192];
  std::snprintf(k, sizeof k, "%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d", sys->kind, sys->n, sys->m, o->precision,
                o->stop_mode, o->max_iter, o->ls_max_trials, b2, Tmax, o->regularization,
                std::isfinite(o->u_max) ? 1 : 0);
  return k;
}

}  // namespace cbic

using namespace cbic;

#define HIP_TRY(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
      return CBIC_E_HIP;                                                \
    }                                                                   \
  } while (0)

extern "C" cbic_status cbic_autotune(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t Tmax,
                                     const int32_t* d_T, const double* d_x0, const double* d_U0,
                                     const cbic_solve_opts* opts, void* stream_v, int32_t* best_group,
                                     double* best_ms) {
  if (!ctx || !sys || !opts || !d_x0) {
    set_error("ctx, sys, opts and d_x0 are required");
    return CBIC_E_INVALID;
  }
  if (B < 1 || Tmax < 1) {
    set_error("B and T_max must be >= 1");
    return CBIC_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_v);
  HIP_TRY(hipSetDevice(ctx->device));
  if (cbic_status rc = check_solve_opts(opts); rc != CBIC_OK) return rc;
  const Launcher* L = find_launcher(sys->kind, sys->n, sys->m, opts->precision, opts->schedule);
  if (!L) {
    set_error("no kernel for this system, precision and schedule");
    return CBIC_E_UNSUPPORTED;
  }
  const bool wg = L->schedule == CBIC_SCHED_GROUP;
  const int n = sys->n, m = sys->m;
  // scratch outputs for the trial solves (a set-up call: it may allocate)
  void* buf = nullptr;
  const size_t nX = size_t(B) * (Tmax + 1) * n, nU = size_t(B) * Tmax * m;
  const size_t bytes = (nX + nU + B) * sizeof(double) + 2 * size_t(B) * sizeof(int32_t) + 512;
  HIP_TRY(hipMalloc(&buf, bytes));
  char* p = static_cast<char*>(buf);
  cbic_outputs out{};
  out.X = reinterpret_cast<double*>(p);
  out.U = out.X + nX;
  out.J = out.U + nU;
  out.iters = reinterpret_cast<int32_t*>(out.J + B);
  out.status = reinterpret_cast<uint32_t*>(out.iters + B);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  cbic_solve_opts o = *opts;
  o.flags &= ~CBIC_FLAG_TIMING;
  int best = 0;
  float bms = 1e30f;
  cbic_status rc = CBIC_OK;
  std::vector<int> cand = {1, 2, 4, 8, 16};
  if (wg) cand = opts->precision == CBIC_FP64 ? std::vector<int>{1} : std::vector<int>{1, 2};
  for (int g : cand) {
    (wg ? o.wg_per_cu : o.group_lanes) = g;
    float mn = 1e30f;
    for (int rep = 0; rep < 3 && rc == CBIC_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) { rc = CBIC_E_HIP; break; }
      rc = cbic_solve_batch(ctx, sys, B, Tmax, d_T, d_x0, d_U0, &o, &out, st);
      if (rc != CBIC_OK) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = CBIC_E_HIP; break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < mn) mn = ms;  // the first run warms caches and allocations
    }
    if (rc != CBIC_OK) break;
    if (mn < bms) {
      bms = mn;
      best = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (rc != CBIC_OK) return rc;
  ctx->tuned[tune_key(sys, B, Tmax, opts)] = best;
  if (best_group) *best_group = best;
  if (best_ms) *best_ms = bms;
  return CBIC_OK;
}
