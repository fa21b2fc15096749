// Iteration-budget calibration (paper Sec. IV-A): the batch runs every
// instance for the same number of iterations, so the budget is read off the
// distribution of the iterations the instances need: solve a large batch with
// the relative-decrease stop under a high cap and take the 99th percentile
// (for the zero-control warm start) and the median (for warm starts from a trained
// actor) of the per-instance iteration counts.
#include <algorithm>
#include <vector>

#include "runtime.hpp"

using namespace cbic;

#define HIP_TRY(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
      return CBIC_E_HIP;                                                \
    }                                                                   \
  } while (0)

namespace {

// nearest-rank percentile of sorted values: the smallest value with at least
// q percent of the values at or below it
int32_t nearest_rank(const std::vector<int32_t>& sorted, int q) {
  const size_t n = sorted.size();
  size_t rank = (size_t(q) * n + 99) / 100;  // ceil(q n / 100)
  if (rank < 1) rank = 1;
  return sorted[rank - 1];
}

}  // namespace

extern "C" cbic_status cbic_calibrate_max_iter(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t Tmax,
                                               const int32_t* d_T, const double* d_x0, const cbic_solve_opts* opts,
                                               int32_t cap, void* stream_v, int32_t* p99, int32_t* p50,
                                               int64_t* hist) {
  if (!ctx || !sys || !opts || !d_x0 || !p99 || !p50) {
    set_error("ctx, sys, opts, d_x0, p99 and p50 are required");
    return CBIC_E_INVALID;
  }
  if (B < 1 || Tmax < 1) {
    set_error("B and T_max must be >= 1");
    return CBIC_E_INVALID;
  }
  if (cap < 1 || cap > 100000) {
    set_error("cap must be in 1..100000");
    return CBIC_E_INVALID;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_v);
  HIP_TRY(hipSetDevice(ctx->device));
  const int n = sys->n, m = sys->m;
  // scratch outputs (a set-up call: it may allocate)
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
  cbic_solve_opts o = *opts;
  o.stop_mode = 1;
  o.max_iter = cap;
  o.flags &= ~CBIC_FLAG_TIMING;
  cbic_status rc = cbic_solve_batch(ctx, sys, B, Tmax, d_T, d_x0, nullptr, &o, &out, st);
  std::vector<int32_t> it(B);
  std::vector<uint32_t> stv(B);
  if (rc == CBIC_OK) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(it.data(), out.iters, B * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(stv.data(), out.status, B * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_error("reading the calibration solve's counts failed: %s", hipGetErrorString(e));
      rc = CBIC_E_HIP;
    }
  }
  (void)hipFree(buf);
  if (rc != CBIC_OK) return rc;
  // the dataset: every instance with a valid horizon; one stopped by the cap
  // counts as the cap
  std::vector<int32_t> v;
  v.reserve(B);
  for (int b = 0; b < B; ++b)
    if (!(stv[b] & CBIC_ST_BAD_INPUT)) v.push_back(it[b]);
  if (v.empty()) {
    set_error("no instance with a valid horizon");
    return CBIC_E_INVALID;
  }
  if (hist) {
    std::fill(hist, hist + cap + 1, int64_t(0));
    for (int32_t k : v) ++hist[std::min(std::max(k, 0), cap)];
  }
  std::sort(v.begin(), v.end());
  *p99 = nearest_rank(v, 99);
  *p50 = nearest_rank(v, 50);
  return CBIC_OK;
}
