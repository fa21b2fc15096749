// extern "C" entry points of include/cbic.h: argument validation, context and
// system objects, workspace management and the batched solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <map>
#include <mutex>
#include <string>

#include "runtime.hpp"

namespace cbic {
const char* last_error();
bool make_device_block(cbic_system* s, double eps);
bool build_device_block(const cbic_system* s, double eps, std::vector<double>& d);
bool validate_params(int kind, const double* p, size_t np, int* n, int* m);
}  // namespace cbic

using namespace cbic;

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                    \
      return CBIC_E_HIP;                                                           \
    }                                                                              \
  } while (0)

namespace cbic {

cbic_status check_solve_opts(const cbic_solve_opts* o) {
  if (!o) { set_error("opts is NULL"); return CBIC_E_INVALID; }
  if (o->struct_size != sizeof(cbic_solve_opts)) {
    set_error("opts.struct_size is %u, expected %zu", o->struct_size, sizeof(cbic_solve_opts));
    return CBIC_E_INVALID;
  }
  if (o->max_iter < 0) { set_error("max_iter must be >= 0"); return CBIC_E_INVALID; }
  if (!(o->psd_eps >= 0.0) || !std::isfinite(o->psd_eps)) { set_error("psd_eps must be finite and >= 0"); return CBIC_E_INVALID; }
  if (o->ls_max_trials < 0) { set_error("ls_max_trials must be >= 0"); return CBIC_E_INVALID; }
  if (!(o->ls_beta > 0.0 && o->ls_beta < 1.0)) { set_error("ls_beta must be in (0,1)"); return CBIC_E_INVALID; }
  if (o->stop_mode != 0 && o->stop_mode != 1) { set_error("stop_mode must be 0 or 1"); return CBIC_E_INVALID; }
  if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) { set_error("rtol must be finite and >= 0"); return CBIC_E_INVALID; }
  if (o->precision != CBIC_FP64 && o->precision != CBIC_MIXED) { set_error("precision must be 0 or 1"); return CBIC_E_INVALID; }
  if (o->schedule < 0 || o->schedule > CBIC_SCHED_GROUP) { set_error("unknown schedule %d", o->schedule); return CBIC_E_INVALID; }
  if (o->group_lanes != 0 && o->group_lanes != 1 && o->group_lanes != 2 && o->group_lanes != 4 &&
      o->group_lanes != 8 && o->group_lanes != 16) {
    set_error("group_lanes must be 0, 1, 2, 4, 8 or 16");
    return CBIC_E_INVALID;
  }
  if (o->wg_per_cu < 0 || o->wg_per_cu > 2) { set_error("wg_per_cu must be 0, 1 or 2"); return CBIC_E_INVALID; }
  if (o->regularization != CBIC_REG_CLIP && o->regularization != CBIC_REG_LM) {
    set_error("regularization must be CBIC_REG_CLIP or CBIC_REG_LM");
    return CBIC_E_INVALID;
  }
  if (o->regularization == CBIC_REG_LM &&
      (!(o->lm_mu0 > 0.0) || !std::isfinite(o->lm_mu0) || !(o->lm_factor > 1.0) || !std::isfinite(o->lm_factor) ||
       !(o->lm_mu_max >= o->lm_mu0) || !std::isfinite(o->lm_mu_max))) {
    set_error("Levenberg-Marquardt needs finite lm_mu0 > 0, lm_factor > 1 and lm_mu_max >= lm_mu0");
    return CBIC_E_INVALID;
  }
  if (!(o->u_max > 0.0)) { set_error("u_max must be > 0 (+infinity: unbounded)"); return CBIC_E_INVALID; }
  return CBIC_OK;
}

// the solve's parameters; the Levenberg-Marquardt variant clips nothing, which
// the kernels read from a negative eps
SolveParamsH solve_params(const cbic_solve_opts* o) {
  SolveParamsH sp{o->max_iter, o->ls_max_trials, o->stop_mode, o->lookahead_K, o->psd_eps, o->ls_beta, o->rtol};
  if (o->regularization == CBIC_REG_LM) {
    sp.eps = -INFINITY;
    sp.reg = 1;
    sp.mu0 = o->lm_mu0;
    sp.mu_fac = o->lm_factor;
    sp.mu_max = o->lm_mu_max;
  }
  sp.umax = o->u_max;
  return sp;
}

}  // namespace cbic

namespace {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

size_t a256(size_t b) { return (b + 255) / 256 * 256; }

// scratch behind the solver's workspace: the horizon sort's histogram and
// permutation, then the iteration order's slot list
size_t sort_bytes(int B, int Tmax) {
  return a256((size_t(Tmax) + 1) * 4) + a256(size_t(B) * 4) + a256(size_t(B) * 4);
}

cbic_status ensure_ws(cbic_context* ctx, size_t need) {
  if (need <= ctx->ws_bytes) return CBIC_OK;
  if (ctx->cap && need > ctx->cap) {
    set_error("workspace of %zu bytes exceeds the context cap of %zu bytes", need, ctx->cap);
    return CBIC_E_OOM;
  }
  if (ctx->ws) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    set_error("hipMalloc of %zu workspace bytes failed: %s", need, hipGetErrorString(e));
    return CBIC_E_OOM;
  }
  ctx->ws_bytes = need;
  // cached graphs refer to the old workspace
  for (auto& kv : ctx->graphs) {
    if (kv.second.ge) (void)hipGraphExecDestroy(kv.second.ge);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  ctx->graphs.clear();
  return CBIC_OK;
}

// Checks shared by both solve entry points (nothing is launched before they
// pass); *L receives the launcher of the system, precision and schedule.
cbic_status check_solve(cbic_context* ctx, const cbic_system* sys, int B, int Tmax, const int32_t* d_T,
                        const double* d_x0, const double* d_U0, const cbic_solve_opts* opts,
                        const cbic_outputs* out, const Launcher** L) {
  if (!ctx || !sys) { set_error("ctx and sys are required"); return CBIC_E_INVALID; }
  if (sys->ctx != ctx || !sys->d_prm) { set_error("sys was not created on this context"); return CBIC_E_INVALID; }
  if (B < 1 || Tmax < 1) { set_error("B and T_max must be >= 1 (got %d, %d)", B, Tmax); return CBIC_E_INVALID; }
  if (!d_x0) { set_error("d_x0 is required"); return CBIC_E_INVALID; }
  if (!out || !out->X || !out->U || !out->J || !out->iters || !out->status) {
    set_error("outputs X, U, J, iters and status are required");
    return CBIC_E_INVALID;
  }
  const void* ptrs[] = {d_T, d_x0, d_U0, out->X, out->U, out->J, out->iters, out->status,
                        out->Vbar, out->Vx, out->xK, out->cost_trace, out->work, out->jtrace};
  for (const void* p : ptrs)
    if (p && !aligned8(p) && p != d_T && p != out->iters && p != out->status && p != out->work &&
        p != out->jtrace) {
      set_error("device pointers must be 8-byte aligned");
      return CBIC_E_INVALID;
    }
  if ((d_T && (reinterpret_cast<uintptr_t>(d_T) & 3u)) || (reinterpret_cast<uintptr_t>(out->iters) & 3u) ||
      (reinterpret_cast<uintptr_t>(out->status) & 3u) || (out->work && (reinterpret_cast<uintptr_t>(out->work) & 3u)) ||
      (out->jtrace && (reinterpret_cast<uintptr_t>(out->jtrace) & 3u))) {
    set_error("int32 device pointers must be 4-byte aligned");
    return CBIC_E_INVALID;
  }
  cbic_status st = check_solve_opts(opts);
  if (st) return st;
  *L = find_launcher(sys->kind, sys->n, sys->m, opts->precision, opts->schedule);
  if (!*L) {
    set_error("no kernel for system kind %d (n=%d, m=%d), precision %d, schedule %d", sys->kind, sys->n,
              sys->m, opts->precision, opts->schedule);
    return CBIC_E_UNSUPPORTED;
  }
  return CBIC_OK;
}

// The device parameter block of a solve with clip floor eps: the system's own
// block, or for an LQ system whose clipped constant Hessians were built for
// another eps, the block for that eps (built, uploaded on the solve's stream
// and kept on first use when may_build; CBIC_E_INVALID otherwise).  No device
// synchronisation: solves with other floors on other streams keep their blocks.
cbic_status param_block(cbic_system* s, double eps, hipStream_t stream, bool may_build, const double** out) {
  if (s->kind != CBIC_SYS_LQ || s->dev_eps == eps) {
    *out = s->d_prm;
    return CBIC_OK;
  }
  auto it = s->lq_blocks.find(eps);
  if (it == s->lq_blocks.end()) {
    if (!may_build) {
      set_error("no parameter block of this LQ system for psd_eps %g yet (cbic_solve_batch builds it)", eps);
      return CBIC_E_INVALID;
    }
    std::vector<double> h;
    if (!build_device_block(s, eps, h)) {
      set_error("cannot build the LQ parameter block");
      return CBIC_E_INVALID;
    }
    double* d = nullptr;
    hipError_t e = hipMalloc(&d, h.size() * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of the LQ parameter block failed: %s", hipGetErrorString(e));
      return CBIC_E_OOM;
    }
    it = s->lq_blocks.emplace(eps, std::make_pair(std::move(h), d)).first;
    HIP_TRY(hipMemcpyAsync(d, it->second.first.data(), it->second.first.size() * sizeof(double),
                           hipMemcpyHostToDevice, stream));
  }
  *out = it->second.second;
  return CBIC_OK;
}

// Enqueue one solve on `stream` with its workspace at `base`: ws_main bytes
// of the launcher's layout followed by the horizon sort's scratch.  The caller
// holds ctx->mu with the context's device current.  Allocates nothing itself
// (a graph launch builds its cached graph on first use).
cbic_status enqueue_solve(cbic_context* ctx, const cbic_system* sys, const double* prm, const Launcher* L,
                          const SolveParamsH& sp, int B, int Tmax, const int32_t* d_T, const double* d_x0,
                          const double* d_U0, const cbic_solve_opts* opts, const cbic_outputs* out, char* base,
                          size_t ws_main, hipStream_t stream) {
  // the launches below report through hipGetLastError: drop an error another
  // call on this thread left behind
  (void)hipGetLastError();
  char* sb = base + ws_main;
  int32_t* hist = reinterpret_cast<int32_t*>(sb);
  sb += a256((size_t(Tmax) + 1) * 4);
  int32_t* perm = reinterpret_cast<int32_t*>(sb);
  sb += a256(size_t(B) * 4);
  int32_t* order = reinterpret_cast<int32_t*>(sb);
  if (d_T) HIP_TRY(launch_horizon_sort(d_T, B, Tmax, hist, perm, stream));
  else perm = nullptr;

  const bool timing = (opts->flags & CBIC_FLAG_TIMING) != 0;
  if (timing) HIP_TRY(hipEventRecord(ctx->phase_ev[0], stream));
  // iterations that never run keep the marker -2
  if (out->jtrace && opts->max_iter > 0) HIP_TRY(launch_fill_i32(out->jtrace, size_t(B) * opts->max_iter, -2, stream));
  const IterTrace tr{out->cost_trace, out->jtrace};
  HIP_TRY(L->init(prm, base, B, Tmax, B, nullptr, Tmax, d_T, perm, d_x0, d_U0, opts->max_iter,
                  out->cost_trace, sp.umax, stream));
  // the iteration launches take the slots in the order of expected work
  // (longest horizon, then highest initial cost first, then highest
  // non-convex share of it) unless the caller asks for the horizon sort's
  // order; results are the same either way
  if ((opts->flags & CBIC_FLAG_INPUT_ORDER) || opts->max_iter <= 0 || !cost_order_supported(d_T != nullptr, Tmax)) {
    order = nullptr;
  } else {
    const LaneLayout lay = lane_layout(L->N, L->M, L->elem, B, Tmax, L->nbuf);
    HIP_TRY(launch_cost_order(reinterpret_cast<const uint32_t*>(base + lay.okey), B, Tmax, d_T != nullptr, order,
                              stream));
  }
  if (timing) HIP_TRY(hipEventRecord(ctx->phase_ev[1], stream));
  int group = requested_group(L, opts);
  if (group <= 0) {
    auto it = ctx->tuned.find(tune_key(sys, B, Tmax, opts));
    group = it != ctx->tuned.end() ? it->second : default_group(L->schedule, B, opts->precision, ctx->device);
  }
  if (opts->max_iter > 0) {
    const int G = opts->iters_per_launch > 0 ? std::min(opts->iters_per_launch, opts->max_iter) : opts->max_iter;
    const int chunks = (opts->max_iter + G - 1) / G;
    const bool graph = (opts->flags & CBIC_FLAG_GRAPH) && stream != nullptr;
    if (!graph && chunks == 1 && L->iterate_final) {
      // one launch: every group finalises its slot as soon as it stops
      // iterating (the finalisation then overlaps the other groups'
      // iterations; the same results as the two launches below).  Timed,
      // the finalisation counts with the iterations and its own phase is 0.
      const FinalOutH fo{out->X,    out->U,  out->J,  out->iters,      out->status,
                         out->Vbar, out->Vx, out->xK, out->cost_trace, out->work};
      HIP_TRY(L->iterate_final(prm, base, B, Tmax, B, order, sp, G, group, tr, Tmax, opts->lookahead_K, fo,
                               stream));
      if (timing) {
        HIP_TRY(hipEventRecord(ctx->phase_ev[2], stream));
        HIP_TRY(hipEventRecord(ctx->phase_ev[3], stream));
      }
      ctx->timed = ctx->timed || timing;
      return CBIC_OK;
    }
    if (!graph) {
      for (int c = 0; c < chunks; ++c)
        HIP_TRY(L->iterate(prm, base, B, Tmax, B, order, sp, G, group, tr, stream));
    } else {
      char key[512];
      std::snprintf(key, sizeof key,
                    "%p|%p|%p|%p|%d|%d|%d|%d|%d|%d|%d|%d|%.17g|%.17g|%.17g|%p|%p|%d|%.17g|%.17g|%.17g|%.17g",
                    (const void*)L, (const void*)prm, (const void*)base, (const void*)order, B, Tmax, G, chunks, group,
                    sp.max_iter, sp.ls_trials, sp.stop_mode, sp.eps, sp.beta, sp.rtol, (void*)out->cost_trace,
                    (void*)out->jtrace, sp.reg, sp.mu0, sp.mu_fac, sp.mu_max, sp.umax);
      auto it = ctx->graphs.find(key);
      if (it == ctx->graphs.end()) {
        cbic_context::GraphEntry ge;
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int c = 0; c < chunks && e == hipSuccess; ++c)
          e = L->iterate(prm, base, B, Tmax, B, order, sp, G, group, tr, stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          set_error("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
          return CBIC_E_HIP;
        }
        ge.g = g;
        HIP_TRY(hipGraphInstantiate(&ge.ge, g, nullptr, nullptr, 0));
        it = ctx->graphs.emplace(key, ge).first;
      }
      HIP_TRY(hipGraphLaunch(it->second.ge, stream));
    }
  }
  if (timing) HIP_TRY(hipEventRecord(ctx->phase_ev[2], stream));
  FinalOutH fo{out->X, out->U, out->J, out->iters, out->status, out->Vbar, out->Vx, out->xK, out->cost_trace,
               out->work};
  HIP_TRY(L->finalize(prm, base, B, Tmax, B, nullptr, Tmax, opts->max_iter, opts->lookahead_K, fo, stream));
  if (timing) HIP_TRY(hipEventRecord(ctx->phase_ev[3], stream));
  ctx->timed = ctx->timed || timing;
  return CBIC_OK;
}

// ---------------------------------------------------------------- allocation-free scratch
// The workspace of cbic_solve_batch_noalloc: a file-scope device array, part
// of the library's code object, so each GPU the library runs on holds one
// copy from module load until the process ends.  In host code its name is
// not a device address; each context takes its device's address from
// hipGetSymbolAddress at creation (scratch_address) and uses only that.
constexpr size_t kScratchBytes = size_t(CBIC_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The array's address on the current device (looked up once per device).
cbic_status scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    it = addr.emplace(device, p).first;
  }
  *out = it->second;
  return CBIC_OK;
}

}  // namespace

cbic_status context_aux(cbic_context* ctx, size_t need, void** p) {
  if (need > ctx->aux_bytes) {
    if (ctx->aux) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->aux));
      ctx->aux = nullptr;
      ctx->aux_bytes = 0;
    }
    const size_t bytes = std::max<size_t>(need, 64 << 10);
    hipError_t e = hipMalloc(&ctx->aux, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ctx->aux = nullptr;
      set_error("hipMalloc of %zu scratch bytes failed: %s", bytes, hipGetErrorString(e));
      return CBIC_E_OOM;
    }
    ctx->aux_bytes = bytes;
  }
  *p = ctx->aux;
  return CBIC_OK;
}

extern "C" {

const char* cbic_last_error(void) { return last_error(); }

int32_t cbic_version(void) { return 10000; }

cbic_status cbic_opts_default(cbic_solve_opts* o) {
  if (!o) { set_error("opts is NULL"); return CBIC_E_INVALID; }
  std::memset(o, 0, sizeof *o);
  o->struct_size = sizeof(cbic_solve_opts);
  o->max_iter = 50;
  o->psd_eps = 1e-6;
  o->ls_max_trials = 16;
  o->ls_beta = 0.5;
  o->stop_mode = 0;
  o->rtol = 1e-10;
  o->lookahead_K = 0;
  o->precision = CBIC_FP64;
  o->schedule = 0;
  o->iters_per_launch = 0;
  o->group_lanes = 0;
  o->flags = 0;
  o->regularization = CBIC_REG_CLIP;
  o->lm_mu0 = 1e-6;
  o->lm_factor = 10.0;
  o->lm_mu_max = 1e10;
  o->u_max = INFINITY;
  o->wg_per_cu = 0;
  return CBIC_OK;
}

cbic_status cbic_context_create(int hip_device, size_t cap, cbic_context** out) {
  if (!out) { set_error("out is NULL"); return CBIC_E_INVALID; }
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) {
    set_error("device %d out of range (%d devices)", hip_device, ndev);
    return CBIC_E_INVALID;
  }
  HIP_TRY(hipSetDevice(hip_device));
  cbic_context* c = new (std::nothrow) cbic_context();
  if (!c) { set_error("out of host memory"); return CBIC_E_OOM; }
  c->device = hip_device;
  c->cap = cap;
  if (scratch_address(hip_device, &c->scratch) != CBIC_OK) {
    delete c;
    return CBIC_E_HIP;
  }
  hipError_t e = hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming);
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&c->phase_ev[i]);
  if (e != hipSuccess) {
    delete c;
    set_error("hipEventCreate failed: %s", hipGetErrorString(e));
    return CBIC_E_HIP;
  }
  *out = c;
  return CBIC_OK;
}

cbic_status cbic_context_destroy(cbic_context* ctx) {
  if (!ctx) { set_error("ctx is NULL"); return CBIC_E_INVALID; }
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->graphs) {
    if (kv.second.ge) (void)hipGraphExecDestroy(kv.second.ge);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->aux) (void)hipFree(ctx->aux);
  if (ctx->done_ev) (void)hipEventDestroy(ctx->done_ev);
  for (int i = 0; i < 4; ++i)
    if (ctx->phase_ev[i]) (void)hipEventDestroy(ctx->phase_ev[i]);
  delete ctx;
  return CBIC_OK;
}

cbic_status cbic_system_create(cbic_context* ctx, cbic_system_kind kind, const double* h_params, size_t np,
                               cbic_system** out) {
  if (!out) { set_error("out is NULL"); return CBIC_E_INVALID; }
  *out = nullptr;
  int n = 0, m = 0;
  if (!validate_params(int(kind), h_params, np, &n, &m)) return CBIC_E_INVALID;
  cbic_system* s = new (std::nothrow) cbic_system();
  if (!s) { set_error("out of host memory"); return CBIC_E_OOM; }
  s->kind = int(kind);
  s->n = n;
  s->m = m;
  s->params.assign(h_params, h_params + np);
  s->ctx = ctx;
  if (!make_device_block(s, 1e-6)) {
    delete s;
    set_error("cannot build the device parameter block");
    return CBIC_E_INVALID;
  }
  s->dev_eps = 1e-6;
  if (ctx) {
    s->device = ctx->device;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc(&s->d_prm, s->dev.size() * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpy(s->d_prm, s->dev.data(), s->dev.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (s->d_prm) (void)hipFree(s->d_prm);
      delete s;
      set_error("uploading system parameters failed: %s", hipGetErrorString(e));
      return CBIC_E_HIP;
    }
  }
  *out = s;
  return CBIC_OK;
}

cbic_status cbic_system_dims(const cbic_system* s, int32_t* n, int32_t* m) {
  if (!s || !n || !m) { set_error("NULL argument"); return CBIC_E_INVALID; }
  *n = s->n;
  *m = s->m;
  return CBIC_OK;
}

cbic_status cbic_system_destroy(cbic_system* s) {
  if (!s) { set_error("sys is NULL"); return CBIC_E_INVALID; }
  if (s->d_prm) {
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(s->d_prm);
    for (auto& kv : s->lq_blocks) (void)hipFree(kv.second.second);
  }
  delete s;
  return CBIC_OK;
}

cbic_status cbic_workspace_size(const cbic_system* s, int32_t B, int32_t Tmax, const cbic_solve_opts* opts,
                                size_t* bytes) {
  if (!s || !bytes) { set_error("NULL argument"); return CBIC_E_INVALID; }
  if (B < 1 || Tmax < 1) { set_error("B and T_max must be >= 1"); return CBIC_E_INVALID; }
  cbic_status st = check_solve_opts(opts);
  if (st) return st;
  const Launcher* L = find_launcher(s->kind, s->n, s->m, opts->precision, opts->schedule);
  if (!L) {
    set_error("no kernel for system kind %d (n=%d, m=%d), precision %d, schedule %d", s->kind, s->n, s->m,
              opts->precision, opts->schedule);
    return CBIC_E_UNSUPPORTED;
  }
  *bytes = L->ws_bytes(B, Tmax) + sort_bytes(B, Tmax);
  return CBIC_OK;
}

cbic_status cbic_solve_batch(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t Tmax,
                             const int32_t* d_T, const double* d_x0, const double* d_U0,
                             const cbic_solve_opts* opts, const cbic_outputs* out, void* stream_v) {
  const Launcher* L = nullptr;
  cbic_status st = check_solve(ctx, sys, B, Tmax, d_T, d_x0, d_U0, opts, out, &L);
  if (st) return st;
  const SolveParamsH sp = solve_params(opts);
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  HIP_TRY(hipSetDevice(ctx->device));
  // the LQ Hessians are constant; a solve with another clip floor (or the
  // Levenberg-Marquardt variant, which clips nothing) uses a block of its own
  const double* prm = nullptr;
  st = param_block(const_cast<cbic_system*>(sys), sp.eps, stream, true, &prm);
  if (st) return st;
  const size_t ws_main = L->ws_bytes(B, Tmax);
  st = ensure_ws(ctx, ws_main + sort_bytes(B, Tmax));
  if (st) return st;
  if (ctx->have_last && ctx->last_stream != stream) HIP_TRY(hipStreamWaitEvent(stream, ctx->done_ev, 0));
  st = enqueue_solve(ctx, sys, prm, L, sp, B, Tmax, d_T, d_x0, d_U0, opts, out, static_cast<char*>(ctx->ws),
                     ws_main, stream);
  if (st) return st;
  HIP_TRY(hipEventRecord(ctx->done_ev, stream));
  ctx->last_stream = stream;
  ctx->have_last = true;
  return CBIC_OK;
}

cbic_status cbic_solve_batch_noalloc(cbic_context* ctx, const cbic_system* sys, int32_t B, int32_t Tmax,
                                     const int32_t* d_T, const double* d_x0, const double* d_U0,
                                     const cbic_solve_opts* opts, const cbic_outputs* out, void* stream_v) {
  const Launcher* L = nullptr;
  cbic_status st = check_solve(ctx, sys, B, Tmax, d_T, d_x0, d_U0, opts, out, &L);
  if (st) return st;
  if (opts->flags & (CBIC_FLAG_GRAPH | CBIC_FLAG_TIMING)) {
    set_error("the allocation-free solve takes neither CBIC_FLAG_GRAPH nor CBIC_FLAG_TIMING");
    return CBIC_E_INVALID;
  }
  const SolveParamsH sp = solve_params(opts);
  const size_t ws_main = L->ws_bytes(B, Tmax);
  const size_t need = ws_main + sort_bytes(B, Tmax);
  if (need > kScratchBytes) {
    set_error("the solve needs %zu workspace bytes; the allocation-free solve has %zu (CBIC_NOALLOC_SCRATCH_BYTES)",
              need, kScratchBytes);
    return CBIC_E_OOM;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->scratch) {
    set_error("no device scratch address for device %d", ctx->device);
    return CBIC_E_HIP;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  const double* prm = nullptr;
  st = param_block(const_cast<cbic_system*>(sys), sp.eps, static_cast<hipStream_t>(stream_v), false, &prm);
  if (st) return st;
  return enqueue_solve(ctx, sys, prm, L, sp, B, Tmax, d_T, d_x0, d_U0, opts, out, static_cast<char*>(ctx->scratch),
                       ws_main, static_cast<hipStream_t>(stream_v));
}

cbic_status cbic_phase_times(cbic_context* ctx, double* ms3) {
  if (!ctx || !ms3) { set_error("NULL argument"); return CBIC_E_INVALID; }
  if (!ctx->timed) { set_error("no solve with CBIC_FLAG_TIMING was launched on this context"); return CBIC_E_INVALID; }
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->phase_ev[3]));
  for (int i = 0; i < 3; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->phase_ev[i], ctx->phase_ev[i + 1]));
    ms3[i] = ms;
  }
  return CBIC_OK;
}

}  // extern "C"
