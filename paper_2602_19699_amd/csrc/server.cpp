// Continuous-batching server: requests (one TO instance each) of any system
// created on the server's context are admitted into per-class device slot
// pools while their device footprint fits under the memory cap, iterate G
// iLQR iterations per launch beside the requests already resident (one
// stream per class, so classes overlap on the GPU), keep their iterates in
// device memory between launches, and are extracted, copied to host and
// freed when they finish.
#include <cmath>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.hpp"

namespace cbic {

hipError_t launch_gather_u32(const uint32_t* src, const int32_t* idx, int n, uint32_t* dst, hipStream_t st);
hipError_t launch_set_index(const int32_t* slots, int n, int32_t* inst, hipStream_t st);

namespace {

struct Request {
  uint64_t ticket = 0;
  const cbic_system* sys = nullptr;
  int T = 0;
  std::vector<double> x0, U0;
  cbic_solve_opts opts{};
  std::string sig;  // the result-affecting options (the class key with sys and precision)
  double t_submit = 0, t_admit = 0;
  size_t bytes = 0;
};

// The options that change a solve's result, as a key: requests that differ in
// them are served by different pools (the lanes-per-instance width, the
// launch split and the flags do not change results).
std::string result_signature(const cbic_solve_opts& o) {
  char b[320];
  std::snprintf(b, sizeof b, "%d|%.17g|%d|%.17g|%d|%.17g|%d|%d|%.17g|%.17g|%.17g|%.17g", o.max_iter, o.psd_eps,
                o.ls_max_trials, o.ls_beta, o.stop_mode, o.rtol, o.lookahead_K, o.regularization, o.lm_mu0,
                o.lm_factor, o.lm_mu_max, o.u_max);
  return b;
}

struct Result {
  std::vector<double> X, U, Vbar, Vx;
  double J = 0;
  int32_t iters = 0;
  uint32_t status = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// per-request device footprint: the slot's state and the trajectory, gain and
// trial-trajectory storage for its own horizon
size_t footprint(int n, int m, int elem, int T, int nbuf) {
  const size_t words = size_t(nbuf) * (T + 1) * n + size_t(nbuf) * T * m + size_t(T) * m * n + size_t(T) * m;
  return words * elem + 40;
}

struct Pool {
  const cbic_system* sys = nullptr;
  int precision = 0;
  const Launcher* L = nullptr;
  cbic_solve_opts opts{};
  int n = 0, m = 0, Bcap = 0, Tcap = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* ws = nullptr;         // solver workspace (lane layout)
  LaneLayout lay{};
  // device staging
  char* dbuf = nullptr;
  int32_t *d_list = nullptr, *d_adm = nullptr, *d_T = nullptr, *d_fin = nullptr, *d_iters = nullptr;
  uint32_t *d_stat = nullptr, *d_statg = nullptr;
  double *d_x0 = nullptr, *d_U0 = nullptr, *d_X = nullptr, *d_U = nullptr, *d_J = nullptr, *d_Vb = nullptr,
         *d_Vx = nullptr;
  // pinned host staging
  char* hbuf = nullptr;
  int32_t *h_list = nullptr, *h_adm = nullptr, *h_T = nullptr, *h_fin = nullptr, *h_iters = nullptr;
  uint32_t *h_statg = nullptr, *h_stat = nullptr;
  double *h_x0 = nullptr, *h_U0 = nullptr, *h_X = nullptr, *h_U = nullptr, *h_J = nullptr, *h_Vb = nullptr,
         *h_Vx = nullptr;
  size_t bytes = 0;  // device bytes of this pool (0 while it holds none)
  std::vector<int> free_slots;
  std::vector<std::unique_ptr<Request>> slot_req;  // request resident in each slot
  std::vector<int> active;                         // slots in use
  std::deque<std::unique_ptr<Request>> pending;
  bool list_dirty = true;
  // 0 idle, 1 iterations launched (event: statuses copied back), 2 outputs of
  // finished slots being copied back (event)
  int phase = 0;
  int nfin = 0;
};

}  // namespace
}  // namespace cbic

using namespace cbic;

struct cbic_server {
  cbic_context* ctx = nullptr;
  cbic_server_opts opts{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<std::unique_ptr<Request>> inbox;
  std::unordered_map<uint64_t, std::unique_ptr<Result>> results;
  uint64_t next_ticket = 1;
  size_t outstanding = 0;  // submitted and not yet done
  size_t inflight_bytes = 0, pool_bytes = 0, peak_inflight = 0, peak_pool = 0;
  uint64_t submitted = 0, completed = 0, rounds = 0, evictions = 0, launches = 0, launched_slots = 0;
  // worker time spent in its rounds (host bookkeeping, staging, launches)
  std::atomic<uint64_t> host_busy_ns{0};
  int max_resident = 0, resident = 0;
  std::map<std::tuple<const cbic_system*, int, std::string>, std::unique_ptr<Pool>> pools;
  std::thread worker;
  bool stop = false;
  int fatal = 0;
  char fatal_msg[256] = "";

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

#define SRV_TRY(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      std::snprintf(srv->fatal_msg, sizeof srv->fatal_msg, "%s: %s", #expr, hipGetErrorString(e_)); \
      srv->fatal = 1;                                                                \
      return false;                                                                  \
    }                                                                                \
  } while (0)

template <class T>
T* carve(char*& p, size_t count) {
  T* r = reinterpret_cast<T*>(p);
  p += (count * sizeof(T) + 255) / 256 * 256;
  return r;
}

size_t staging_bytes(int B, int T, int n, int m) {
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  return a(4 * size_t(B)) * 5 + a(4 * size_t(B)) * 2 + a(8 * size_t(B) * n) + a(8 * size_t(B) * T * m) +
         a(8 * size_t(B) * (T + 1) * n) * 2 + a(8 * size_t(B) * T * m) + a(8 * size_t(B)) + a(8 * size_t(B) * (T + 1));
}

// device bytes of a pool of Bcap slots: the launcher's workspace and staging
size_t pool_bytes(const Launcher* L, int Bcap, int Tcap, int n, int m) {
  return L->ws_bytes(Bcap, Tcap) + staging_bytes(Bcap, Tcap, n, m);
}

bool make_pool(cbic_server* srv, Pool* p) {
  const int elem = p->precision ? 4 : 8;
  p->lay = lane_layout(p->n, p->m, elem, p->Bcap, p->Tcap, p->L->nbuf);
  if (!p->stream) SRV_TRY(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
  if (!p->ev) SRV_TRY(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming));
  // the launcher's workspace: the lane layout plus whatever it keeps per slot
  const size_t wsb = p->L->ws_bytes(p->Bcap, p->Tcap);
  SRV_TRY(hipMalloc(&p->ws, wsb));
  const size_t sb = staging_bytes(p->Bcap, p->Tcap, p->n, p->m);
  SRV_TRY(hipMalloc(&p->dbuf, sb));
  SRV_TRY(hipHostMalloc(&p->hbuf, sb, hipHostMallocDefault));
  p->bytes = wsb + sb;
  for (int pass = 0; pass < 2; ++pass) {
    char* q = pass ? p->hbuf : p->dbuf;
    int32_t** i32[] = {pass ? &p->h_list : &p->d_list, pass ? &p->h_adm : &p->d_adm, pass ? &p->h_T : &p->d_T,
                       pass ? &p->h_fin : &p->d_fin, pass ? &p->h_iters : &p->d_iters};
    for (auto ptr : i32) *ptr = carve<int32_t>(q, p->Bcap);
    (pass ? p->h_statg : p->d_statg) = carve<uint32_t>(q, p->Bcap);
    (pass ? p->h_stat : p->d_stat) = carve<uint32_t>(q, p->Bcap);
    (pass ? p->h_x0 : p->d_x0) = carve<double>(q, size_t(p->Bcap) * p->n);
    (pass ? p->h_U0 : p->d_U0) = carve<double>(q, size_t(p->Bcap) * p->Tcap * p->m);
    (pass ? p->h_X : p->d_X) = carve<double>(q, size_t(p->Bcap) * (p->Tcap + 1) * p->n);
    (pass ? p->h_Vx : p->d_Vx) = carve<double>(q, size_t(p->Bcap) * (p->Tcap + 1) * p->n);
    (pass ? p->h_U : p->d_U) = carve<double>(q, size_t(p->Bcap) * p->Tcap * p->m);
    (pass ? p->h_J : p->d_J) = carve<double>(q, p->Bcap);
    (pass ? p->h_Vb : p->d_Vb) = carve<double>(q, size_t(p->Bcap) * (p->Tcap + 1));
  }
  p->slot_req.clear();
  p->slot_req.resize(p->Bcap);
  p->free_slots.clear();
  p->free_slots.reserve(p->Bcap);
  for (int s = p->Bcap - 1; s >= 0; --s) p->free_slots.push_back(s);
  return true;
}

// Release a pool's device and pinned memory (its stream and event too when
// `all`); an idle pool released this way is rebuilt when requests return.
void free_pool(Pool* p, bool all = true) {
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->ws) (void)hipFree(p->ws);
  if (p->dbuf) (void)hipFree(p->dbuf);
  if (p->hbuf) (void)hipHostFree(p->hbuf);
  p->ws = nullptr;
  p->dbuf = nullptr;
  p->hbuf = nullptr;
  p->bytes = 0;
  p->free_slots.clear();
  p->slot_req.clear();
  p->list_dirty = true;
  if (all) {
    if (p->ev) (void)hipEventDestroy(p->ev);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    p->ev = nullptr;
    p->stream = nullptr;
  }
}

// Largest slot count (<= want) whose pool fits beside the memory the other
// pools hold, 0 if not even one slot fits.
int fit_slots(const cbic_server* srv, const Pool* p, int want) {
  const size_t cap = srv->opts.mem_cap_bytes;
  auto fits = [&](int b) { return srv->pool_bytes + pool_bytes(p->L, b, p->Tcap, p->n, p->m) <= cap; };
  if (!fits(1)) return 0;
  int lo = 1, hi = want;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (fits(mid)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

void collect_inbox(cbic_server* srv) {
  std::lock_guard<std::mutex> lk(srv->mu);
  while (!srv->inbox.empty()) {
    std::unique_ptr<Request> r = std::move(srv->inbox.front());
    srv->inbox.pop_front();
    auto key = std::make_tuple(r->sys, int(r->opts.precision), r->sig);
    auto it = srv->pools.find(key);
    if (it == srv->pools.end()) {
      auto p = std::make_unique<Pool>();
      p->sys = r->sys;
      p->precision = r->opts.precision;
      p->L = find_launcher(r->sys->kind, r->sys->n, r->sys->m, r->opts.precision, 0);
      p->opts = r->opts;
      p->n = r->sys->n;
      p->m = r->sys->m;
      p->Bcap = 0;
      p->Tcap = srv->opts.t_max;
      it = srv->pools.emplace(key, std::move(p)).first;
    }
    it->second->pending.push_back(std::move(r));
  }
}

// Give a class with waiting requests its pool: as many slots (up to
// slots_per_class) as fit beside the memory the other pools hold, releasing
// idle pools (nothing resident, nothing waiting) when not even one slot fits.
// The device memory of all pools together never exceeds the cap; a class
// that finds no room keeps waiting until another pool goes idle.
bool ensure_pool(cbic_server* srv, Pool* p) {
  if (p->ws || p->pending.empty()) return true;
  int b = fit_slots(srv, p, srv->opts.slots_per_class);
  if (b == 0)
    for (auto& kv : srv->pools) {
      Pool* q = kv.second.get();
      if (q == p || !q->ws || !q->active.empty() || !q->pending.empty() || q->phase != 0) continue;
      srv->pool_bytes -= q->bytes;
      free_pool(q, false);
      ++srv->evictions;
      if ((b = fit_slots(srv, p, srv->opts.slots_per_class)) > 0) break;
    }
  if (b == 0) return true;
  p->Bcap = b;
  if (!make_pool(srv, p)) return false;
  srv->pool_bytes += p->bytes;
  srv->peak_pool = std::max(srv->peak_pool, srv->pool_bytes);
  return true;
}

// Admit pending requests of class p (FIFO) while a slot of its pool is free;
// stage their inputs and run init.
bool admit(cbic_server* srv, Pool* p) {
  if (!ensure_pool(srv, p)) return false;
  if (!p->ws) return true;
  const double tnow = srv->now();
  int nadm = 0;
  while (!p->pending.empty() && !p->free_slots.empty()) {
    Request* r = p->pending.front().get();
    const int s = p->free_slots.back();
    p->free_slots.pop_back();
    srv->inflight_bytes += r->bytes;
    srv->peak_inflight = std::max(srv->peak_inflight, srv->inflight_bytes);
    ++srv->resident;
    srv->max_resident = std::max(srv->max_resident, srv->resident);
    r->t_admit = tnow;
    std::memcpy(p->h_x0 + size_t(nadm) * p->n, r->x0.data(), sizeof(double) * p->n);
    double* u0 = p->h_U0 + size_t(nadm) * p->Tcap * p->m;
    if (r->U0.empty()) std::memset(u0, 0, sizeof(double) * size_t(r->T) * p->m);
    else std::memcpy(u0, r->U0.data(), sizeof(double) * size_t(r->T) * p->m);
    p->h_T[nadm] = r->T;
    p->h_adm[nadm] = s;
    p->slot_req[s] = std::move(p->pending.front());
    p->pending.pop_front();
    p->active.push_back(s);
    ++nadm;
  }
  if (!nadm) return true;
  p->list_dirty = true;
  SRV_TRY(hipMemcpyAsync(p->d_x0, p->h_x0, sizeof(double) * nadm * p->n, hipMemcpyHostToDevice, p->stream));
  SRV_TRY(hipMemcpyAsync(p->d_U0, p->h_U0, sizeof(double) * size_t(nadm) * p->Tcap * p->m, hipMemcpyHostToDevice,
                         p->stream));
  SRV_TRY(hipMemcpyAsync(p->d_T, p->h_T, 4 * nadm, hipMemcpyHostToDevice, p->stream));
  SRV_TRY(hipMemcpyAsync(p->d_adm, p->h_adm, 4 * nadm, hipMemcpyHostToDevice, p->stream));
  SRV_TRY(p->L->init(p->sys->d_prm, p->ws, p->Bcap, p->Tcap, nadm, p->d_adm, p->Tcap, p->d_T, nullptr, p->d_x0,
                     p->d_U0, p->opts.max_iter, nullptr, p->opts.u_max, p->stream));
  return true;
}

// G iterations for every resident slot of the class on its stream, then the
// statuses of those slots back to the host (event).
bool launch_iterations(cbic_server* srv, Pool* p) {
  const int na = int(p->active.size());
  if (p->list_dirty) {
    std::memcpy(p->h_list, p->active.data(), 4 * na);
    SRV_TRY(hipMemcpyAsync(p->d_list, p->h_list, 4 * na, hipMemcpyHostToDevice, p->stream));
    p->list_dirty = false;
  }
  const SolveParamsH sp = solve_params(&p->opts);
  ++srv->launches;
  srv->launched_slots += uint64_t(na);
  const int req = requested_group(p->L, &p->opts);
  const int group = req > 0 ? req : default_group(p->L->schedule, na, p->precision, srv->ctx->device);
  SRV_TRY(p->L->iterate(p->sys->d_prm, p->ws, p->Bcap, p->Tcap, na, p->d_list, sp,
                        std::max(1, srv->opts.iters_per_launch), group, IterTrace{nullptr, nullptr}, p->stream));
  const uint32_t* st = reinterpret_cast<const uint32_t*>(static_cast<char*>(p->ws) + p->lay.status);
  SRV_TRY(launch_gather_u32(st, p->d_list, na, p->d_statg, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_statg, p->d_statg, 4 * na, hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipEventRecord(p->ev, p->stream));
  p->phase = 1;
  return true;
}

// Statuses are back: finished slots get their targets extracted into compact
// rows and copied to host (event).
bool launch_finalize(cbic_server* srv, Pool* p) {
  const int na = int(p->active.size());
  int nf = 0;
  std::vector<int> keep;
  keep.reserve(na);
  for (int i = 0; i < na; ++i) {
    if (p->h_statg[i] != 0) p->h_fin[nf++] = p->active[i];
    else keep.push_back(p->active[i]);
  }
  p->nfin = nf;
  if (!nf) {
    p->phase = 0;
    return true;
  }
  p->active.swap(keep);
  p->list_dirty = true;
  SRV_TRY(hipMemcpyAsync(p->d_fin, p->h_fin, 4 * nf, hipMemcpyHostToDevice, p->stream));
  int32_t* inst = reinterpret_cast<int32_t*>(static_cast<char*>(p->ws) + p->lay.inst);
  SRV_TRY(launch_set_index(p->d_fin, nf, inst, p->stream));
  FinalOutH fo{p->d_X, p->d_U, p->d_J, p->d_iters, p->d_stat, p->d_Vb, p->d_Vx, nullptr, nullptr, nullptr};
  SRV_TRY(p->L->finalize(p->sys->d_prm, p->ws, p->Bcap, p->Tcap, nf, p->d_fin, p->Tcap, p->opts.max_iter,
                         p->opts.lookahead_K, fo, p->stream));
  const size_t sx = size_t(p->Tcap + 1) * p->n, su = size_t(p->Tcap) * p->m;
  SRV_TRY(hipMemcpyAsync(p->h_X, p->d_X, 8 * sx * nf, hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_U, p->d_U, 8 * su * nf, hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_Vb, p->d_Vb, 8 * size_t(p->Tcap + 1) * nf, hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_Vx, p->d_Vx, 8 * sx * nf, hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_J, p->d_J, 8 * size_t(nf), hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_iters, p->d_iters, 4 * size_t(nf), hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipMemcpyAsync(p->h_stat, p->d_stat, 4 * size_t(nf), hipMemcpyDeviceToHost, p->stream));
  SRV_TRY(hipEventRecord(p->ev, p->stream));
  p->phase = 2;
  return true;
}

// Outputs are on the host: hand the results over and free the slots.
void retire(cbic_server* srv, Pool* p) {
  const double td = srv->now();
  const size_t sx = size_t(p->Tcap + 1) * p->n, su = size_t(p->Tcap) * p->m;
  std::vector<std::pair<uint64_t, std::unique_ptr<Result>>> done;
  for (int f = 0; f < p->nfin; ++f) {
    const int s = p->h_fin[f];
    std::unique_ptr<Request> r = std::move(p->slot_req[s]);
    auto res = std::make_unique<Result>();
    const int T = r->T, n = p->n, m = p->m;
    res->X.assign(p->h_X + f * sx, p->h_X + f * sx + size_t(T + 1) * n);
    res->U.assign(p->h_U + f * su, p->h_U + f * su + size_t(T) * m);
    res->Vbar.assign(p->h_Vb + size_t(f) * (p->Tcap + 1), p->h_Vb + size_t(f) * (p->Tcap + 1) + T + 1);
    res->Vx.assign(p->h_Vx + f * sx, p->h_Vx + f * sx + size_t(T + 1) * n);
    res->J = p->h_J[f];
    res->iters = p->h_iters[f];
    res->status = p->h_stat[f];
    res->t_submit = r->t_submit;
    res->t_admit = r->t_admit;
    res->t_done = td;
    srv->inflight_bytes -= r->bytes;
    --srv->resident;
    p->free_slots.push_back(s);
    done.emplace_back(r->ticket, std::move(res));
  }
  p->nfin = 0;
  p->phase = 0;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto& d : done) srv->results[d.first] = std::move(d.second);
    srv->outstanding -= done.size();
    srv->completed += done.size();
  }
  srv->done_cv.notify_all();
}

// One pass over the classes: every class advances its own state machine
// (idle -> iterations -> finalisation -> idle) as soon as its stream has
// finished the previous step, so fast classes are never held back by slow
// ones.  Returns false on a fatal HIP error.
bool round(cbic_server* srv, bool& progressed) {
  progressed = false;
  ++srv->rounds;
  collect_inbox(srv);
  for (auto& kv : srv->pools) {
    Pool* p = kv.second.get();
    if (p->phase != 0) {
      const hipError_t q = hipEventQuery(p->ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) SRV_TRY(q);
      progressed = true;
      if (p->phase == 1) {
        if (!launch_finalize(srv, p)) return false;
        if (p->phase == 2) continue;
      } else {
        retire(srv, p);
      }
    }
    // idle: admit newcomers, then iterate everything resident
    if (!admit(srv, p)) return false;
    if (!p->active.empty()) {
      if (!launch_iterations(srv, p)) return false;
      progressed = true;
    }
  }
  return true;
}

void worker_main(cbic_server* srv) {
  if (hipSetDevice(srv->ctx->device) != hipSuccess) {
    srv->fatal = 1;
    return;
  }
  while (true) {
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      if (srv->stop) break;
      bool idle = srv->inbox.empty();
      if (idle)
        for (auto& kv : srv->pools)
          if (!kv.second->active.empty() || !kv.second->pending.empty() || kv.second->phase != 0) idle = false;
      if (idle) {
        srv->cv.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
    }
    bool progressed = false;
    const auto t_round = std::chrono::steady_clock::now();
    const bool ok = round(srv, progressed);
    srv->host_busy_ns += uint64_t(
        std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t_round).count());
    if (!ok) {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->done_cv.notify_all();
      break;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

cbic_status cbic_server_opts_default(cbic_server_opts* o) {
  if (!o) { set_error("opts is NULL"); return CBIC_E_INVALID; }
  o->struct_size = sizeof(cbic_server_opts);
  o->mem_cap_bytes = size_t(32) << 30;
  o->slots_per_class = 4096;
  o->t_max = 200;
  o->iters_per_launch = 4;
  return CBIC_OK;
}

cbic_status cbic_server_create(cbic_context* ctx, const cbic_server_opts* o, cbic_server** out) {
  if (!out) { set_error("out is NULL"); return CBIC_E_INVALID; }
  *out = nullptr;
  if (!ctx || !o) { set_error("ctx and opts are required"); return CBIC_E_INVALID; }
  if (o->struct_size != sizeof(cbic_server_opts)) { set_error("server opts struct_size mismatch"); return CBIC_E_INVALID; }
  if (o->slots_per_class < 1 || o->t_max < 1 || o->mem_cap_bytes == 0) {
    set_error("slots_per_class, t_max and mem_cap_bytes must be positive");
    return CBIC_E_INVALID;
  }
  auto* s = new (std::nothrow) cbic_server();
  if (!s) { set_error("out of host memory"); return CBIC_E_OOM; }
  s->ctx = ctx;
  s->opts = *o;
  s->t0 = std::chrono::steady_clock::now();
  s->worker = std::thread(worker_main, s);
  *out = s;
  return CBIC_OK;
}

cbic_status cbic_server_submit(cbic_server* srv, const cbic_system* sys, int32_t T, const double* h_x0,
                               const double* h_U0, const cbic_solve_opts* opts, uint64_t* ticket) {
  if (!srv || !sys || !h_x0 || !opts || !ticket) { set_error("NULL argument"); return CBIC_E_INVALID; }
  if (sys->ctx != srv->ctx || !sys->d_prm) { set_error("sys was not created on the server's context"); return CBIC_E_INVALID; }
  const cbic_status cs = check_solve_opts(opts);
  if (cs) return cs;
  if (T < 1 || T > srv->opts.t_max) { set_error("T must be in 1..%d", srv->opts.t_max); return CBIC_E_INVALID; }
  const Launcher* L = find_launcher(sys->kind, sys->n, sys->m, opts->precision, 0);
  if (!L) {
    set_error("no kernel for this system and precision");
    return CBIC_E_UNSUPPORTED;
  }
  if (sys->kind == CBIC_SYS_LQ && sys->dev_eps != solve_params(opts).eps) {
    set_error("this LQ system's clipped Hessians were built for psd_eps %g (a served request cannot rebuild "
              "them under running solves)", sys->dev_eps);
    return CBIC_E_INVALID;
  }
  if (srv->fatal) { set_error("server stopped: %s", srv->fatal_msg); return CBIC_E_HIP; }
  auto r = std::make_unique<Request>();
  r->sys = sys;
  r->T = T;
  r->x0.assign(h_x0, h_x0 + sys->n);
  if (h_U0) r->U0.assign(h_U0, h_U0 + size_t(T) * sys->m);
  r->opts = *opts;
  r->sig = result_signature(*opts);
  r->bytes = footprint(sys->n, sys->m, opts->precision ? 4 : 8, T, L->nbuf) + L->slot_extra;
  // a request that can never fit: a one-slot pool of its class over the cap
  const size_t one = pool_bytes(L, 1, srv->opts.t_max, sys->n, sys->m);
  if (one > srv->opts.mem_cap_bytes) {
    set_error("a one-slot pool of this class needs %zu B, over the memory cap of %zu B", one,
              srv->opts.mem_cap_bytes);
    return CBIC_E_BUSY;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    r->t_submit = srv->now();
    *ticket = r->ticket;
    srv->inbox.push_back(std::move(r));
    ++srv->outstanding;
    ++srv->submitted;
  }
  srv->cv.notify_one();
  return CBIC_OK;
}

cbic_status cbic_server_poll(cbic_server* srv, uint64_t ticket, cbic_result* out) {
  if (!srv || !out) { set_error("NULL argument"); return CBIC_E_INVALID; }
  std::unique_ptr<Result> r;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->results.find(ticket);
    if (it == srv->results.end()) {
      if (ticket == 0 || ticket >= srv->next_ticket) { set_error("unknown ticket"); return CBIC_E_INVALID; }
      if (srv->fatal) { set_error("server stopped: %s", srv->fatal_msg); return CBIC_E_HIP; }
      return CBIC_NOT_READY;
    }
    r = std::move(it->second);
    srv->results.erase(it);
  }
  if (out->X) std::memcpy(out->X, r->X.data(), sizeof(double) * r->X.size());
  if (out->U) std::memcpy(out->U, r->U.data(), sizeof(double) * r->U.size());
  if (out->Vbar) std::memcpy(out->Vbar, r->Vbar.data(), sizeof(double) * r->Vbar.size());
  if (out->Vx) std::memcpy(out->Vx, r->Vx.data(), sizeof(double) * r->Vx.size());
  out->J = r->J;
  out->iters = r->iters;
  out->status = r->status;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  return CBIC_OK;
}

double cbic_server_clock(const cbic_server* srv) { return srv ? srv->now() : 0.0; }

cbic_status cbic_server_get_stats(cbic_server* srv, cbic_server_stats* out) {
  if (!srv || !out) { set_error("NULL argument"); return CBIC_E_INVALID; }
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->rounds = srv->rounds;
  out->inflight_bytes = srv->inflight_bytes;
  out->peak_inflight_bytes = srv->peak_inflight;
  out->pool_bytes = srv->pool_bytes;
  out->classes = int32_t(srv->pools.size());
  out->max_resident = srv->max_resident;
  out->peak_pool_bytes = srv->peak_pool;
  out->evictions = srv->evictions;
  out->launches = srv->launches;
  out->launched_slots = srv->launched_slots;
  out->host_busy_s = 1e-9 * double(srv->host_busy_ns.load());
  return CBIC_OK;
}

cbic_status cbic_server_drain(cbic_server* srv) {
  if (!srv) { set_error("NULL argument"); return CBIC_E_INVALID; }
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->done_cv.wait(lk, [&] { return srv->outstanding == 0 || srv->fatal; });
  if (srv->fatal) { set_error("server stopped: %s", srv->fatal_msg); return CBIC_E_HIP; }
  return CBIC_OK;
}

cbic_status cbic_server_destroy(cbic_server* srv) {
  if (!srv) { set_error("NULL argument"); return CBIC_E_INVALID; }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& kv : srv->pools) free_pool(kv.second.get());
  delete srv;
  return CBIC_OK;
}

}  // extern "C"
