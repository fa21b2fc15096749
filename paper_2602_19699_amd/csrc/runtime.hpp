// Host-side runtime of the solver library: contexts, systems, workspace
// layout and the table of kernel launchers per (system, precision).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cbic.h"
#include "dev_common.hpp"

namespace cbic {

void set_error(const char* fmt, ...);

struct SolveParams;  // ilqr_lane.hpp

// Per-slot stride, in elements of `elem` bytes, of `count` elements padded to
// whole 128-byte cache lines (the lane schedule's trajectories and gains are
// slot-major, so that one slot's steps fill whole lines).
inline int lane_stride(int count, int elem) { return int((size_t(count) * elem + 127) / 128 * 128 / elem); }

// Byte offsets of the per-slot state, trajectories and gains inside one
// workspace allocation (lane schedule).  All sub-arrays are 256-byte aligned.
struct LaneLayout {
  size_t T, inst, J, iters, status, cur, work, mu, okey;
  size_t X, U, K, kf;
  size_t total;
};
// nbuf trajectory buffers (X, U): the iterate and the trial trajectories
LaneLayout lane_layout(int N, int M, int elem, int Bcap, int Tcap, int nbuf = 2);

// Group schedule (one workgroup per instance) for large systems.
struct GroupLayout {
  size_t T, inst, J, iters, status, cur, work, mu;
  size_t X, U, K, kf;
  size_t total;
};
GroupLayout group_layout(int N, int M, int elem, int Bcap, int Tcap);

struct SolveParamsH {
  int32_t max_iter, ls_trials, stop_mode, lookahead;
  double eps, beta, rtol;
  // Levenberg-Marquardt (reg = 1; eps is then negative: no clipping)
  int32_t reg = 0;
  double mu0 = 0.0, mu_fac = 1.0, mu_max = 0.0;
  // control bound of eq. 1 (infinite: none)
  double umax = __builtin_inf();
};

struct FinalOutH {
  double *X, *U, *J;
  int32_t* iters;
  uint32_t* status;
  double *Vbar, *Vx, *xK, *trace;
  int32_t* work;
};

// Launchers for one (system, precision).  `base` is the workspace; `slots`
// (optional) lists the slots to work on; `perm` (optional) maps a thread to
// the caller's instance index when initialising from caller arrays.
struct Launcher {
  int N, M, elem;
  int schedule;  // CBIC_SCHED_*
  size_t (*ws_bytes)(int Bcap, int Tcap);
  hipError_t (*init)(const double* prm, void* base, int Bcap, int Tcap, int nthreads, const int32_t* slots,
                     int Tmax, const int32_t* Tin, const int32_t* perm, const double* x0, const double* U0,
                     int max_iter, double* trace, double umax, hipStream_t st);
  hipError_t (*iterate)(const double* prm, void* base, int Bcap, int Tcap, int nthreads, const int32_t* slots,
                        const SolveParamsH& sp, int G, int group, const IterTrace& tr, hipStream_t st);
  hipError_t (*finalize)(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                         const int32_t* slots, int Tmax, int max_iter, int lookahead, const FinalOutH& o,
                         hipStream_t st);
  // device bytes per slot that ws_bytes holds beyond the lane layout
  size_t slot_extra = 0;
  // trajectory buffers of the lane layout
  int nbuf = 2;
  // optional: the iterations of a solve's only launch with every group
  // finalising its slot as soon as it stops (iterate then finalize in one
  // kernel; the same results)
  hipError_t (*iterate_final)(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                              const int32_t* slots, const SolveParamsH& sp, int G, int group, const IterTrace& tr,
                              int Tmax, int lookahead, const FinalOutH& o, hipStream_t st) = nullptr;
};

const Launcher* find_launcher(int kind, int n, int m, int precision, int schedule);

// validation of a cbic_solve_opts (CBIC_E_INVALID with the message set)
cbic_status check_solve_opts(const cbic_solve_opts* o);
// the kernels' solve parameters for valid options (the Levenberg-Marquardt
// variant clips nothing: eps is then negative)
SolveParamsH solve_params(const cbic_solve_opts* o);

// the schedule choice when the caller leaves it to the library: lanes per
// instance of the lane schedule (enough groups to give every SIMD of the chip
// a wave or two), instances per compute unit of the workgroup schedule (one
// while the batch fits the device's compute units one instance each, two
// above; always one in FP64)
int default_group(int schedule, int B, int precision, int device);
// the caller's own choice for the launcher's schedule (0: none)
int requested_group(const Launcher* L, const cbic_solve_opts* o);
// compute units of a device (cached)
int cu_count(int device);

// key of the autotuning table for a solve (system kind and size, precision,
// stop rule, batch rounded up to a power of two, horizon capacity)
std::string tune_key(const cbic_system* sys, int B, int Tmax, const cbic_solve_opts* o);

// horizon sort (longest first) of B instances -> perm (device)
hipError_t launch_horizon_sort(const int32_t* dT, int B, int Tmax, int32_t* hist, int32_t* perm, hipStream_t st);

// iteration order of B initialised slots from the keys their warm start
// wrote (`ragged`: the slots hold several horizons, longest first; the key is
// then the horizon above the J^0 octave, else the J^0 quarter octave above
// the half octave of the non-convex share of J^0): within each horizon,
// highest J^0 first in coarse levels, and for a batch of one horizon highest
// non-convex share first within each level -> order (device, B entries).  One
// workgroup; every horizon up to Tmax must have a level in its shared-memory
// histogram (cost_order_supported).
bool cost_order_supported(bool ragged, int Tmax);
hipError_t launch_cost_order(const uint32_t* keys, int B, int Tmax, bool ragged, int32_t* order, hipStream_t st);

// p[0..n) = v on the device, by a kernel
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t st);

}  // namespace cbic

struct cbic_context {
  int device = 0;
  size_t cap = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t last_stream = nullptr;
  bool have_last = false;
  hipEvent_t done_ev = nullptr;
  hipEvent_t phase_ev[4] = {nullptr, nullptr, nullptr, nullptr};  // timing events
  bool timed = false;
  std::mutex mu;
  // graph cache for the iteration chain
  struct GraphEntry {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
  };
  std::map<std::string, GraphEntry> graphs;
  // autotuned lanes per instance, keyed by problem class (see autotune.cpp)
  std::map<std::string, int> tuned;
  // small device scratch of the calls beside the solver (the selection of
  // biased initial states), grown on demand
  void* aux = nullptr;
  size_t aux_bytes = 0;
  // this device's address of the allocation-free solve's scratch array
  void* scratch = nullptr;
};

// At least `need` bytes of the context's auxiliary device scratch in *p
// (allocated or grown here; the caller holds ctx->mu and orders its stream
// after the context's previous call).
cbic_status context_aux(cbic_context* ctx, size_t need, void** p);

struct cbic_system {
  int kind = -1;
  int n = 0, m = 0;
  std::vector<double> params;  // user's vector
  std::vector<double> dev;     // derived device block
  double dev_eps = 1e-6;       // eps the LQ block was clipped with
  cbic_context* ctx = nullptr;
  int device = -1;             // the context's device (the system may outlive its context)
  double* d_prm = nullptr;     // device copy of `dev`
  // LQ systems: the blocks for other clip floors solved with (their clipped
  // constant Hessians depend on it), keyed by psd_eps; each host copy lives as
  // long as the system, since an asynchronous upload reads it
  std::map<double, std::pair<std::vector<double>, double*>> lq_blocks;
};
