// Host launchers for the lane-per-instance kernels of one (system, precision).
#pragma once
#include "ilqr_lane.hpp"
#include "runtime.hpp"

namespace cbic {

// Trajectory buffers of the lane kernels: for a system whose trial lanes
// write their own trajectories, the iterate plus one per lane of the widest
// group (the accepted trial is then already written wherever it was found);
// otherwise the iterate and one trial trajectory.
template <class Sys>
constexpr int lane_bufs() { return Sys::kOwnTrialBuffers ? 17 : 2; }

template <class R>
inline LaneState<R> lane_state(void* base, int N, int M, int Bcap, int Tcap, int nbuf) {
  const LaneLayout L = lane_layout(N, M, int(sizeof(R)), Bcap, Tcap, nbuf);
  char* b = static_cast<char*>(base);
  LaneState<R> w;
  w.T = reinterpret_cast<int32_t*>(b + L.T);
  w.inst = reinterpret_cast<int32_t*>(b + L.inst);
  w.J = reinterpret_cast<double*>(b + L.J);
  w.iters = reinterpret_cast<int32_t*>(b + L.iters);
  w.status = reinterpret_cast<uint32_t*>(b + L.status);
  w.cur = reinterpret_cast<int32_t*>(b + L.cur);
  w.work = reinterpret_cast<int32_t*>(b + L.work);
  w.mu = reinterpret_cast<double*>(b + L.mu);
  w.okey = reinterpret_cast<uint32_t*>(b + L.okey);
  w.X = reinterpret_cast<R*>(b + L.X);
  w.U = reinterpret_cast<R*>(b + L.U);
  w.K = reinterpret_cast<R*>(b + L.K);
  w.kf = reinterpret_cast<R*>(b + L.kf);
  w.Bcap = Bcap;
  w.Tcap = Tcap;
  w.nbuf = nbuf;
  w.xs = lane_stride((Tcap + 1) * N, int(sizeof(R)));
  w.us = lane_stride(Tcap * M, int(sizeof(R)));
  w.Ks = lane_stride(Tcap * M * N, int(sizeof(R)));
  w.ks = lane_stride(Tcap * M, int(sizeof(R)));
  return w;
}

inline SolveParams to_dev(const SolveParamsH& h) {
  SolveParams s;
  s.max_iter = h.max_iter;
  s.ls_trials = h.ls_trials;
  s.stop_mode = h.stop_mode;
  s.lookahead = h.lookahead;
  s.eps = h.eps;
  s.beta = h.beta;
  s.rtol = h.rtol;
  s.reg = h.reg;
  s.mu0 = h.mu0;
  s.mu_fac = h.mu_fac;
  s.mu_max = h.mu_max;
  s.umax = h.umax;
  return s;
}

template <class Sys, class R>
struct LaneLaunch {
  static constexpr int N = Sys::N, M = Sys::M;
  static constexpr int WG = 64;

  static size_t ws_bytes(int Bcap, int Tcap) {
    return lane_layout(N, M, int(sizeof(R)), Bcap, Tcap, lane_bufs<Sys>()).total;
  }

  static hipError_t init(const double* prm, void* base, int Bcap, int Tcap, int nthreads, const int32_t* slots,
                         int Tmax, const int32_t* Tin, const int32_t* perm, const double* x0, const double* U0,
                         int max_iter, double* trace, double umax, hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, lane_bufs<Sys>());
    // eight lanes per instance share the stage costs and the stores
    constexpr int IG = 8;
    const long total = long(nthreads) * IG;
    hipLaunchKernelGGL((lane_init<Sys, R, IG>), dim3((total + WG - 1) / WG), dim3(WG), 0, st, prm, w, nthreads,
                       slots, Tmax, Tin, perm, x0, U0, max_iter, trace, umax);
    return hipGetLastError();
  }

  // the bounded variant (eq. 1) is a kernel of its own, so that the
  // unbounded one keeps its register allocation; FIN finalises in the same
  // kernel (fo, Tmax, lookahead)
  template <int GL, bool FIN>
  static hipError_t iterate_g(const double* prm, const LaneState<R>& w, int nthreads, const int32_t* slots,
                              const SolveParams& sp, int G, const IterTrace& tr, int Tmax, int lookahead,
                              const FinalOut& fo, hipStream_t st) {
    const long total = long(nthreads) * GL;
    if (__builtin_isfinite(sp.umax))
      hipLaunchKernelGGL((lane_iterate<Sys, R, GL, true, FIN>), dim3((total + WG - 1) / WG), dim3(WG), 0, st, prm,
                         w, nthreads, slots, sp, G, tr, Tmax, lookahead, fo);
    else
      hipLaunchKernelGGL((lane_iterate<Sys, R, GL, false, FIN>), dim3((total + WG - 1) / WG), dim3(WG), 0, st,
                         prm, w, nthreads, slots, sp, G, tr, Tmax, lookahead, fo);
    return hipGetLastError();
  }

  template <bool FIN>
  static hipError_t iterate_any(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                                const int32_t* slots, const SolveParamsH& sp, int G, int group, const IterTrace& tr,
                                int Tmax, int lookahead, const FinalOut& fo, hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, lane_bufs<Sys>());
    const SolveParams d = to_dev(sp);
    switch (group) {
      case 1: return iterate_g<1, FIN>(prm, w, nthreads, slots, d, G, tr, Tmax, lookahead, fo, st);
      case 2: return iterate_g<2, FIN>(prm, w, nthreads, slots, d, G, tr, Tmax, lookahead, fo, st);
      case 4: return iterate_g<4, FIN>(prm, w, nthreads, slots, d, G, tr, Tmax, lookahead, fo, st);
      case 8: return iterate_g<8, FIN>(prm, w, nthreads, slots, d, G, tr, Tmax, lookahead, fo, st);
      case 16: return iterate_g<16, FIN>(prm, w, nthreads, slots, d, G, tr, Tmax, lookahead, fo, st);
      default: return hipErrorInvalidValue;
    }
  }

  static hipError_t iterate(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                            const int32_t* slots, const SolveParamsH& sp, int G, int group, const IterTrace& tr,
                            hipStream_t st) {
    return iterate_any<false>(prm, base, Bcap, Tcap, nthreads, slots, sp, G, group, tr, 0, 0, FinalOut{}, st);
  }

  static hipError_t iterate_final(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                                  const int32_t* slots, const SolveParamsH& sp, int G, int group,
                                  const IterTrace& tr, int Tmax, int lookahead, const FinalOutH& o,
                                  hipStream_t st) {
    const FinalOut fo{o.X, o.U, o.J, o.iters, o.status, o.Vbar, o.Vx, o.xK, o.trace, o.work};
    return iterate_any<true>(prm, base, Bcap, Tcap, nthreads, slots, sp, G, group, tr, Tmax, lookahead, fo, st);
  }

  static hipError_t finalize(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                             const int32_t* slots, int Tmax, int max_iter, int lookahead, const FinalOutH& o,
                             hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, lane_bufs<Sys>());
    FinalOut fo{o.X, o.U, o.J, o.iters, o.status, o.Vbar, o.Vx, o.xK, o.trace, o.work};
    // eight lanes per instance share the output copies and the stage costs
    constexpr int FG = 8;
    const long total = long(nthreads) * FG;
    hipLaunchKernelGGL((lane_final<Sys, R, FG>), dim3((total + WG - 1) / WG), dim3(WG), 0, st, prm, w, nthreads,
                       slots, Tmax, max_iter, lookahead, fo);
    return hipGetLastError();
  }

  static const Launcher* get() {
    static const Launcher L{N,         M,       int(sizeof(R)), CBIC_SCHED_LANE, &ws_bytes, &init, &iterate,
                            &finalize, 0,       lane_bufs<Sys>(), &iterate_final};
    return &L;
  }
};

}  // namespace cbic
