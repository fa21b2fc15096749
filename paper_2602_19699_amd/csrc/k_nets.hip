// Biased initial-state selection and the actor warm start (paper Sec. II,
// III-C/D): std-critic scoring of candidate initial states, selection of the
// N highest scores, and closed-loop rollouts of the system under the actor.
#include <cmath>
#include <cstring>

#include "dev_systems.hpp"
#include "nets.hpp"
#include "runtime.hpp"

namespace cbic {

namespace {

#define HIP_TRY(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
      return CBIC_E_HIP;                                                \
    }                                                                   \
  } while (0)

constexpr int kScoreWG = 256;
constexpr int kSelectWG = 1024;

// ------------------------------------------------------------------ scoring
// score[b] = net(x_b, tau_b) for one candidate per lane (FP64 inputs rounded
// to FP32, as the network computes in FP32).
template <int W>
__global__ void __launch_bounds__(kScoreWG) mlp_score(MlpDev net, int B, int n, const double* __restrict__ x,
                                                      const double* __restrict__ tau, float* __restrict__ score) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* xb = x + size_t(b) * n;
  mlp_eval<W, 0, 1>(
      net, [&](int i) { return i < n ? float(xb[i]) : float(tau[b]); },
      [&](int, float v) { score[b] = v; });
}

// out[b][:] = net(in[b][:]) for FP32 rows.
template <int W>
__global__ void __launch_bounds__(kScoreWG) mlp_rows(MlpDev net, int B, const float* __restrict__ in,
                                                     float* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float* ib = in + size_t(b) * net.in_dim;
  float* ob = out + size_t(b) * net.out_dim;
  mlp_eval<W, 0, 0>(net, [&](int i) { return ib[i]; }, [&](int o, float v) { ob[o] = v; });
}

// ------------------------------------------------------------------ selection
// Order-preserving key of a score: a larger score has a larger key; -0 and +0
// share a key; NaN gets the smallest key.
__device__ __forceinline__ uint32_t score_key(float s) {
  if (!(s == s)) return 0u;
  if (s == 0.0f) s = 0.0f;
  const uint32_t u = __float_as_uint(s);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exclusive prefix count of `flag` over the workgroup's threads (in thread
// order) and the workgroup's total; `wtot` holds one slot per wave.
__device__ __forceinline__ uint32_t block_scan(bool flag, uint32_t* wtot, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long bits = __ballot(flag);
  const uint32_t below = __popcll(bits & ((1ull << lane) - 1ull));
  if (lane == 0) wtot[wave] = __popcll(bits);
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int v = 0; v < kSelectWG / 64; ++v) {
    const uint32_t t = wtot[v];
    before += v < wave ? t : 0u;
    total += t;
  }
  __syncthreads();
  return before + below;
}

// The N highest scores of Bc, in ascending index order (equal scores: lower
// index first), by a radix select of the N-th largest key (11 + 11 + 10 bits)
// and an order-preserving compaction.  One workgroup; 1 <= N <= Bc.
__global__ void __launch_bounds__(kSelectWG) topn_select(const float* __restrict__ score, int Bc, int N,
                                                         int32_t* __restrict__ sel) {
  __shared__ uint32_t hist[2048];
  __shared__ uint32_t wtot[kSelectWG / 64];
  __shared__ uint32_t s_bin, s_left;
  const int t = threadIdx.x;
  uint32_t prefix = 0, mask = 0, left = uint32_t(N);
  for (int pass = 0; pass < 3; ++pass) {
    const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const uint32_t nb = pass < 2 ? 2048u : 1024u;
    for (uint32_t i = t; i < nb; i += kSelectWG) hist[i] = 0u;
    __syncthreads();
    for (int i = t; i < Bc; i += kSelectWG) {
      const uint32_t k = score_key(score[i]);
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & (nb - 1u)], 1u);
    }
    __syncthreads();
    if (t == 0) {
      // the bin holding the left-th largest remaining key, from the top
      uint32_t above = 0;
      int b = int(nb) - 1;
      for (; b > 0; --b) {
        if (above + hist[b] >= left) break;
        above += hist[b];
      }
      s_bin = uint32_t(b);
      s_left = left - above;
    }
    __syncthreads();
    prefix |= s_bin << shift;
    mask |= (nb - 1u) << shift;
    left = s_left;
    __syncthreads();
  }
  // prefix is the N-th largest key; `left` keys equal to it are taken
  uint32_t out_base = 0, tie_base = 0;
  for (int c = 0; c < Bc; c += kSelectWG) {
    const int i = c + t;
    const uint32_t k = i < Bc ? score_key(score[i]) : 0u;
    const bool gt = i < Bc && k > prefix;
    const bool eq = i < Bc && k == prefix;
    uint32_t eq_total, take_total;
    const uint32_t eq_rank = tie_base + block_scan(eq, wtot, eq_total);
    const bool take = gt || (eq && eq_rank < left);
    const uint32_t pos = out_base + block_scan(take, wtot, take_total);
    if (take && pos < uint32_t(N)) sel[pos] = i;
    out_base += take_total;
    tie_base += eq_total;
  }
}

// ------------------------------------------------------------------ actor rollout
// One instance per lane: u_k = actor(x_k, tau_k) in FP32, x_{k+1} = f(x_k, u_k)
// in FP64.  Outputs are zero past the horizon (all zero for a horizon outside
// 1..T_max).
template <class Sys, int W>
__global__ void __launch_bounds__(64) actor_rollout(const double* __restrict__ prm, MlpDev net, int B, int Tmax,
                                                    const int32_t* __restrict__ Tin, const double* __restrict__ x0,
                                                    double* __restrict__ U, double* __restrict__ X) {
  constexpr int N = Sys::N, M = Sys::M;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const typename Sys::template Model<double> mdl{prm};
  const int Tr = Tin ? Tin[b] : Tmax;
  const int T = (Tr < 1 || Tr > Tmax) ? 0 : Tr;
  double* Ub = U + size_t(b) * Tmax * M;
  double* Xb = X ? X + size_t(b) * (Tmax + 1) * N : nullptr;
  double x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = T > 0 ? x0[size_t(b) * N + i] : 0.0;
  if (Xb)
#pragma unroll
    for (int i = 0; i < N; ++i) Xb[i] = x[i];
  const float inv_T = 1.0f / float(Tmax);
  for (int k = 0; k < T; ++k) {
    const float tau = float(Tmax - T + k) * inv_T;
    double u[M];
    mlp_eval<W, N + 1, M>(
        net, [&](int i) { return i < N ? float(x[i < N ? i : 0]) : tau; }, [&](int o, float v) { u[o] = double(v); });
    double xn[N];
    mdl.dyn(x, u, xn);
#pragma unroll
    for (int i = 0; i < M; ++i) Ub[size_t(k) * M + i] = u[i];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = xn[i];
    if (Xb)
#pragma unroll
      for (int i = 0; i < N; ++i) Xb[size_t(k + 1) * N + i] = x[i];
  }
  for (int k = T; k < Tmax; ++k)
#pragma unroll
    for (int i = 0; i < M; ++i) Ub[size_t(k) * M + i] = 0.0;
  if (Xb)
    for (int k = T + 1; k <= Tmax; ++k)
#pragma unroll
      for (int i = 0; i < N; ++i) Xb[size_t(k) * N + i] = 0.0;
}

template <class Sys>
hipError_t launch_actor(const double* prm, const MlpDev& net, int width, int B, int Tmax, const int32_t* d_T,
                        const double* x0, double* U, double* X, hipStream_t st) {
  const dim3 grid((B + 63) / 64), block(64);
  if (width == 32)
    hipLaunchKernelGGL((actor_rollout<Sys, 32>), grid, block, 0, st, prm, net, B, Tmax, d_T, x0, U, X);
  else
    hipLaunchKernelGGL((actor_rollout<Sys, 64>), grid, block, 0, st, prm, net, B, Tmax, d_T, x0, U, X);
  return hipGetLastError();
}

int64_t param_count(const cbic_mlp& m) {
  const int64_t W = m.width;
  return m.in_dim * W + W + (m.depth - 1) * (W * W + W) + W * m.out_dim + m.out_dim;
}

cbic_status check_mlp(const cbic_mlp* m) {
  if (!m) {
    set_error("network description is NULL");
    return CBIC_E_INVALID;
  }
  if (m->in_dim < 1 || m->in_dim > 64 || (m->width != 32 && m->width != 64) || m->depth < 1 || m->depth > 4 ||
      m->out_dim < 1 || m->out_dim > 16 || m->act < CBIC_ACT_TANH || m->act > CBIC_ACT_RELU ||
      m->out_act < CBIC_OUT_LINEAR || m->out_act > CBIC_OUT_SOFTPLUS || !std::isfinite(m->out_scale)) {
    set_error("network must have in_dim 1..64, width 32 or 64, depth 1..4, out_dim 1..16, known activations "
              "and a finite out_scale");
    return CBIC_E_INVALID;
  }
  return CBIC_OK;
}

MlpDev dev_mlp(const cbic_mlp& m) {
  return MlpDev{m.params, m.in_dim, m.depth, m.out_dim, m.act, m.out_act, float(m.out_scale)};
}

}  // namespace
}  // namespace cbic

using namespace cbic;

extern "C" {

cbic_status cbic_mlp_param_count(const cbic_mlp* net, int64_t* count) {
  if (cbic_status st = check_mlp(net)) return st;
  if (!count) {
    set_error("count is NULL");
    return CBIC_E_INVALID;
  }
  *count = param_count(*net);
  return CBIC_OK;
}

cbic_status cbic_mlp_forward(cbic_context* ctx, const cbic_mlp* net, int32_t B, const float* d_in, float* d_out,
                             void* stream) {
  if (cbic_status st = check_mlp(net)) return st;
  if (!ctx || !net->params || (B > 0 && (!d_in || !d_out)) || B < 0) {
    set_error("ctx, params, d_in and d_out are required and B >= 0");
    return CBIC_E_INVALID;
  }
  if (B == 0) return CBIC_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*net);
  const dim3 grid((B + kScoreWG - 1) / kScoreWG), block(kScoreWG);
  if (net->width == 32) hipLaunchKernelGGL((mlp_rows<32>), grid, block, 0, st, d, B, d_in, d_out);
  else hipLaunchKernelGGL((mlp_rows<64>), grid, block, 0, st, d, B, d_in, d_out);
  HIP_TRY(hipGetLastError());
  return CBIC_OK;
}

cbic_status cbic_bic_select(cbic_context* ctx, const cbic_mlp* net, int32_t Bc, int32_t n, const double* d_x,
                            const double* d_tau, int32_t N, float* d_score, int32_t* d_sel, void* stream) {
  if (cbic_status st = check_mlp(net)) return st;
  if (!ctx || !net->params || Bc < 1 || n < 1 || N < 0 || N > Bc || !d_x || !d_score || (N > 0 && !d_sel)) {
    set_error("ctx, params, d_x, d_score and d_sel are required; Bc >= 1, n >= 1, 0 <= N <= Bc");
    return CBIC_E_INVALID;
  }
  if (net->in_dim != n + (d_tau ? 1 : 0) || net->out_dim != 1) {
    set_error("the std-critic must take %d inputs and give one output", n + (d_tau ? 1 : 0));
    return CBIC_E_INVALID;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*net);
  const dim3 grid((Bc + kScoreWG - 1) / kScoreWG), block(kScoreWG);
  if (net->width == 32) hipLaunchKernelGGL((mlp_score<32>), grid, block, 0, st, d, Bc, n, d_x, d_tau, d_score);
  else hipLaunchKernelGGL((mlp_score<64>), grid, block, 0, st, d, Bc, n, d_x, d_tau, d_score);
  HIP_TRY(hipGetLastError());
  if (N > 0) {
    hipLaunchKernelGGL(topn_select, dim3(1), dim3(kSelectWG), 0, st, d_score, Bc, N, d_sel);
    HIP_TRY(hipGetLastError());
  }
  return CBIC_OK;
}

cbic_status cbic_actor_rollout(cbic_context* ctx, const cbic_system* sys, const cbic_mlp* actor, int32_t B,
                               int32_t T_max, const int32_t* d_T, const double* d_x0, double* d_U, double* d_X,
                               void* stream) {
  if (cbic_status st = check_mlp(actor)) return st;
  if (!ctx || !sys || !actor->params || B < 1 || T_max < 1 || !d_x0 || !d_U) {
    set_error("ctx, sys, params, d_x0 and d_U are required; B, T_max >= 1");
    return CBIC_E_INVALID;
  }
  if (actor->in_dim != sys->n + 1 || actor->out_dim != sys->m) {
    set_error("the actor must take n + 1 = %d inputs and give m = %d outputs", sys->n + 1, sys->m);
    return CBIC_E_INVALID;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*actor);
  const int w = actor->width;
  hipError_t e;
  if (sys->kind == CBIC_SYS_POINT_MASS) {
    e = launch_actor<PointMass>(sys->d_prm, d, w, B, T_max, d_T, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_PLANAR3) {
    e = launch_actor<Arm3>(sys->d_prm, d, w, B, T_max, d_T, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_LQ && sys->n == 2 && sys->m == 1) {
    e = launch_actor<LinQuad<2, 1>>(sys->d_prm, d, w, B, T_max, d_T, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_LQ && sys->n == 4 && sys->m == 2) {
    e = launch_actor<LinQuad<4, 2>>(sys->d_prm, d, w, B, T_max, d_T, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_LQ && sys->n == 6 && sys->m == 3) {
    e = launch_actor<LinQuad<6, 3>>(sys->d_prm, d, w, B, T_max, d_T, d_x0, d_U, d_X, st);
  } else {
    set_error("no actor rollout for system kind %d (n=%d, m=%d)", sys->kind, sys->n, sys->m);
    return CBIC_E_UNSUPPORTED;
  }
  HIP_TRY(e);
  return CBIC_OK;
}

}  // extern "C"
