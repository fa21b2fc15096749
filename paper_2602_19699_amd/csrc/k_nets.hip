// Biased initial-state selection and the actor warm start (paper Sec. II,
// III-C/D): std-critic scoring of candidate initial states, selection of the
// N highest scores, and closed-loop rollouts of the system under the actor.
#include <cmath>
#include <cstring>
#include <mutex>

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

constexpr int kNetWG = 256;  // four waves of 16 samples

// Dynamic LDS beyond 64 KiB (the largest networks take up to 79 KiB of the
// CU's 160 KiB) has to be allowed per kernel before the launch.
template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(bytes));
}
constexpr int kSelectWG = 1024;

// score[b] = net(x_b, tau_b), tau_b = (T_max - T_b) / T_max (FP64 inputs
// rounded to FP32, as the network computes in FP32); without T the network
// takes the state alone.  16 candidates per wave.
template <int W, int ACT>
__global__ void __launch_bounds__(kNetWG) mlp_score(MlpDev net, MlpLds L, int B, int n,
                                                    const double* __restrict__ x, const int32_t* __restrict__ T,
                                                    int Tmax, float* __restrict__ score) {
  extern __shared__ float lds[];
  mlp_stage(net, L, lds);
  const int lane = threadIdx.x & 63;
  const int b = (blockIdx.x * (kNetWG / 64) + (threadIdx.x >> 6)) * 16 + (lane & 15);
  const bool valid = b < B;
  const double* xb = x + size_t(valid ? b : 0) * n;
  const float tau = (T && valid) ? float(Tmax - T[b]) * (1.0f / float(Tmax)) : 0.0f;
  const nf4 y = mlp_tile<W, 0, ACT>(net, L, lds, [&](int s, int g) {
    const int f = 4 * s + g;
    return !valid ? 0.0f : (f < n ? float(xb[f]) : (f == n && T ? tau : 0.0f));
  });
  if (valid && lane < 16) score[b] = y[0];
}

// out[b][:] = net(in[b][:]) for FP32 rows, 16 rows per wave.
template <int W, int ACT>
__global__ void __launch_bounds__(kNetWG) mlp_rows(MlpDev net, MlpLds L, int B, const float* __restrict__ in,
                                                   float* __restrict__ out) {
  extern __shared__ float lds[];
  mlp_stage(net, L, lds);
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int b = (blockIdx.x * (kNetWG / 64) + (threadIdx.x >> 6)) * 16 + (lane & 15);
  const bool valid = b < B;
  const float* ib = in + size_t(valid ? b : 0) * net.in_dim;
  const nf4 y = mlp_tile<W, 0, ACT>(net, L, lds, [&](int s, int gg) {
    const int f = 4 * s + gg;
    return valid && f < net.in_dim ? ib[f] : 0.0f;
  });
  if (valid)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * g + r < net.out_dim) out[size_t(b) * net.out_dim + 4 * g + r] = y[r];
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

// Exclusive prefix sum of v over the workgroup's WG threads (in thread
// order) and the workgroup's total; `wtot` holds one slot per wave.
template <int WG>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* wtot, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) {
    const uint32_t t = wtot[w];
    before += w < wave ? t : 0u;
    total += t;
  }
  __syncthreads();
  return before + inc - v;
}

// The N highest scores of Bc, in ascending index order (equal scores: lower
// index first): a radix select of the N-th largest key (11 + 11 + 10 bits)
// and an order-preserving compaction that also gathers the selected rows of
// x (n wide) and T.  The work is spread over blocks of kSelChunk keys; a
// one-block kernel between the histogram passes finds the digit.  Scratch
// (uint32): hist [2048], state {prefix, mask, left} at kSelState, then per
// block: greater count, equal count, output base, tie base.
constexpr int kSelWG = 256, kSelE = 16, kSelChunk = kSelWG * kSelE;
constexpr int kSelState = 2048, kSelBlocks = 2056;

__global__ void __launch_bounds__(kSelectWG) sel_init(uint32_t* __restrict__ sc, int N) {
  for (int i = threadIdx.x; i < 2048; i += kSelectWG) sc[i] = 0u;
  if (threadIdx.x == 0) {
    sc[kSelState] = 0u;
    sc[kSelState + 1] = 0u;
    sc[kSelState + 2] = uint32_t(N);
  }
}

__global__ void __launch_bounds__(kSelWG) sel_hist(const float* __restrict__ score, int Bc, uint32_t* __restrict__ sc,
                                                   int shift, uint32_t nb) {
  __shared__ uint32_t h[2048];
  const int t = threadIdx.x;
  for (uint32_t i = t; i < nb; i += kSelWG) h[i] = 0u;
  const uint32_t prefix = sc[kSelState], mask = sc[kSelState + 1];
  __syncthreads();
  const int base = blockIdx.x * kSelChunk;
  uint32_t k[kSelE];
#pragma unroll
  for (int j = 0; j < kSelE; ++j) {
    const int i = base + j * kSelWG + t;
    k[j] = i < Bc ? score_key(score[i]) : 0u;
  }
#pragma unroll
  for (int j = 0; j < kSelE; ++j)
    if (base + j * kSelWG + t < Bc && (k[j] & mask) == prefix) atomicAdd(&h[(k[j] >> shift) & (nb - 1u)], 1u);
  __syncthreads();
  for (uint32_t i = t; i < nb; i += kSelWG)
    if (h[i]) atomicAdd(&sc[i], h[i]);
}

// One block: the digit of the left-th largest remaining key.  Thread t owns
// bins 2t + 1 and 2t (bin t in the 1024-bin pass); the keys in the bins above
// them come from a suffix sum over the threads.  Clears the histogram.
__global__ void __launch_bounds__(kSelectWG) sel_find(uint32_t* __restrict__ sc, int shift, uint32_t nb) {
  __shared__ uint32_t wtot[kSelectWG / 64];
  __shared__ uint32_t s_bin, s_left;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t left = sc[kSelState + 2];
  const int per = int(nb) / kSelectWG;
  const int hi = per == 2 ? 2 * t + 1 : t;
  const uint32_t hh = sc[hi], hl = per == 2 ? sc[hi - 1] : 0u;
  const uint32_t mine = hh + hl;
  uint32_t inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_down(inc, o, 64);
    if (lane + o < 64) inc += u;
  }
  if (lane == 0) wtot[wave] = inc;
  if (t == 0) {
    s_bin = 0u;
    s_left = left;
  }
  __syncthreads();
  uint32_t above = inc - mine;
#pragma unroll
  for (int w = 0; w < kSelectWG / 64; ++w) above += w > wave ? wtot[w] : 0u;
  __syncthreads();
  if (above < left && left <= above + hh) {
    s_bin = uint32_t(hi);
    s_left = left - above;
  } else if (per == 2 && above + hh < left && left <= above + hh + hl) {
    s_bin = uint32_t(hi - 1);
    s_left = left - above - hh;
  }
  __syncthreads();
  for (uint32_t i = t; i < nb; i += kSelectWG) sc[i] = 0u;
  if (t == 0) {
    sc[kSelState] |= s_bin << shift;
    sc[kSelState + 1] |= (nb - 1u) << shift;
    sc[kSelState + 2] = s_left;
  }
}

// Per block: keys above the threshold key and keys equal to it.
__global__ void __launch_bounds__(kSelWG) sel_count(const float* __restrict__ score, int Bc,
                                                    uint32_t* __restrict__ sc, int G) {
  __shared__ uint32_t wtot[kSelWG / 64];
  const int t = threadIdx.x;
  const uint32_t thr = sc[kSelState];
  const int base = blockIdx.x * kSelChunk;
  uint32_t gt = 0, eq = 0;
#pragma unroll
  for (int j = 0; j < kSelE; ++j) {
    const int i = base + j * kSelWG + t;
    const uint32_t k = i < Bc ? score_key(score[i]) : 0u;
    gt += (i < Bc && k > thr) ? 1u : 0u;
    eq += (i < Bc && k == thr) ? 1u : 0u;
  }
  uint32_t tg, te;
  block_scan<kSelWG>(gt, wtot, tg);
  block_scan<kSelWG>(eq, wtot, te);
  if (t == 0) {
    sc[kSelBlocks + blockIdx.x] = tg;
    sc[kSelBlocks + G + blockIdx.x] = te;
  }
}

// One block: each block's first output position and first tie rank.
__global__ void __launch_bounds__(kSelectWG) sel_offsets(uint32_t* __restrict__ sc, int G) {
  __shared__ uint32_t wtot[kSelectWG / 64];
  const uint32_t left = sc[kSelState + 2];
  uint32_t out_run = 0, tie_run = 0;
  for (int c = 0; c < G; c += kSelectWG) {
    const int b = c + threadIdx.x;
    const uint32_t gt = b < G ? sc[kSelBlocks + b] : 0u, eq = b < G ? sc[kSelBlocks + G + b] : 0u;
    uint32_t te, tt;
    const uint32_t tie0 = tie_run + block_scan<kSelectWG>(eq, wtot, te);
    const uint32_t ties_taken = tie0 >= left ? 0u : min(eq, left - tie0);
    const uint32_t out0 = out_run + block_scan<kSelectWG>(gt + ties_taken, wtot, tt);
    if (b < G) {
      sc[kSelBlocks + 2 * G + b] = out0;
      sc[kSelBlocks + 3 * G + b] = tie0;
    }
    out_run += tt;
    tie_run += te;
  }
}

// Per block: write the selected indices (and rows) in ascending index order;
// thread t handles keys [base + E t, base + E t + E).
__global__ void __launch_bounds__(kSelWG) sel_scatter(const float* __restrict__ score, int Bc, int N,
                                                      int32_t* __restrict__ sel, int n, const double* __restrict__ x,
                                                      const int32_t* __restrict__ T, double* __restrict__ xs,
                                                      int32_t* __restrict__ Ts, const uint32_t* __restrict__ sc,
                                                      int G) {
  __shared__ uint32_t wtot[kSelWG / 64];
  const int t = threadIdx.x;
  const uint32_t thr = sc[kSelState], left = sc[kSelState + 2];
  const int i0 = blockIdx.x * kSelChunk + kSelE * t;
  uint32_t gt = 0, eq = 0, neq = 0;
#pragma unroll
  for (int j = 0; j < kSelE; ++j) {
    const int i = i0 + j;
    const uint32_t k = i < Bc ? score_key(score[i]) : 0u;
    if (i < Bc && k > thr) gt |= 1u << j;
    if (i < Bc && k == thr) {
      eq |= 1u << j;
      ++neq;
    }
  }
  uint32_t te, tt;
  uint32_t rank = sc[kSelBlocks + 3 * G + blockIdx.x] + block_scan<kSelWG>(neq, wtot, te);
  uint32_t take = gt;
#pragma unroll
  for (int j = 0; j < kSelE; ++j)
    if ((eq >> j) & 1u) {
      if (rank < left) take |= 1u << j;
      ++rank;
    }
  uint32_t pos = sc[kSelBlocks + 2 * G + blockIdx.x] + block_scan<kSelWG>(__popc(take), wtot, tt);
#pragma unroll
  for (int j = 0; j < kSelE; ++j)
    if ((take >> j) & 1u) {
      const int i = i0 + j;
      if (pos < uint32_t(N)) {
        sel[pos] = i;
        if (xs)
          for (int q = 0; q < n; ++q) xs[size_t(pos) * n + q] = x[size_t(i) * n + q];
        if (Ts) Ts[pos] = T[i];
      }
      ++pos;
    }
}

// ------------------------------------------------------------------ actor rollout
// 16 instances per wave, four lanes per instance: the lanes of an instance
// keep its state and step the FP64 dynamics redundantly, and the wave
// evaluates u_k = actor(x_k, tau_k) for its 16 instances on the matrix cores.
// The wave runs until its longest horizon, so ragged batches are taken in
// horizon order (perm, longest first) and a wave holds similar horizons.
// Outputs are zero past each horizon (all zero for a horizon outside
// 1..T_max).
template <class Sys, int W, int ACT>
__global__ void __launch_bounds__(kNetWG) actor_rollout(const double* __restrict__ prm, MlpDev net, MlpLds L, int B,
                                                        int Tmax, const int32_t* __restrict__ Tin,
                                                        const int32_t* __restrict__ perm,
                                                        const double* __restrict__ x0, double* __restrict__ U,
                                                        double* __restrict__ X) {
  constexpr int N = Sys::N, M = Sys::M;
  constexpr int IN4 = (N + 1 + 3) & ~3;
  static_assert(M <= 4, "outputs of lane group 0");
  extern __shared__ float lds[];
  mlp_stage(net, L, lds);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int slot = (blockIdx.x * (kNetWG / 64) + (threadIdx.x >> 6)) * 16 + c;
  const bool valid = slot < B;
  const int b = valid ? (perm ? perm[slot] : slot) : 0;
  const typename Sys::template Model<double> mdl{prm};
  const int Tr = valid ? (Tin ? Tin[b] : Tmax) : 0;
  const int T = (Tr < 1 || Tr > Tmax) ? 0 : Tr;
  int Tw = T;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) Tw = max(Tw, __shfl_xor(Tw, o, 64));
  const bool writer = valid && g == 0;
  double* Ub = U + size_t(valid ? b : 0) * Tmax * M;
  double* Xb = X ? X + size_t(valid ? b : 0) * (Tmax + 1) * N : nullptr;
  double x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = T > 0 ? x0[size_t(b) * N + i] : 0.0;
  if (writer && Xb)
#pragma unroll
    for (int i = 0; i < N; ++i) Xb[i] = x[i];
  const float inv_T = 1.0f / float(Tmax);
  for (int k = 0; k < Tw; ++k) {
    float f[IN4];
#pragma unroll
    for (int i = 0; i < IN4; ++i) f[i] = i < N ? float(x[i < N ? i : 0]) : (i == N ? float(Tmax - T + k) * inv_T : 0.0f);
    const nf4 y = mlp_tile<W, IN4, ACT>(net, L, lds, [&](int s, int gg) {
      return gg == 0 ? f[4 * s] : (gg == 1 ? f[4 * s + 1] : (gg == 2 ? f[4 * s + 2] : f[4 * s + 3]));
    });
    // outputs 0..M-1 of instance c sit in lane c (group 0), registers 0..M-1
    double u[M];
#pragma unroll
    for (int o = 0; o < M; ++o) u[o] = double(__shfl(y[o], c, 64));
    if (k < T) {
      double xn[N];
      mdl.dyn(x, u, xn);
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = xn[i];
      if (writer) {
#pragma unroll
        for (int i = 0; i < M; ++i) Ub[size_t(k) * M + i] = u[i];
        if (Xb)
#pragma unroll
          for (int i = 0; i < N; ++i) Xb[size_t(k + 1) * N + i] = x[i];
      }
    }
  }
  if (writer) {
    for (int k = T; k < Tmax; ++k)
#pragma unroll
      for (int i = 0; i < M; ++i) Ub[size_t(k) * M + i] = 0.0;
    if (Xb)
      for (int k = T + 1; k <= Tmax; ++k)
#pragma unroll
        for (int i = 0; i < N; ++i) Xb[size_t(k) * N + i] = 0.0;
  }
}

template <class Sys, int W, int ACT>
hipError_t launch_actor_k(const double* prm, const MlpDev& net, const MlpLds& L, int B, int Tmax,
                          const int32_t* d_T, const int32_t* perm, const double* x0, double* U, double* X,
                          hipStream_t st) {
  const dim3 grid((B + kNetWG / 4 - 1) / (kNetWG / 4)), block(kNetWG);
  const size_t lds = size_t(L.total()) * sizeof(float);
  hipError_t e = allow_lds(actor_rollout<Sys, W, ACT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((actor_rollout<Sys, W, ACT>), grid, block, lds, st, prm, net, L, B, Tmax, d_T, perm, x0, U, X);
  return hipGetLastError();
}

template <class Sys>
hipError_t launch_actor(const double* prm, const MlpDev& net, const MlpLds& L, int B, int Tmax, const int32_t* d_T,
                        const int32_t* perm, const double* x0, double* U, double* X, hipStream_t st) {
#define CBIC_ACTOR(WW, AA) launch_actor_k<Sys, WW, AA>(prm, net, L, B, Tmax, d_T, perm, x0, U, X, st)
  if (L.W == 32) return net.act == 0 ? CBIC_ACTOR(32, 0) : (net.act == 1 ? CBIC_ACTOR(32, 1) : CBIC_ACTOR(32, 2));
  return net.act == 0 ? CBIC_ACTOR(64, 0) : (net.act == 1 ? CBIC_ACTOR(64, 1) : CBIC_ACTOR(64, 2));
#undef CBIC_ACTOR
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
  (void)hipGetLastError();  // launch errors below are this call's, not a stale one
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*net);
  const MlpLds L = mlp_lds(net->in_dim, net->width, net->depth, net->out_dim);
  const dim3 grid((B + kNetWG / 4 - 1) / (kNetWG / 4)), block(kNetWG);
  const size_t lds = size_t(L.total()) * sizeof(float);
#define CBIC_ROWS(WW, AA)                                                                  \
  do {                                                                                     \
    HIP_TRY(allow_lds(mlp_rows<WW, AA>, lds));                                             \
    hipLaunchKernelGGL((mlp_rows<WW, AA>), grid, block, lds, st, d, L, B, d_in, d_out);    \
  } while (0)
  if (net->width == 32) {
    if (net->act == 0) CBIC_ROWS(32, 0);
    else if (net->act == 1) CBIC_ROWS(32, 1);
    else CBIC_ROWS(32, 2);
  } else {
    if (net->act == 0) CBIC_ROWS(64, 0);
    else if (net->act == 1) CBIC_ROWS(64, 1);
    else CBIC_ROWS(64, 2);
  }
#undef CBIC_ROWS
  HIP_TRY(hipGetLastError());
  return CBIC_OK;
}

cbic_status cbic_bic_select(cbic_context* ctx, const cbic_mlp* net, int32_t Bc, int32_t n, const double* d_x,
                            const int32_t* d_T, int32_t T_max, int32_t N, float* d_score, int32_t* d_sel,
                            double* d_x_sel, int32_t* d_T_sel, void* stream) {
  if (cbic_status st = check_mlp(net)) return st;
  if (!ctx || !net->params || Bc < 1 || n < 1 || N < 0 || N > Bc || !d_x || !d_score || (N > 0 && !d_sel) ||
      (d_T && T_max < 1) || (d_T_sel && !d_T)) {
    set_error("ctx, params, d_x, d_score and d_sel are required (d_T with d_T_sel, T_max >= 1 with d_T); "
              "Bc >= 1, n >= 1, 0 <= N <= Bc");
    return CBIC_E_INVALID;
  }
  if (net->in_dim != n + (d_T ? 1 : 0) || net->out_dim != 1) {
    set_error("the std-critic must take %d inputs and give one output", n + (d_T ? 1 : 0));
    return CBIC_E_INVALID;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  (void)hipGetLastError();  // launch errors below are this call's, not a stale one
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*net);
  const MlpLds L = mlp_lds(net->in_dim, net->width, net->depth, net->out_dim);
  const dim3 grid((Bc + kNetWG / 4 - 1) / (kNetWG / 4)), block(kNetWG);
  const size_t lds = size_t(L.total()) * sizeof(float);
#define CBIC_SCORE(WW, AA)                                                                           \
  do {                                                                                               \
    HIP_TRY(allow_lds(mlp_score<WW, AA>, lds));                                                      \
    hipLaunchKernelGGL((mlp_score<WW, AA>), grid, block, lds, st, d, L, Bc, n, d_x, d_T, T_max, d_score); \
  } while (0)
  if (net->width == 32) {
    if (net->act == 0) CBIC_SCORE(32, 0);
    else if (net->act == 1) CBIC_SCORE(32, 1);
    else CBIC_SCORE(32, 2);
  } else {
    if (net->act == 0) CBIC_SCORE(64, 0);
    else if (net->act == 1) CBIC_SCORE(64, 1);
    else CBIC_SCORE(64, 2);
  }
#undef CBIC_SCORE
  HIP_TRY(hipGetLastError());
  if (N > 0) {
    const int G = (Bc + kSelChunk - 1) / kSelChunk;
    std::lock_guard<std::mutex> lk(ctx->mu);
    void* aux = nullptr;
    if (cbic_status e = context_aux(ctx, (size_t(kSelBlocks) + 4 * size_t(G)) * sizeof(uint32_t), &aux)) return e;
    uint32_t* sc = static_cast<uint32_t*>(aux);
    if (ctx->have_last && ctx->last_stream != st) HIP_TRY(hipStreamWaitEvent(st, ctx->done_ev, 0));
    hipLaunchKernelGGL(sel_init, dim3(1), dim3(kSelectWG), 0, st, sc, N);
    for (int pass = 0; pass < 3; ++pass) {
      const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
      const uint32_t nb = pass < 2 ? 2048u : 1024u;
      hipLaunchKernelGGL(sel_hist, dim3(G), dim3(kSelWG), 0, st, d_score, Bc, sc, shift, nb);
      hipLaunchKernelGGL(sel_find, dim3(1), dim3(kSelectWG), 0, st, sc, shift, nb);
    }
    hipLaunchKernelGGL(sel_count, dim3(G), dim3(kSelWG), 0, st, d_score, Bc, sc, G);
    hipLaunchKernelGGL(sel_offsets, dim3(1), dim3(kSelectWG), 0, st, sc, G);
    hipLaunchKernelGGL(sel_scatter, dim3(G), dim3(kSelWG), 0, st, d_score, Bc, N, d_sel, n, d_x, d_T, d_x_sel,
                       d_T_sel, sc, G);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ctx->done_ev, st));
    ctx->last_stream = st;
    ctx->have_last = true;
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
  (void)hipGetLastError();  // launch errors below are this call's, not a stale one
  hipStream_t st = static_cast<hipStream_t>(stream);
  const MlpDev d = dev_mlp(*actor);
  const MlpLds w = mlp_lds(actor->in_dim, actor->width, actor->depth, actor->out_dim);
  const bool known = sys->kind == CBIC_SYS_POINT_MASS || sys->kind == CBIC_SYS_PLANAR3 ||
                     (sys->kind == CBIC_SYS_LQ && ((sys->n == 2 && sys->m == 1) || (sys->n == 4 && sys->m == 2) ||
                                                   (sys->n == 6 && sys->m == 3)));
  if (!known) {
    set_error("no actor rollout for system kind %d (n=%d, m=%d)", sys->kind, sys->n, sys->m);
    return CBIC_E_UNSUPPORTED;
  }
  // a ragged batch is taken in horizon order (sorted on the device)
  std::lock_guard<std::mutex> lk(ctx->mu);
  int32_t* perm = nullptr;
  if (d_T) {
    const size_t hb = (size_t(T_max) + 1) * 4, hb_al = (hb + 255) / 256 * 256;
    void* aux = nullptr;
    if (cbic_status e = context_aux(ctx, hb_al + size_t(B) * 4, &aux)) return e;
    if (ctx->have_last && ctx->last_stream != st) HIP_TRY(hipStreamWaitEvent(st, ctx->done_ev, 0));
    int32_t* hist = static_cast<int32_t*>(aux);
    perm = reinterpret_cast<int32_t*>(static_cast<char*>(aux) + hb_al);
    HIP_TRY(launch_horizon_sort(d_T, B, T_max, hist, perm, st));
  }
  hipError_t e;
  if (sys->kind == CBIC_SYS_POINT_MASS) {
    e = launch_actor<PointMass>(sys->d_prm, d, w, B, T_max, d_T, perm, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_PLANAR3) {
    e = launch_actor<Arm3>(sys->d_prm, d, w, B, T_max, d_T, perm, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_LQ && sys->n == 2 && sys->m == 1) {
    e = launch_actor<LinQuad<2, 1>>(sys->d_prm, d, w, B, T_max, d_T, perm, d_x0, d_U, d_X, st);
  } else if (sys->kind == CBIC_SYS_LQ && sys->n == 4 && sys->m == 2) {
    e = launch_actor<LinQuad<4, 2>>(sys->d_prm, d, w, B, T_max, d_T, perm, d_x0, d_U, d_X, st);
  } else {
    e = launch_actor<LinQuad<6, 3>>(sys->d_prm, d, w, B, T_max, d_T, perm, d_x0, d_U, d_X, st);
  }
  HIP_TRY(e);
  if (perm) {
    HIP_TRY(hipEventRecord(ctx->done_ev, st));
    ctx->last_stream = st;
    ctx->have_last = true;
  }
  return CBIC_OK;
}

}  // extern "C"
