// Multilayer perceptrons of the biased initial-state selection and the actor
// warm start (paper Sec. II and III): FP32, evaluated as dense products on
// the matrix cores.  A wave evaluates the network for 16 samples at once: each
// layer is H_out^T = act(W^T H_in^T + b) in 16 x 16 x 4 FP32 MFMA tiles
// (neurons x samples), with the weights staged in LDS.  Lane l works for
// sample l % 16; its accumulator register r of neuron tile t holds neuron
// 16 t + 4 (l / 16) + r.  The next layer reads its K dimension in that same
// order (its weight rows are fetched permuted), so a layer's accumulators are
// the next layer's B operand as they stand: no data moves between layers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbic {

struct MlpDev {
  const float* __restrict__ p;  // packed parameters (see cbic_mlp)
  int in_dim, depth, out_dim, act, out_act;
  float out_scale;
};

typedef float nf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ nf4 mfma_f32_16x16x4(float a, float b, nf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// tanh(z) = 1 - 2 / (1 + e^(2z)) with the hardware exponential: a few
// instructions, no branches, absolute error a few units of 2^-24 (saturates
// to +-1, keeps NaN).
__device__ __forceinline__ float fast_tanh(float z) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * z));
}

// hidden activation, fixed at compile time: 0 tanh, 1 ELU, 2 ReLU
template <int ACT>
__device__ __forceinline__ float mlp_act(float z) {
  if constexpr (ACT == 0) return fast_tanh(z);
  else if constexpr (ACT == 1) return z > 0.0f ? z : __expf(z) - 1.0f;
  else return z > 0.0f ? z : 0.0f;
}

__device__ __forceinline__ float mlp_out(float z, int out_act, float scale) {
  if (out_act == 1) return scale * fast_tanh(z);
  // softplus log(1 + e^z) in the overflow-free form max(z, 0) + log(1 + e^-|z|)
  if (out_act == 2) return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
  return z;
}

// LDS image of a network (floats).  Row strides are padded so that the four
// lane groups of a wave (l / 16) read disjoint LDS banks: the input layer's
// rows (one per group) by W + 16, hidden rows (four apart per group) by W + 4,
// output rows by 20.
//   W0 [in4][W + 16], b0 [W], then per hidden layer Wl [W][W + 4], bl [W],
//   then Wo [W][20] (columns >= out_dim zero), bo [16] (zero-padded).
// in4 = in_dim rounded up to a multiple of 4; rows >= in_dim are zero.
struct MlpLds {
  int W, in4, depth, out_dim;
  __host__ __device__ int s0() const { return W + 16; }
  __host__ __device__ int sh() const { return W + 4; }
  __host__ __device__ int b0() const { return in4 * s0(); }
  __host__ __device__ int hid(int l) const { return b0() + W + (l - 1) * (W * sh() + W); }  // l >= 1
  __host__ __device__ int out() const { return hid(depth); }
  __host__ __device__ int bout() const { return out() + W * 20; }
  __host__ __device__ int total() const { return bout() + 16; }
};

__host__ __device__ inline MlpLds mlp_lds(int in_dim, int W, int depth, int out_dim) {
  return MlpLds{W, (in_dim + 3) & ~3, depth, out_dim};
}

// Copy the packed parameters into the padded LDS image (whole workgroup).
__device__ inline void mlp_stage(const MlpDev& net, const MlpLds& L, float* lds) {
  const int W = L.W, in = net.in_dim, out = net.out_dim;
  const float* __restrict__ p = net.p;
  const int n0 = L.in4 * L.s0(), nh = (L.depth - 1) * (W * L.sh() + W);
  for (int i = threadIdx.x; i < L.total(); i += blockDim.x) {
    float v = 0.0f;
    if (i < n0) {
      const int r = i / L.s0(), c = i % L.s0();
      if (r < in && c < W) v = p[r * W + c];
    } else if (i < L.b0() + W) {
      v = p[in * W + (i - L.b0())];
    } else if (i < L.b0() + W + nh) {
      const int q = i - (L.b0() + W), l = q / (W * L.sh() + W), e = q % (W * L.sh() + W);
      const float* pl = p + in * W + W + l * (W * W + W);
      if (e < W * L.sh()) {
        const int r = e / L.sh(), c = e % L.sh();
        if (c < W) v = pl[r * W + c];
      } else {
        v = pl[W * W + (e - W * L.sh())];
      }
    } else {
      const float* po = p + in * W + W + (L.depth - 1) * (W * W + W);
      if (i < L.bout()) {
        const int r = (i - L.out()) / 20, c = (i - L.out()) % 20;
        if (c < out) v = po[r * out + c];
      } else {
        const int c = i - L.bout();
        if (c < out) v = po[W * out + c];
      }
    }
    lds[i] = v;
  }
  __syncthreads();
}

// The network for the wave's 16 samples.  feat(s, g) returns input feature
// 4 s + g of this lane's sample (zero past in_dim); IN4 > 0 fixes in4 at
// compile time (the loop over s is then unrolled, so feat may pick registers
// with a constant s).  Returns, in lane l, outputs 4 (l / 16) + r (r = 0..3)
// of sample l % 16 after the output map.
template <int W, int IN4, int ACT, class Feat>
__device__ __forceinline__ nf4 mlp_tile(const MlpDev& net, const MlpLds& L, const float* lds, Feat feat) {
  constexpr int NT = W / 16;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  nf4 h[NT];
  // input layer
  {
    const float* w = lds;
    const float* b = lds + L.b0();
#pragma unroll
    for (int t = 0; t < NT; ++t) h[t] = *reinterpret_cast<const nf4*>(b + 16 * t + 4 * g);
    auto kstep = [&](int s) {
      const float bv = feat(s, g);
      const float* row = w + (4 * s + g) * L.s0() + c;
#pragma unroll
      for (int t = 0; t < NT; ++t) h[t] = mfma_f32_16x16x4(row[16 * t], bv, h[t]);
    };
    if constexpr (IN4 > 0) {
#pragma unroll
      for (int s = 0; s < IN4 / 4; ++s) kstep(s);
    } else {
      for (int s = 0; s < L.in4 / 4; ++s) kstep(s);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) h[t][r] = mlp_act<ACT>(h[t][r]);
  }
  // hidden layers: K runs in the accumulators' neuron order
  for (int l = 1; l < L.depth; ++l) {
    const float* w = lds + L.hid(l);
    const float* b = w + W * L.sh();
    nf4 o[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) o[t] = *reinterpret_cast<const nf4*>(b + 16 * t + 4 * g);
#pragma unroll
    for (int s = 0; s < W / 4; ++s) {
      const float* row = w + (16 * (s >> 2) + 4 * g + (s & 3)) * L.sh() + c;
      const float bv = h[s >> 2][s & 3];
#pragma unroll
      for (int t = 0; t < NT; ++t) o[t] = mfma_f32_16x16x4(row[16 * t], bv, o[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) h[t][r] = mlp_act<ACT>(o[t][r]);
  }
  // output layer (16 padded outputs)
  const float* w = lds + L.out();
  nf4 y = *reinterpret_cast<const nf4*>(lds + L.bout() + 4 * g);
#pragma unroll
  for (int s = 0; s < W / 4; ++s) {
    const float* row = w + (16 * (s >> 2) + 4 * g + (s & 3)) * 20 + c;
    y = mfma_f32_16x16x4(row[0], h[s >> 2][s & 3], y);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = mlp_out(y[r], net.out_act, net.out_scale);
  return y;
}

}  // namespace cbic
