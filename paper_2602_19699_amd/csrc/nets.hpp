// Multilayer perceptrons of the biased initial-state selection and the actor
// warm start (paper Sec. II and III): FP32, one sample per lane.  Every lane of
// a wave reads the same parameter at the same time, so the parameter loads
// are wave-uniform (the compiler serves them through scalar loads) and the
// hidden activations stay in registers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbic {

struct MlpDev {
  const float* __restrict__ p;  // packed parameters (see cbic_mlp)
  int in_dim, depth, out_dim, act, out_act;
  float out_scale;
};

__device__ __forceinline__ float mlp_act(float z, int act) {
  if (act == 0) return tanhf(z);
  if (act == 1) return z > 0.0f ? z : expm1f(z);  // ELU
  return z > 0.0f ? z : 0.0f;                     // ReLU
}

__device__ __forceinline__ float mlp_out(float z, int out_act, float scale) {
  if (out_act == 1) return scale * tanhf(z);
  // softplus log(1 + e^z) in the overflow-free form max(z, 0) + log(1 + e^-|z|)
  if (out_act == 2) return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
  return z;
}

// y = net(x) for one sample.  W is the hidden width; IN (> 0) fixes the input
// width at compile time, otherwise net.in_dim is used; OUT likewise for the
// output.  in(i) returns input i; out(o, v) receives output o.
template <int W, int IN, int OUT, class In, class Out>
__device__ __forceinline__ void mlp_eval(const MlpDev& net, In in, Out out) {
  const int in_dim = IN > 0 ? IN : net.in_dim;
  const int out_dim = OUT > 0 ? OUT : net.out_dim;
  const float* __restrict__ p = net.p;
  float h[W];
#pragma unroll
  for (int j = 0; j < W; ++j) h[j] = p[in_dim * W + j];
  if constexpr (IN > 0) {
#pragma unroll
    for (int i = 0; i < IN; ++i) {
      const float xi = in(i);
#pragma unroll
      for (int j = 0; j < W; ++j) h[j] += xi * p[i * W + j];
    }
  } else {
    for (int i = 0; i < in_dim; ++i) {
      const float xi = in(i);
#pragma unroll
      for (int j = 0; j < W; ++j) h[j] += xi * p[i * W + j];
    }
  }
#pragma unroll
  for (int j = 0; j < W; ++j) h[j] = mlp_act(h[j], net.act);
  p += in_dim * W + W;
  for (int l = 1; l < net.depth; ++l) {
    float g[W];
#pragma unroll
    for (int j = 0; j < W; ++j) g[j] = p[W * W + j];
#pragma unroll
    for (int i = 0; i < W; ++i)
#pragma unroll
      for (int j = 0; j < W; ++j) g[j] += h[i] * p[i * W + j];
#pragma unroll
    for (int j = 0; j < W; ++j) h[j] = mlp_act(g[j], net.act);
    p += W * W + W;
  }
  auto emit = [&](int o) {
    float z = p[W * out_dim + o];
#pragma unroll
    for (int j = 0; j < W; ++j) z += h[j] * p[j * out_dim + o];
    out(o, mlp_out(z, net.out_act, net.out_scale));
  };
  if constexpr (OUT > 0) {
#pragma unroll
    for (int o = 0; o < OUT; ++o) emit(o);
  } else {
    for (int o = 0; o < out_dim; ++o) emit(o);
  }
}

}  // namespace cbic
